"""HIP path vs the FP64 oracle at the full sizes of the rotor workloads.  The
slab cases run the launch configuration the benchmark times (mass reduction
and finite check every step) and also compare the force and torque records
of the rotors inside the compared window.

The 256x128x128 channel fits the oracle whole.  The 1024x512x384 wake and the
1536x768x256 rotor array do not; there the oracle runs an x-slab of the
domain (all of y and z) for a few steps.  One step moves information at most
five cells (one by streaming, four by the wall-model probe stencil: probe at
most y_s = 3 cells off the wall cell, plus the trilinear corner), so after n
steps the slab's cells farther than 6n + 2 planes from its cut faces hold
the same values as the full run; those cells are compared.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W
from parity_metrics import force_torque_error

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}
# FP16 / BF16 storage: stated errors under the linear-growth bound of the
# storage rounding, 4 n u (unit roundoff u = 2^-11, 2^-8)
UNIT = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def _tol(storage, n):
    return TOL[storage] if storage in TOL else 4.0 * n * UNIT[storage]
THREADS = min(16, os.cpu_count() or 1)


def _hl():
    from paper_2510_13726_amd import hlbm
    return hlbm


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _free(lat):
    import torch
    lat.close()
    del lat
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage,diag", [("f64", 1), ("f32", 0), ("f32", 1)])
def test_rotor_channel_full_domain(storage, diag):
    """256x128x128 channel, rotor R = 40 with the wall model, 6 steps."""
    hl = _hl()
    w = W.config2()
    n = 6
    print(f"[fullsize] {w.name} {storage} diag={diag} {n} steps", flush=True)
    lat = hl.setup(w, storage=storage, diag_every=diag)
    lat.step(n)
    hg = lat.get_populations().cpu().numpy()
    it_g, nw_g = lat.wall_stats()
    hist_g = lat.history() if diag else None
    safe_g = lat.wall_safeguards()
    _free(lat)
    o = O.setup(w, threads=THREADS)
    o.step(n)
    ho = o.get_populations()
    e = rel(hg, ho)
    print(f"[fullsize] {w.name} {storage}: h rel err {e:.3e}", flush=True)
    assert e < TOL[storage]
    halv, caps, near = o.wall_safeguards()
    print(f"[fullsize] oracle Newton halvings {halv}, caps {caps}; slips within [0.5e-6, 2e-6]: {near}", flush=True)
    assert (halv, caps) == (0, 0)
    if diag:
        eF, eT = force_torque_error(hist_g, o.history(), o.history_scale())
        print(f"[fullsize] F err {eF:.3e} T err {eT:.3e}; newton {it_g}/{o.newton_stats()[0]} wall cells {nw_g}",
              flush=True)
        assert eF < TOL[storage] and eT < TOL[storage]
        assert safe_g == (0, 0)
        # equal Newton counts are an FP64 property: FP32 probe velocities
        # may flip a stop decision
        if storage == "f64":
            assert (it_g, nw_g) == o.newton_stats()
        assert nw_g > 1000


def _slab_case(w, x0, length, n, storage, box):
    """Run `w` on the GPU for n steps and the x-slab [x0, x0 + length) on the
    oracle; compare the slab's interior cells inside the y-z window `box`, and
    the force / torque records of the rotors whose boxes lie in the slab's
    interior (their cells hold the same values in both runs)."""
    hl = _hl()
    m = 6 * n + 2
    lo = x0 + (m if x0 != 0 else 0)
    hi = x0 + length - m
    assert hi > lo
    (y0, y1), (z0, z1) = box
    zz, yy, xx = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(lo, hi), indexing="ij")
    cells = ((zz * w.ny + yy) * w.nx + xx).reshape(-1).astype(np.int64)
    print(f"[fullsize] {w.name} D3Q{getattr(w, 'q', 27)} {storage}: {n} steps, slab x [{x0}, {x0 + length}), "
          f"compare x [{lo}, {hi}) ({cells.size} cells)", flush=True)
    lat = hl.setup(w, storage=storage, diag_every=1, check_nonfinite=1)
    lat.step(n)
    hg = lat.get_populations_at(cells).cpu().numpy()          # [cells][27]
    hist_g = lat.history()
    _free(lat)
    s = W.x_slab(w, x0, length)
    o = O.setup(s, threads=THREADS)
    o.step(n)
    ho = o.get_populations()                                   # [27][slab cells]
    lc = ((zz * s.ny + yy) * s.nx + (xx - x0)).reshape(-1)
    ho = ho[:, lc].T
    e = rel(hg, ho)
    tol = _tol(storage, n)
    halv, caps, near = o.wall_safeguards()
    print(f"[fullsize] {w.name} {storage}: h rel err {e:.3e} (max |h| {np.abs(ho).max():.3e}); "
          f"slab newton {o.newton_stats()}, halvings {halv}, caps {caps}, slips within [0.5e-6, 2e-6]: {near}",
          flush=True)
    assert (halv, caps) == (0, 0)
    if e >= tol:
        err = np.abs(hg - ho).max(axis=1)
        bad = np.argsort(-err)[:8]
        for b in bad:
            c = int(cells[b])
            x, y, z = c % w.nx, (c // w.nx) % w.ny, c // (w.nx * w.ny)
            near = min(((x - r.center[0]) ** 2 + (y - r.center[1]) ** 2 + (z - r.center[2]) ** 2) ** 0.5
                       for r in w.rotors) if w.rotors else -1
            print(f"[fullsize]   cell ({x},{y},{z}) err {err[b]:.3e} dist to nearest rotor centre {near:.1f}",
                  flush=True)
        print(f"[fullsize]   cells above tolerance: {(err > tol * np.abs(ho).max()).sum()}", flush=True)
    # rotors whose marking boxes (centre +- 6 cells along the x axis) lie in
    # the compared planes
    tags = {r.tag for r in w.rotors if lo + 6 <= r.center[0] < hi - 6}
    if tags:
        eF, eT = force_torque_error(hist_g, o.history(), o.history_scale(), tags)
        print(f"[fullsize] {w.name} {storage}: tags {sorted(tags)} F err {eF:.3e} T err {eT:.3e}", flush=True)
        assert eF < tol and eT < tol
    return e, o, tags


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_wake_rotor_slab(storage):
    """1024x512x384 wake workload (rotor R = 120, inflow turbulence), slab
    around the rotor plane."""
    w = W.config3()
    n = 4
    xc = int(w.rotors[0].center[0])
    e, o, tags = _slab_case(w, xc - 16 - (6 * n + 2), 32 + 2 * (6 * n + 2), n, storage, ((128, 384), (64, 320)))
    assert o.newton_stats()[1] > 1000 and tags == {1}
    assert e < _tol(storage, n)


def test_wake_inflow_slab():
    """1024x512x384 wake workload: slab at the inlet (turbulent equilibrium
    inflow drawn from the counter-based generator of every (step, y, z))."""
    w = W.config3()
    n = 4
    e, _, _ = _slab_case(w, 0, 24 + 6 * n + 2, n, "f32", ((0, 512), (100, 160)))
    assert e < TOL["f32"]


@pytest.mark.parametrize("storage,q", [("f32", 27), ("f16", 27), ("bf16", 27), ("f32", 19), ("f16", 19)])
def test_rotor_array_slab(storage, q):
    """1536x768x256 array of 8 rotors (R = 48): slab around the first column
    of two rotors with different phases, in each storage type and velocity
    set the benchmark times."""
    w = W.config5()
    w.q = q
    n = 4
    xc = int(w.rotors[0].center[0])
    e, o, tags = _slab_case(w, xc - 10 - (6 * n + 2), 20 + 2 * (6 * n + 2), n, storage, ((250, 520), (70, 190)))
    assert o.newton_stats()[1] > 1000 and len(tags) == 2
    assert e < _tol(storage, n)


def test_rotor_array_slab_reference_grid():
    """The same slab with every rotor's body on a half-cell reference grid
    (hub sphere and capsule blades of the same parameters), as the benchmark
    times it: one grid shared by the eight rotors."""
    w = W.config5()
    g = W.capsule_rotor_grid(w.rotors[0], spacing=0.5, eps_h=w.params.eps_h)
    for r in w.rotors:
        r.grid = g
    n = 4
    xc = int(w.rotors[0].center[0])
    e, o, tags = _slab_case(w, xc - 10 - (6 * n + 2), 20 + 2 * (6 * n + 2), n, "f32", ((250, 520), (70, 190)))
    assert o.newton_stats()[1] > 1000 and len(tags) == 2
    assert e < TOL["f32"]
