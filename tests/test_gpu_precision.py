"""Reduced-precision population storage (FP16 / BF16 normalized deviations,
FP32 compute) against the FP64 oracle, with FP32 storage alongside.

The errors are stated, not a parity claim: each step rounds every stored
deviation g = (f - w) / w once (unit roundoff 2^-11 in FP16, 2^-8 in BF16),
and the collision neither amplifies the conserved moments nor the damped
non-equilibrium part, so the error of h = f - w grows at most linearly with
the number of steps.  The asserted bounds are that linear growth,
n * u * |h|_max, with a factor 4 for the reconstruction and moment sums;
the measured errors are printed.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
UNIT = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}

CASES = {
    "tgv_sphere_32": (lambda: W.config1(), 100),
    "rotor_channel_256x128x128": (lambda: W.config2(), 10),
    "rotor_wake_256x128x96": (lambda: W.config3(coarse=True), 20),
    "rotor_adjoint_128x64x64": (lambda: W.config4(), 50),
}

_oracle_cache = {}


def _oracle(case):
    if case not in _oracle_cache:
        make, n = CASES[case]
        w = make()
        o = O.setup(w, threads=THREADS)
        o.step(n)
        rho, u = o.moments()
        _oracle_cache[case] = (o.get_populations(), rho, u, o.history())
    return _oracle_cache[case]


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_storage_error_vs_fp64_oracle(case, storage):
    import torch
    from paper_2510_13726_amd import hlbm
    make, n = CASES[case]
    w = make()
    print(f"[precision] {case} {storage} {n} steps", flush=True)
    lat = hlbm.setup(w, storage=storage, diag_every=1)
    lat.step(n)
    hg = lat.get_populations().cpu().numpy()
    rho_g, u_g = (t.cpu().numpy().astype(np.float64) for t in lat.moments())
    hist_g = lat.history()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ho, rho_o, u_o, hist_o = _oracle(case)
    e_h = rel(hg, ho)
    e_u = rel(u_g, u_o)
    e_rho = float(np.abs(rho_g - rho_o).max())
    tags = [1] if w.sphere is not None else [r.tag for r in w.rotors]
    cols = np.concatenate([np.arange(1 + 6 * (t - 1), 7 + 6 * (t - 1)) for t in tags])
    e_F = rel(hist_g[:, cols], hist_o[:, cols])
    e_m = float(np.abs(hist_g[:, 0] - hist_o[:, 0]).max() / w.cells)
    print(f"[precision] {case} {storage}: h {e_h:.3e} u {e_u:.3e} rho(abs) {e_rho:.3e} "
          f"F,T {e_F:.3e} mass/cell {e_m:.3e}", flush=True)
    bound = 4.0 * n * UNIT[storage] + (1e-6 if storage == "f32" else 0.0)
    assert np.isfinite(hg).all()
    assert e_h < bound
    assert e_u < 4 * bound
