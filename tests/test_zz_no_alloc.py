"""hlbm_lattice_create_static (the lattice on the library's static device
workspace, for callers that cannot allocate) against hlbm_lattice_create with
a caller workspace on the same inputs: bit-identical populations and force
history, on two lattices in a row, the second smaller; oversized lattices
and a second concurrent static lattice are refused."""
import numpy as np
import pytest

from paper_2510_13726_amd import workloads as W

pytestmark = pytest.mark.gpu


def _hl():
    from paper_2510_13726_amd import hlbm
    return hlbm


def _run(w, storage, steps, static):
    hl = _hl()
    lat = hl.setup(w, storage=storage, check_nonfinite=1, static_workspace=static)
    lat.step(steps)
    h = lat.get_populations().cpu().numpy()
    hist = lat.history()
    stats = lat.wall_stats()
    lat.close()
    return h, hist, stats


@pytest.mark.parametrize("case", [(56, 44, 40, 10.0, "f64", 9), (40, 32, 32, 8.0, "f32", 7)])
def test_static_workspace_matches_caller_workspace(case):
    nx, ny, nz, R, storage, steps = case
    print(f"[no-alloc] {nx}x{ny}x{nz} {storage} {steps} steps", flush=True)
    w = W.small_rotor(nx=nx, ny=ny, nz=nz, R=R, chord=3.0, hub=2.0, tau0=0.51, turb=0.05)
    h0, hist0, st0 = _run(w, storage, steps, static=False)
    h1, hist1, st1 = _run(w, storage, steps, static=True)
    assert np.array_equal(h0, h1)
    assert np.array_equal(hist0, hist1, equal_nan=True)
    assert st0 == st1 and st0[1] > 0


def test_two_static_lattices_in_a_row_second_smaller():
    """The second static lattice starts from the cleared array: its result is
    that of a fresh caller-workspace lattice."""
    hl = _hl()
    big = W.small_rotor(nx=64, ny=48, nz=48, R=12.0, chord=4.0, hub=2.0, tau0=0.51, turb=0.05)
    small = W.small_rotor(nx=36, ny=28, nz=28, R=7.0, chord=3.0, hub=1.5, tau0=0.52)
    a = hl.setup(big, storage="f32", static_workspace=True)
    a.step(6)
    ha = a.get_populations().cpu().numpy()
    a.close()
    b = hl.setup(small, storage="f32", static_workspace=True)
    b.step(6)
    hb = b.get_populations().cpu().numpy()
    b.close()
    ref_a, _, _ = _run(big, "f32", 6, static=False)
    ref_b, _, _ = _run(small, "f32", 6, static=False)
    assert np.array_equal(ha, ref_a)
    assert np.array_equal(hb, ref_b)


def test_static_workspace_limits():
    hl = _hl()
    with pytest.raises(hl.HlbmError) as e:
        hl.Lattice(256, 128, 128, storage="f32", static_workspace=True)
    assert e.value.code == hl.HLBM_ERR_INVALID and "static workspace" in str(e.value)
    a = hl.Lattice(32, 16, 16, storage="f32", static_workspace=True)
    with pytest.raises(hl.HlbmError) as e:
        hl.Lattice(32, 16, 16, storage="f32", static_workspace=True)
    assert e.value.code == hl.HLBM_ERR_STATE
    a.close()
    b = hl.Lattice(32, 16, 16, storage="f32", static_workspace=True)
    b.close()
