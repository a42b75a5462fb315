"""The history ring read back across its wrap: one call over a range that
crosses the end of the ring returns the same records, bit for bit, as
single-record calls, and ranges outside the ring are refused.  The force
records of the range also agree with the oracle's (Sec. 2.2.2 and Sec. 3.1:
per-element force and torque each step)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W
from parity_metrics import force_torque_error

pytestmark = pytest.mark.gpu


def test_history_across_the_ring_wrap():
    from paper_2510_13726_amd import hlbm as hl
    w = W.small_rotor(nx=24, ny=20, nz=20, R=6.0, chord=3.0, hub=1.5, tau0=0.52, turb=0.05)
    cap = 64
    lat = hl.setup(w, storage="f64", history=cap)
    n = 150
    lat.step(n)
    lo, hi = n - cap, n
    assert (lo % cap) > (hi - 1) % cap    # the range wraps around the ring's end
    bulk = lat.history(lo, hi)
    single = np.concatenate([lat.history(s, s + 1) for s in range(lo, hi)])
    assert np.array_equal(bulk, single)
    assert np.array_equal(lat.history(lo + 5, lo + 40), bulk[5:40])
    with pytest.raises(hl.HlbmError):
        lat.history(lo - 1, hi)
    with pytest.raises(hl.HlbmError):
        lat.history(lo, hi + 1)
    o = O.setup(w)
    o.step(n)
    eF, eT = force_torque_error(bulk, o.history()[lo:hi], o.history_scale()[lo:hi])
    print(f"[history] wrap at {cap}: F {eF:.2e} T {eT:.2e}", flush=True)
    assert eF < 1e-12 and eT < 1e-12
