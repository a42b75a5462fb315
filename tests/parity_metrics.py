"""Error metrics shared by the GPU parity tests.

Fields: max |x_gpu - x_oracle| / max |x_oracle| (populations as h = f* - w,
velocities).  Forces and torques: per step and tag, the error of each
component of F divided by the sum over the tag's cells of |dP|, and of T by
the sum of |(x - x_c) x dP| (the oracle's history scales): the forces of the
cells of a solid largely cancel, so a norm of the net force says nothing
about the precision of the sum.
"""
import numpy as np


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def force_torque_error(hist_gpu, hist_or, scale_or, tags=None):
    """Largest normalized force and torque error over steps and tags with a
    nonzero scale: returns (eF, eT)."""
    hg = np.asarray(hist_gpu)[:, 1:].reshape(len(hist_gpu), 15, 6)
    ho = np.asarray(hist_or)[:, 1:].reshape(len(hist_or), 15, 6)
    sc = np.asarray(scale_or)
    assert hg.shape == ho.shape and sc.shape == (len(hist_or), 15, 2)
    eF = eT = 0.0
    for t in range(15):
        if tags is not None and (t + 1) not in tags:
            continue
        m = sc[:, t, 0] > 0
        if not m.any():
            continue
        eF = max(eF, float((np.abs(hg[m, t, :3] - ho[m, t, :3]).max(axis=1) / sc[m, t, 0]).max()))
        eT = max(eT, float((np.abs(hg[m, t, 3:] - ho[m, t, 3:]).max(axis=1) / sc[m, t, 1]).max()))
    return eF, eT
