"""Pins of the oracle's momentum-exchange force (Sec. 2.2.2, read per link
between a tag-0 cell and a cell of the element, Galilean-invariant form).

For a solid at rest (u_s = 0) the estimator of a step is exactly the
momentum that streaming then carries into the element's cell set S minus
the momentum it carries out: M_S(pre-collision, n+1) - M_S(post-collision,
n), with M_S the summed momentum of the cells of S.  In a steady flow the
momentum inside S is steady, so the estimator and the momentum the
collision hands to the solid (sum of j - rho u_hat) agree; in general they
differ by the change of that momentum."""
import numpy as np

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W


def test_momentum_exchange_is_the_momentum_flux_into_the_solid():
    w = W.config1(noise=True)
    o = O.setup(w)
    o.set_force_mode(1)
    S = o.geometry()["tag"] == 1
    assert S.sum() > 500
    worst, scale = 0.0, 0.0
    for n in range(6):
        rho, u, uh = o.moments(uhat=True)
        post = (rho * uh)[:, S].sum(axis=1)           # sum over S of rho u_hat = sum c f*
        o.step(1)
        rho1, u1 = o.moments()
        pre1 = (rho1 * u1)[:, S].sum(axis=1)           # sum over S of the pulled momentum
        F = o.history_me()[-1][0]
        ref = pre1 - post
        scale = max(scale, np.abs(ref).max())
        worst = max(worst, np.abs(F - ref).max())
    # rounding: each cell's momentum in the two sums over S comes from O(1)
    # populations (an eps each), the estimator sums O(1) populations per link
    bound = 8 * np.finfo(float).eps * S.sum()
    print(f"momentum exchange vs flux into S: max abs err {worst:.2e} (flux scale {scale:.2e}, rounding "
          f"bound {bound:.1e})")
    assert scale > 1e-6
    assert worst < bound


def test_momentum_exchange_minus_collision_force_is_the_change_inside_the_solid():
    """The collision hands F_col = M_S(pre, n) - M_S(post, n) to the solid, so
    F_ME - F_col = M_S(pre, n+1) - M_S(pre, n): the two force definitions
    differ exactly by the rate of change of the momentum inside the element
    (zero in a steady flow)."""
    w = W.config1(noise=True)
    o = O.setup(w)
    o.set_force_mode(1)
    S = o.geometry()["tag"] == 1
    bound = 8 * np.finfo(float).eps * S.sum()
    rho, u = o.moments()
    pre = (rho * u)[:, S].sum(axis=1)
    for n in range(6):
        o.step(1)
        rho1, u1 = o.moments()
        pre1 = (rho1 * u1)[:, S].sum(axis=1)
        F_col = o.history()[-1][1:4]
        F_me = o.history_me()[-1][0]
        assert np.abs((F_me - F_col) - (pre1 - pre)).max() < bound
        pre = pre1
