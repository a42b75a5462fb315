"""Pins of the oracle's D3Q19 instantiation (the paper's stencil, Sec. 2.2,
Fig. 2): quadrature, the moments of the equilibrium and of the collision
that the 19-velocity set represents, the BGK special case, the shear-wave
viscosity, and the momentum and angular-momentum balances with a solid.

The third-order Hermite terms on D3Q19 are the projection onto H_aab + H_ccb
and H_aab - H_ccb (the recursive-regularized D3Q19 scheme the paper builds
on); its defining property is that the six represented third moments
sum_i c_a^2 c_b f_i come out exactly as the continuous Hermite series gives
them, which is what these tests check (independently of the projection
formula itself)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

CS2 = 1.0 / 3.0


def _mom(f, c):
    return f.sum(), c.T @ f, np.einsum("i,ia,ib->ab", f, c, c), np.einsum("i,ia,ib,ic->abc", f, c, c, c)


def _sym(P6):
    xx, yy, zz, xy, xz, yz = P6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _tables():
    c, w = O.lattice_tables(19)
    return c.astype(float), w


def test_d3q19_quadrature():
    """19 velocities with |c|^2 <= 2 in the order of the 27-velocity cube
    restricted; weights 1/3, 1/18, 1/36; isotropy up to the fourth moment
    with cs^2 = 1/3; opposite of k is 18 - k."""
    c, w = _tables()
    assert c.shape == (19, 3)
    idx27 = [9 * (a + 1) + 3 * (b + 1) + (d + 1) for a, b, d in c.astype(int)]
    assert idx27 == sorted(idx27) and all((c ** 2).sum(axis=1) <= 2)
    assert set(np.round(w * 36).astype(int)) == {12, 2, 1}
    for k in range(19):
        assert np.all(c[18 - k] == -c[k])
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(c.T @ w, 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(3), atol=1e-16)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)


def _third_expect(rho, u):
    d = np.eye(3)
    return rho * CS2 * (np.einsum("a,bc->abc", u, d) + np.einsum("b,ac->abc", u, d) + np.einsum("c,ab->abc", u, d)) \
        + rho * np.einsum("a,b,c->abc", u, u, u)


@pytest.mark.parametrize("rho,u", [(1.03, (0.05, -0.02, 0.03)), (0.97, (-0.11, 0.07, 0.04)), (1.0, (0, 0, 0))])
def test_d3q19_equilibrium_moments(rho, u):
    """rho, rho u, rho cs^2 I + rho u u exactly; of the third moments, the six
    c_a^2 c_b (a != b) equal rho cs^2 u_b + rho u_a^2 u_b exactly, and
    c_x c_y c_z vanishes on every D3Q19 velocity."""
    c, w = _tables()
    u = np.array(u, dtype=float)
    feq = O.equilibrium(rho, u, q=19)
    r, j, P, T3 = _mom(feq, c)
    assert abs(r - rho) < 1e-15
    assert np.allclose(j, rho * u, atol=1e-16)
    assert np.allclose(P, rho * CS2 * np.eye(3) + rho * np.outer(u, u), atol=1e-16)
    expect = _third_expect(rho, u)
    for a in range(3):
        for b in range(3):
            if a != b:
                assert abs(T3[a, a, b] - expect[a, a, b]) < 1e-16, (a, b)
    assert T3[0, 1, 2] == 0.0


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("sigma", [1.0, 0.0])
def test_d3q19_collision_moments(seed, sigma):
    """Mass kept; momentum rho u_hat (eq. convexVelocity); second moment
    rho cs^2 I + rho u_hat u_hat + (1 - 1/tau)(sigma Pi - (1 - sigma) 2 rho tau
    cs^2 S); represented third moments rho u_a^2 u_b + cs^2 rho u_b +
    (1 - 1/tau) sigma (2 u_a Pi_ab + u_b Pi_aa) (recursive a1^(3))."""
    rng = np.random.default_rng(100 + seed)
    c, w = _tables()
    rho0 = 1.0 + 0.05 * rng.standard_normal()
    u0 = 0.05 * rng.standard_normal(3)
    f = O.equilibrium(rho0, u0, q=19) * (1.0 + 0.02 * rng.standard_normal(19))
    m = O.moments_of(f, q=19)
    d, uB, uwm, S = rng.uniform(0, 1), 0.05 * rng.standard_normal(3), 0.02 * rng.standard_normal(3), \
        1e-3 * rng.standard_normal(6)
    tau0, Cs = 0.53, 0.12
    fs, dP = O.collide_cell(m, d, uB, uwm, S, sigma, tau0, Cs, q=19)
    rho, j, P, T3 = _mom(fs, c)
    r0 = m[0]
    uh = (1 - d) * m[1:4] / r0 + d * (uB + uwm)
    assert abs(rho - r0) < 1e-14
    assert np.allclose(j, r0 * uh, atol=1e-15)
    assert np.allclose(dP, m[1:4] - r0 * uh, atol=1e-15)
    Pi = _sym(m[4:10]) - r0 * CS2 * np.eye(3) - r0 * np.outer(uh, uh)
    Q = math.sqrt(np.sum(Pi * Pi))
    tau = 0.5 * (tau0 + math.sqrt(tau0 ** 2 + 18 * math.sqrt(2) * Cs ** 2 * Q / r0))
    om = 1 - 1 / tau
    Peq = r0 * CS2 * np.eye(3) + r0 * np.outer(uh, uh)
    expectP = Peq + om * (sigma * Pi - (1 - sigma) * 2 * r0 * tau * CS2 * _sym(S))
    assert np.allclose(P, expectP, atol=1e-15)
    eq3 = _third_expect(r0, uh)
    for a in range(3):
        for b in range(3):
            if a != b:
                a1 = 2 * uh[a] * Pi[a, b] + uh[b] * Pi[a, a]
                assert abs(T3[a, a, b] - eq3[a, a, b] - om * sigma * a1) < 1e-15, (a, b)


def test_d3q19_bgk_special_case():
    """tau0 = 1, C_S = 0: the collision returns the equilibrium at u_hat."""
    rng = np.random.default_rng(5)
    f = O.equilibrium(1.02, (0.03, -0.04, 0.02), q=19) * (1 + 0.03 * rng.standard_normal(19))
    m = O.moments_of(f, q=19)
    fs, _ = O.collide_cell(m, 0.0, (0, 0, 0), (0, 0, 0), (0,) * 6, 1.0, 1.0, 0.0, q=19)
    feq = O.equilibrium(m[0], m[1:4] / m[0], q=19)
    assert np.abs(fs - feq).max() < 1e-16


@pytest.mark.parametrize("tau0", [0.55, 0.8])
def test_d3q19_shear_wave_viscosity(tau0):
    """A shear wave on D3Q19 decays as exp(-nu k^2 t), nu = cs^2 (tau0 - 1/2)."""
    n, steps = 64, 200
    p = W.Params(tau0=tau0, cs_smag=0.0)
    o = O.OracleLattice(2, n, 1, 0, q=19)
    o.set_params(p)
    o.set_rotors([])
    y = np.arange(n)
    basis = np.tile(np.sin(2 * math.pi * y / n)[:, None], (1, 2)).reshape(-1)
    u = np.stack([1e-3 * basis, np.zeros_like(basis), np.zeros_like(basis)])
    o.init_equilibrium(np.ones(2 * n), u)
    amps = []
    for _ in range(steps):
        amps.append(np.dot(o.moments()[1][0], basis) / np.dot(basis, basis))
        o.step(1)
    k = 2 * math.pi / n
    rate = -np.polyfit(np.arange(50, steps), np.log(np.array(amps[50:])), 1)[0]
    nu = CS2 * (tau0 - 0.5)
    assert abs(rate / (nu * k * k) - 1) < 0.01, rate / (nu * k * k)


def _d3q19_rotor_box(n=40):
    w = W.small_rotor(nx=n, ny=n, nz=n, R=7.0, chord=3.0, hub=1.5, tau0=0.52, wall=1)
    w.bc_x = W.BC_PERIODIC
    w.q = 19
    r = w.rotors[0]
    r.center = (20.3, 19.6, 20.2)
    r.axis = (1.0, 0.2, 0.1)
    r.omega = 0.02
    w.u0 = 0.0
    return w, r


def test_d3q19_momentum_and_angular_momentum_balance():
    """Periodic box with a spinning rotor (wall model on): every step the total
    momentum changes by -F and the angular momentum about the rotor centre
    by -T, to rounding on the scales sum |dP| and sum |r x dP|."""
    n = 40
    w, r = _d3q19_rotor_box(n)
    o = O.setup(w)
    c, wts = _tables()
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rr = np.stack([x.reshape(-1) - r.center[0], y.reshape(-1) - r.center[1], z.reshape(-1) - r.center[2]])

    def PL(h):
        j = c.T @ h
        return j.sum(axis=1), np.array([np.sum(rr[1] * j[2] - rr[2] * j[1]), np.sum(rr[2] * j[0] - rr[0] * j[2]),
                                        np.sum(rr[0] * j[1] - rr[1] * j[0])])
    P0, L0 = PL(o.get_populations())
    worst = 0.0
    for _ in range(10):
        o.step(1)
        P1, L1 = PL(o.get_populations())
        rec, sc = o.history()[-1], o.history_scale()[-1][0]
        eF = np.abs(P1 - P0 + rec[1:4]).max() / sc[0]
        eT = np.abs(L1 - L0 + rec[4:7]).max() / sc[1]
        worst = max(worst, eF, eT)
        P0, L0 = P1, L1
    assert np.abs(o.history()[:, 4:7]).max() > 0
    assert worst < 1e-12, worst
