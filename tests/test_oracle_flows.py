"""Whole-lattice pins of the oracle: conservation, momentum balance with the
solid, viscous decay rates, Couette flow between moving porous walls, the
uniform-flow fixed point of the outer boundaries, determinism and restart."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

CS2 = 1.0 / 3.0


def test_mass_and_momentum_balance_periodic():
    """Fully periodic box with a tagged porous sphere: mass is conserved and the
    change of total momentum over a step equals minus the force handed to the
    solid (streaming is a permutation; the collision moves exactly
    j - rho u_hat into the solid, Sec. 2.2 eq. convexVelocity)."""
    w = W.config1(noise=True)
    o = O.setup(w)
    rho0, u0 = o.moments()
    M0 = rho0.sum()
    for n in range(12):
        rho, u = o.moments()
        P0 = (rho * u).sum(axis=1)
        o.step(1)
        rho1, u1 = o.moments()
        P1 = (rho1 * u1).sum(axis=1)
        rec = o.history()[-1]
        F = rec[1:4]
        assert abs(rec[0] - rho.sum()) / rho.sum() < 1e-13
        assert abs(rho1.sum() - M0) / M0 < 1e-14
        scale = max(np.abs(F).max(), 1e-8)
        assert np.allclose(P1 - P0, -F, atol=1e-13 * rho.size * 1e-2 + 1e-12 * scale), (n, P1 - P0, F)
    assert np.abs(o.history()[:, 1:4]).max() > 1e-6  # the sphere does take momentum


def test_solid_cells_move_with_the_solid():
    """u_hat (the post-collision velocity) is exactly the solid velocity where
    d = 1 (zero for the static sphere)."""
    w = W.config1(noise=True)
    o = O.setup(w)
    o.step(3)
    g = o.geometry()
    rho, u, uh = o.moments(uhat=True)
    solid = g["d"] == 1.0
    assert solid.sum() > 100
    assert np.abs(uh[:, solid]).max() == 0.0
    assert np.abs(u[:, solid]).max() > 1e-6  # streaming carries fluid momentum into the solid


def _shear_wave(tau0, steps, n=64):
    p = W.Params(tau0=tau0, cs_smag=0.0)
    o = O.OracleLattice(2, n, 1, 0)
    o.set_params(p)
    o.set_rotors([])
    y = np.arange(n)
    U0 = 1e-3
    ux = np.tile(U0 * np.sin(2 * math.pi * y / n)[:, None], (1, 2)).reshape(-1)
    u = np.stack([ux, np.zeros_like(ux), np.zeros_like(ux)])
    o.init_equilibrium(np.ones(2 * n), u)
    amps = []
    basis = np.tile(np.sin(2 * math.pi * y / n)[:, None], (1, 2)).reshape(-1)
    for t in range(steps):
        rho, uu = o.moments()
        amps.append(np.dot(uu[0], basis) / np.dot(basis, basis))
        o.step(1)
    return np.array(amps), 2 * math.pi / n


@pytest.mark.parametrize("tau0", [0.55, 0.8])
def test_shear_wave_viscosity(tau0):
    """A shear wave decays as exp(-nu k^2 t) with nu = cs^2 (tau0 - 1/2)
    (relation of tau and viscosity, eq. tauEff with nu_turb = 0)."""
    amps, k = _shear_wave(tau0, 1500)
    t = np.arange(len(amps))
    sel = t >= 100
    slope = np.polyfit(t[sel], np.log(amps[sel]), 1)[0]
    nu = -slope / k ** 2
    assert abs(nu / (CS2 * (tau0 - 0.5)) - 1) < 0.01


def test_taylor_green_2d_decay():
    """z-invariant Taylor-Green vortex: kinetic energy decays as exp(-4 nu k^2 t)."""
    n = 32
    tau0 = 0.6
    o = O.OracleLattice(n, n, 1, 0)
    o.set_params(W.Params(tau0=tau0, cs_smag=0.0))
    o.set_rotors([])
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k = 2 * math.pi / n
    U0 = 5e-3
    ux = U0 * np.sin(k * x) * np.cos(k * y)
    uy = -U0 * np.cos(k * x) * np.sin(k * y)
    rho = 1.0 + 3.0 * U0 ** 2 / 4.0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    o.init_equilibrium(rho.reshape(-1), np.stack([ux, uy, 0 * ux]).reshape(3, -1))
    E = []
    for t in range(600):
        r, u = o.moments()
        E.append(np.sum(r * (u ** 2).sum(axis=0)))
        o.step(1)
    E = np.array(E)
    t = np.arange(len(E))
    sel = t >= 100
    slope = np.polyfit(t[sel], np.log(E[sel]), 1)[0]
    nu = -slope / (4 * k ** 2)
    assert abs(nu / (CS2 * (tau0 - 0.5)) - 1) < 0.01


def test_couette_between_moving_porous_slabs():
    """Two porous slabs (d = 1 inside, tanh band, the d = 1/2 level set is the
    wall, Def. Lattice Porosity) moving at -U and +U drive linear Couette
    profiles in the two channels between them."""
    n = 32
    U = 0.01
    tau0 = 1.0
    o = O.OracleLattice(2, n, 1, 0)
    o.set_params(W.Params(tau0=tau0, cs_smag=0.0, eps_h=2.0))
    o.set_rotors([])
    y = np.arange(n)
    distA = np.minimum(np.abs(y - 0), n - np.abs(y - 0))
    distB = np.abs(y - 16)
    phiA, phiB = 3.0 - distA, 3.0 - distB
    phi = np.maximum(phiA, phiB)

    def s(p):
        v = 0.5 * (1 + np.tanh(4 * p / 2.0) / np.tanh(2.0))
        return np.where(p <= -1, 0.0, np.where(p >= 1, 1.0, v))

    d = np.tile(s(phi)[:, None], (1, 2)).reshape(-1)
    uBx = np.tile(np.where(phiA > phiB, -U, U)[:, None], (1, 2)).reshape(-1)
    uB = np.stack([uBx, 0 * uBx, 0 * uBx])
    o.set_porosity_field(d, np.zeros(2 * n, dtype=np.uint8))
    o.set_solid_velocity(uB)
    o.init_equilibrium(None, None)
    o.step(6000)
    rho, u = o.moments()
    ux = u[0].reshape(n, 2)[:, 0]
    dd = d.reshape(n, 2)[:, 0]
    for lo, hi, ulo, uhi in ((3.0, 13.0, -U, U), (19.0, 29.0, U, -U)):
        ys = np.array([v for v in range(int(lo) + 2, int(hi) - 1) if dd[v] == 0.0])
        coef = np.polyfit(ys, ux[ys], 1)
        resid = ux[ys] - np.polyval(coef, ys)
        assert np.abs(resid).max() < 1e-3 * U
        # the line meets the wall velocities near the d = 1/2 level sets
        y_at_lo = (ulo - coef[1]) / coef[0]
        y_at_hi = (uhi - coef[1]) / coef[0]
        assert abs(y_at_lo - lo) < 0.6 and abs(y_at_hi - hi) < 0.6, (y_at_lo, y_at_hi)


def test_uniform_flow_is_a_fixed_point():
    """With equilibrium inflow, zero-gradient outflow and no solid, a uniform
    stream at the inflow velocity stays exactly uniform."""
    w = W.small_rotor(nx=24, ny=12, nz=10, steps=5)
    w.rotors = []
    o = O.setup(w)
    h0 = o.get_populations()
    o.step(15)
    assert np.abs(o.get_populations() - h0).max() < 5e-15  # rounding of f = w + h only


def test_restart_and_determinism():
    """Restoring populations + wall state + step reproduces the trajectory bit
    for bit, and two runs of the same input agree bit for bit."""
    w = W.small_rotor(nx=40, ny=32, nz=32, R=9.0, chord=3.0, hub=2.0, tau0=0.51, turb=0.05)
    o = O.setup(w)
    o.step(6)
    h = o.get_populations()
    ut, ac = o.wall_state()
    assert ac.sum() > 10
    st = o.step_count
    o.step(6)
    ref = o.get_populations()
    o.set_populations(h)
    o.set_wall_state(ut, ac, st)
    o.step(6)
    assert np.array_equal(o.get_populations(), ref)
    o2 = O.setup(w)
    o2.step(12)
    assert np.array_equal(o2.get_populations(), ref)


def test_inflow_turbulence_statistics():
    """The inflow plane carries the seeded perturbation: its velocity has mean
    U e_x and standard deviation I U per component."""
    w = W.small_rotor(nx=8, ny=32, nz=32, turb=0.05)
    w.rotors = []
    o = O.setup(w)
    o.step(1)
    rho, u = o.moments()
    # pre-collision velocity at x = 0 mixes inflow populations with the
    # interior; check the population-level inflow instead through x = 0 of the
    # next step's pull: compare with the time-averaged statistics of the
    # interior cell after a step
    ux = u[0].reshape(w.nz, w.ny, w.nx)[:, :, 0]
    assert abs(ux.mean() - 0.05) < 0.05 * 0.05 * 0.5
    assert 0.2 * 0.05 * 0.05 < ux.std() < 0.05 * 0.05 * 1.5


@pytest.mark.parametrize("x0", [0, 10])
def test_light_cone_of_an_x_slab(x0):
    """The dependency reach the full-size GPU comparisons rely on: after n
    steps, an x-slab run on its own agrees with the full run on every cell
    farther than 6n + 2 planes from the slab's cut faces (streaming moves one
    cell per step, the wall-model probe stencil four more)."""
    w = W.small_rotor(nx=100, ny=36, nz=36, R=9.0, chord=3.0, hub=2.0, tau0=0.51, turb=0.05)
    w.rotors[0].center = (30.0, w.rotors[0].center[1], w.rotors[0].center[2])
    n = 3
    m = 6 * n + 2
    length = 2 * m + 14 if x0 else m + 14
    full = O.setup(w)
    full.step(n)
    s = W.x_slab(w, x0, length)
    assert s.bc_x == (w.bc_x if x0 == 0 else W.BC_PERIODIC)
    o = O.setup(s)
    o.step(n)
    assert o.newton_stats()[1] > 50 or x0 == 0
    lo = m if x0 else 0
    hf = full.get_populations().reshape(27, w.nz, w.ny, w.nx)[..., x0 + lo:x0 + length - m]
    hs = o.get_populations().reshape(27, s.nz, s.ny, s.nx)[..., lo:length - m]
    assert hf.shape == hs.shape and hf.shape[-1] == 14
    assert np.abs(hf - hs).max() <= 1e-13 * np.abs(hf).max()
    # the compared planes hold the rotor's disturbance, not only free stream
    assert np.abs(hf - hf[:, :1, :1, :1]).max() > 1e-4 * np.abs(hf).max()


@pytest.mark.parametrize("case", ["poiseuille", "brinkman"])
def test_channel_driven_by_a_weak_porosity(case):
    """A periodic channel between two porous walls (a d = 1 slab with the
    tanh band; its d = 1/2 level set 17 cells from the axis, Def. Lattice
    Porosity), the fluid held by a weak uniform porosity delta toward the
    solid velocity V: each step the collision hands rho delta (V - u) to the
    fluid (eq. convexVelocity), a body force.  The steady profile solves
    nu u'' + delta (V - u) = 0 with u = 0 at the walls,
    u = V (1 - cosh(k y) / cosh(k h)), k = sqrt(delta / nu), nu =
    cs^2 (tau0 - 1/2): the Poiseuille parabola u = delta V (h^2 - y^2) /
    (2 nu) for k h -> 0 (delta = 2e-5), a distinctly flatter profile for
    k h = 1.9 (delta = 2e-3).  The wall position h is fitted; it must lie
    within 0.6 cells of the level set, as for the Couette flow."""
    from scipy.optimize import brentq
    delta, V, steps = {"poiseuille": (2e-5, 1.0, 18000), "brinkman": (2e-3, 0.01, 6000)}[case]
    n, tau0 = 40, 1.0
    o = O.OracleLattice(2, n, 1, 0)
    o.set_params(W.Params(tau0=tau0, cs_smag=0.0, eps_h=2.0))
    o.set_rotors([])
    y = np.arange(n)
    phi = 3.0 - np.minimum(y, n - y)

    def s(p):
        v = 0.5 * (1 + np.tanh(4 * p / 2.0) / np.tanh(2.0))
        return np.where(p <= -1, 0.0, np.where(p >= 1, 1.0, v))

    dw = s(phi)
    d = np.tile(np.maximum(dw, delta)[:, None], (1, 2)).reshape(-1)
    uBx = np.tile(np.where(dw > 0, 0.0, V)[:, None], (1, 2)).reshape(-1)
    o.set_porosity_field(d, np.zeros(2 * n, dtype=np.uint8))
    o.set_solid_velocity(np.stack([uBx, 0 * uBx, 0 * uBx]))
    o.init_equilibrium(None, None)
    o.step(steps)
    ux = o.moments()[1][0].reshape(n, 2)[:, 0]
    o.step(100)
    assert np.abs(o.moments()[1][0].reshape(n, 2)[:, 0] - ux).max() < 1e-9 * V   # steady
    nu = CS2 * (tau0 - 0.5)
    k = np.sqrt(delta / nu)
    yc, h_set = 20.0, 17.0
    ys = np.array([v for v in range(5, 36) if dw[v] == 0.0])

    def model(h):
        return V * (1 - np.cosh(k * (ys - yc)) / np.cosh(k * h))

    h = brentq(lambda hh: np.sum((ux[ys] - model(hh)) * np.cosh(k * (ys - yc))), 15.0, 19.0)
    umax = ux[ys].max()
    resid = np.abs(ux[ys] - model(h)).max() / umax
    par = np.polyfit(ys, ux[ys], 2)
    par_resid = np.abs(ux[ys] - np.polyval(par, ys)).max() / umax
    print(f"{case}: wall at {h:.3f} (level set {h_set}), residual {resid:.1e} of u_max {umax:.4e}, "
          f"parabola residual {par_resid:.1e}")
    assert abs(h - h_set) < 0.6
    assert resid < 1e-3
    if case == "poiseuille":
        assert par_resid < 1e-3
        assert abs(umax / (delta * V * h ** 2 / (2 * nu)) - 1) < 0.02
    else:
        assert par_resid > 1e-2
