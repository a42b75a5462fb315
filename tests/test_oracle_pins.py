"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: lattice
quadrature identities, exact moment identities of the equilibrium and of the
collision, asymptotes of the wall law, the Smagorinsky fixed point, viscous
decay rates, Couette flow between moving porous walls, conservation laws and
rigid-body kinematics.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

CS2 = 1.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))


def _sym(P6):
    xx, yy, zz, xy, xz, yz = P6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _mom(f, c):
    rho = f.sum()
    j = c.T @ f
    P = np.einsum("i,ia,ib->ab", f, c, c)
    T3 = np.einsum("i,ia,ib,ic->abc", f, c, c, c)
    return rho, j, P, T3


# ------------------------------------------------------------------ P1
def test_d3q27_quadrature():
    """Weights sum to one; isotropy of the 2nd and 4th moments with cs^2 = 1/3;
    odd moments vanish; H3_aaa vanishes identically on the 27-velocity cube
    (Sec. 2.2: Hermite expansion on the discrete velocities)."""
    c, w = O.lattice_tables()
    c = c.astype(float)
    assert sorted(map(tuple, c.astype(int).tolist())) == sorted(
        (a, b, d) for a in (-1, 0, 1) for b in (-1, 0, 1) for d in (-1, 0, 1))
    for i in range(27):  # canonical order i = 9(cx+1) + 3(cy+1) + (cz+1)
        assert i == 9 * (c[i, 0] + 1) + 3 * (c[i, 1] + 1) + (c[i, 2] + 1)
        assert np.all(c[26 - i] == -c[i])
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(c.T @ w, 0, atol=1e-16)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2, CS2 * np.eye(3), atol=1e-16)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(M4, iso, atol=1e-16)
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.allclose(M3, 0, atol=1e-16)
    for a in range(3):
        assert np.allclose(c[:, a] ** 3 - 3 * CS2 * c[:, a], 0)


# ------------------------------------------------------------------ P2
@pytest.mark.parametrize("rho,u", [(1.03, (0.05, -0.02, 0.03)), (0.97, (-0.11, 0.07, 0.0)), (1.0, (0, 0, 0))])
def test_equilibrium_moments(rho, u):
    """The third-order equilibrium reproduces rho, rho u, rho cs^2 I + rho u u and,
    for every third moment the 27-velocity cube represents (aab with a != b,
    and xyz), rho cs^2 (u_a d_bc + u_b d_ac + u_c d_ab) + rho u_a u_b u_c
    (Sec. 2.2, equilibrium; Hermite coefficients a0^(n) = rho u^n)."""
    c, w = O.lattice_tables()
    c = c.astype(float)
    u = np.array(u, dtype=float)
    feq = O.equilibrium(rho, u)
    r, j, P, T3 = _mom(feq, c)
    assert abs(r - rho) < 1e-15
    assert np.allclose(j, rho * u, atol=1e-16)
    assert np.allclose(P, rho * CS2 * np.eye(3) + rho * np.outer(u, u), atol=1e-16)
    d = np.eye(3)
    expect = rho * CS2 * (np.einsum("a,bc->abc", u, d) + np.einsum("b,ac->abc", u, d) + np.einsum("c,ab->abc", u, d)) \
        + rho * np.einsum("a,b,c->abc", u, u, u)
    for a in range(3):
        for b in range(3):
            for cc in range(3):
                if a == b == cc:
                    continue  # c_a^3 = c_a: not represented by the lattice
                assert abs(T3[a, b, cc] - expect[a, b, cc]) < 1e-16, (a, b, cc)


def _random_cell(rng, d=None):
    rho = 1.0 + 0.05 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    feq = O.equilibrium(rho, u)
    f = feq * (1.0 + 0.02 * rng.standard_normal(27))
    m = O.moments_of(f)
    dd = rng.uniform(0, 1) if d is None else d
    uB = 0.05 * rng.standard_normal(3)
    uwm = 0.02 * rng.standard_normal(3)
    S = 1e-3 * rng.standard_normal(6)
    return f, m, dd, uB, uwm, S


# ------------------------------------------------------------------ P3/P4
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("sigma", [1.0, 0.0])
def test_collision_moments(seed, sigma):
    """Mass is kept, the post-collision momentum is rho u_hat with u_hat the
    porosity-weighted velocity (eq. convexVelocity), the second moment is the
    equilibrium one plus (1 - 1/tau) times the non-equilibrium stress (sigma=1)
    or minus (1 - 1/tau) 2 rho tau cs^2 S (sigma=0, FD part), and the
    momentum handed to the solid is j - rho u_hat (Sec. 2.2, eq. hlbm)."""
    rng = np.random.default_rng(seed)
    c, w = O.lattice_tables()
    c = c.astype(float)
    f, m, d, uB, uwm, S = _random_cell(rng)
    tau0, Cs = 0.53, 0.12
    fs, dP = O.collide_cell(m, d, uB, uwm, S, sigma, tau0, Cs)
    rho, j, P, T3 = _mom(fs, c)
    r0 = m[0]
    u = m[1:4] / r0
    uh = (1 - d) * u + d * (uB + uwm)
    assert abs(rho - r0) < 1e-14
    assert np.allclose(j, r0 * uh, atol=1e-15)
    assert np.allclose(dP, m[1:4] - r0 * uh, atol=1e-15)
    Pi = _sym(m[4:10]) - r0 * CS2 * np.eye(3) - r0 * np.outer(uh, uh)
    # recover tau from the second moment (sigma = 1) and check it is the
    # Smagorinsky fixed point tau = tau0 + Cs^2 |S|/cs^2, |S| = sqrt(2 S:S),
    # S = -Pi / (2 rho cs^2 tau)    (eqs. sgsStress, turbVisc, tauEff)
    Peq = r0 * CS2 * np.eye(3) + r0 * np.outer(uh, uh)
    if sigma == 1.0:
        om = np.sum((P - Peq) * Pi) / np.sum(Pi * Pi)
        assert np.allclose(P - Peq, om * Pi, atol=1e-15)
        tau = 1.0 / (1.0 - om)
        Sst = -Pi / (2 * r0 * CS2 * tau)
        nu_t = Cs ** 2 * math.sqrt(2 * np.sum(Sst * Sst))
        assert abs(tau - (tau0 + nu_t / CS2)) < 1e-12
        # recursive third-order non-equilibrium: a1^(3) = u_a Pi_bc + u_b Pi_ac + u_c Pi_ab
        d3 = np.eye(3)
        eq3 = r0 * CS2 * (np.einsum("a,bc->abc", uh, d3) + np.einsum("b,ac->abc", uh, d3)
                          + np.einsum("c,ab->abc", uh, d3)) + r0 * np.einsum("a,b,c->abc", uh, uh, uh)
        a3 = np.einsum("a,bc->abc", uh, Pi) + np.einsum("b,ac->abc", uh, Pi) + np.einsum("c,ab->abc", uh, Pi)
        for a in range(3):
            for b in range(3):
                for cc in range(3):
                    if not (a == b == cc):
                        assert abs(T3[a, b, cc] - eq3[a, b, cc] - om * a3[a, b, cc]) < 1e-15
    else:
        Sm = _sym(S)
        # tau is still the local Smagorinsky value: recover it from Pi via the fixed point
        Q = math.sqrt(np.sum(Pi * Pi))
        tau = 0.5 * (tau0 + math.sqrt(tau0 ** 2 + 18 * math.sqrt(2) * Cs ** 2 * Q / r0))
        Sloc = -Pi / (2 * r0 * CS2 * tau)
        assert abs(tau - (tau0 + Cs ** 2 * math.sqrt(2 * np.sum(Sloc * Sloc)) / CS2)) < 1e-12
        expect = Peq - (1 - 1 / tau) * 2 * r0 * tau * CS2 * Sm
        assert np.allclose(P, expect, atol=1e-15)


def test_solid_cell_velocity():
    """A fully solid cell (d = 1) at rest hands back zero momentum; a moving one
    the solid's momentum (Sec. 2.2, eq. convexVelocity with d = 1)."""
    rng = np.random.default_rng(11)
    c, w = O.lattice_tables()
    c = c.astype(float)
    f, m, _, uB, _, S = _random_cell(rng)
    fs, dP = O.collide_cell(m, 1.0, (0, 0, 0), (0, 0, 0), S, 1.0, 0.55, 0.1)
    assert np.allclose(c.T @ fs, 0, atol=1e-16)
    assert np.allclose(dP, m[1:4], atol=1e-16)
    fs, dP = O.collide_cell(m, 1.0, uB, (0, 0, 0), S, 1.0, 0.55, 0.1)
    assert np.allclose(c.T @ fs, m[0] * uB, atol=1e-16)


def test_bgk_special_case():
    """tau0 = 1 and C_S = 0: the update is the equilibrium of (rho, u_hat)."""
    rng = np.random.default_rng(3)
    f, m, d, uB, uwm, S = _random_cell(rng)
    fs, _ = O.collide_cell(m, d, uB, (0, 0, 0), S, 1.0, 1.0, 0.0)
    uh = (1 - d) * m[1:4] / m[0] + d * uB
    assert np.allclose(fs, O.equilibrium(m[0], uh), atol=1e-16)


# ------------------------------------------------------------------ P11
def test_spalding_asymptotes():
    """Spalding's law (eq. spalding): viscous sublayer y+ -> u+ (the bracket is
    O(u+^4)), log law u+ -> ln(E y+)/kappa for large u+."""
    for up in (1e-3, 1e-2, 0.1):
        yp = O.spalding_yplus(up)
        assert abs(yp - up) <= (0.41 * up) ** 4 / 24 / 9.8 * 1.01 + 1e-18
    # relative distance to the log law y+ = exp(kappa u+)/E shrinks like a
    # polynomial over an exponential
    rels = []
    for up in (20.0, 30.0, 40.0, 50.0):
        yp = O.spalding_yplus(up)
        rels.append(abs(yp - math.exp(0.41 * up) / 9.8) / yp)
    assert all(b < a for a, b in zip(rels, rels[1:])) and rels[-1] < 2e-6
    # monotone increasing
    ups = np.linspace(0, 30, 301)
    yps = np.array([O.spalding_yplus(v) for v in ups])
    assert np.all(np.diff(yps) > 0)


def _params(**kw):
    p = W.Params(tau0=0.5005, wall_model=1)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_wall_newton_root_and_log_law():
    """Newton for u_tau (eq. implicitWF) lands on the wall law at the sampling
    distance, and the reconstructed velocity at y1 follows the same law; for a
    log-law profile u(y) = u_tau*/kappa ln(E y u_tau*/nu) the model recovers
    u_tau* (Sec. 2.2.1)."""
    p = _params(tol=1e-12, maxit=50)
    nu = CS2 * (p.tau0 - 0.5)
    n = np.array([0.0, 1.0, 0.0])
    errs = {}
    for ut_star in (2e-3, 5e-3, 1e-2, 1.5e-2):  # U up to ~0.3
        for y1 in (0.3, 0.6, 0.95):
            ys = p.y_s
            us_mag = ut_star / 0.41 * math.log(9.8 * ys * ut_star / nu)
            r = O.wall_cell((us_mag, 0.02, 0.0), (0, 0, 0), n, y1, p)
            assert r["active"]
            ut = r["utau"]
            # root of the wall law at y_s
            assert abs(O.spalding_yplus(us_mag / ut) - ys * ut / nu) < 1e-8 * ys * ut / nu
            # large y+: the Spalding root approaches the log-law friction velocity
            errs[ut_star] = abs(ut - ut_star) / ut_star
            up = np.linalg.norm(r["uwm"]) / ut
            assert abs(O.spalding_yplus(up) - y1 * ut / nu) < 1e-8 * max(1, y1 * ut / nu)
            assert np.allclose(r["uwm"] / np.linalg.norm(r["uwm"]), (1, 0, 0))   # tangential, normal part dropped
            # strain: (U - u_wm)/(y_s - y1) on the t-n off-diagonal
            dudn = (us_mag - np.linalg.norm(r["uwm"])) / (ys - y1)
            assert abs(r["S"][3] - 0.5 * dudn) < 1e-12  # S_xy
            assert np.allclose(r["S"][[0, 1, 2, 4, 5]], 0, atol=1e-15)
    e = [errs[k] for k in sorted(errs)]
    assert all(b < a for a, b in zip(e, e[1:])) and e[-1] < 5e-3


def test_wall_laminar_guess_exact():
    """In the viscous sublayer the laminar guess u0 = sqrt(nu U / y) makes the
    linear part of the wall law vanish, leaving f(u0) = bracket(kappa p0)/E =
    (kappa p0)^4 / (24 E) + ... with p0 = y u0 / nu; one Newton step (f' =
    -2 y / nu there) moves u0 by the relative amount kappa^4 p0^3 / (48 E),
    after which the stop rule ends the iteration."""
    p = _params()
    nu = CS2 * (p.tau0 - 0.5)
    for U in (1.5e-6, 6e-6):
        r = O.wall_cell((U, 0, 0), (0, 0, 0), (0, 0, 1.0), 0.5, p)
        assert r["active"] and r["iters"] == 1
        u0 = math.sqrt(nu * U / p.y_s)
        p0 = p.y_s * u0 / nu
        dev = (r["utau"] - u0) / u0
        expect = p.kappa ** 4 * p0 ** 3 / (48.0 * p.E)
        assert 0 < dev and abs(dev / expect - 1.0) < 0.05


def test_wall_stop_rule_and_guess():
    """Stop rule |f(u^{j+1}) - f(u^j)| < 1e-4 with at most 10 iterations; a
    previous friction velocity is used as the guess when the cell was active
    (eq. guess); below a tangential slip U = 1e-6 the cell is inactive."""
    p = _params()
    r1 = O.wall_cell((0.05, 0, 0), (0, 0, 0), (0, 1.0, 0), 0.5, p)
    assert 1 <= r1["iters"] <= 10
    r2 = O.wall_cell((0.05, 0, 0), (0, 0, 0), (0, 1.0, 0), 0.5, p, utau_prev=r1["utau"], prev_active=True)
    assert r2["iters"] == 1 and abs(r2["utau"] - r1["utau"]) / r1["utau"] < 1e-6
    r3 = O.wall_cell((1e-12, 0, 0), (1e-12, 0, 0), (0, 1.0, 0), 0.5, p)
    assert not r3["active"] and np.all(r3["uwm"] == 0)
    # the bound is on the tangential part of the slip only
    assert not O.wall_cell((0.06 + 9e-7, 0.02, 0), (0.06, 0.0, 0), (0, 1.0, 0), 0.5, p)["active"]
    assert O.wall_cell((0.06 + 2e-6, 0.02, 0), (0.06, 0.0, 0), (0, 1.0, 0), 0.5, p)["active"]
    # a moving wall: only the velocity relative to the wall counts
    r4 = O.wall_cell((0.07, 0.01, 0), (0.02, 0.0, 0), (0, 1.0, 0), 0.5, p)
    r5 = O.wall_cell((0.05, 0.03, 0), (0.0, 0.0, 0), (0, 1.0, 0), 0.5, p)
    assert np.allclose(r4["uwm"], r5["uwm"], rtol=1e-12)


# ------------------------------------------------------------------ P12
def _rotor(**kw):
    r = W.Rotor(center=(20.0, 30.0, 30.0), R=16.0, r_hub=2.0, chord=5.0, thick=3.0, omega=0.01)
    for k, v in kw.items():
        setattr(r, k, v)
    return r


def test_transition_function():
    """Lattice porosity (Def. Lattice Porosity): 0 and 1 outside the band,
    1/2 on the surface, monotone; linear s = phi/eps + 1/2."""
    for kind in (0, 1):
        assert O.transition(-1.0, 2.0, kind) == 0.0 and O.transition(1.0, 2.0, kind) == 1.0
        assert abs(O.transition(0.0, 2.0, kind) - 0.5) < 1e-16
        xs = np.linspace(-1.2, 1.2, 97)
        ds = [O.transition(v, 2.0, kind) for v in xs]
        assert np.all(np.diff(ds) >= 0) and min(ds) >= 0 and max(ds) <= 1
    assert abs(O.transition(0.3, 2.0, 1) - (0.3 / 2.0 + 0.5)) < 1e-16


def test_rotor_sdf_closed_forms():
    """Signed distance of a flat-plate blade: mid-section centre is t/2 inside;
    along the plate normal a point delta outside the face has phi = -delta;
    past the tip phi = -(r - R)."""
    r = _rotor(n_blades=1, twist_root=0.3, twist_tip=0.3, phase0=0.0)
    # axis +x, e1 = +y, e2 = +z; blade 0 points along +y at step 0
    xc = np.array(r.center)
    rm = 0.5 * (r.R + r.r_hub)
    phi, _ = O.rotor_phi(r, xc + np.array([0, rm, 0]))
    assert abs(phi - r.thick / 2) < 1e-12
    beta = 0.3
    # plate normal in the (psi, axis) plane: cos(beta) e_axis + sin(beta) e_psi, e_psi = +z here
    nrm = np.array([math.cos(beta), 0.0, math.sin(beta)])
    for delta in (0.25, 1.0, 2.0):
        phi, g = O.rotor_phi(r, xc + np.array([0, rm, 0]) + (r.thick / 2 + delta) * nrm)
        assert abs(phi + delta) < 1e-12
        assert np.allclose(-g / np.linalg.norm(g), nrm, atol=1e-12)
    phi, _ = O.rotor_phi(r, xc + np.array([0, r.R + 1.5, 0]))
    assert abs(phi + 1.5) < 1e-12


def test_rotor_sdf_gradient_fd():
    """The analytic gradient (including the twist's radial derivative) matches
    central differences of phi away from kinks."""
    r = _rotor()
    rng = np.random.default_rng(2)
    checked = cand = 0
    for _ in range(400):
        x = np.array(r.center) + rng.uniform(-18, 18, size=3) * np.array([0.3, 1, 1])
        phi, g = O.rotor_phi(r, x, n=7)
        if phi < -3:
            continue
        cand += 1
        h = 1e-6
        gfd = np.array([(O.rotor_phi(r, x + h * e, n=7)[0] - O.rotor_phi(r, x - h * e, n=7)[0]) / (2 * h)
                        for e in np.eye(3)])
        if np.linalg.norm(gfd - g) < 1e-5:
            checked += 1
    assert cand >= 100 and checked >= cand - 3  # a few points may sit on a kink of the max/abs


def test_rotor_rotation_covariance():
    """phi(x, n) = phi(R(-Omega n) x, 0): the geometry rotates rigidly about its axis."""
    r = _rotor(omega=0.037, phase0=0.4)
    rng = np.random.default_rng(4)
    xc = np.array(r.center)
    for n in (1, 13, 100):
        a = -r.omega * n
        Rm = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
        for _ in range(20):
            x = xc + rng.uniform(-17, 17, size=3)
            p1, _ = O.rotor_phi(r, x, n=n)
            p0, _ = O.rotor_phi(r, xc + Rm @ (x - xc), n=0)
            assert abs(p1 - p0) < 1e-10


def test_rotor_volume_and_solid_velocity():
    """Sum of porosities approximates the solid volume (the d = 1/2 level set is
    the wall); u_B is the rigid rotation Omega e x (x - x_c)."""
    w = W.small_rotor(nx=48, ny=48, nz=48, R=16.0, chord=5.0, hub=3.0)
    r = w.rotors[0]
    o = O.setup(w)
    g = o.geometry()
    V = r.n_blades * r.chord * r.thick * (r.R - r.r_hub) + 4.0 / 3.0 * math.pi * r.r_hub ** 3
    # the diffuse band adds O(eps * curvature * area): about +8 pi r_hub eps^2/24
    # for the hub sphere and a little along the blade edges
    assert abs(g["d"].sum() - V) / V < 0.06
    assert np.all((g["d"] >= 0) & (g["d"] <= 1))
    N = w.cells
    idx = np.nonzero(g["d"] > 0)[0]
    z, y, x = np.unravel_index(idx, (w.nz, w.ny, w.nx))
    rel = np.stack([x, y, z]).astype(float) - np.array(r.center)[:, None]
    uB = g["uB"][:, idx]
    assert np.allclose(np.einsum("ai,ai->i", uB, rel - np.array([[1.0], [0], [0]]) * rel[0]), 0, atol=1e-14)
    assert np.allclose(uB[0], 0, atol=1e-16)
    assert np.allclose(np.linalg.norm(uB, axis=0), r.omega * np.linalg.norm(rel[1:], axis=0), rtol=1e-12)
    assert np.all(g["tag"][idx] == 1)
    # wall cells: fluid side of the band, phi in (-eps/2, 0)
    wc = np.nonzero(g["wall"])[0]
    assert len(wc) > 0 and np.all((g["phi"][wc] > -1.0) & (g["phi"][wc] < 0))
    assert np.allclose(np.linalg.norm(g["n"][:, wc], axis=0), 1.0)


# ------------------------------------------------------------------ RNG
def test_splitmix64_vectors():
    """splitmix64 matches the published reference outputs for seed 1234567."""
    with open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")) as fh:
        vals = [int(l) for l in fh if l.strip() and not l.startswith("#")]
    assert [O.splitmix64(1234567, k) for k in range(5)] == vals


def test_inflow_gaussian_statistics():
    """Box-Muller normals from the counter generator: mean 0, variance 1,
    reproducible, distinct per (step, y, z, component)."""
    xs = np.array([O.gaussian(3, n, y, z, c, 16, 16) for n in range(40) for y in range(16)
                   for z in range(16) for c in range(3)])
    assert abs(xs.mean()) < 0.02 and abs(xs.std() - 1) < 0.02
    assert abs(np.mean(xs ** 4) - 3) < 0.1
    assert O.gaussian(3, 5, 2, 1, 0, 16, 16) == O.gaussian(3, 5, 2, 1, 0, 16, 16)
    assert O.gaussian(3, 5, 2, 1, 0, 16, 16) != O.gaussian(3, 5, 2, 1, 1, 16, 16)


def test_newton_safeguard_counters():
    """The safeguards of the wall-law Newton iterations (Sec. 2.2.1; a
    non-positive iterate is halved, an exponential argument above 80 is
    capped) are counted: a wildly wrong previous friction velocity takes them,
    the guesses of the method do not."""
    p = W.Params(tau0=0.5005, wall_model=1)
    good = O.wall_cell((0.05, 0.0, 0.0), (0, 0, 0), (0, 1, 0), 1.0, p)
    assert good["active"] and good["halvings"] == 0 and good["capped"] == 0
    prev = O.wall_cell((0.05, 0.0, 0.0), (0, 0, 0), (0, 1, 0), 1.0, p, utau_prev=good["utau"], prev_active=True)
    assert prev["halvings"] == 0 and prev["capped"] == 0
    big = O.wall_cell((0.05, 0.0, 0.0), (0, 0, 0), (0, 1, 0), 1.0, p, utau_prev=10.0, prev_active=True)
    assert big["halvings"] >= 1 and big["capped"] >= 1
    tiny = O.wall_cell((0.05, 0.0, 0.0), (0, 0, 0), (0, 1, 0), 1.0, p, utau_prev=1e-8, prev_active=True)
    assert tiny["capped"] >= 1


def test_rotor_run_takes_no_newton_safeguard():
    """On a rotor channel with the wall model and inflow turbulence the
    Newton solves never need the halving or the cap (reading of the stop
    rule: they are safeguards only)."""
    w = W.small_rotor(nx=48, ny=36, nz=36, R=9.0, chord=3.0, hub=2.0, tau0=0.51, turb=0.05)
    o = O.setup(w)
    o.step(12)
    halv, caps, near = o.wall_safeguards()
    it, cells = o.newton_stats()
    assert cells > 100
    assert (halv, caps) == (0, 0)
