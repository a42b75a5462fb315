"""Pins of the oracle's two-way rotor coupling (the structure update of the
FSI time loop, Sec. 3.2, for a rigid rotation about a fixed axis).

A rotor with moment of inertia I > 0 turns with the state (theta, Omega):
I (Omega_{n+1} - Omega_n) = e . T_n - T_gen, theta_{n+1} = theta_n + Omega_n,
T_n the torque the fluid handed to it in step n.  Two facts fix it from
outside the update itself:

* the fluid loses exactly the angular momentum the rotor gains: streaming
  conserves L = sum (x - x_c) x j while nothing wraps, and the collision
  removes T_n (the balance pinned in test_oracle_torque_probe), so
  e . L + I Omega + n T_gen stays constant;
* the element is drawn at the coupled angle with the coupled speed: its
  porosity, tags and solid velocity at step n equal those of a prescribed
  rotor started at phase theta_n with speed Omega_n.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

from test_oracle_torque_probe import _angular_momentum


def _coupled(n=48, inertia=2.5e5, torque_gen=5.0, tag=3):
    w = W.small_rotor(nx=n, ny=n, nz=n, R=8.0, chord=3.0, hub=1.5, tau0=0.52, wall=1)
    w.bc_x = W.BC_PERIODIC
    r = w.rotors[0]
    r.center = (24.31, 23.62, 24.47)
    r.axis = (1.0, 0.3, -0.2)
    r.omega = 0.02
    r.phase0 = 0.4
    r.tag = tag          # the torque record of a tag other than 1
    r.inertia = inertia
    r.torque_gen = torque_gen
    w.u0 = 0.0
    return w


def test_coupled_rotor_conserves_angular_momentum():
    """Periodic 48^3 box at rest, a coupled rotor (tag 3, tilted axis, wall
    model on, generator torque 5) spinning down: e . L_fluid + I Omega + n
    T_gen is constant to rounding for 16 steps while Omega changes by
    several percent."""
    n = 48
    w = _coupled(n)
    r = w.rotors[0]
    I, Tg = r.inertia, r.torque_gen
    e = np.array(r.axis) / np.linalg.norm(r.axis)
    o = O.setup(w)
    shape = (n, n, n)
    h = o.get_populations()
    L0, b0 = _angular_momentum(h, shape, r.center)
    th0, om0 = o.rotor_state()
    assert th0[0] == r.phase0 and om0[0] == r.omega
    first = om0[0]
    worst = 0.0
    for k in range(16):
        o.step(1)
        L1, b1 = _angular_momentum(o.get_populations(), shape, r.center)
        th1, om1 = o.rotor_state()
        scale = o.history_scale()[-1][r.tag - 1, 1]
        # the fluid's loss and the rotor's gain: I dOmega + T_gen + e . dL = 0
        err = abs(I * (om1[0] - om0[0]) + Tg + e @ (L1 - L0))
        bound = 1e-13 * scale + (b0 + b1) + 4 * np.finfo(float).eps * I * (abs(om0[0]) + abs(om1[0]))
        assert err < bound, (k, err, bound)
        worst = max(worst, err / bound)
        # the angle advances by the speed of the step
        assert th1[0] == th0[0] + om0[0]
        L0, b0, th0, om0 = L1, b1, th1, om1
    print(f"coupled balance: worst error / rounding bound {worst:.2e}; Omega {first} -> {om0[0]:.6f}")
    assert abs(om0[0] - first) > 0.02 * first   # the coupling does act


def test_coupled_geometry_is_the_prescribed_one_at_the_coupled_angle():
    """After 10 coupled steps the element (porosity, tags, wall cells, solid
    velocity) is the one of a prescribed rotor with phase0 = theta_10 and
    omega = Omega_10 at step 0, bit for bit."""
    n = 48
    w = _coupled(n)
    o = O.setup(w)
    o.step(10)
    th, om = o.rotor_state()
    g = o.geometry()
    w2 = _coupled(n)
    r2 = w2.rotors[0]
    r2.phase0, r2.omega, r2.inertia = float(th[0]), float(om[0]), 0.0
    g2 = O.setup(w2).geometry()
    assert np.count_nonzero(g["d"]) > 100
    for key in ("d", "tag", "wall", "phi", "uB"):
        assert np.array_equal(g[key], g2[key]), key


def test_prescribed_rotor_state_follows_its_law():
    """inertia 0: the rotor keeps phase0 + omega n and omega."""
    w = _coupled(32, inertia=0.0)
    w.rotors[0].center = (16.2, 15.7, 16.1)
    w.rotors[0].R = 6.0
    o = O.setup(w)
    o.step(3)
    th, om = o.rotor_state()
    r = w.rotors[0]
    assert th[0] == r.phase0 + r.omega * 3.0 and om[0] == r.omega


def test_adjoint_refuses_coupled_rotors():
    w = _coupled(32)
    w.rotors[0].center = (16.2, 15.7, 16.1)
    w.rotors[0].R = 6.0
    o = O.setup(w)
    with pytest.raises(RuntimeError):
        o.adjoint_run(4, 1, 3)
    with pytest.raises(RuntimeError):
        o.complex_step_J(4, 1, 3, cell=0)
