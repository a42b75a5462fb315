"""GPU discrete adjoint vs the oracle's adjoint (itself pinned by complex-step
derivatives), the autograd wrapper, and finite differences through the
porosity control."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

pytestmark = pytest.mark.gpu


def _hl():
    from paper_2510_13726_amd import hlbm
    return hlbm


def _torque_scale(o, t0, t1):
    """Mean over the window [t0, t1) of the summed |(x - x_c) x dP| of all tags."""
    sc = o.history_scale()
    return float(sc[t0:t1, :, 1].sum(axis=1).mean())


def _cases():
    a = W.config1(noise=True, n=12)
    a.params.cs_smag = 0.15
    b = W.small_rotor(nx=24, ny=20, nz=20, R=6.0, chord=3.0, hub=1.5, tau0=0.52, turb=0.05)
    return {"sphere": (a, 12, 4, 12), "rotor": (b, 10, 3, 10)}


@pytest.mark.parametrize("q", [27, 19])
@pytest.mark.parametrize("case", ["sphere", "rotor"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_matches_oracle(case, storage, q):
    hl = _hl()
    w, n, t0, t1 = _cases()[case]
    w.q = q
    print(f"[adjoint] {case} D3Q{q} {storage}", flush=True)
    o = O.setup(w)
    J_or, G_or = o.adjoint_run(n, t0, t1, obj_tag=0, ckpt_every=4)
    lat = hl.setup(w, storage=storage, flags=hl.WITH_ADJOINT)
    J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=4)
    G = lat.adjoint(1.0).cpu().numpy()
    # J sums torques of cells of opposite sign: its error is measured on the
    # scale of the summed |(x - x_c) x dP| over the window
    eJ = abs(J - J_or) / _torque_scale(o, t0, t1)
    eG = np.abs(G - G_or).max() / np.abs(G_or).max()
    print(f"[adjoint] {case} D3Q{q} {storage}: J {J:.6e} vs {J_or:.6e} (rel {eJ:.2e}); G rel err {eG:.2e}",
          flush=True)
    tol = {"f64": 1e-12, "f32": 2e-5}[storage]
    assert eJ < tol
    assert eG < tol
    # the lattice is left in the forward final state
    h = lat.get_populations().cpu().numpy()
    assert np.abs(h - o.get_populations()).max() / np.abs(o.get_populations()).max() < tol


def test_autograd_function_and_finite_differences():
    hl = _hl()
    torch = pytest.importorskip("torch")
    w, n, t0, t1 = _cases()["rotor"]
    lat = hl.setup(w, storage="f64", flags=hl.WITH_ADJOINT | hl.WITH_CONTROL)
    state0 = lat.get_state().clone()
    TorqueObjective = hl.torque_objective_function()
    dd = torch.zeros(w.cells, dtype=torch.float64, device=lat.device, requires_grad=True)
    J = TorqueObjective.apply(dd, lat, state0, n, t0, t1, 0, 4)
    J.backward()
    g = dd.grad.cpu().numpy()
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    # central differences of the GPU forward at the largest-gradient cells
    cells = np.argsort(-np.abs(g))[:3]
    eps = 1e-6
    for c in cells:
        Js = []
        for sgn in (1.0, -1.0):
            pert = torch.zeros(w.cells, dtype=torch.float64, device=lat.device)
            pert[int(c)] = sgn * eps
            Js.append(float(TorqueObjective.apply(pert, lat, state0, n, t0, t1, 0, 4)))
        fd = (Js[0] - Js[1]) / (2 * eps)
        print(f"[adjoint] cell {c}: adjoint {g[c]:.8e} fd {fd:.8e}", flush=True)
        assert abs(fd - g[c]) < 1e-5 * abs(g[c]) + 1e-9


def test_adjoint_independent_of_checkpoint_spacing():
    """Segments of one step (no recompute, no geometry carried between
    reverse steps), of three and of the whole run give the same gradient:
    the recompute reproduces the forward states exactly, and the probe-velocity
    adjoints are summed in fixed point, so the gradients agree bit for bit."""
    hl = _hl()
    w, n, t0, t1 = _cases()["rotor"]
    lat = hl.setup(w, storage="f64", flags=hl.WITH_ADJOINT)
    state0 = lat.get_state().clone()
    res = {}
    for ce in (1, 3, 4, n):
        lat.set_state(state0)
        J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=ce)
        res[ce] = (J, lat.adjoint(1.0).cpu().numpy())
        print(f"[adjoint] ckpt_every {ce}: J {J:.12e} |G| {np.abs(res[ce][1]).max():.6e}", flush=True)
    J4, G4 = res[4]
    for ce, (J, G) in res.items():
        assert J == J4
        assert np.array_equal(G, G4), (ce, np.abs(G - G4).max())
    # and a repeated run gives the same gradient
    lat.set_state(state0)
    J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=4)
    assert J == J4 and np.array_equal(lat.adjoint(1.0).cpu().numpy(), G4)


def test_adjoint_across_blade_angle_table_reload():
    """A recorded window across step 2048, where the device table of blade
    angles (2048 steps) is reloaded: forwards in the recorded run, backwards
    during the reverse sweep.  After 2056 steps the FP64 rounding of the two
    forward runs has grown beyond the 1e-12 bar of the short parity cases
    (elementwise parity applies to runs of up to 50 steps), so the gradient
    is held to 1e-11 here; J stays at 1e-12."""
    hl = _hl()
    w, _, _, _ = _cases()["rotor"]
    n0, n, t0, t1 = 2040, 16, 2, 16
    o = O.setup(w)
    o.step(n0)
    J_or, G_or = o.adjoint_run(n, t0, t1, obj_tag=0, ckpt_every=4)
    lat = hl.setup(w, storage="f64", flags=hl.WITH_ADJOINT)
    lat.step(n0)
    J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=4)
    G = lat.adjoint(1.0).cpu().numpy()
    eJ = abs(J - J_or) / _torque_scale(o, n0 + t0, n0 + t1)
    eG = np.abs(G - G_or).max() / np.abs(G_or).max()
    print(f"[adjoint] steps {n0}..{n0 + n}: J rel {eJ:.2e}, G rel err {eG:.2e}", flush=True)
    assert eJ < 1e-12
    assert eG < 1e-11


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_with_reference_grid_rotor_matches_oracle(storage):
    """A rotor whose body is a reference grid (Sec. 3.1): the porosity and
    the wall normals come from the sampled grid, the adjoint is unchanged."""
    hl = _hl()
    w, n, t0, t1 = _cases()["rotor"]
    w.rotors[0].grid = W.capsule_rotor_grid(w.rotors[0], spacing=0.5, eps_h=w.params.eps_h)
    print(f"[adjoint-grid] {storage}", flush=True)
    o = O.setup(w)
    J_or, G_or = o.adjoint_run(n, t0, t1, obj_tag=0, ckpt_every=4)
    lat = hl.setup(w, storage=storage, flags=hl.WITH_ADJOINT)
    J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=4)
    G = lat.adjoint(1.0).cpu().numpy()
    eJ = abs(J - J_or) / _torque_scale(o, t0, t1)
    eG = np.abs(G - G_or).max() / np.abs(G_or).max()
    print(f"[adjoint-grid] {storage}: J {J:.6e} vs {J_or:.6e} (rel {eJ:.2e}); G rel err {eG:.2e}", flush=True)
    tol = {"f64": 1e-12, "f32": 2e-5}[storage]
    assert eJ < tol and eG < tol


@pytest.mark.parametrize("case,storage,q", [("sphere", "f64", 27), ("sphere", "f32", 27), ("rotor", "f64", 27),
                                            ("rotor", "f32", 27), ("rotor", "f64", 19)])
def test_adjoint_with_hybrid_strain_matches_oracle(case, storage, q):
    """fd_share > 0 (the hybrid non-equilibrium of Sec. 2.2 off the wall):
    the strain of the element cells is the central difference of the
    neighbours' velocities, so the adjoint reaches them through it; the
    oracle's adjoint of the same scheme is pinned by complex step."""
    hl = _hl()
    w, n, t0, t1 = _cases()[case]
    w.q = q
    w.params.fd_share = 0.4 if case == "sphere" else 0.3
    print(f"[adjoint-fd] {case} D3Q{q} {storage}", flush=True)
    o = O.setup(w)
    J_or, G_or = o.adjoint_run(n, t0, t1, obj_tag=0, ckpt_every=4)
    lat = hl.setup(w, storage=storage, flags=hl.WITH_ADJOINT)
    J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=4)
    G = lat.adjoint(1.0).cpu().numpy()
    eJ = abs(J - J_or) / _torque_scale(o, t0, t1)
    eG = np.abs(G - G_or).max() / np.abs(G_or).max()
    print(f"[adjoint-fd] {case} D3Q{q} {storage}: J {J:.6e} vs {J_or:.6e} (rel {eJ:.2e}); G rel err {eG:.2e}",
          flush=True)
    tol = {"f64": 1e-12, "f32": 2e-5}[storage]
    assert eJ < tol
    assert eG < tol
    # the strain does change the gradient: the local scheme's differs
    w.params.fd_share = 0.0
    _, G_loc = O.setup(w).adjoint_run(n, t0, t1, obj_tag=0, ckpt_every=4)
    assert np.abs(G_loc - G_or).max() > 100 * tol * np.abs(G_or).max()


def test_adjoint_with_hybrid_strain_independent_of_checkpoint_spacing():
    """The strain's velocity adjoints join the fixed-point sums of the probe
    velocities: gradients agree bit for bit across checkpoint spacings."""
    hl = _hl()
    w, n, t0, t1 = _cases()["rotor"]
    w.params.fd_share = 0.3
    lat = hl.setup(w, storage="f64", flags=hl.WITH_ADJOINT)
    state0 = lat.get_state().clone()
    res = {}
    for ce in (1, 4, n):
        lat.set_state(state0)
        J = lat.forward_record(n, t0, t1, obj_tag=0, ckpt_every=ce)
        res[ce] = (J, lat.adjoint(1.0).cpu().numpy())
    J4, G4 = res[4]
    for ce, (J, G) in res.items():
        assert J == J4
        assert np.array_equal(G, G4), (ce, np.abs(G - G4).max())
