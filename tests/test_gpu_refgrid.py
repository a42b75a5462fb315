"""Reference-grid rotors (Sec. 3.1: a moving element voxelized once on its
own reference grid and embedded into the lattice porosity at its position
and orientation every step) on the device against the oracle on the same
seeded inputs: a capsule-blade rotor on a half-cell grid (the paper
resolves its reference grid at twice the lattice resolution), with the wall
model and inflow turbulence.  Populations, forces and torques at FP64
1e-12 and FP32 2e-5, as for the flat-plate rotors."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W
from parity_metrics import force_torque_error, rel

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}


def _hl():
    from paper_2510_13726_amd import hlbm
    return hlbm


def _grid_rotor(q=27):
    w = W.small_rotor(nx=72, ny=44, nz=40, R=12.0, chord=4.0, hub=2.0, tau0=0.51, turb=0.05)
    w.q = q
    r = w.rotors[0]
    r.grid = W.capsule_rotor_grid(r, spacing=0.5, eps_h=w.params.eps_h)
    return w


@pytest.mark.parametrize("storage,q", [("f64", 27), ("f32", 27), ("f64", 19)])
def test_reference_grid_rotor_parity(storage, q):
    hl = _hl()
    w = _grid_rotor(q)
    n = 24
    print(f"[refgrid] {w.name} q={q} storage={storage} grid {w.rotors[0].grid.phi.shape} steps={n}", flush=True)
    lat = hl.setup(w, storage=storage, check_nonfinite=1)
    o = O.setup(w)
    lat.step(n)
    o.step(n)
    eF, eT = force_torque_error(lat.history(), o.history(), o.history_scale())
    ep = rel(lat.get_populations().cpu().numpy(), o.get_populations())
    it, cells = lat.wall_stats()
    print(f"[refgrid] D3Q{q} {storage}: pops {ep:.2e} F {eF:.2e} T {eT:.2e}, wall cells {cells}, newton {it}",
          flush=True)
    assert cells > 0
    assert ep < TOL[storage] and eF < TOL[storage] and eT < TOL[storage]
    assert lat.wall_safeguards() == (0, 0)


def test_coupled_reference_grid_rotor_parity():
    """Two-way coupling (Sec. 3.2) turns the grid body with the torque it
    receives: the angle and speed follow the oracle within the torque
    tolerance carried through the rotor ODE."""
    hl = _hl()
    w = _grid_rotor()
    w.rotors[0].inertia = 1e6
    w.rotors[0].torque_gen = 2.0
    n = 24
    lat = hl.setup(w, storage="f64", check_nonfinite=1)
    o = O.setup(w)
    om_g, om_o = [], []
    for _ in range(n):
        lat.step(1)
        o.step(1)
        om_g.append(lat.rotor_state()[1][0])
        om_o.append(o.rotor_state()[1][0])
    om_g, om_o = np.array(om_g), np.array(om_o)
    scale = o.history_scale()[:, 0, 1]
    bound = np.cumsum(1e-12 * scale) / w.rotors[0].inertia + 4e-16 * np.abs(om_o)
    ep = rel(lat.get_populations().cpu().numpy(), o.get_populations())
    eF, eT = force_torque_error(lat.history(), o.history(), o.history_scale())
    print(f"[refgrid] coupled: Omega {om_o[0]:.6f} -> {om_o[-1]:.6f}, speed err {np.abs(om_g - om_o).max():.2e}, "
          f"pops {ep:.2e} F {eF:.2e} T {eT:.2e}", flush=True)
    assert om_o[-1] != om_o[0]
    assert np.all(np.abs(om_g - om_o) <= bound)
    assert ep < 1e-12 and eF < 1e-12 and eT < 1e-12


def test_reference_grid_kept_across_a_parameter_change():
    """eps_h raised from 2 to 3 mid-run rebuilds the rotor boxes; the grid
    stays with its rotor and the run continues as the oracle's (the grid
    reaches eps_h/2 + 2 = 3 cells beyond the body, enough for eps_h = 3)."""
    hl = _hl()
    w = _grid_rotor()
    lat = hl.setup(w, storage="f64", check_nonfinite=1)
    o = O.setup(w)
    lat.step(6)
    o.step(6)
    w.params.eps_h = 3.0
    lat.set_params(w.params, check_nonfinite=1)
    o.set_params(w.params)
    lat.step(6)
    o.step(6)
    ep = rel(lat.get_populations().cpu().numpy(), o.get_populations())
    eF, eT = force_torque_error(lat.history(), o.history(), o.history_scale())
    print(f"[refgrid] eps_h 2 -> 3: pops {ep:.2e} F {eF:.2e} T {eT:.2e}", flush=True)
    assert ep < 1e-12 and eF < 1e-12 and eT < 1e-12
    assert lat.wall_stats() == o.newton_stats()


def test_reference_grid_differs_from_the_flat_plates_and_removal_restores_them():
    """The grid body is another solid than the flat-plate rotor of the same
    parameters; removing the grid gives back the flat-plate run bit for bit."""
    hl = _hl()
    w = _grid_rotor()
    grid = w.rotors[0].grid
    w.rotors[0].grid = None
    ref = hl.setup(w, storage="f64")
    ref.step(6)
    h_ref = ref.get_populations().cpu().numpy()
    lat = hl.setup(w, storage="f64")
    state0 = lat.get_state().clone()
    lat.set_rotor_grid(0, grid)
    lat.step(3)
    h_grid = lat.get_populations().cpu().numpy()
    lat.set_rotor_grid(0, None)
    lat.set_state(state0)
    lat.step(6)
    assert np.array_equal(lat.get_populations().cpu().numpy(), h_ref)
    ref3 = hl.setup(w, storage="f64")
    ref3.step(3)
    assert np.abs(h_grid - ref3.get_populations().cpu().numpy()).max() > 1e-6


def test_reference_grid_arguments_are_checked():
    hl = _hl()
    w = _grid_rotor()
    g = w.rotors[0].grid
    w.rotors[0].grid = None
    lat = hl.setup(w, storage="f32")
    bad = [W.RefGrid(phi=g.phi[:1], spacing=0.5, origin=g.origin),
           W.RefGrid(phi=g.phi, spacing=0.0, origin=g.origin),
           W.RefGrid(phi=g.phi, spacing=0.5, origin=(float("nan"), 0.0, 0.0))]
    for b in bad:
        with pytest.raises(hl.HlbmError) as e:
            lat.set_rotor_grid(0, b)
        assert e.value.code == hl.HLBM_ERR_INVALID
    with pytest.raises(hl.HlbmError):
        lat.set_rotor_grid(8, g)
    # a rotor without blades cannot orient a grid
    w.rotors[0].n_blades = 0
    lat.set_rotors(w.rotors)
    with pytest.raises(hl.HlbmError):
        lat.set_rotor_grid(0, g)
