"""Pins of the oracle's reference-grid embedding (Sec. 3.1: a moving element
voxelized once on its own reference grid, embedded into the lattice
porosity at its position and orientation every step).

The sample is the trilinear interpolant of the grid in the rotor's body
frame (blade 0's radial direction, the tangential direction, the axis) at
the rotor's angle.  The pins rest on facts that hold apart from the code:
- trilinear interpolation reproduces an affine field exactly, value and
  gradient, so a transposed index, a wrong origin or spacing, or a rotation
  of the wrong sense changes the result;
- the body turns rigidly: the sample at angle theta at the point rotated by
  theta about the axis (Rodrigues' formula) equals the sample at angle 0;
- at grid nodes the sample is the stored value;
- a capsule body agrees with its closed-form distance within the
  interpolation error of a half-cell grid.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W


def _rotor(axis=(0.0, 0.0, 1.0), center=(20.0, 18.0, 16.0)):
    return W.Rotor(center=center, axis=axis, R=8.0, r_hub=1.5, chord=3.0, thick=2.0, n_blades=3, tag=2)


def _affine_grid(a, b, origin, n, h):
    i0 = np.arange(n[0]); i1 = np.arange(n[1]); i2 = np.arange(n[2])
    p2, p1, p0 = np.meshgrid(origin[2] + h * i2, origin[1] + h * i1, origin[0] + h * i0, indexing="ij")
    return W.RefGrid(phi=a + b[0] * p0 + b[1] * p1 + b[2] * p2, spacing=h, origin=tuple(origin))


def _rodrigues(k, v, ang):
    k = np.asarray(k, dtype=float) / np.linalg.norm(k)
    v = np.asarray(v, dtype=float)
    return v * math.cos(ang) + np.cross(k, v) * math.sin(ang) + k * np.dot(k, v) * (1.0 - math.cos(ang))


def test_affine_field_is_sampled_exactly_about_the_z_axis():
    """Axis z: blade 0 points along (cos t, sin t, 0) at angle t, the
    tangential direction along (-sin t, cos t, 0)."""
    r = _rotor()
    a, b = 0.37, np.array([0.61, -1.13, 2.29])
    origin, n, h = (-6.3, -5.1, -3.7), (27, 23, 17), 0.5
    g = _affine_grid(a, b, origin, n, h)
    th = 0.7
    er = np.array([math.cos(th), math.sin(th), 0.0])
    ep = np.array([-math.sin(th), math.cos(th), 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(5)
    for _ in range(40):
        rel = rng.uniform(-3.0, 3.0, 3) * np.array([1.0, 1.0, 0.8])
        x = np.asarray(r.center) + rel
        phi, grad = O.grid_rotor_phi(r, g, x, th)
        p = np.array([rel @ er, rel @ ep, rel @ ez])
        assert abs(phi - (a + b @ p)) < 1e-12
        assert np.abs(grad - (b[0] * er + b[1] * ep + b[2] * ez)).max() < 1e-12
    # the opposite sense of rotation would give another value
    rel = np.array([2.0, 1.0, 0.5])
    p_wrong = np.array([rel @ (er * [1, -1, 1]), rel @ (ep * [-1, 1, 1]), rel[2]])
    phi, _ = O.grid_rotor_phi(r, g, np.asarray(r.center) + rel, th)
    assert abs(phi - (a + b @ p_wrong)) > 0.1


def test_axial_field_on_a_tilted_axis_and_rigid_rotation():
    """On a tilted axis an affine field of the axial coordinate alone is
    sampled exactly; any field turns rigidly with the rotor angle."""
    axis = (0.3, 1.0, 0.2)
    e = np.asarray(axis) / np.linalg.norm(axis)
    r = _rotor(axis=axis)
    g_ax = _affine_grid(0.2, np.array([0.0, 0.0, 1.7]), (-5.0, -5.0, -3.0), (21, 21, 13), 0.5)
    rng = np.random.default_rng(7)
    for _ in range(20):
        rel = rng.uniform(-2.0, 2.0, 3)
        phi, grad = O.grid_rotor_phi(r, g_ax, np.asarray(r.center) + rel, 1.1)
        assert abs(phi - (0.2 + 1.7 * rel @ e)) < 1e-12
        assert np.abs(grad - 1.7 * e).max() < 1e-12
    # a random (non-affine) grid: the sample at angle th at the point turned
    # by th about the axis equals the sample at angle 0 at the point
    grid = W.RefGrid(phi=rng.normal(size=(13, 21, 21)), spacing=0.5, origin=(-5.0, -5.0, -3.0))
    for th in (0.4, -1.3, 2.9):
        for _ in range(10):
            rel0 = rng.uniform(-2.5, 2.5, 3)
            x0 = np.asarray(r.center) + rel0
            x = np.asarray(r.center) + _rodrigues(e, rel0, th)
            v0, g0 = O.grid_rotor_phi(r, grid, x0, 0.0)
            v1, g1 = O.grid_rotor_phi(r, grid, x, th)
            assert abs(v1 - v0) < 1e-12
            assert np.abs(g1 - _rodrigues(e, g0, th)).max() < 1e-11


def test_nodes_return_the_stored_values_and_outside_is_not_body():
    """Axis z, angle 0 (blade 0 along x), spacing 1 and an integer origin:
    lattice points fall on nodes, (x, y, z) - c - origin = (i0, i1, i2)."""
    r = _rotor(center=(10.0, 12.0, 9.0))
    rng = np.random.default_rng(11)
    n = (9, 7, 5)
    phi = rng.normal(size=(n[2], n[1], n[0]))
    g = W.RefGrid(phi=phi, spacing=1.0, origin=(-4.0, -3.0, -2.0))
    for i0, i1, i2 in [(0, 0, 0), (8, 6, 4), (3, 5, 1), (7, 2, 3), (4, 3, 2)]:
        x = np.array([10.0 - 4.0 + i0, 12.0 - 3.0 + i1, 9.0 - 2.0 + i2])
        v, _ = O.grid_rotor_phi(r, g, x, 0.0)
        assert v == phi[i2, i1, i0]
    # beyond the last node along any axis: not in the body
    for x in ([10.0 + 4.5, 12.0, 9.0], [10.0, 12.0 - 3.25, 9.0], [10.0, 12.0, 9.0 + 2.01]):
        v, gr = O.grid_rotor_phi(r, g, np.asarray(x), 0.0)
        assert v == -1e300 and not np.any(gr)


def test_capsule_body_matches_its_closed_form_within_the_interpolation_error():
    r = W.Rotor(center=(30.0, 30.0, 30.0), axis=(1.0, 0.0, 0.0), R=12.0, r_hub=2.0, chord=4.0, thick=2.0,
                n_blades=3, phase0=0.3, tag=1)
    g = W.capsule_rotor_grid(r, spacing=0.5)
    e = np.array([1.0, 0.0, 0.0])
    # blade 0's radial direction at angle th, read off as the gradient of the
    # affine field p0 (so the test does not restate the frame's construction)
    probe = _affine_grid(0.0, np.array([1.0, 0.0, 0.0]), g.origin, g.phi.shape[::-1], g.spacing)
    th = 0.9
    _, er = O.grid_rotor_phi(r, probe, np.asarray(r.center), th)
    ep = np.cross(e, er)
    rad, tilt, h = 1.0, 1.0, g.spacing
    rng = np.random.default_rng(3)
    errs, smooth = [], []
    for _ in range(4000):
        rel = rng.uniform(-13.0, 13.0, 3) * np.array([0.25, 1.0, 1.0])
        p = np.array([rel @ er, rel @ ep, rel @ e])
        pieces = [(r.r_hub - np.linalg.norm(p), False)]
        for b in range(3):
            a = 2.0 * math.pi * b / 3
            d = np.array([math.cos(a), math.sin(a), 0.0])
            A = 0.5 * r.r_hub * d - np.array([0.0, 0.0, tilt])
            B = (r.R - rad) * d + np.array([0.0, 0.0, tilt])
            t = np.clip((p - A) @ (B - A) / ((B - A) @ (B - A)), 0.0, 1.0)
            dist = np.linalg.norm(p - (A + t * (B - A)))
            # the lateral surface of the capsule, away from its axis and caps
            pieces.append((rad - dist, 0.05 < t < 0.95 and dist > 1.0))
        pieces.sort(key=lambda q: -q[0])
        best = pieces[0][0]
        if abs(best) > 1.5:
            continue
        v, _ = O.grid_rotor_phi(r, g, np.asarray(r.center) + rel, th)
        errs.append(abs(v - best))
        # one smooth piece wins by more than the cell diagonal: no crease in reach
        if pieces[0][1] and pieces[0][0] - pieces[1][0] > 2.0 * math.sqrt(3.0) * h:
            smooth.append(abs(v - best))
    errs, smooth = np.array(errs), np.array(smooth)
    print(f"capsule: {len(errs)} points in the band, max error {errs.max():.3e}, mean {errs.mean():.3e}; "
          f"{len(smooth)} on smooth surface, max {smooth.max():.3e}")
    assert len(errs) > 200 and len(smooth) > 100
    # a distance is 1-Lipschitz: no sample is farther from it than a corner
    assert errs.max() < math.sqrt(3.0) * h and errs.mean() < 0.03
    # where the distance is smooth with |d2 phi| <= 1 / dist <= 1, trilinear
    # error <= h^2 / 8 (sum of the three second derivatives) <= 3 h^2 / 8
    assert smooth.max() < 3.0 * h * h / 8.0
