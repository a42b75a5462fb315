"""Pins of the oracle's hybrid non-equilibrium off the wall (Sec. 2.2:
f~(1) = sigma f(1) - (1 - sigma) f(1,FD), f(1,FD) = rho tau / cs^2 H2 : S^FD
with a non-local finite-difference strain).  The strain and the second
moment the collision must produce are computed here independently with
numpy from the state: pulled populations by periodic shifts, velocity
moments, central differences by np.roll."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_13726_amd import workloads as W

CS2 = 1.0 / 3.0


def _box(fd_share, n=(12, 10, 8), seed=3, Cs=0.12):
    nx, ny, nz = n
    p = W.Params(tau0=0.62, cs_smag=Cs, eps_h=2.0, fd_share=fd_share)
    w = W.Workload("fd_box", nx, ny, nz, W.BC_PERIODIC, p, [], 1, init="uniform", u0=0.0)
    o = O.OracleLattice(nx, ny, nz, 0)
    o.set_params(p)
    o.set_rotors([])
    # every cell belongs to element 1 (tag 1) with porosity d = 0
    o.set_porosity_field(np.zeros(w.cells), np.ones(w.cells, dtype=np.uint8))
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.stack([0.03 * np.sin(2 * math.pi * y / ny + 0.3) + 0.01 * np.cos(2 * math.pi * z / nz),
                  0.02 * np.cos(2 * math.pi * x / nx) * np.sin(2 * math.pi * z / nz),
                  0.015 * np.sin(2 * math.pi * (x / nx + y / ny))]).reshape(3, -1)
    rho = 1.0 + 0.01 * np.cos(2 * math.pi * x / nx).reshape(-1)
    o.init_equilibrium(rho, u)
    h = o.get_populations()
    o.set_populations(h + 1e-4 * rng.standard_normal(h.shape) * (np.abs(h) + 1e-3))
    return o, (nx, ny, nz), p


def _pulled(o, shape):
    """Pre-collision populations f_i(x) = w_i + h_i(x - c_i) (periodic)."""
    nx, ny, nz = shape
    c, wts = O.lattice_tables()
    h = o.get_populations().reshape(27, nz, ny, nx)
    f = np.empty_like(h)
    for i in range(27):
        f[i] = wts[i] + np.roll(h[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
    return f.reshape(27, -1), c.astype(float), wts


@pytest.mark.parametrize("fd_share", [1.0, 0.5])
def test_fd_strain_second_moment(fd_share):
    o, shape, p = _box(fd_share)
    nx, ny, nz = shape
    f, c, wts = _pulled(o, shape)
    rho = f.sum(axis=0)
    j = c.T @ f
    u = j / rho
    P = np.einsum("ia,ib,in->abn", c, c, f)
    Pi = P - rho * CS2 * np.eye(3)[:, :, None] - rho * np.einsum("an,bn->abn", u, u)
    Q = np.sqrt(np.einsum("abn,abn->n", Pi, Pi))
    tau = 0.5 * (p.tau0 + np.sqrt(p.tau0 ** 2 + 18 * math.sqrt(2) * p.cs_smag ** 2 * Q / rho))
    ug = u.reshape(3, nz, ny, nx)
    du = np.empty((3, 3, nz, ny, nx))   # du[a][b] = d_b u_a, axes b: x, y, z
    for a in range(3):
        for b, ax in ((0, 2), (1, 1), (2, 0)):
            du[a, b] = 0.5 * (np.roll(ug[a], -1, axis=ax) - np.roll(ug[a], 1, axis=ax))
    S = 0.5 * (du + du.transpose(1, 0, 2, 3, 4))
    S = S.reshape(3, 3, -1)
    o.step(1)
    fs = o.get_populations() + wts[:, None]
    Ps = np.einsum("ia,ib,in->abn", c, c, fs)
    sig = 1.0 - fd_share
    expect = rho * CS2 * np.eye(3)[:, :, None] + rho * np.einsum("an,bn->abn", u, u) + \
        (1 - 1 / tau) * (sig * Pi - (1 - sig) * 2 * rho * tau * CS2 * S)
    err = np.abs(Ps - expect).max()
    print(f"fd_share {fd_share}: max |P* - expected| {err:.2e}, |S| max {np.abs(S).max():.2e}")
    assert np.abs(S).max() > 1e-3
    assert err < 1e-14


def test_fd_share_zero_is_the_local_scheme():
    a, _, _ = _box(0.0)
    b, _, _ = _box(0.0)
    b_params = W.Params(tau0=0.62, cs_smag=0.12, eps_h=2.0)
    b.set_params(b_params)
    a.step(3)
    b.step(3)
    assert np.array_equal(a.get_populations(), b.get_populations())


def test_fd_strain_only_in_element_cells():
    """Cells of tag 0 keep sigma = 1: with no tagged cell, fd_share changes
    nothing."""
    a, shape, _ = _box(1.0)
    b, _, _ = _box(0.0)
    n = a.N
    for o in (a, b):
        o.set_porosity_field(np.zeros(n), np.zeros(n, dtype=np.uint8))
        o.step(2)
    assert np.array_equal(a.get_populations(), b.get_populations())
