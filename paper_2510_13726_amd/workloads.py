"""Seeded synthetic workloads: lattice sizes, parameters, rotor tables and
initial fields.

This module holds only input recipes (sizes, constants, seeded random
numbers, initial density/velocity fields and static porosity inputs).  It
contains none of the method's arithmetic, so both the HIP path and the
oracle read their inputs from here.

The rotors are synthetic flat-plate turbines standing in for the paper's
model wind turbine (Sec. 4: rotor geometry from an STL file that is not
available); the parameters follow the paper's setup where it states one
(lattice velocity 0.05, Sec. 4; rotor 20 % of the domain length behind the
inlet, Sec. 4, Fig. domain).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

BC_PERIODIC = 0
BC_INFLOW_OUTFLOW = 1
TRANSITION_TANH = 0
TRANSITION_LINEAR = 1


@dataclasses.dataclass
class Params:
    tau0: float = 0.55
    cs_smag: float = 0.1
    eps_h: float = 2.0
    transition: int = TRANSITION_TANH
    wall_model: int = 0
    E: float = 9.8
    kappa: float = 0.41
    y_s: float = 3.0
    tol: float = 1e-4
    maxit: int = 10
    u_in: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    turb_I: float = 0.0
    seed: int = 0
    force_mode: int = 0         # 1: also record the momentum-exchange force
    fd_share: float = 0.0       # 1 - sigma off the wall in element cells (hybrid f~(1))


@dataclasses.dataclass
class RefGrid:
    """A moving element on its own reference grid: signed distance phi
    (positive inside), shape (n2, n1, n0), at body coordinates
    origin + spacing (i0, i1, i2); body axes the radial direction of blade 0,
    the tangential direction (axis x radial) and the rotor axis."""
    phi: np.ndarray
    spacing: float
    origin: Tuple[float, float, float]


@dataclasses.dataclass
class Rotor:
    center: Tuple[float, float, float]
    axis: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    R: float = 40.0
    r_hub: float = 4.0
    chord: float = 6.0
    thick: float = 3.0
    twist_root: float = math.radians(20.0)
    twist_tip: float = math.radians(5.0)
    omega: float = 0.0075
    phase0: float = 0.0
    n_blades: int = 3
    tag: int = 1
    inertia: float = 0.0        # > 0: rotation driven by the fluid torque (two-way coupling)
    torque_gen: float = 0.0     # opposing generator torque of a coupled rotor
    grid: Optional[RefGrid] = None  # reference-grid body replacing the flat-plate blades and hub


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    bc_x: int
    params: Params
    rotors: List[Rotor]
    steps: int
    init: str = "uniform"          # "uniform" or "tgv"
    u0: float = 0.05               # initial / free-stream velocity (x) or TGV amplitude
    sphere: Optional[Tuple[float, float, float, float]] = None  # static sphere (cx, cy, cz, R), tag 1
    noise_seed: Optional[int] = None  # seeded non-equilibrium perturbation of the initial state
    noise_amp: float = 1e-5
    q: int = 27                    # velocity set: 27 (D3Q27) or 19 (D3Q19)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


def capsule_rotor_grid(r: Rotor, spacing: float = 0.5, eps_h: float = 2.0) -> RefGrid:
    """A synthetic element on a reference grid of `spacing` lattice units
    (the paper resolves its reference grid at twice the lattice resolution,
    Sec. 3.1), standing in for the voxelized STL rotor: a hub sphere of
    radius r_hub and n_blades capsule blades of radius thick/2 whose axes
    run from r_hub/2 to R - thick/2 along each blade's radial direction,
    tilted axially from root to tip by +-min(chord/4, h_c - thick/2), h_c =
    sqrt((chord/2)^2 + (thick/2)^2).  The body lies within the
    flat-plate rotor's envelope (radius R, axial half extent
    max(sqrt((chord/2)^2 + (thick/2)^2), r_hub)); the grid reaches
    eps_h/2 + 2 cells beyond it."""
    rad = 0.5 * r.thick
    hc = math.sqrt(0.25 * r.chord ** 2 + 0.25 * r.thick ** 2)
    tilt = max(0.0, min(0.25 * r.chord, hc - rad))
    ha = max(hc, r.r_hub)
    m = 0.5 * eps_h + 2.0
    lo = np.array([-(r.R + m), -(r.R + m), -(ha + m)])
    n = [int(math.ceil(-2.0 * lo[k] / spacing)) + 1 for k in range(3)]
    ax = [lo[k] + spacing * np.arange(n[k]) for k in range(3)]
    p2, p1, p0 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    P = np.stack([p0, p1, p2], axis=-1)
    phi = r.r_hub - np.linalg.norm(P, axis=-1)
    for b in range(max(r.n_blades, 1)):
        a = 2.0 * math.pi * b / max(r.n_blades, 1)
        d = np.array([math.cos(a), math.sin(a), 0.0])
        A = 0.5 * r.r_hub * d + np.array([0.0, 0.0, -tilt])
        B = (r.R - rad) * d + np.array([0.0, 0.0, tilt])
        AB = B - A
        t = np.clip(((P - A) @ AB) / (AB @ AB), 0.0, 1.0)
        dist = np.linalg.norm(P - (A + t[..., None] * AB), axis=-1)
        phi = np.maximum(phi, rad - dist)
    return RefGrid(phi=np.ascontiguousarray(phi), spacing=spacing, origin=(float(lo[0]), float(lo[1]), float(lo[2])))


# ----------------------------------------------------------------- configs
def config1(noise: bool = False, n: int = 32) -> Workload:
    """Periodic n^3 box, 3D Taylor-Green vortex (U0 = 0.02), tau0 = 0.55,
    C_S = 0.1, static porous sphere (R = 6, tanh edge over 2 cells) at rest,
    wall model off, 100 steps."""
    c = n / 2.0
    return Workload("tgv_sphere_32", n, n, n, BC_PERIODIC,
                    Params(tau0=0.55, cs_smag=0.1, eps_h=2.0, wall_model=0),
                    [], 100, init="tgv", u0=0.02, sphere=(c, c, c, 6.0 * n / 32.0),
                    noise_seed=1 if noise else None)


def _rotor_channel(name, nx, ny, nz, R, chord, hub, omega, steps, turb=0.0, seed=0,
                   centers=None, phases=None, thick=3.0, tau0=0.5005) -> Workload:
    if centers is None:
        centers = [(0.2 * nx, ny / 2.0, nz / 2.0)]
    if phases is None:
        phases = [0.0] * len(centers)
    rotors = [Rotor(center=tuple(float(v) for v in cc), R=R, r_hub=hub, chord=chord, thick=thick,
                    omega=omega, phase0=float(ph), tag=k + 1)
              for k, (cc, ph) in enumerate(zip(centers, phases))]
    p = Params(tau0=tau0, cs_smag=0.1, eps_h=2.0, wall_model=1, u_in=(0.05, 0.0, 0.0),
               turb_I=turb, seed=seed)
    return Workload(name, nx, ny, nz, BC_INFLOW_OUTFLOW, p, rotors, steps, init="uniform", u0=0.05)


def config2() -> Workload:
    """256x128x128 channel, inflow U = 0.05, 3-blade rotor R = 40 (chord 6,
    hub 4, twist 20->5 deg) at tip-speed ratio 6, tau0 = 0.5005, C_S = 0.1,
    wall model on, 20k steps."""
    return _rotor_channel("rotor_channel_256x128x128", 256, 128, 128, R=40.0, chord=6.0, hub=4.0,
                          omega=6 * 0.05 / 40.0, steps=20000, centers=[(51.0, 64.0, 64.0)])


def config3(coarse: bool = False) -> Workload:
    """1024x512x384 channel, rotor R = 120 (chord 18, hub 12), 5 % seeded
    inflow turbulence, 2k steps.  `coarse` gives the 4x-coarsened copy."""
    if coarse:
        return _rotor_channel("rotor_wake_256x128x96", 256, 128, 96, R=30.0, chord=4.5, hub=3.0,
                              omega=6 * 0.05 / 30.0, steps=2000, turb=0.05, seed=3,
                              centers=[(51.25, 64.0, 48.0)])
    return _rotor_channel("rotor_wake_1024x512x384", 1024, 512, 384, R=120.0, chord=18.0, hub=12.0,
                          omega=6 * 0.05 / 120.0, steps=2000, turb=0.05, seed=3,
                          centers=[(205.0, 256.0, 192.0)])


def config4() -> Workload:
    """128x64x64 channel, rotor R = 20 (chord 3, hub 2); objective = axial
    torque averaged over steps [1000, 2000)."""
    return _rotor_channel("rotor_adjoint_128x64x64", 128, 64, 64, R=20.0, chord=3.0, hub=2.0,
                          omega=6 * 0.05 / 20.0, steps=2000, centers=[(26.0, 32.0, 32.0)])


def config5() -> Workload:
    """1536x768x256 domain, 4x2 array of rotors R = 48 (spacing 5R streamwise,
    3R spanwise), seeded phase offsets in [0, 2pi/3), 5k steps."""
    rng = np.random.default_rng(5)
    centers = [(x, y, 128.0) for x in (230.0, 470.0, 710.0, 950.0) for y in (312.0, 456.0)]
    phases = rng.uniform(0.0, 2.0 * math.pi / 3.0, size=len(centers))
    return _rotor_channel("rotor_array_1536x768x256", 1536, 768, 256, R=48.0, chord=7.2, hub=4.8,
                          omega=6 * 0.05 / 48.0, steps=5000, centers=centers, phases=phases)


def small_rotor(nx=64, ny=48, nz=48, R=12.0, chord=4.0, hub=2.0, tau0=0.51, turb=0.0,
                wall=1, steps=20) -> Workload:
    """A few-tile rotor channel the oracle finishes in seconds (parity case)."""
    w = _rotor_channel(f"small_rotor_{nx}x{ny}x{nz}", nx, ny, nz, R=R, chord=chord, hub=hub,
                       omega=6 * 0.05 / R, steps=steps, turb=turb, seed=7,
                       centers=[(0.3 * nx, ny / 2.0 + 0.37, nz / 2.0 - 0.21)], tau0=tau0)
    w.params.wall_model = wall
    return w


ALL = {"1": config1, "2": config2, "3": config3, "4": config4, "5": config5}


# ----------------------------------------------------------- input fields
def initial_fields(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """Initial density (N,) and velocity (3, N) as FP64, layout [z][y][x]."""
    z, y, x = np.meshgrid(np.arange(w.nz), np.arange(w.ny), np.arange(w.nx), indexing="ij")
    if w.init == "tgv":
        k = 2.0 * math.pi / w.nx
        U0 = w.u0
        ux = U0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
        uy = -U0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
        uz = np.zeros_like(ux)
        rho = 1.0 + 3.0 * (U0 ** 2 / 16.0) * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    else:
        rho = np.ones(x.shape)
        ux = np.full(x.shape, w.u0)
        uy = np.zeros(x.shape)
        uz = np.zeros(x.shape)
    u = np.stack([ux, uy, uz]).reshape(3, -1)
    return rho.reshape(-1).astype(np.float64), u.astype(np.float64)


def static_porosity(w: Workload) -> Tuple[Optional[np.ndarray], Optional[np.ndarray]]:
    """Static porosity input (N,) and tags (N,) for a workload with a sphere:
    d = 1 inside, 0 outside, tanh edge of width eps_h centred on the surface
    (d = 1/2 there)."""
    if w.sphere is None:
        return None, None
    cx, cy, cz, R = w.sphere
    z, y, x = np.meshgrid(np.arange(w.nz), np.arange(w.ny), np.arange(w.nx), indexing="ij")
    dist = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    phi = (R - dist).reshape(-1)
    eps = w.params.eps_h
    d = 0.5 * (1.0 + np.tanh(4.0 * phi / eps) / np.tanh(2.0))
    d = np.where(phi <= -eps / 2, 0.0, np.where(phi >= eps / 2, 1.0, d))
    tag = (d > 0).astype(np.uint8)
    return d.astype(np.float64), tag


def population_noise(w: Workload) -> Optional[np.ndarray]:
    """Seeded perturbation (27, N) added to the initial shifted populations."""
    if w.noise_seed is None:
        return None
    rng = np.random.default_rng(w.noise_seed)
    return rng.uniform(-w.noise_amp, w.noise_amp, size=(27, w.cells))


def random_cells(w: Workload, count: int, seed: int, region: str = "rotor") -> np.ndarray:
    """Seeded cell indices; region "rotor" draws inside the first rotor's
    bounding cylinder, "any" anywhere."""
    rng = np.random.default_rng(seed)
    if region == "any" or not w.rotors:
        return rng.choice(w.cells, size=count, replace=False)
    r = w.rotors[0]
    out = set()
    while len(out) < count:
        th = rng.uniform(0, 2 * math.pi)
        rad = r.R * math.sqrt(rng.uniform(0, 1))
        ax = rng.uniform(-r.chord, r.chord)
        x = int(round(r.center[0] + ax))
        y = int(round(r.center[1] + rad * math.cos(th)))
        z = int(round(r.center[2] + rad * math.sin(th)))
        out.add((z * w.ny + y) * w.nx + x)
    return np.array(sorted(out), dtype=np.int64)


def x_slab(w: Workload, x0: int, length: int) -> Workload:
    """The cells x0 <= x < x0 + length of `w` (all of y and z) as a workload
    of its own, for light-cone comparisons of a large run against a small
    one: rotors are moved by -x0, and the slab is periodic in x unless it
    starts at the inlet (then it keeps the inflow, and its last plane is an
    outflow that the large run does not have).  After n steps the cells
    farther than the per-step dependency reach times n from the slab's cut
    faces hold the same values as in `w`."""
    import copy
    s = copy.deepcopy(w)
    s.name = f"{w.name}_x{x0}+{length}"
    s.nx = int(length)
    if x0 != 0:
        s.bc_x = BC_PERIODIC
    for r in s.rotors:
        r.center = (r.center[0] - x0, r.center[1], r.center[2])
    return s
