"""Wake velocity profiles of the rotor wake workload on its 4x-coarsened copy
(256x128x96, rotor R = 30): the streamwise velocity u_x averaged over
azimuth on radial lines in the planes x_c + 2R and x_c + 5R downstream of
the rotor, and over the last 500 of 2000 steps (the counterpart of the
radial-line velocity comparisons of the paper's Sec. 4).

`profile` and `planes` are the post-processing both sides of the check use.
Run as a script, this module writes the FP64 oracle's profiles to
wake_profiles_256x128x96.json next to it; it calls only the oracle and the
input recipes (about two hours on 8 host cores).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
FIXTURE = os.path.join(HERE, "wake_profiles_256x128x96.json")
STEPS = 2000
AVERAGE = 500        # last steps averaged
NBINS = 45           # radial bins of one cell, r in [0, 45) = [0, 1.5 R)


def planes(w):
    """x indices of the planes x_c + 2R and x_c + 5R."""
    r = w.rotors[0]
    return [int(round(r.center[0] + 2 * r.R)), int(round(r.center[0] + 5 * r.R))]


def profile(ux_plane, w, nbins=NBINS):
    """Azimuthal mean of u_x over annuli of unit width around the rotor axis
    (cells at distance r from the axis in bin floor(r)), ux_plane (nz, ny)."""
    r0 = w.rotors[0]
    z, y = np.meshgrid(np.arange(w.nz), np.arange(w.ny), indexing="ij")
    rad = np.sqrt((y - r0.center[1]) ** 2 + (z - r0.center[2]) ** 2)
    b = np.floor(rad).astype(int)
    out = np.full(nbins, np.nan)
    for k in range(nbins):
        m = b == k
        if m.any():
            out[k] = float(np.asarray(ux_plane)[m].mean())
    return out


def main():
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_2510_13726_amd import workloads as W
    w = W.config3(coarse=True)
    o = O.setup(w, threads=os.cpu_count())
    xs = planes(w)
    acc = np.zeros((2, NBINS))
    t0 = time.time()
    for n in range(STEPS):
        if n >= STEPS - AVERAGE:
            rho, u = o.moments()
            ux = u[0].reshape(w.nz, w.ny, w.nx)
            for k, x in enumerate(xs):
                acc[k] += profile(ux[:, :, x], w)
        o.step(1)
        if n % 100 == 0:
            print(f"step {n} {time.time() - t0:.0f} s", flush=True)
    acc /= AVERAGE
    rec = {
        "what": "u_x(r) azimuthal mean over unit annuli, mean of the pre-collision velocity over steps "
                f"[{STEPS - AVERAGE}, {STEPS}) of the FP64 oracle",
        "workload": w.name, "planes_x": xs, "R": w.rotors[0].R, "bins": NBINS,
        "made_by": "python tests/golden/wake_profiles.py (oracle only)",
        "profiles": acc.tolist(),
    }
    with open(FIXTURE, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", FIXTURE, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
