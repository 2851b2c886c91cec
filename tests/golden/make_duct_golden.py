"""Write the oracle's reference values for the long rectangular-duct parity runs.

Runs the CPU oracle (oracle/, FP64) on the seeded duct workloads and stores,
per case, the invariants (flux, mass, mass deviation), the largest axial
velocity over the whole box and the fields (rho - rho0, u_x, u_y, u_z) at a
seeded sample of cells.  Nothing here touches the GPU library: the stored
values come from the oracle alone, and the GPU tests compare with them.

Cases (the duct workload: D3Q19, walls on y and z, x periodic, tau 0.7,
body force 1e-6 along x, wall friction a smooth random field of mean 0.05 and
std 0.02 on the unrolled wall surface):
  duct_256x128x64_2000   the full 256 x 128 x 64 duct, 2,000 steps,
                         friction field of correlation length 16;
  duct_64x32x16_20000    a 64 x 32 x 16 replica (every side a quarter),
                         20,000 steps, correlation length 4.

Usage: python tests/golden/make_duct_golden.py CASE [CASE ...]
(the full-size case takes about half an hour of one core).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2403_15768_amd import inputs  # noqa: E402

CASES = {
    "duct_256x128x64_2000": dict(box=(256, 128, 64), steps=2000, friction_index=0, sigma=16.0),
    "duct_64x32x16_20000": dict(box=(64, 32, 16), steps=20000, friction_index=13, sigma=4.0),
}
TAU, G = 0.7, 1e-6
NSAMPLE = 1024


def sample_cells(shape, n, seed=20240315):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    flat = rng.choice(nz * ny * nx, size=n, replace=False)
    z, rem = np.divmod(flat, ny * nx)
    y, x = np.divmod(rem, nx)
    return np.stack([z, y, x], axis=1)


def run(name: str) -> str:
    c = CASES[name]
    nx, ny, nz = c["box"]
    o = oracle.Lattice(19, oracle.DUCT, nx, ny, nz, tau=TAU, force=(G, 0, 0))
    lam = inputs.duct_friction(o.wall_coords(), nx, ny, nz,
                               inputs.rng_for("duct", c["friction_index"]), sigma=c["sigma"])
    o.set_friction(lam)
    t0 = time.perf_counter()
    left = c["steps"]
    while left > 0:
        k = min(left, 100)
        o.step(k)
        left -= k
        print(f"{name}: step {c['steps'] - left} of {c['steps']} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    rho, ux, uy, uz = o.fields()
    flux, mass, dmass = o.invariants()
    cells = sample_cells(o.shape, NSAMPLE)
    z, y, x = cells[:, 0], cells[:, 1], cells[:, 2]
    rec = {
        "source": "written by tests/golden/make_duct_golden.py from the CPU oracle (FP64)",
        "case": name, "lattice": "D3Q19", "geometry": "duct", "box": [nx, ny, nz],
        "tau": TAU, "force": [G, 0.0, 0.0], "rho0": 1.0, "steps": c["steps"],
        "friction": {"generator": "inputs.duct_friction", "workload": "duct",
                     "index": c["friction_index"], "sigma": c["sigma"],
                     "mean": 0.05, "std": 0.02},
        "flux": flux, "mass": mass, "mass_deviation": dmass,
        "max_abs_ux": float(np.max(np.abs(ux))),
        "cells_zyx": cells.tolist(),
        "rho_minus_rho0": (rho[z, y, x] - 1.0).tolist(),
        "ux": ux[z, y, x].tolist(), "uy": uy[z, y, x].tolist(), "uz": uz[z, y, x].tolist(),
        "oracle_seconds": round(time.perf_counter() - t0, 1),
    }
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(path + ".tmp", path)
    return path


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        print(run(nm), flush=True)
