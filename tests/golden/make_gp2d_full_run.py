"""Writes gp2d_2048_2000steps.json: the FP64 oracle's state after the full 2D Gross-Pitaevskii
benchmark run (2049^2 nodes, a = 0.5, s = -1, omega = 0.05 on [-40, 40]^2, Dirichlet 0,
vortex + 1e-3 noise with seed 2; dt = 0.5 x the bound of Eq. kdfull, 2000 RK4 steps of
Sec. 3.1), sampled on a coarse lattice of nodes (every 128th node on each axis) and on the
16 x 16 nodes around the vortex core, plus the mass and energy before and after.

Only the oracle computes these values.  Run from the repository root:
    python tests/golden/make_gp2d_full_run.py
(about ten minutes on eight cores)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import nlse_inputs as I  # noqa: E402
import oracle as O  # noqa: E402

N, STEPS = 2048, 2000
LATTICE = list(range(0, N + 1, 128))
CORE = list(range(N // 2 - 8, N // 2 + 8))


def sample_nodes():
    nodes = [(iy, ix) for iy in LATTICE for ix in LATTICE]
    nodes += [(iy, ix) for iy in CORE for ix in CORE]
    return nodes


def main():
    sp = I.config_gp2d(n=N)
    P = O.Problem.from_spec(sp)
    dt = 0.5 * P.max_dt(sp.psi0)
    t0 = time.time()
    psi = sp.psi0
    for chunk in range(STEPS // 100):
        psi = P.rk4(psi, 100, dt)
        print(f"steps {100 * (chunk + 1)} of {STEPS}, {time.time() - t0:.0f} s", flush=True)
    nodes = sample_nodes()
    vals = [psi[iy, ix] for iy, ix in nodes]
    out = {
        "what": "FP64 oracle, 2D GP 2049^2 benchmark workload after 2000 RK4 steps (Sec. 3.1) with the "
                "2SHOC Laplacian (Sec. 2.2), dt = 0.5 k_max (Eq. kdfull); sampled nodes [iy, ix]",
        "n": N, "steps": STEPS, "dt": dt,
        "nodes": [[int(a), int(b)] for a, b in nodes],
        "re": [float(v.real) for v in vals], "im": [float(v.imag) for v in vals],
        "mass0": P.mass(sp.psi0), "energy0": P.energy(sp.psi0),
        "mass": P.mass(psi), "energy": P.energy(psi),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gp2d_2048_2000steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} ({len(nodes)} nodes)")


if __name__ == "__main__":
    main()
