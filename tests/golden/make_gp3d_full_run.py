"""Writes gp3d_512_500steps.json: the FP64 oracle's state after the full 3D Gross-Pitaevskii run
(513^3 nodes, a = 0.5, s = -1, omega = 0.1 on [-24, 24]^3, Dirichlet 0, Thomas-Fermi cloud with the
phase of a vortex ring of radius 6; dt = 0.5 x the bound of Eq. kdfull, 500 RK4 steps of Sec. 3.1),
sampled on a coarse lattice of nodes (every 64th node on each axis) and on the 8 x 8 x 8 nodes
around a point of the ring's core (x = 6, y = z = 0), plus the mass before and after.

Only the oracle computes these values.  Run from the repository root:
    python tests/golden/make_gp3d_full_run.py
(about 80 minutes and 20 GB of memory on eight cores)."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import nlse_inputs as I  # noqa: E402
import oracle as O  # noqa: E402

N, STEPS = 512, 500
LATTICE = list(range(0, N + 1, 64))
CORE_X = list(range(320 - 4, 320 + 4))        # x = -24 + 320 h = 6
CORE_YZ = list(range(N // 2 - 4, N // 2 + 4))


def sample_nodes():
    nodes = [(iz, iy, ix) for iz in LATTICE for iy in LATTICE for ix in LATTICE]
    nodes += [(iz, iy, ix) for iz in CORE_YZ for iy in CORE_YZ for ix in CORE_X]
    return nodes


def main():
    sp = I.config_gp3d(n=N)
    P = O.Problem.from_spec(sp)
    dt = 0.5 * P.max_dt(sp.psi0)
    t0 = time.time()
    psi = sp.psi0
    for chunk in range(STEPS // 25):
        psi = P.rk4(psi, 25, dt)
        print(f"steps {25 * (chunk + 1)} of {STEPS}, {time.time() - t0:.0f} s", flush=True)
    nodes = sample_nodes()
    vals = [psi[iz, iy, ix] for iz, iy, ix in nodes]
    out = {
        "what": "FP64 oracle, 3D GP 513^3 workload after 500 RK4 steps (Sec. 3.1) with the 2SHOC "
                "Laplacian (Sec. 2.3), dt = 0.5 k_max (Eq. kdfull); sampled nodes [iz, iy, ix]",
        "n": N, "steps": STEPS, "dt": dt,
        "nodes": [[int(a), int(b), int(c)] for a, b, c in nodes],
        "re": [float(v.real) for v in vals], "im": [float(v.imag) for v in vals],
        "mass0": P.mass(sp.psi0), "mass": P.mass(psi),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gp3d_512_500steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} ({len(nodes)} nodes)")


if __name__ == "__main__":
    main()
