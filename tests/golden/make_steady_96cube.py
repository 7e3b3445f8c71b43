"""Writes steady_96cube.txt: the FP64 oracle's steady-state permeability of a 96^3 sphere pack.

The pack has the radius and porosity of the 384^3 precision workload (r = 8,
porosity 0.6, seed 4; SplitMix64 overlapping spheres, periodic box), omega = 1,
body force 1e-6 in x, rest start.  The oracle (two-step, FP64) runs in windows
of K = 100 steps; the mean velocity U = (J_x + M g / 2) / M after every
window is recorded.  The run stops when three consecutive windows each
change U by less than 1e-9 of itself (FP64 carries no rounding noise at that
level), or at 10000 steps.  Darcy's law gives k = nu * phi * U / g with
nu = (1/omega - 1/2) / 3 and phi = N_f / N_c.

Only the oracle and the seeded input generator are called.  Run from the
repository root:  python tests/golden/make_steady_96cube.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lbm_inputs  # noqa: E402
import oracle  # noqa: E402

N, RADIUS, POROSITY, SEED = 96, 8, 0.6, 4
OMEGA, G, K, TOL, CAP = 1.0, 1e-6, 100, 1e-9, 10000


def main():
    solid, spheres = lbm_inputs.sphere_pack(N, RADIUS, POROSITY, SEED)
    nf = int((solid == 0).sum())
    phi = nf / solid.size
    f = oracle.init_equilibrium(lbm_inputs.rho_u_field(solid.shape), solid)
    hist, steps = [], 0
    t0 = time.perf_counter()
    while steps < CAP:
        f = oracle.run_ts(f, solid, K, OMEGA, (G, 0.0, 0.0))
        steps += K
        hist.append(float(oracle.mean_velocity(oracle.moments(f, solid), (G, 0.0, 0.0))[0]))
        print(f"step {steps}: U {hist[-1]:.17e}", flush=True)
        if len(hist) > 3 and all(abs(hist[-j] - hist[-j - 1]) < TOL * abs(hist[-1]) for j in (1, 2, 3)):
            break
    nu = (1.0 / OMEGA - 0.5) / 3.0
    k = nu * phi * hist[-1] / G
    out = os.path.join(HERE, "steady_96cube.txt")
    with open(out, "w") as fh:
        fh.write("# FP64 oracle steady state of a 96^3 sphere pack; written by make_steady_96cube.py\n")
        fh.write("# (oracle and input generator only).  U after every window of K steps, then the result.\n")
        fh.write(f"lattice {N}\nradius {RADIUS}\nporosity_target {POROSITY}\nseed {SEED}\nspheres {spheres}\n")
        fh.write(f"n_fluid {nf}\nomega {OMEGA!r}\ng {G!r}\nK {K}\ntol {TOL!r}\nsteps {steps}\n")
        fh.write(f"U {hist[-1]!r}\npermeability {k!r}\n")
        for j, u in enumerate(hist):
            fh.write(f"U_at {(j + 1) * K} {u!r}\n")
    print(f"{out}: {steps} steps, k = {k:.12g}, {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main()
