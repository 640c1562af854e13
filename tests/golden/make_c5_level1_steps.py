"""Write tests/golden/c5_level1_steps.npz: two fine steps of the 3d workload
(c5 geometry and physics at refinement level 1, 32x8x8 hexahedra) from two
seeded admissible states, computed by the FP64 oracle only.

The 3d oracle step takes about a minute per slice on a few host cores, too
slow to repeat inside a GPU test, so its output is stored here.  Run from the
repository root:  python tests/golden/make_c5_level1_steps.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.residual import Discretization  # noqa: E402
from oracle import propagate as P  # noqa: E402

SEEDS = (11, 12)
T0 = 0.15          # after the inflow ramp
STEPS = 2


def main():
    p = synth.workload("c5", seed=0, level=1)
    D = Discretization(p)
    k = p["k_fine"]
    U_in, U_out = [], []
    for s in SEEDS:
        u0 = D.apply_dirichlet(synth.random_state(p, s), T0)
        u1 = P.propagate(D, u0, T0, STEPS * k, STEPS)
        U_in.append(u0)
        U_out.append(u1)
        print("seed", s, "done", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_level1_steps.npz")
    np.savez_compressed(out, U_in=np.stack(U_in), U_out=np.stack(U_out), t0=T0, k=k, steps=STEPS,
                        seeds=np.array(SEEDS))


if __name__ == "__main__":
    main()
