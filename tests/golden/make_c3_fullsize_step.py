"""Write tests/golden/c3_fullsize_step.npz: one fine step of the c3 workload
(2d, 256x64 cells, 83,525 unknowns, seed 0) for two sampled slices of the
64-slice batch, each from a seeded smooth state (synth.smooth_state) with the
Dirichlet data of its slice start, computed by the FP64 oracle only.

One oracle step at this size takes minutes on a few host cores, too slow to
repeat inside a GPU test, so its output is stored here.  The GPU test rebuilds
the inputs from the same seeds.  Run from the repository root:
    python tests/golden/make_c3_fullsize_step.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.residual import Discretization  # noqa: E402
from oracle import propagate as P  # noqa: E402

SLICES = (5, 37)         # sampled slices of the batch
SEED_BASE = 300          # slice l starts from synth.smooth_state(p, SEED_BASE + l)


def main():
    p = synth.workload("c3", seed=0)
    D = Discretization(p)
    k, dl = p["k_fine"], p["slice_len"]
    U_out = []
    for l in SLICES:
        t0 = l * dl
        u0 = D.apply_dirichlet(synth.smooth_state(p, SEED_BASE + l), t0)
        U_out.append(P.propagate(D, u0, t0, k, 1))
        print("slice", l, "done", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_fullsize_step.npz")
    np.savez_compressed(out, U_out=np.stack(U_out), slices=np.array(SLICES), seed_base=SEED_BASE, k=k, dl=dl)


if __name__ == "__main__":
    main()
