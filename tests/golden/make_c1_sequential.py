"""Write tests/golden/c1_sequential.npz: the oracle's sequential fine solution of the
full c1 workload (2d, 32x8 cells, N = 8 slices of m = 13 fine steps on [0, 1], inflow
peak of seed SEED) at the slice boundaries, from rest.  Section 4.1: Parareal after
N iterations reproduces exactly this sequence, so the GPU test runs parareal_run
with K = N on the same workload and compares its boundary states with these.

Computed by the FP64 oracle only (oracle.propagate.sequential, 104 Newton-SuperLU
steps, about a minute on the host).  Run from the repository root:
    python tests/golden/make_c1_sequential.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.residual import Discretization  # noqa: E402
from oracle import propagate as P  # noqa: E402

SEED = 3


def main():
    p = synth.workload("c1", seed=SEED)
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    seq = np.stack(P.sequential(D, p, U0))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_sequential.npz")
    np.savez_compressed(out, states=seq, seed=SEED, N=p["N"], m=p["m"], M=p["M"], T=p["T"])
    print("wrote", out, seq.shape)


if __name__ == "__main__":
    main()
