"""Write tests/golden/c4_adjoint.npz: the oracle's discrete adjoint of the
time-integrated drag on the c4 mesh (2d, 128x32 cells, 21,285 unknowns, fine
step 2^-9 as in c4), shortened to N = 2 slices of m = 2 steps.  The start state
is a seeded smooth state (synth.smooth_state, seed SEED) with the Dirichlet data
of t = 0, so that the drag and its sensitivities are not those of a fluid at
rest.  Stored: J and dJ/d(inflow peak, mu_s, lambda_s), computed by the FP64
oracle only (oracle.adjoint.adjoint_gradient).

The oracle's complex-step Jacobians at this size take about a minute, too slow
to repeat inside a GPU test.  The GPU test rebuilds the start state from the
same seed.  Run from the repository root:
    python tests/golden/make_c4_adjoint.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.residual import Discretization  # noqa: E402
from oracle import adjoint as A  # noqa: E402

N, M_STEPS, SEED = 2, 2, 400


def workload():
    k = 2.0 ** -9
    return synth.workload("c4", seed=0, T=N * M_STEPS * k, N=N, dt_fine=k)


def start_state(p, D):
    return D.apply_dirichlet(synth.smooth_state(p, SEED), 0.0)


def main():
    p = workload()
    assert p["m"] == M_STEPS
    D = Discretization(p)
    J, grad = A.adjoint_gradient(D, p, start_state(p, D))
    print("J", J, "grad", grad, flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_adjoint.npz")
    np.savez_compressed(out, J=J, grad=grad, N=N, m=M_STEPS, seed=SEED, k=p["k_fine"], T=p["T"])


if __name__ == "__main__":
    main()
