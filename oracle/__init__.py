"""FP64 CPU oracle for the ALE fluid-structure fine propagator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the GPU library: the
mesh, basis functions, quadrature, residual, Jacobian, Newton solver and
Parareal loop are all written here again, plainly, in NumPy/SciPy.

What it computes (Margenberg & Richter, "Parallel time-stepping for
fluid-structure interactions"):
  * the monolithic ALE system, eqs. (ALE), (ALE:stress), in the variational
    form of eqs. (variational), (test), Section 2.2;
  * equal-order Q1 elements on an interface-fitted tensor mesh (Section 2.2),
    with a local-projection pressure stabilisation (Section 2.2, last
    paragraph; the form is a reading, documented in residual.py);
  * one shifted Crank-Nicolson step, the time-step equation of Section 2.3
    with the semi-linear forms of eq. (semiforms), theta = 1/2 + theta0 k;
  * Newton's method with a direct sparse LU (SuperLU) per step;
  * the fine and coarse propagators and the Parareal iteration of eq.
    (parareal:iteration), Section 3;
  * the time-integrated drag functional and its discrete adjoint gradient.

Every floating-point quantity is float64 (complex128 where the complex-step
derivative is taken).

Parity pins live in tests/test_oracle_*.py; each function states which
passage it follows.
"""
