"""Oracle pins for the time stepping and the Parareal iteration (Sections 2.3, 3)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle.residual import Discretization
from oracle import propagate as P


def _q1_laplacian_fluid(m):
    """Q1 stiffness over the fluid cells, from 1d P1 matrices (Kronecker form)."""
    def k1(h):
        return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h

    def m1(h):
        return np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0

    def glob1(x, f):
        n = len(x)
        A = np.zeros((n, n))
        for i in range(n - 1):
            A[i:i + 2, i:i + 2] += f(x[i + 1] - x[i])
        return A

    x, y = m.axes
    K = np.kron(glob1(y, m1), glob1(x, k1)) + np.kron(glob1(y, k1), glob1(x, m1))
    for c in np.nonzero(m.solid)[0]:
        hx, hy = m.h[c]
        Kl = np.kron(m1(hy), k1(hx)) + np.kron(k1(hy), m1(hx))
        n = m.conn[c]
        K[np.ix_(n, n)] -= Kl
    return sp.csr_matrix(K)


def test_kinematic_and_harmonic_invariants():
    """After every step: solid nodes move with the trapezoidal velocity, fluid u is discrete-harmonic."""
    p = synth.workload("c1")
    D = Discretization(p)
    m = D.mesh
    L = _q1_laplacian_fluid(m)
    k = p["k_fine"]
    th = 0.5 + p["theta0"] * k
    U = np.zeros((m.n_nodes, 5))
    solid_rows = m.in_NS & ~D.dirichlet[:, 2]
    fluid_rows = ~m.in_NS & ~D.dirichlet[:, 2]
    for n in range(1, 6):
        Un = P.newton_step(D, U, n * k, k)
        du = Un[:, 2:4] - U[:, 2:4]
        kin = k * (th * Un[:, 0:2] + (1 - th) * U[:, 0:2])
        assert np.abs(du[solid_rows] - kin[solid_rows]).max() <= 1e-12 * np.abs(kin[solid_rows]).max()
        Lu = L @ Un[:, 2:4]
        scale = abs(L).max() * np.abs(Un[:, 2:4]).max()
        assert np.abs(Lu[fluid_rows]).max() <= 1e-11 * scale
        U = Un
    assert np.abs(U[:, 2:4]).max() > 0  # the bar did move


def _self_convergence(theta_fixed):
    """Ratios of successive differences ||U_k - U_{k/2}|| at T for v and u.

    A softer bar (mu_s = 5e3) and a more viscous fluid (nu_f = 1e-2) put the
    step sizes 0.1/4 .. 0.1/32 in the asymptotic range of the scheme; with the
    workload's stiff bar the solid's own period (~0.05) is not resolved by
    these steps.
    """
    p = synth.workload("c1", theta_fixed=theta_fixed, mu_s=5e3, nu_f=1e-2, ramp_time=0.2)
    p["lambda_s"] = synth.lame_lambda(p["mu_s"], p["nu_s"])
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    T = 0.1
    sols = [P.propagate(D, U0, 0.0, T, n) for n in (4, 8, 16, 32)]
    ratios = []
    for sl in (slice(0, 2), slice(2, 4)):
        e = [np.linalg.norm(sols[j][:, sl] - sols[j + 1][:, sl]) for j in range(3)]
        ratios.append(e[1] / e[2])
    return ratios


def test_shifted_cn_second_order():
    """theta = 1/2 + k: self-convergence ratio -> 4 (second order, Section 2.3)."""
    r = _self_convergence(None)
    for x in r:
        assert 3.3 < x < 4.7, r


def test_backward_euler_first_order():
    """theta = 1 is backward Euler, first order (Section 2.3): ratio -> 2."""
    r = _self_convergence(1.0)
    for x in r:
        assert 1.7 < x < 2.3, r


def _small_parareal_problem():
    return synth.workload("c1", T=0.2, N=4, dt_fine=0.0125, dt_coarse=0.05)


def test_parareal_finite_termination_and_K_equals_N():
    """After i iterations slices 0..i are exact; K = N gives the sequential fine solution."""
    p = _small_parareal_problem()
    assert (p["m"], p["M"]) == (4, 1)
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    seq = P.sequential(D, p, U0)
    hist = []
    Upar, it = P.parareal(D, p, U0, tol=0.0, history=hist)
    assert it == p["N"]

    def rel(a, b):
        nb = np.linalg.norm(b)
        return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)

    for i, (Ui, _) in enumerate(hist):
        for l in range(0, i + 2):
            assert rel(Ui[l][:, :4], seq[l][:, :4]) <= 1e-12, (i, l)
    # the iterate before convergence is not yet exact on the last slice
    assert rel(hist[0][0][p["N"]][:, :4], seq[p["N"]][:, :4]) > 1e-8
    for l in range(p["N"] + 1):
        assert rel(Upar[l][:, :4], seq[l][:, :4]) <= 1e-12


def test_theta_weight_definitions():
    """Least squares weight minimises |F_c - th C_c| per component; the cosine weight is <= 1 and 1 for parallel fields."""
    rng = np.random.default_rng(3)
    F = rng.normal(size=(50, 5))
    C = F + 0.3 * rng.normal(size=(50, 5))
    lsq = [np.linalg.lstsq(C[:, [c]], F[:, c], rcond=None)[0][0] for c in range(4)]
    assert abs(P.theta_weight(F, C, 2, "lsq") - np.mean(lsq)) <= 1e-14
    cosv = [F[:, c] @ C[:, c] / (np.linalg.norm(F[:, c]) * np.linalg.norm(C[:, c])) for c in range(4)]
    assert abs(P.theta_weight(F, C, 2, "cosine") - np.mean(cosv)) <= 1e-14
    assert P.theta_weight(F, C, 2, "cosine") <= 1.0
    assert abs(P.theta_weight(F, 2.5 * F, 2, "cosine") - 1.0) <= 1e-14
    assert abs(P.theta_weight(F, 2.5 * F, 2, "lsq") - 0.4) <= 1e-14
    # the pressure column does not enter; zero components are left out
    G = C.copy()
    G[:, 4] = 1e9
    assert P.theta_weight(F, G, 2, "lsq") == P.theta_weight(F, C, 2, "lsq")
    Z = np.zeros_like(F)
    assert P.theta_weight(Z, C, 2, "cosine") == 1.0 and P.theta_weight(F, Z, 2, "lsq") == 1.0


@pytest.mark.parametrize("mode", ["cosine", "lsq"])
def test_theta_parareal_finite_termination(mode):
    """Weighted Parareal keeps finite termination: slices 0..i exact after i iterations, K = N sequential."""
    p = _small_parareal_problem()
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    seq = P.sequential(D, p, U0)
    hist, th = [], []
    Upar, it = P.parareal(D, p, U0, tol=0.0, history=hist, theta=mode, thetas=th)
    assert it == p["N"]

    def rel(a, b):
        nb = np.linalg.norm(b)
        return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)

    for i, (Ui, _) in enumerate(hist):
        for l in range(0, i + 2):
            assert rel(Ui[l][:, :4], seq[l][:, :4]) <= 1e-12, (i, l)
    # the weights are genuinely different from 1 on the corrected slices
    assert any(abs(t - 1.0) > 1e-6 for (i, l, t) in th if l >= i)
    if mode == "cosine":
        assert all(t <= 1.0 + 1e-15 for (_, _, t) in th)


def test_plain_parareal_is_theta_one():
    p = _small_parareal_problem()
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    a, ia = P.parareal(D, p, U0, tol=0.0, max_iter=2)
    th = []
    b, ib = P.parareal(D, p, U0, tol=0.0, max_iter=2, theta="plain", thetas=th)
    assert ia == ib and np.array_equal(a, b) and all(t == 1.0 for (_, _, t) in th)


def test_dissipation_matched_theta():
    """theta(k) = 1/2 + theta0 k_r^2 / k damps an oscillation per unit time like steps of k_r (to leading order)."""
    p = synth.workload("c2")
    kr, K = 2.0 ** -9, 2.0 ** -6
    D = Discretization(dict(p, theta_ref_k=kr))
    D0 = Discretization(p)
    assert D.theta(kr) == D0.theta(kr)

    def rate(theta, k, w):
        z = 1j * w * k
        return np.log(abs((1 + (1 - theta) * z) / (1 - theta * z))) / k

    for wK in (0.02, 0.05, 0.1):
        w = wK / K
        fine = rate(D0.theta(kr), kr, w)
        matched = rate(D.theta(K), K, w)
        default = rate(D0.theta(K), K, w)
        assert fine < 0 and matched < 0
        assert abs(matched / fine - 1.0) <= 2 * wK ** 2, (wK, matched / fine)
        assert default / fine > 50.0        # the default large step damps ~ (K / k_r)^2 = 64 times more


def test_parareal_change_norm_hand_example():
    """The stopping quantity of the Parareal iteration (Section 3) on a hand-worked
    two-boundary, two-node example: per boundary and per field (v and u separately,
    p left out), the Euclidean norm of the change over the norm of the NEW iterate;
    the largest of these is 1/5 (boundary 1, velocity).

    Each plausible mistake gives a different number: dividing by the old iterate
    1/sqrt(18), max-norms 1/4, v and u in one norm sqrt(1.01)/sqrt(26), one norm over
    all boundaries 1/sqrt(26), the pressure included 10.
    """
    new = np.zeros((2, 2, 5))
    old = np.zeros((2, 2, 5))
    # boundary 0: nonzero, unchanged
    new[0, 0, 0] = old[0, 0, 0] = 1.0
    # boundary 1: v_new = ((3, 0), (0, 4)), v_old = ((3, 0), (0, 3))
    new[1, 0, 0:2] = (3.0, 0.0)
    new[1, 1, 0:2] = (0.0, 4.0)
    old[1, 0, 0:2] = (3.0, 0.0)
    old[1, 1, 0:2] = (0.0, 3.0)
    # u_new = ((0.6, 0.8), 0), u_old = ((0.6, 0.7), 0): change 0.1 of norm 1
    new[1, 0, 2:4] = (0.6, 0.8)
    old[1, 0, 2:4] = (0.6, 0.7)
    # the pressure changes by ten times its new size
    new[1, 1, 4] = 1.0
    old[1, 1, 4] = 11.0
    assert P.relative_change(new, old, 2) == pytest.approx(0.2, rel=1e-15, abs=0.0)
    # a change in one boundary's displacement alone is seen with its own norm
    old2 = new.copy()
    old2[0, 1, 3] = 0.5
    new2 = new.copy()
    new2[0, 1, 2:4] = (0.0, 2.0)
    assert P.relative_change(new2, old2, 2) == pytest.approx(1.5 / 2.0, rel=1e-15, abs=0.0)
