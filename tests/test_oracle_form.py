"""Oracle pins for the ALE time-step form (Section 2.3).

Each check recomputes a piece of the residual by a route that does not use
the oracle's formulas: finite differences, an Eulerian Navier-Stokes residual
written from eq. (fluid), the same Eulerian form on the moved mesh, an
invariance of the ALE time derivative, and the St. Venant-Kirchhoff strain
energy.  The helpers below use their own loops and basis evaluation.
"""
import numpy as np
import pytest

import synth
from oracle.residual import Discretization

G2 = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]


def _basis(xi, eta):
    """Bilinear basis on the unit square, local order (0,0),(1,0),(0,1),(1,1)."""
    N = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta])
    dxi = np.array([-(1 - eta), (1 - eta), -eta, eta])
    deta = np.array([-(1 - xi), -xi, (1 - xi), xi])
    return N, np.stack([dxi, deta], axis=1)


def _rows_to_check(D):
    m = D.mesh
    mom = np.zeros((m.n_nodes, D.nc), dtype=bool)
    free = ~D.dirichlet
    mom[:, 0:2] = (~m.in_NS)[:, None] & free[:, 0:2]
    mom[:, 4] = m.in_NF & free[:, 4]
    return mom


def _eulerian_moved(D, U, k, p, moved=True):
    """k * [A_NS + A_div] of eq. (fluid) in Eulerian form on the mesh X + u.

    Isoparametric bilinear cells in physical coordinates: grad_x N =
    (dx/dxi)^{-T} grad_xi N, dx = det(dx/dxi) dxi; the do-nothing correction
    -rho nu <grad v^T n, phi> uses the moved outflow edge's normal.
    """
    m = D.mesh
    rf, nu = p["rho_f"], p["nu_f"]
    R = np.zeros((m.n_nodes, 5))
    Xn = m.X + (U[:, 2:4] if moved else 0.0)
    for c in np.nonzero(m.fluid)[0]:
        nodes = m.conn[c]
        xe = Xn[nodes]
        ve = U[nodes, 0:2]
        pe = U[nodes, 4]
        for xi in G2:
            for eta in G2:
                N, dN = _basis(xi, eta)
                Jm = xe.T @ dN                       # dx/dxi, 2x2
                det = Jm[0, 0] * Jm[1, 1] - Jm[0, 1] * Jm[1, 0]
                gN = dN @ np.linalg.inv(Jm)          # [a, r] physical gradients
                v = N @ ve
                gv = ve.T @ gN                       # gv[i, r] = d_r v_i
                pr = N @ pe
                sig = rf * nu * (gv + gv.T) - pr * np.eye(2)
                w = 0.25 * det
                conv = gv @ v
                for a in range(4):
                    R[nodes[a], 0:2] += k * w * (rf * conv * N[a] + sig @ gN[a])
                    R[nodes[a], 4] += k * w * np.trace(gv) * N[a]
    for c in m.outflow_cells:
        nodes = m.conn[c]
        xe = Xn[nodes]
        ve = U[nodes, 0:2]
        for eta in G2:
            N, dN = _basis(1.0, eta)
            Jm = xe.T @ dN
            gN = dN @ np.linalg.inv(Jm)
            gv = ve.T @ gN
            t = Jm[:, 1]                             # d x / d eta along the edge
            nds = np.array([t[1], -t[0]]) * 0.5      # outward normal times ds, weight 1/2
            b = rf * nu * gv.T @ nds
            for a in range(4):
                R[nodes[a], 0:2] -= k * b * N[a]
    return R


@pytest.mark.parametrize("level,alpha0", [(0, 0.0), (1, 0.1)])
def test_jacobian_vs_central_fd(level, alpha0):
    """The complex-step Jacobian equals central differences of the global residual."""
    p = synth.workload("c1", lps_alpha0=alpha0, level=level)
    D = Discretization(p)
    U = synth.random_state(p, 21)
    Uo = synth.random_state(p, 22)
    k = p["k_fine"]
    A = D.jacobian(U, Uo, 0.07, k)
    Ao = D.jacobian_old(U, Uo, 0.07, k)
    rng = np.random.default_rng(5)
    scale = np.abs(U).max(axis=0)
    for _ in range(3):
        x = rng.normal(size=U.shape) * scale
        eps = 1e-6
        fd = (D.residual(U + eps * x, Uo, 0.07, k) - D.residual(U - eps * x, Uo, 0.07, k)) / (2 * eps)
        an = (A @ x.ravel()).reshape(U.shape)
        assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()
        fdo = (D.residual(U, Uo + eps * x, 0.07, k) - D.residual(U, Uo - eps * x, 0.07, k)) / (2 * eps)
        ano = (Ao @ x.ravel()).reshape(U.shape)
        assert np.abs(fdo - ano).max() <= 1e-6 * np.abs(ano).max()
    # old pressure enters nowhere (the pressure is implicit in both theta parts)
    assert abs(Ao[:, 4::5]).max() == 0.0


def test_zero_displacement_reduces_to_eulerian_ns():
    """With u = u° = 0 the ALE step is the Eulerian Navier-Stokes CN step."""
    p = synth.workload("c1", lps_alpha0=0.0)
    D = Discretization(p)
    U = synth.random_state(p, 31)
    Uo = synth.random_state(p, 32)
    U[:, 2:4] = 0.0
    Uo[:, 2:4] = 0.0
    k = p["k_fine"]
    th = 0.5 + p["theta0"] * k
    R = D.residual(U, Uo, 0.2, k, with_dirichlet=False)
    # Eulerian: rho (v - v°) phi + k th A(v, p) + k (1 - th) A(v°, p) (pressure new in both)
    Uop = Uo.copy()
    Uop[:, 4] = U[:, 4]
    A_new = _eulerian_moved(D, U, 1.0, p, moved=False)
    A_old = _eulerian_moved(D, Uop, 1.0, p, moved=False)
    E = th * k * A_new + (1 - th) * k * A_old
    E[:, 4] = k * A_new[:, 4]
    m = D.mesh
    for c in np.nonzero(m.fluid)[0]:
        nodes = m.conn[c]
        h = m.h[c]
        for xi in G2:
            for eta in G2:
                N, _ = _basis(xi, eta)
                dv = N @ (U[nodes, 0:2] - Uo[nodes, 0:2])
                for a in range(4):
                    E[nodes[a], 0:2] += p["rho_f"] * 0.25 * h[0] * h[1] * dv * N[a]
    rows = _rows_to_check(D)
    err = np.abs(R[rows] - E[rows]).max()
    assert err <= 1e-12 * np.abs(E[rows]).max(), err


def test_ale_stationary_terms_equal_eulerian_on_moved_mesh():
    """A_NS + A_div in ALE form on the reference mesh = Eulerian form on X + u."""
    p = synth.workload("c1", lps_alpha0=0.0)
    D = Discretization(p)
    U = synth.random_state(p, 41, grad_u_max=0.2)
    k = p["k_fine"]
    # old = new: the time-difference terms vanish and theta parts add up to k A(U)
    R = D.residual(U, U, 0.2, k, with_dirichlet=False)
    E = _eulerian_moved(D, U, k, p, moved=True)
    rows = _rows_to_check(D)
    err = np.abs(R[rows] - E[rows]).max()
    assert err <= 1e-12 * np.abs(E[rows]).max(), err
    # and the moved mesh matters: the unmoved Eulerian form differs
    E0 = _eulerian_moved(D, U, k, p, moved=False)
    assert np.abs(R[rows] - E0[rows]).max() > 1e-4 * np.abs(E[rows]).max()


def test_ale_time_derivative_vanishes_for_steady_affine_flow():
    """rho J̄ ((v - v°) - grad v̄ F̄^{-1} (u - u°)) = 0 when v(X, t) = c + G (X + u(X, t)).

    An affine Eulerian field that is steady in time has zero ALE time
    derivative, for any mesh motion; with Q1 displacements this holds
    exactly in the discrete scheme (mean F̄ of Section 2.3).
    """
    p = synth.workload("c1", lps_alpha0=0.0)
    D = Discretization(p)
    rng = np.random.default_rng(7)
    c = rng.normal(size=2)
    Gm = rng.normal(size=(2, 2))
    U = synth.random_state(p, 51, grad_u_max=0.2)
    Uo = synth.random_state(p, 52, grad_u_max=0.2)
    X = D.mesh.X
    U[:, 0:2] = c + (X + U[:, 2:4]) @ Gm.T
    Uo[:, 0:2] = c + (X + Uo[:, 2:4]) @ Gm.T
    R = D.residual(U, Uo, 0.2, 0.0, theta=0.5, with_dirichlet=False)
    rows = _rows_to_check(D)
    rows[:, 4] = False
    ref = p["rho_f"] * np.abs(U[:, 0:2] - Uo[:, 0:2]).max() * np.prod(D.mesh.h, 1).max()
    assert np.abs(R[rows]).max() <= 1e-13 * ref
    # a non-affine field does not satisfy it
    U2 = U.copy()
    U2[:, 0] += 0.1 * np.sin(7 * X[:, 1])
    R2 = D.residual(U2, Uo, 0.2, 0.0, theta=0.5, with_dirichlet=False)
    assert np.abs(R2[rows]).max() > 1e-3 * ref


def test_solid_stress_is_strain_energy_gradient():
    """(F Sigma(u), grad phi)_S is the derivative of the St. Venant-Kirchhoff energy.

    W(E) = mu tr(E^2) + lambda/2 tr(E)^2 (eq. (stress)); the energy is
    integrated with its own loops and differentiated by complex step.
    """
    p = synth.workload("c1")
    D = Discretization(p)
    U = synth.random_state(p, 61, grad_u_max=0.2)
    U[:, 0:2] = 0.0
    U[:, 4] = 0.0
    k = p["k_fine"]
    R = D.residual(U, U, 0.2, k, with_dirichlet=False)
    m = D.mesh
    mu, lam = p["mu_s"], p["lambda_s"]

    def energy(u):
        e = 0.0
        for c in np.nonzero(m.solid)[0]:
            nodes = m.conn[c]
            h = m.h[c]
            for xi in G2:
                for eta in G2:
                    _, dN = _basis(xi, eta)
                    gN = dN / h
                    F = np.eye(2) + u[nodes].T @ gN
                    E = 0.5 * (F.T @ F - np.eye(2))
                    e = e + 0.25 * h[0] * h[1] * (mu * np.sum(E * E) + 0.5 * lam * np.trace(E) ** 2)
        return e

    rng = np.random.default_rng(9)
    for _ in range(3):
        w = rng.normal(size=(m.n_nodes, 2))
        dpsi = energy(U[:, 2:4] + 1e-30j * w).imag / 1e-30
        assert abs(np.sum(R[:, 0:2] * w) - k * dpsi) <= 1e-12 * abs(k * dpsi)


@pytest.mark.parametrize("dim", [2, 3])
def test_displacement_rows_do_not_depend_on_the_state(dim):
    """The displacement rows of the step Jacobian (harmonic extension, kinematic
    equation, Dirichlet identity) are linear in (v, u) with coefficients fixed by
    the mesh, k and theta: two unrelated states give the same rows, and the rows
    touch only v_i and u_i of their own component i.  The GPU path stores these
    rows once for all slices of a call and relies on exactly this."""
    if dim == 2:
        p = synth.workload("c1")
    else:
        p = synth.workload("c5", level=0)
    D = Discretization(p)
    nc = 2 * dim + 1
    k = p["k_fine"]
    A1 = D.jacobian(synth.random_state(p, 31), synth.random_state(p, 32), 0.05, k).tocsr()
    A2 = D.jacobian(synth.random_state(p, 33), synth.random_state(p, 34), 0.11, k).tocsr()
    n = A1.shape[0]
    rows = np.array([r for r in range(n) if dim <= r % nc < 2 * dim])
    R1, R2 = A1[rows], A2[rows]
    diff = abs(R1 - R2).max()
    assert diff <= 1e-14 * abs(R1).max(), diff
    # structure: row of component i (u_i) couples only to v_i and u_i
    R1 = R1.tocoo()
    comp_row = (rows[R1.row] % nc) - dim
    comp_col = R1.col % nc
    nz = R1.data != 0
    assert np.all((comp_col[nz] == comp_row[nz]) | (comp_col[nz] == comp_row[nz] + dim))


def test_solid_inertia_is_consistent_mass():
    """Momentum rows of the solid with no stiffness (mu_s = lambda_s = 0), the fluid at
    rest and no displacement: the residual reduces to rho_s M_S (v - v°), M_S the
    consistent Q1 mass matrix of the solid cells, here built from 1d P1 mass matrices
    (tensor form) on the bar's own node grid.  A lumped or missing inertia term, a
    wrong density or a wrong sign fails.  The velocity is put only on nodes that touch
    no fluid cell, so every fluid term vanishes.
    """
    p = synth.workload("c1", mu_s=0.0, lambda_s=0.0, rho_s=1234.5)
    D = Discretization(p)
    m = D.mesh
    x, y = m.axes
    ix = np.nonzero((x >= 0.4 - 1e-12) & (x <= 0.5 + 1e-12))[0]
    iy = np.nonzero(y <= 0.25 + 1e-12)[0]

    def mass1(pts):
        n = len(pts)
        A = np.zeros((n, n))
        for i in range(n - 1):
            A[i:i + 2, i:i + 2] += np.array([[2.0, 1.0], [1.0, 2.0]]) * (pts[i + 1] - pts[i]) / 6.0
        return A

    Ms = np.kron(mass1(y[iy]), mass1(x[ix]))               # x fastest, as the node numbering
    nodes = (ix[None, :] + (len(x)) * iy[:, None]).ravel()
    rng = np.random.default_rng(7)
    U = np.zeros((m.n_nodes, 5))
    Uo = np.zeros((m.n_nodes, 5))
    strict = ~m.in_NF
    U[strict, 0:2] = rng.uniform(-1.0, 1.0, size=(strict.sum(), 2))
    Uo[strict, 0:2] = rng.uniform(-1.0, 1.0, size=(strict.sum(), 2))
    assert strict[nodes].sum() == strict.sum() > 0
    k = p["k_fine"]
    R = D.residual(U, Uo, 0.5, k, with_dirichlet=False)
    expect = np.zeros((m.n_nodes, 2))
    expect[nodes] = p["rho_s"] * (Ms @ (U[nodes, 0:2] - Uo[nodes, 0:2]))
    scale = np.abs(expect).max()
    assert np.abs(R[:, 0:2] - expect).max() <= 1e-13 * scale
    # the consistent mass couples neighbours: a lumped mass would differ by a lot
    lumped = np.zeros_like(expect)
    lumped[nodes] = p["rho_s"] * (Ms.sum(axis=1)[:, None] * (U[nodes, 0:2] - Uo[nodes, 0:2]))
    assert np.abs(lumped - expect).max() > 0.1 * scale
