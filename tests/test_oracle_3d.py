"""Oracle pins for the 3d form (Q1 hexahedra, Section 2.3 time-step equation).

The 3d oracle is the same dimension-generic code as the 2d one; these checks
pin its 3d branch (cofactor inverse of F, trilinear basis, the outflow face,
the 7-unknown node layout) against routes that do not use its formulas:
central differences, an Eulerian Navier-Stokes residual on isoparametric
trilinear cells written here with its own loops (on the reference mesh and on
the mesh moved by u), the invariance of the ALE time derivative for steady
affine flows, and the St. Venant-Kirchhoff strain energy.  The workload is the
c5 duct-with-block geometry at level 0 (16x4x4 cells, 4 of them solid).
"""
import numpy as np

import synth
from oracle.residual import Discretization

G2 = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
OFF = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]


def _basis(xi):
    """Trilinear basis on the unit cube and its reference gradients [a, r]."""
    N = np.empty(8)
    dN = np.empty((8, 3))
    for a, o in enumerate(OFF):
        f = [xi[r] if o[r] else 1.0 - xi[r] for r in range(3)]
        d = [1.0 if o[r] else -1.0 for r in range(3)]
        N[a] = f[0] * f[1] * f[2]
        dN[a] = [d[0] * f[1] * f[2], f[0] * d[1] * f[2], f[0] * f[1] * d[2]]
    return N, dN


def _workload(**kw):
    return synth.workload("c5", seed=0, level=0, **kw)


def _rows_to_check(D):
    m = D.mesh
    rows = np.zeros((m.n_nodes, D.nc), dtype=bool)
    free = ~D.dirichlet
    rows[:, 0:3] = (~m.in_NS)[:, None] & free[:, 0:3]
    rows[:, 6] = m.in_NF & free[:, 6]
    return rows


def _eulerian(D, U, k, p, moved=True):
    """k * [A_NS + A_div] of eq. (fluid) in Eulerian form on the mesh X + u
    (or X), isoparametric trilinear cells; the do-nothing correction
    -rho nu <grad v^T n, phi> on the outflow face with n dS from the cross
    product of the moved face's tangents."""
    m = D.mesh
    rf, nu = p["rho_f"], p["nu_f"]
    R = np.zeros((m.n_nodes, 7))
    Xn = m.X + (U[:, 3:6] if moved else 0.0)
    for c in np.nonzero(m.fluid)[0]:
        nodes = m.conn[c]
        xe, ve, pe = Xn[nodes], U[nodes, 0:3], U[nodes, 6]
        for x0 in G2:
            for x1 in G2:
                for x2 in G2:
                    N, dN = _basis((x0, x1, x2))
                    Jm = xe.T @ dN
                    det = np.linalg.det(Jm)
                    gN = dN @ np.linalg.inv(Jm)
                    v = N @ ve
                    gv = ve.T @ gN
                    pr = N @ pe
                    sig = rf * nu * (gv + gv.T) - pr * np.eye(3)
                    w = det / 8.0
                    conv = gv @ v
                    for a in range(8):
                        R[nodes[a], 0:3] += k * w * (rf * conv * N[a] + sig @ gN[a])
                        R[nodes[a], 6] += k * w * np.trace(gv) * N[a]
    for c in m.outflow_cells:
        nodes = m.conn[c]
        xe, ve = Xn[nodes], U[nodes, 0:3]
        for x1 in G2:
            for x2 in G2:
                N, dN = _basis((1.0, x1, x2))
                Jm = xe.T @ dN
                gN = dN @ np.linalg.inv(Jm)
                gv = ve.T @ gN
                nds = np.cross(Jm[:, 1], Jm[:, 2]) / 4.0   # outward (+x) normal times dS, weight 1/4
                b = rf * nu * gv.T @ nds
                for a in range(8):
                    R[nodes[a], 0:3] -= k * b * N[a]
    return R


def test_mesh_and_layout_3d():
    p = _workload()
    D = Discretization(p)
    m = D.mesh
    assert m.shape == (16, 4, 4) and m.n_nodes == 17 * 5 * 5
    assert int(m.solid.sum()) == 4 and D.nc == 7
    # node index i + 17 j + 85 k; local node a at (a & 1, a >> 1 & 1, a >> 2 & 1)
    c = 3 + 16 * (1 + 4 * 2)
    i, j, kk = m.cell_ijk[c]
    for a, o in enumerate(OFF):
        assert m.conn[c, a] == (i + o[0]) + 17 * (j + o[1]) + 85 * (kk + o[2])


def test_jacobian_vs_central_fd_3d():
    p = _workload(lps_alpha0=0.1)
    D = Discretization(p)
    U = synth.random_state(p, 21)
    Uo = synth.random_state(p, 22)
    k = p["k_fine"]
    A = D.jacobian(U, Uo, 0.07, k)
    Ao = D.jacobian_old(U, Uo, 0.07, k)
    rng = np.random.default_rng(5)
    scale = np.abs(U).max(axis=0)
    for _ in range(2):
        x = rng.normal(size=U.shape) * scale
        eps = 1e-6
        fd = (D.residual(U + eps * x, Uo, 0.07, k) - D.residual(U - eps * x, Uo, 0.07, k)) / (2 * eps)
        an = (A @ x.ravel()).reshape(U.shape)
        assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()
        fdo = (D.residual(U, Uo + eps * x, 0.07, k) - D.residual(U, Uo - eps * x, 0.07, k)) / (2 * eps)
        ano = (Ao @ x.ravel()).reshape(U.shape)
        assert np.abs(fdo - ano).max() <= 1e-6 * np.abs(ano).max()
    assert abs(Ao[:, 6::7]).max() == 0.0


def test_zero_displacement_reduces_to_eulerian_ns_3d():
    p = _workload(lps_alpha0=0.0)
    D = Discretization(p)
    U = synth.random_state(p, 31)
    Uo = synth.random_state(p, 32)
    U[:, 3:6] = 0.0
    Uo[:, 3:6] = 0.0
    k = p["k_fine"]
    th = 0.5 + p["theta0"] * k
    R = D.residual(U, Uo, 0.2, k, with_dirichlet=False)
    Uop = Uo.copy()
    Uop[:, 6] = U[:, 6]
    A_new = _eulerian(D, U, 1.0, p, moved=False)
    A_old = _eulerian(D, Uop, 1.0, p, moved=False)
    E = th * k * A_new + (1 - th) * k * A_old
    E[:, 6] = k * A_new[:, 6]
    m = D.mesh
    for c in np.nonzero(m.fluid)[0]:
        nodes = m.conn[c]
        vol = np.prod(m.h[c])
        for x0 in G2:
            for x1 in G2:
                for x2 in G2:
                    N, _ = _basis((x0, x1, x2))
                    dv = N @ (U[nodes, 0:3] - Uo[nodes, 0:3])
                    for a in range(8):
                        E[nodes[a], 0:3] += p["rho_f"] * vol / 8.0 * dv * N[a]
    rows = _rows_to_check(D)
    err = np.abs(R[rows] - E[rows]).max()
    assert err <= 1e-12 * np.abs(E[rows]).max(), err


def test_ale_stationary_terms_equal_eulerian_on_moved_mesh_3d():
    p = _workload(lps_alpha0=0.0)
    D = Discretization(p)
    U = synth.random_state(p, 41, grad_u_max=0.2)
    k = p["k_fine"]
    R = D.residual(U, U, 0.2, k, with_dirichlet=False)
    E = _eulerian(D, U, k, p, moved=True)
    rows = _rows_to_check(D)
    err = np.abs(R[rows] - E[rows]).max()
    assert err <= 1e-12 * np.abs(E[rows]).max(), err
    E0 = _eulerian(D, U, k, p, moved=False)
    assert np.abs(R[rows] - E0[rows]).max() > 1e-4 * np.abs(E[rows]).max()


def test_ale_time_derivative_vanishes_for_steady_affine_flow_3d():
    p = _workload(lps_alpha0=0.0)
    D = Discretization(p)
    rng = np.random.default_rng(7)
    c = rng.normal(size=3)
    Gm = rng.normal(size=(3, 3))
    U = synth.random_state(p, 51, grad_u_max=0.2)
    Uo = synth.random_state(p, 52, grad_u_max=0.2)
    X = D.mesh.X
    U[:, 0:3] = c + (X + U[:, 3:6]) @ Gm.T
    Uo[:, 0:3] = c + (X + Uo[:, 3:6]) @ Gm.T
    R = D.residual(U, Uo, 0.2, 0.0, theta=0.5, with_dirichlet=False)
    rows = _rows_to_check(D)
    rows[:, 6] = False
    ref = p["rho_f"] * np.abs(U[:, 0:3] - Uo[:, 0:3]).max() * np.prod(D.mesh.h, 1).max()
    assert np.abs(R[rows]).max() <= 1e-13 * ref
    U2 = U.copy()
    U2[:, 0] += 0.1 * np.sin(7 * X[:, 1])
    R2 = D.residual(U2, Uo, 0.2, 0.0, theta=0.5, with_dirichlet=False)
    assert np.abs(R2[rows]).max() > 1e-3 * ref


def test_solid_stress_is_strain_energy_gradient_3d():
    p = _workload()
    D = Discretization(p)
    U = synth.random_state(p, 61, grad_u_max=0.2)
    U[:, 0:3] = 0.0
    U[:, 6] = 0.0
    k = p["k_fine"]
    R = D.residual(U, U, 0.2, k, with_dirichlet=False)
    m = D.mesh
    mu, lam = p["mu_s"], p["lambda_s"]

    def energy(u):
        e = 0.0
        for c in np.nonzero(m.solid)[0]:
            nodes = m.conn[c]
            h = m.h[c]
            for x0 in G2:
                for x1 in G2:
                    for x2 in G2:
                        _, dN = _basis((x0, x1, x2))
                        gN = dN / h
                        F = np.eye(3) + u[nodes].T @ gN
                        E = 0.5 * (F.T @ F - np.eye(3))
                        e = e + np.prod(h) / 8.0 * (mu * np.sum(E * E) + 0.5 * lam * np.trace(E) ** 2)
        return e

    rng = np.random.default_rng(9)
    for _ in range(2):
        w = rng.normal(size=(m.n_nodes, 3))
        dpsi = energy(U[:, 3:6] + 1e-30j * w).imag / 1e-30
        assert abs(np.sum(R[:, 0:3] * w) - k * dpsi) <= 1e-12 * abs(k * dpsi)


def test_inflow_profile_3d():
    """v_x = s(t) peak 16 y (H - y) z (W - z) / (H^2 W^2) on the inflow face, zero on its edges."""
    p = _workload()
    D = Discretization(p)
    X = D.mesh.X
    g = D.dirichlet_values(1.0, peak=0.3)
    inflow = np.abs(X[:, 0]) < 1e-12
    H = W = 0.4
    expect = 0.3 * 16 * X[:, 1] * (H - X[:, 1]) * X[:, 2] * (W - X[:, 2]) / (H * H * W * W)
    assert np.allclose(g[inflow, 0], expect[inflow], rtol=0, atol=1e-15)
    assert g[inflow, 0].max() == 0.3 * 16 * 0.2 * 0.2 * 0.2 * 0.2 / 0.4 ** 4
    assert np.all(g[:, 1:] == 0.0)
