"""Oracle pins for the biquadratic (Q2) equal-order discretisation of Section 2.2
(the paper's own element, V_h^(2) for v, u and p), 2d.

The checks recompute what the Q2 oracle does by routes that do not use its
basis or quadrature code: Gauss-Legendre exactness against the integrals of
monomials, nodal interpolation of biquadratics, the textbook 1d quadratic
element matrices in tensor form against whole residual rows, exact discrete
harmonicity of a harmonic quadratic, central differences of the residual, an
Eulerian Navier-Stokes residual written here with its own Q2 basis loops, the
properties of the one-level local projection, and the order of the time
stepping.
"""
import numpy as np
import pytest

import synth
from oracle.fe import gauss_rule, q2_basis
from oracle.residual import Discretization
from oracle import propagate as P


def _q2p(**kw):
    """The c1 channel with Q2 cells on level 0 (16 x 4 cells, 33 x 9 nodes: the nodes of c1)."""
    kw.setdefault("level", 0)
    return synth.workload("c1", degree=2, **kw)


def test_gauss3_exact_to_degree_5():
    x, w = gauss_rule(1, 3)
    for kdeg in range(6):
        assert abs(np.sum(w * x[:, 0] ** kdeg) - 1.0 / (kdeg + 1)) < 1e-15
    assert abs(np.sum(w * x[:, 0] ** 6) - 1.0 / 7) > 1e-5
    x2, w2 = gauss_rule(2, 3)
    for i in range(6):
        for j in range(6):
            assert abs(np.sum(w2 * x2[:, 0] ** i * x2[:, 1] ** j) - 1.0 / ((i + 1) * (j + 1))) < 1e-15


def test_q2_basis_nodal_and_reproduces_biquadratics():
    nodes = np.array([[(a % 3) / 2.0, (a // 3) / 2.0] for a in range(9)])
    N, dN = q2_basis(2, nodes)
    assert np.allclose(N, np.eye(9), atol=1e-15)
    rng = np.random.default_rng(3)
    c = rng.normal(size=(3, 3))

    def q(x, y):
        return sum(c[i, j] * x ** i * y ** j for i in range(3) for j in range(3))

    def dq(x, y):
        return (sum(i * c[i, j] * x ** (i - 1) * y ** j for i in range(1, 3) for j in range(3)),
                sum(j * c[i, j] * x ** i * y ** (j - 1) for i in range(3) for j in range(1, 3)))

    pts = rng.uniform(0, 1, size=(20, 2))
    Np, dNp = q2_basis(2, pts)
    vals = q(nodes[:, 0], nodes[:, 1])
    assert np.allclose(Np @ vals, q(pts[:, 0], pts[:, 1]), atol=1e-13)
    gx, gy = dq(pts[:, 0], pts[:, 1])
    assert np.allclose(dNp[:, :, 0] @ vals, gx, atol=1e-12)
    assert np.allclose(dNp[:, :, 1] @ vals, gy, atol=1e-12)
    assert np.allclose(Np.sum(axis=1), 1.0) and np.allclose(dNp.sum(axis=1), 0.0, atol=1e-13)


def _mass1(pts):
    """Assembled 1d quadratic-element mass matrix on nodes pts (cells = pairs of node intervals):
    the textbook element matrix h/30 [[4, 2, -1], [2, 16, 2], [-1, 2, 4]]."""
    n = len(pts)
    A = np.zeros((n, n))
    for i in range(0, n - 2, 2):
        h = pts[i + 2] - pts[i]
        A[i:i + 3, i:i + 3] += h / 30.0 * np.array([[4.0, 2.0, -1.0], [2.0, 16.0, 2.0], [-1.0, 2.0, 4.0]])
    return A


def _stiff1(pts):
    """The same for the Laplace stiffness, 1/(3 h) [[7, -8, 1], [-8, 16, -8], [1, -8, 7]]."""
    n = len(pts)
    A = np.zeros((n, n))
    for i in range(0, n - 2, 2):
        h = pts[i + 2] - pts[i]
        A[i:i + 3, i:i + 3] += 1.0 / (3.0 * h) * np.array([[7.0, -8.0, 1.0], [-8.0, 16.0, -8.0], [1.0, -8.0, 7.0]])
    return A


def test_q2_solid_inertia_is_tensor_mass():
    """Solid momentum rows with mu_s = lambda_s = 0, the fluid at rest and no displacement:
    rho_s (M_y x M_x)(v - v°) on the bar's nodes, with the textbook 1d quadratic mass matrices.
    A lumped mass, a lower-order rule or wrong basis fails."""
    p = _q2p(mu_s=0.0, lambda_s=0.0, rho_s=1234.5)
    D = Discretization(p)
    m = D.mesh
    x, y = m.naxes
    ix = np.nonzero((x >= 0.4 - 1e-12) & (x <= 0.5 + 1e-12))[0]
    iy = np.nonzero(y <= 0.25 + 1e-12)[0]
    Ms = np.kron(_mass1(y[iy]), _mass1(x[ix]))
    nodes = (ix[None, :] + len(x) * iy[:, None]).ravel()
    rng = np.random.default_rng(7)
    U = np.zeros((m.n_nodes, 5))
    Uo = np.zeros((m.n_nodes, 5))
    strict = ~m.in_NF
    assert strict.sum() > 0 and strict[nodes].sum() == strict.sum()
    U[strict, 0:2] = rng.uniform(-1.0, 1.0, size=(strict.sum(), 2))
    Uo[strict, 0:2] = rng.uniform(-1.0, 1.0, size=(strict.sum(), 2))
    R = D.residual(U, Uo, 0.5, p["k_fine"], with_dirichlet=False)
    expect = np.zeros((m.n_nodes, 2))
    expect[nodes] = p["rho_s"] * (Ms @ (U[nodes, 0:2] - Uo[nodes, 0:2]))
    assert np.abs(R[:, 0:2] - expect).max() <= 1e-13 * np.abs(expect).max()


def test_q2_harmonic_extension_rows_are_tensor_stiffness():
    """Displacement rows of nodes outside the bar with v = 0, p = 0 and u = u° (so the row is
    k grad u : grad psi over fluid cells): the Kronecker form K_y x M_x + M_y x K_x of the
    textbook 1d quadratic matrices, on a field u supported away from the bar."""
    p = _q2p()
    D = Discretization(p)
    m = D.mesh
    x, y = m.naxes
    k = p["k_fine"]
    rng = np.random.default_rng(11)
    # u nonzero only on nodes with x >= 0.75 (all their cells are fluid cells)
    ix = np.nonzero(x >= 0.75 - 1e-12)[0]
    iy = np.arange(len(y))
    nodes = (ix[None, :] + len(x) * iy[:, None]).ravel()
    U = np.zeros((m.n_nodes, 5))
    sel = m.X[:, 0] >= 0.875 - 1e-12
    U[sel, 2:4] = rng.uniform(-1e-3, 1e-3, size=(sel.sum(), 2))
    R = D.residual(U, U, 0.5, k, with_dirichlet=False)
    A = np.kron(_stiff1(y[iy]), _mass1(x[ix])) + np.kron(_mass1(y[iy]), _stiff1(x[ix]))
    expect = k * (A @ U[nodes, 2:4])
    rows = m.X[nodes, 0] >= 0.75 + 1e-9     # rows whose whole support lies in the block of nodes
    got = R[nodes, 2:4]
    assert np.abs(got[rows] - expect[rows]).max() <= 1e-13 * np.abs(expect[rows]).max()


def test_q2_reproduces_a_harmonic_quadratic():
    """u = u° = eps (x^2 - y^2, 2 x y) is harmonic and lies in the Q2 space: the harmonic-extension
    rows of every node outside the bar and off the outer boundary vanish to round-off (Galerkin
    orthogonality with exact quadrature).  The tensor-form rows above are the discriminating pin;
    this one checks the assembly around the bar."""
    p = _q2p()
    D = Discretization(p)
    m = D.mesh
    X = m.X
    U = np.zeros((m.n_nodes, 5))
    U[:, 2] = 1e-3 * (X[:, 0] ** 2 - X[:, 1] ** 2)
    U[:, 3] = 1e-3 * 2 * X[:, 0] * X[:, 1]
    R = D.residual(U, U, 0.5, p["k_fine"], with_dirichlet=False)
    rows = ~m.in_NS & ~D.dirichlet[:, 2]
    scale = p["k_fine"] * 1e-3 * 4       # k |grad u| |grad psi| |K| ~ k eps O(1)
    assert rows.sum() > 100
    assert np.abs(R[rows, 2:4]).max() <= 1e-12 * scale
    # a harmonic quartic (not in Q2, and beyond the stencils' exactness on this tensor mesh,
    # which also covers the harmonic cubics) leaves a residual
    U[:, 2] = 1e-3 * (X[:, 0] ** 4 - 6 * X[:, 0] ** 2 * X[:, 1] ** 2 + X[:, 1] ** 4)
    U[:, 3] = 0.0
    R = D.residual(U, U, 0.5, p["k_fine"], with_dirichlet=False)
    assert np.abs(R[rows, 2]).max() > 1e-9 * scale


@pytest.mark.parametrize("alpha0", [0.0, 0.1])
def test_q2_jacobian_vs_central_fd(alpha0):
    p = _q2p(lps_alpha0=alpha0)
    D = Discretization(p)
    U = synth.random_state(p, 21)
    Uo = synth.random_state(p, 22)
    k = p["k_fine"]
    A = D.jacobian(U, Uo, 0.07, k)
    Ao = D.jacobian_old(U, Uo, 0.07, k)
    rng = np.random.default_rng(5)
    scale = np.abs(U).max(axis=0)
    for _ in range(2):
        xv = rng.normal(size=U.shape) * scale
        eps = 1e-6
        fd = (D.residual(U + eps * xv, Uo, 0.07, k) - D.residual(U - eps * xv, Uo, 0.07, k)) / (2 * eps)
        an = (A @ xv.ravel()).reshape(U.shape)
        assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()
        fdo = (D.residual(U, Uo + eps * xv, 0.07, k) - D.residual(U, Uo - eps * xv, 0.07, k)) / (2 * eps)
        ano = (Ao @ xv.ravel()).reshape(U.shape)
        assert np.abs(fdo - ano).max() <= 1e-6 * np.abs(ano).max()


def _lag(x):
    """Quadratic Lagrange polynomials on 0, 1/2, 1 and derivatives, written out here."""
    return (np.array([2 * (x - 0.5) * (x - 1.0), -4 * x * (x - 1.0), 2 * x * (x - 0.5)]),
            np.array([4 * x - 3.0, -8 * x + 4.0, 4 * x - 1.0]))


def test_q2_zero_displacement_reduces_to_eulerian_ns():
    """With u = u° = 0 the Q2 ALE step is the Eulerian Navier-Stokes CN step, here assembled
    cell by cell with this file's own Q2 basis and numpy's Gauss-Legendre points."""
    p = _q2p(lps_alpha0=0.0)
    D = Discretization(p)
    m = D.mesh
    U = synth.random_state(p, 31)
    Uo = synth.random_state(p, 32)
    U[:, 2:4] = 0.0
    Uo[:, 2:4] = 0.0
    k = p["k_fine"]
    th = 0.5 + p["theta0"] * k
    rf, nu = p["rho_f"], p["nu_f"]
    R = D.residual(U, Uo, 0.2, k, with_dirichlet=False)
    gx, gw = np.polynomial.legendre.leggauss(3)
    gx, gw = 0.5 * (gx + 1.0), 0.5 * gw
    E = np.zeros_like(R)
    for c in np.nonzero(m.fluid)[0]:
        nodes = m.conn[c]
        hx, hy = m.h[c]
        for qx, wx in zip(gx, gw):
            for qy, wy in zip(gx, gw):
                Lx, dLx = _lag(qx)
                Ly, dLy = _lag(qy)
                N = np.array([Lx[a % 3] * Ly[a // 3] for a in range(9)])
                G = np.array([[dLx[a % 3] * Ly[a // 3] / hx, Lx[a % 3] * dLy[a // 3] / hy] for a in range(9)])
                w = wx * wy * hx * hy
                v, vo = N @ U[nodes, 0:2], N @ Uo[nodes, 0:2]
                gv, gvo = U[nodes, 0:2].T @ G, Uo[nodes, 0:2].T @ G
                pr = N @ U[nodes, 4]
                sig = rf * nu * (gv + gv.T) - pr * np.eye(2)
                sigo = rf * nu * (gvo + gvo.T) - pr * np.eye(2)
                mom = rf * (v - vo) + k * th * rf * gv @ v + k * (1 - th) * rf * gvo @ vo
                for a in range(9):
                    E[nodes[a], 0:2] += w * (mom * N[a] + (k * th * sig + k * (1 - th) * sigo) @ G[a])
                    E[nodes[a], 4] += w * k * np.trace(gv) * N[a]
    for c in m.outflow_cells:
        nodes = m.conn[c]
        hy = m.h[c][1]
        for qy, wy in zip(gx, gw):
            Lx, dLx = _lag(1.0)
            Ly, dLy = _lag(qy)
            N = np.array([Lx[a % 3] * Ly[a // 3] for a in range(9)])
            G = np.array([[dLx[a % 3] * Ly[a // 3] / m.h[c][0], Lx[a % 3] * dLy[a // 3] / hy] for a in range(9)])
            gv, gvo = U[nodes, 0:2].T @ G, Uo[nodes, 0:2].T @ G
            b = k * th * rf * nu * gv.T @ np.array([1.0, 0.0]) + k * (1 - th) * rf * nu * gvo.T @ np.array([1.0, 0.0])
            for a in range(9):
                E[nodes[a], 0:2] -= wy * hy * b * N[a]
    rows = np.zeros_like(D.dirichlet)
    free = ~D.dirichlet
    rows[:, 0:2] = (~m.in_NS)[:, None] & free[:, 0:2]
    rows[:, 4] = m.in_NF & free[:, 4]
    err = np.abs(R[rows] - E[rows]).max()
    assert err <= 1e-12 * np.abs(E[rows]).max(), err


def test_q2_lps_properties():
    """Symmetric, positive semi-definite, zero on every function that is bilinear on each cell
    (the Q1 functions of the cells, continuous), positive on the checkerboard of the nodes."""
    p = _q2p()
    D = Discretization(p)
    m = D.mesh
    S = D.S.toarray()
    assert np.allclose(S, S.T, atol=1e-12 * np.abs(S).max())
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() > -1e-10 * ev.max()
    # a continuous cellwise-bilinear function: random vertex values, midpoints interpolated
    rng = np.random.default_rng(4)
    nx, ny = m.nshape
    P = np.zeros((nx, ny))
    P[0::2, 0::2] = rng.normal(size=((nx + 1) // 2, (ny + 1) // 2))
    P[1::2, 0::2] = 0.5 * (P[0:-1:2, 0::2] + P[2::2, 0::2])
    P[:, 1::2] = 0.5 * (P[:, 0:-1:2] + P[:, 2::2])
    pq = P.ravel(order="F")
    assert np.abs(S @ pq).max() <= 1e-12 * np.abs(S).max() * np.abs(pq).max()
    chk = (-1.0) ** (m.node_ijk[:, 0] + m.node_ijk[:, 1])
    assert chk @ S @ chk > 1e-3 * np.abs(S).max()


def test_q2_shifted_cn_second_order():
    """theta = 1/2 + k with Q2 cells: the self-convergence ratio of the time stepping -> 4."""
    p = _q2p(mu_s=5e3, nu_f=1e-2, ramp_time=0.2)
    p["lambda_s"] = synth.lame_lambda(p["mu_s"], p["nu_s"])
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    sols = [P.propagate(D, U0, 0.0, 0.1, n) for n in (4, 8, 16, 32)]
    for sl in (slice(0, 2), slice(2, 4)):
        e = [np.linalg.norm(sols[j][:, sl] - sols[j + 1][:, sl]) for j in range(3)]
        assert 3.3 < e[1] / e[2] < 4.7, e
