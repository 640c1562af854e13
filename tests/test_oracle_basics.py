"""Oracle pins: quadrature, basis, mesh, data, stabilisation, linear solve, speedup model."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.fe import gauss_rule, q1_basis
from oracle.mesh import Mesh
from oracle.residual import Discretization, ramp
from oracle.propagate import speedup_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_gauss_exact_to_degree_3(dim):
    x, w = gauss_rule(dim)
    assert abs(w.sum() - 1.0) < 1e-15
    rng = np.random.default_rng(dim)
    for _ in range(10):
        e = rng.integers(0, 4, size=dim)         # degree <= 3 per direction
        exact = np.prod(1.0 / (e + 1.0))
        approx = np.sum(w * np.prod(x ** e, axis=1))
        assert abs(approx - exact) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_basis_partition_and_nodal(dim):
    rng = np.random.default_rng(0)
    xi = rng.uniform(size=(7, dim))
    N, dN = q1_basis(dim, xi)
    assert np.allclose(N.sum(1), 1.0, atol=1e-15)
    assert np.allclose(dN.sum(1), 0.0, atol=1e-15)
    corners = np.asarray([[(a >> r) & 1 for r in range(dim)] for a in range(2 ** dim)], float)
    Nc, _ = q1_basis(dim, corners)
    assert np.allclose(Nc, np.eye(2 ** dim))
    # gradient of the interpolant of a linear function is exact
    g = rng.normal(size=dim)
    vals = corners @ g
    grad = np.einsum("qar,a->qr", dN, vals)
    assert np.allclose(grad, g[None, :], atol=1e-14)


@pytest.mark.parametrize("name,shape,solid", [
    ("c1", (32, 8), 8), ("c2", (128, 32), 128), ("c3", (256, 64), 512),
    ("c4", (128, 32), 128), ("c5", (64, 16, 16), 256)])
def test_mesh_sizes(name, shape, solid):
    p = synth.workload(name)
    m = Mesh(p)
    assert m.shape == shape
    assert int(m.solid.sum()) == solid


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_mesh_interface_fitted(level):
    """The bar faces x = 0.4, 0.5 and y = 0.25 are mesh lines on every level."""
    p = synth.workload("c1")
    m = Mesh(p, level)
    for x in (0.4, 0.5):
        assert np.min(np.abs(m.axes[0] - x)) < 1e-14
    assert np.min(np.abs(m.axes[1] - 0.25)) < 1e-14
    # every cell is wholly fluid or wholly solid and the bar area is resolved
    area = np.sum(np.prod(m.h[m.solid], axis=1))
    assert abs(area - 0.1 * 0.25) < 1e-14


def test_node_classes_c1():
    p = synth.workload("c1")
    m = Mesh(p)
    # bar 2 x 4 cells -> 3 x 5 nodes; interface nodes = bar nodes minus strictly solid
    assert m.in_NS.sum() == 15
    interface = m.in_NS & m.in_NF
    strictly_solid = m.in_NS & ~m.in_NF
    # strictly solid: the bar's interior column (x = 0.45) below the top, incl. floor node
    assert strictly_solid.sum() == 4
    assert interface.sum() == 11


def test_inflow_profile_and_ramp():
    p = synth.workload("c1")
    D = Discretization(p)
    assert ramp(0.0, 0.1) == 0.0
    assert abs(ramp(0.05, 0.1) - 0.5) < 1e-15
    assert ramp(0.1, 0.1) == 1.0 and ramp(0.7, 0.1) == 1.0
    g = D.dirichlet_values(0.5)
    X = D.mesh.X
    mid = np.nonzero((np.abs(X[:, 0]) < 1e-14) & (np.abs(X[:, 1] - 0.25) < 1e-14))[0]
    assert abs(g[mid[0], 0] - p["inflow_peak"]) < 1e-15
    quarter = np.nonzero((np.abs(X[:, 0]) < 1e-14) & (np.abs(X[:, 1] - 0.125) < 1e-14))[0]
    assert abs(g[quarter[0], 0] - 0.75 * p["inflow_peak"]) < 1e-15
    assert np.all(g[:, 1:] == 0.0)


def test_lps_properties():
    """s_h is symmetric PSD, vanishes on parent-patch Q1 functions, sees the fine scale."""
    p = synth.workload("c1")
    D = Discretization(p)
    S = D.S.toarray()
    assert np.abs(S - S.T).max() < 1e-18
    ev = np.linalg.eigvalsh(S)
    assert ev.min() > -1e-12 * ev.max()
    # a function that is Q1 on every level-0 cell: interpolate a random level-0 field
    m = D.mesh
    m0 = Mesh(p, 0)
    rng = np.random.default_rng(3)
    f0 = rng.normal(size=m0.n_nodes)
    ix = np.clip(np.searchsorted(m0.axes[0], m.X[:, 0], side="right") - 1, 0, m0.shape[0] - 1)
    iy = np.clip(np.searchsorted(m0.axes[1], m.X[:, 1], side="right") - 1, 0, m0.shape[1] - 1)
    sx = (m.X[:, 0] - m0.axes[0][ix]) / np.diff(m0.axes[0])[ix]
    sy = (m.X[:, 1] - m0.axes[1][iy]) / np.diff(m0.axes[1])[iy]
    n = lambda i, j: m0.node_index(np.stack([i, j], -1))
    f = ((1 - sx) * (1 - sy) * f0[n(ix, iy)] + sx * (1 - sy) * f0[n(ix + 1, iy)]
         + (1 - sx) * sy * f0[n(ix, iy + 1)] + sx * sy * f0[n(ix + 1, iy + 1)])
    # only fluid patches contribute; the function is parent-Q1 everywhere
    assert np.abs(S @ f).max() < 1e-12 * np.abs(S).max() * np.abs(f).max()
    # a checkerboard is not parent-Q1 and must be penalised
    chk = (-1.0) ** (m.node_ijk[:, 0] + m.node_ijk[:, 1])
    assert chk @ S @ chk > 1e-3 * np.abs(S).max()
    # alpha scaling: alpha_K = alpha0 h_K^2 / (rho nu) with the Laplacian of the fluctuation
    p2 = dict(p, lps_alpha0=2 * p["lps_alpha0"])
    assert np.allclose(Discretization(p2).S.toarray(), 2 * S, rtol=0, atol=1e-18)


def test_dense_vs_sparse_lu():
    p = synth.workload("c1")
    D = Discretization(p)
    U = synth.random_state(p, 11)
    Uo = synth.random_state(p, 12)
    A = D.jacobian(U, Uo, 0.3, p["k_fine"])
    x_true = synth.random_state(p, 13).ravel()
    b = A @ x_true
    x1 = spla.splu(A.tocsc()).solve(b)
    x2 = np.linalg.solve(A.toarray(), b)
    # rows span many orders of magnitude (pressure rows ~ k h, solid rows ~ k mu_s):
    # the unscaled condition number is ~1e15, so compare backward errors with row
    # scaling and forward errors against cond * eps
    r = 1.0 / abs(A).max(axis=1).toarray().ravel()
    for x in (x1, x2):
        assert np.linalg.norm(r * (A @ x - b)) <= 1e-10 * np.linalg.norm(r * b)
    assert np.linalg.norm(x1 - x2) <= 1e-6 * np.linalg.norm(x2)


def test_speedup_model_golden():
    """eq. (eq:speedup) at the 2d example's values gives the printed 5.78."""
    with open(os.path.join(GOLDEN, "speedup_model.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        s = speedup_model(c["r"], c["K"], c["N"])
        assert abs(s - c["S"]) <= c["abs_tol"], (c, s)


def test_workload_time_grids():
    """T/L = m k = M K (Section 3) with the requested steps rounded down."""
    expect = {"c1": (8, 13, 2), "c2": (32, 32, 4), "c3": (64, 32, 4), "c4": (32, 16, 2), "c5": (16, 10, 1)}
    for name, (N, m, M) in expect.items():
        p = synth.workload(name)
        assert (p["N"], p["m"], p["M"]) == (N, m, M)
        assert abs(p["m"] * p["k_fine"] - p["T"] / N) < 1e-15
        assert abs(p["M"] * p["k_coarse"] - p["T"] / N) < 1e-15
        assert p["k_fine"] <= p["dt_fine"] + 1e-15
