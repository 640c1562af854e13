"""Q1 and Q2 basis functions and Gauss-Legendre quadrature on the unit cell.

Section 2.2: equal-order iso-parametric tensor-product elements Q^(r).  The
workloads use the lowest order (bilinear / trilinear, Q1); the paper's own
choice, biquadratic Q2, is here for 2d.  On the axis-aligned cells of the
tensor mesh the reference map is affine, so physical gradients are reference
gradients divided by the cell widths.
"""
from __future__ import annotations

import itertools

import numpy as np

# two-point Gauss-Legendre rule on [0, 1]
GAUSS1_X = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
GAUSS1_W = np.array([0.5, 0.5])


# three-point Gauss-Legendre rule on [0, 1] (exact to degree 5)
GAUSS3_X = np.array([0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)])
GAUSS3_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


def gauss_rule(dim: int, npts: int = 2):
    """Tensor Gauss rule on [0,1]^dim with npts (2 or 3) points per axis: points [nq, dim], weights [nq].

    Point q has coordinate r from digit r of q in base npts (the first axis fastest)."""
    x1, w1 = (GAUSS1_X, GAUSS1_W) if npts == 2 else (GAUSS3_X, GAUSS3_W)
    pts = np.array(list(itertools.product(x1, repeat=dim)))[:, ::-1]
    wts = np.array([np.prod(w) for w in itertools.product(w1, repeat=dim)])
    return pts.copy(), wts


def lagrange2_1d(x):
    """Quadratic Lagrange basis on the nodes 0, 1/2, 1 and its derivatives: [3, ...] each."""
    x = np.asarray(x, dtype=np.result_type(x, np.float64))
    L = np.stack([(2 * x - 1) * (x - 1), 4 * x * (1 - x), x * (2 * x - 1)])
    dL = np.stack([4 * x - 3, 4 - 8 * x, 4 * x - 1])
    return L, dL


def q2_basis(dim: int, xi: np.ndarray):
    """Values [nq, 3^d] and reference gradients [nq, 3^d, d] of the Q2 (tensor Lagrange) basis.

    Local node a sits at offset o_r / 2 on axis r, o_r the base-3 digit r of a
    (the first axis fastest); its basis function is prod_r L_{o_r}(xi_r)."""
    xi = np.atleast_2d(xi)
    nq = xi.shape[0]
    nloc = 3 ** dim
    L, dL = zip(*[lagrange2_1d(xi[:, r]) for r in range(dim)])
    N = np.ones((nq, nloc))
    dN = np.ones((nq, nloc, dim))
    for a in range(nloc):
        o = [(a // 3 ** r) % 3 for r in range(dim)]
        for r in range(dim):
            N[:, a] *= L[r][o[r]]
            for s in range(dim):
                dN[:, a, s] *= dL[r][o[r]] if s == r else L[r][o[r]]
    return N, dN


def q1_basis(dim: int, xi: np.ndarray):
    """Values [nq, 2^d] and reference gradients [nq, 2^d, d] of the Q1 basis.

    Local node a sits at the corner whose coordinate r is bit r of a; its
    basis function is prod_r (xi_r if bit set else 1 - xi_r).
    """
    xi = np.atleast_2d(xi)
    nq = xi.shape[0]
    nloc = 2 ** dim
    N = np.ones((nq, nloc))
    dN = np.ones((nq, nloc, dim))
    for a in range(nloc):
        for r in range(dim):
            bit = (a >> r) & 1
            f = xi[:, r] if bit else 1.0 - xi[:, r]
            df = 1.0 if bit else -1.0
            N[:, a] *= f
            for s in range(dim):
                dN[:, a, s] *= (df if s == r else f)
    return N, dN
