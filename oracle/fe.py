"""Q1 basis functions and Gauss-Legendre quadrature on the unit cell.

Section 2.2: equal-order iso-parametric tensor-product elements.  The
workloads use the lowest order (bilinear / trilinear, Q1).  On the
axis-aligned cells of the tensor mesh the reference map is affine, so
physical gradients are reference gradients divided by the cell widths.
"""
from __future__ import annotations

import itertools

import numpy as np

# two-point Gauss-Legendre rule on [0, 1]
GAUSS1_X = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
GAUSS1_W = np.array([0.5, 0.5])


def gauss_rule(dim: int):
    """Tensor Gauss rule on [0,1]^dim: points [nq, dim], weights [nq]."""
    pts = np.array(list(itertools.product(GAUSS1_X, repeat=dim)))[:, ::-1]
    wts = np.array([np.prod(w) for w in itertools.product(GAUSS1_W, repeat=dim)])
    return pts.copy(), wts


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
