"""Local-projection pressure stabilisation (two-level, reference domain).

Section 2.2 adds a local-projection stabilisation (Becker & Braack) to the
equal-order pair without stating its form.  The reading used here is the
two-level variant on the interface-fitted hierarchy:

    s_h(p, xi) = sum over fluid cells K of  alpha_K (grad(p - i_2h p), grad(xi - i_2h xi))_K,

where i_2h is bilinear (trilinear) interpolation on the parent cell of K
(the level l-1 cell made of 2^d level-l cells), alpha_K = alpha0 h_K^2 /
(rho_f nu_f) and h_K = |K|^(1/d).  It lives on the fixed reference domain,
so it does not depend on the state or on the solid parameters: one constant
symmetric positive semi-definite matrix on the pressure unknowns.  It enters
the pressure rows of the time-step residual as k s_h(p, xi), with the same
factor k as the divergence term, and vanishes on functions that are Q1 on
every parent cell.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def lps_matrix(disc) -> sp.csr_matrix:
    m = disc.mesh
    d = m.dim
    p = disc.p
    nloc = 2 ** d
    offs = np.asarray([[(a >> r) & 1 for r in range(d)] for a in range(nloc)])
    # fine-cell Laplace stiffness [cells, a, b] with the 2-point Gauss rule (exact)
    K = np.einsum("cq,cqar,cqbr->cab", disc.W, disc.G, disc.G)
    hK = np.prod(m.h, axis=1) ** (1.0 / d)
    alpha = p["lps_alpha0"] * hK ** 2 / (p["rho_f"] * p["nu_f"])
    rows, cols, vals = [], [], []
    patch_offs = np.asarray(list(itertools.product(range(3), repeat=d)))[:, ::-1]
    npn = patch_offs.shape[0]
    flu = np.nonzero(m.fluid)[0]
    cij = m.cell_ijk[flu]
    child = cij % 2
    origin = cij - child                                    # patch origin node (multi-index)
    # global node index of every patch node [cells, npn]
    pnode = m.node_index(origin[:, None, :] + patch_offs[None, :, :])
    # patch-local index of an offset vector in {0,1,2}^d
    def pidx(o):
        idx = np.zeros(o.shape[:-1], dtype=np.int64)
        mul = 1
        for r in range(d):
            idx = idx + mul * o[..., r]
            mul *= 3
        return idx
    kappa = np.zeros((flu.size, nloc, npn))
    for a in range(nloc):
        off = child + offs[a]                                # offset of fine node a in the patch
        kappa[np.arange(flu.size), a, pidx(off)] += 1.0
        s = off / 2.0                                        # position in the parent cell
        for b in range(nloc):
            w = np.ones(flu.size)
            for r in range(d):
                w = w * (s[:, r] if offs[b, r] else 1.0 - s[:, r])
            kappa[np.arange(flu.size), a, pidx(2 * offs[b][None, :])] -= w
    SK = alpha[flu, None, None] * np.einsum("cap,cab,cbq->cpq", kappa, K[flu], kappa)
    rows = np.broadcast_to(pnode[:, :, None], SK.shape).ravel()
    cols = np.broadcast_to(pnode[:, None, :], SK.shape).ravel()
    S = sp.csr_matrix((SK.ravel(), (rows, cols)), shape=(m.n_nodes, m.n_nodes))
    S.sum_duplicates()
    return S


def lps_matrix_q2(disc) -> sp.csr_matrix:
    """One-level local projection for the Q2 pair (2d):

        s_h(p, xi) = sum over fluid cells K of alpha_K (grad(p - i_h p), grad(xi - i_h xi))_K,

    i_h the bilinear (Q1) interpolation on K from its four vertex values: the Q2
    functions of a cell against the Q1 ones of the same cell play the part that the
    Q1 functions of a patch of four cells play against the parent cell's in the Q1
    case (a Q2 cell carries the nine nodes of such a patch).  alpha_K as there,
    alpha_K = alpha0 h_K^2 / (rho_f nu_f) with h_K = |K|^(1/2); the 3-point Gauss rule
    integrates the Q2 Laplace stiffness exactly.  Constant, symmetric, positive
    semi-definite, zero on the functions that are Q1 on every fluid cell."""
    m = disc.mesh
    d = m.dim
    p = disc.p
    nloc = m.nloc
    K = np.einsum("cq,cqar,cqbr->cab", disc.W, disc.G, disc.G)         # Q2 Laplace stiffness [cells, a, b]
    hK = np.prod(m.h, axis=1) ** (1.0 / d)
    alpha = p["lps_alpha0"] * hK ** 2 / (p["rho_f"] * p["nu_f"])
    # kappa = I - i_h on the local nodes: node a at position o/2 gets the bilinear
    # combination of the four vertex values (vertex = all offsets 0 or 2)
    kappa = np.eye(nloc)
    for a in range(nloc):
        s_ = [((a // 3 ** r) % 3) / 2.0 for r in range(d)]
        for b in range(nloc):
            ob = [(b // 3 ** r) % 3 for r in range(d)]
            if any(o == 1 for o in ob):
                continue
            w = 1.0
            for r in range(d):
                w *= s_[r] if ob[r] == 2 else 1.0 - s_[r]
            kappa[a, b] -= w
    flu = np.nonzero(m.fluid)[0]
    SK = alpha[flu, None, None] * np.einsum("ap,cab,bq->cpq", kappa, K[flu], kappa)
    nodes = m.conn[flu]
    rows = np.broadcast_to(nodes[:, :, None], SK.shape).ravel()
    cols = np.broadcast_to(nodes[:, None, :], SK.shape).ravel()
    S = sp.csr_matrix((SK.ravel(), (rows, cols)), shape=(m.n_nodes, m.n_nodes))
    S.sum_duplicates()
    return S
