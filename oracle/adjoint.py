"""Time-integrated drag on the elastic bar and its discrete adjoint gradient.

The paper reports the drag of the fsi-3 benchmark (Section 4.2, Figure
"fsi3") without a formula; the reading used here:

    D(U) = sum over the bar faces shared with a fluid cell of
           int_face e_x . (J sigma(v, p; F) F^{-T} n_s) ds,

with sigma of eq. (ALE:stress), the gradients of the adjacent fluid cell, n_s
the outward normal of the solid (pointing into the fluid), 2-point Gauss per
face on the reference configuration; D > 0 for flow in +x.  The functional
is J = k sum_{n=1}^{N m} D(U^n) (right-endpoint rule) along the sequential
fine trajectory.

Discrete adjoint of the fine time stepping R_n(U^n, U^{n-1}; q) = 0:
    lambda_{Nm+1} = 0,
    (dR_n/dU^n)^T lambda_n = -k dD/dU(U^n) - (dR_{n+1}/dU^n)^T lambda_{n+1},
    dJ/dq = sum_n lambda_n^T dR_n/dq,
for q = inflow peak (Dirichlet rows only), mu_s and lambda_s (solid rows).
Every derivative here is a complex-step derivative of the oracle's own
residual or drag, evaluated exactly (no subtractive cancellation).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fe import gauss_rule, q1_basis
from .residual import det_inv
from .propagate import newton_step

PARAMS = ("inflow_peak", "mu_s", "lambda_s")


def drag_faces(disc):
    """Bar faces shared with a fluid cell: (fluid cell, face axis, face side in the fluid cell, n_s sign)."""
    m = disc.mesh
    d = m.dim
    faces = []
    for c in np.nonzero(m.solid)[0]:
        ijk = m.cell_ijk[c]
        for ax in range(d):
            for sgn in (-1, 1):
                nb = ijk.copy()
                nb[ax] += sgn
                if nb[ax] < 0 or nb[ax] >= m.shape[ax]:
                    continue
                cf = _cell_index(m, nb)
                if m.fluid[cf]:
                    # the face lies at the fluid cell's side opposite to sgn; n_s = sgn e_ax
                    faces.append((cf, ax, 0 if sgn > 0 else 1, sgn))
    return faces


def _cell_index(m, ijk):
    idx, stride = 0, 1
    for q in range(m.dim):
        idx += stride * int(ijk[q])
        stride *= m.shape[q]
    return idx


def drag(disc, U, params=None):
    """D(U): fluid traction on the bar, x-component (real or complex U)."""
    p = dict(disc.p)
    if params:
        p.update(params)
    m, d = disc.mesh, disc.dim
    rn = p["rho_f"] * p["nu_f"]
    xf, wf = gauss_rule(d - 1)
    total = 0.0
    for (c, ax, side, sgn) in drag_faces(disc):
        h = m.h[c]
        # face points in the fluid cell's reference coordinates
        pts = np.zeros((xf.shape[0], d))
        others = [q for q in range(d) if q != ax]
        pts[:, ax] = float(side)
        for t, q in enumerate(others):
            pts[:, q] = xf[:, t]
        N, dN = q1_basis(d, pts)
        G = dN / h[None, None, :]
        area = np.prod([h[q] for q in others])
        Ue = U[m.conn[c]]
        for q in range(pts.shape[0]):
            gv = np.einsum("ar,ai->ir", G[q], Ue[:, :d])
            gu = np.einsum("ar,ai->ir", G[q], Ue[:, d:2 * d])
            pr = N[q] @ Ue[:, 2 * d]
            J, Fi = det_inv(np.eye(d) + gu)
            A = gv @ Fi
            sig = rn * (A + A.T) - pr * np.eye(d)
            n = np.zeros(d)
            n[ax] = sgn
            traction = J * (sig @ Fi.T @ n)
            total = total + wf[q] * area * traction[0]
    return total


def drag_gradient(disc, U, h=1e-30):
    """dD/dU (complex step over the unknowns of the cells next to the bar)."""
    g = np.zeros(U.shape)
    nodes = sorted({int(n) for (c, *_r) in drag_faces(disc) for n in disc.mesh.conn[c]})
    for n in nodes:
        for comp in range(U.shape[1]):
            Uc = U.astype(np.complex128)
            Uc[n, comp] += 1j * h
            g[n, comp] = drag(disc, Uc).imag / h
    return g


def trajectory(disc, p, U0, N=None, m=None, params=None, rtol=1e-10):
    """Sequential fine solve: states U^0..U^{N m} and their times."""
    N = p["N"] if N is None else N
    m = p["m"] if m is None else m
    k = p["slice_len"] / m
    states, times = [np.array(U0)], [0.0]
    for l in range(N):
        for n in range(1, m + 1):
            t = l * p["slice_len"] + n * k
            states.append(newton_step(disc, states[-1], t, k, rtol=rtol, params=params))
            times.append(t)
    return states, times, k


def functional(disc, states, k, params=None):
    """J = k sum_{n>=1} D(U^n)."""
    return k * sum(drag(disc, U, params) for U in states[1:])


def param_derivative(disc, U, Uo, t, k, q, h=1e-30):
    """dR/dq at (U, Uo) by complex step in the parameter q."""
    base = disc.p[q]
    return disc.residual(U.astype(np.complex128), Uo.astype(np.complex128), t, k,
                         params={q: base + 1j * h}).imag / h


def adjoint_gradient(disc, p, U0, N=None, m=None):
    """Return (J, dJ/d(peak, mu_s, lambda_s)) by the discrete adjoint."""
    states, times, k = trajectory(disc, p, U0, N, m)
    J = functional(disc, states, k)
    S = len(states) - 1
    grad = np.zeros(len(PARAMS))
    lam_next = None
    for n in range(S, 0, -1):
        U, Uo, t = states[n], states[n - 1], times[n]
        rhs = -k * drag_gradient(disc, U).ravel()
        if lam_next is not None:
            Aold = disc.jacobian_old(states[n + 1], U, times[n + 1], k)
            rhs = rhs - Aold.T @ lam_next
        A = disc.jacobian(U, Uo, t, k)
        lam = _solve_transposed(A, rhs)
        for i, q in enumerate(PARAMS):
            grad[i] += lam @ param_derivative(disc, U, Uo, t, k, q).ravel()
        lam_next = lam
    return J, grad


def _solve_transposed(A, rhs):
    """A^T x = rhs with row equilibration of A^T and one step of iterative refinement.

    The rows of the step Jacobian span ~10 orders of magnitude (pressure rows ~
    k h, solid rows ~ k mu_s); equilibrating A^T's rows keeps SuperLU's
    pivoting meaningful for the transposed system.
    """
    At = A.T.tocsr()
    c = 1.0 / abs(At).max(axis=1).toarray().ravel()
    import scipy.sparse as sp
    M = (sp.diags(c) @ At).tocsc()
    lu = spla.splu(M)
    x = lu.solve(c * rhs)
    x = x + lu.solve(c * (rhs - At @ x))
    return x


def _solve(A, rhs):
    """A x = rhs with row equilibration and one step of iterative refinement."""
    A = A.tocsr()
    c = 1.0 / abs(A).max(axis=1).toarray().ravel()
    import scipy.sparse as sp
    lu = spla.splu((sp.diags(c) @ A).tocsc())
    x = lu.solve(c * rhs)
    x = x + lu.solve(c * (rhs - A @ x))
    return x


def tangent_gradient(disc, p, U0, N=None, m=None):
    """Forward (tangent-linear) sensitivities dJ/dq, one linearised sweep per parameter."""
    states, times, k = trajectory(disc, p, U0, N, m)
    grad = np.zeros(len(PARAMS))
    for i, q in enumerate(PARAMS):
        dU = np.zeros(states[0].size)
        acc = 0.0
        for n in range(1, len(states)):
            U, Uo, t = states[n], states[n - 1], times[n]
            rhs = -param_derivative(disc, U, Uo, t, k, q).ravel() - disc.jacobian_old(U, Uo, t, k) @ dU
            dU = _solve(disc.jacobian(U, Uo, t, k), rhs)
            acc += k * (drag_gradient(disc, U).ravel() @ dU)
        grad[i] = acc
    return grad


def complex_step_gradient(disc, p, U0, N=None, m=None, h=1e-30):
    """dJ/dq by complex step through the whole forward Newton solve."""
    grad = np.zeros(len(PARAMS))
    for i, q in enumerate(PARAMS):
        params = {q: disc.p[q] + 1j * h}
        states, times, k = trajectory(disc, p, U0.astype(np.complex128), N, m, params=params)
        grad[i] = functional(disc, states, k, params).imag / h
    return grad
