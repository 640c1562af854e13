"""Newton's method per time step, the propagators and the Parareal iteration.

Section 3: the interval is split into L slices of length T/L = m k = M K;
the fine propagator takes m steps of size k, the coarse one M steps of size
K, both with the same shifted Crank-Nicolson scheme (theta = 1/2 + theta0 *
step).  Each step is solved by Newton's method (Section 4.1 names Newton as
the nonlinear solver; its settings are not given).  Newton here uses the
exact Jacobian and a direct sparse LU (SuperLU), full steps, and stops once
the update just applied is below rtol times the field's size for every
field (v, u, p).  With quadratic convergence the error left after that
update is at round-off level; rtol = 1e-10 sits above the round-off floor of
the update (about 1e-11 relative when the pressure is large against the
velocity, as in the first steps of the inflow ramp).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .residual import Discretization


class NewtonFailure(RuntimeError):
    pass


def field_slices(dim):
    return {"v": slice(0, dim), "u": slice(dim, 2 * dim), "p": slice(2 * dim, 2 * dim + 1)}


def newton_step(disc: Discretization, Uo, t_new, k, rtol=1e-10, maxit=30, theta=None,
                params=None, stats=None):
    """Solve R(U; Uo) = 0 for the state at t_new = t_old + k.

    The initial guess is the old state with the Dirichlet data of t_new
    imposed.  Accepts complex Uo / params (complex-step sensitivities): the
    Jacobian is then evaluated at the real part and the iteration runs until
    both real and imaginary parts of the update have converged.
    """
    U = disc.apply_dirichlet(Uo, t_new, peak=(params or {}).get("inflow_peak"))
    if params and any(np.iscomplexobj(v) for v in params.values()):
        U = U.astype(np.complex128)
    fs = field_slices(disc.dim)
    prev = None
    for it in range(1, maxit + 1):
        R = disc.residual(U, Uo, t_new, k, theta=theta, params=params)
        A = disc.jacobian(U.real, Uo.real, t_new, k, theta=theta) if params is None \
            else _jac_params(disc, U.real, Uo.real, t_new, k, theta, params)
        lu = spla.splu(A.tocsc())
        if np.iscomplexobj(R):
            dU = -(lu.solve(np.ascontiguousarray(R.real.ravel()))
                   + 1j * lu.solve(np.ascontiguousarray(R.imag.ravel())))
        else:
            dU = -lu.solve(R.ravel())
        dU = dU.reshape(U.shape)
        U = U + dU
        if not np.all(np.isfinite(U)):
            raise NewtonFailure("non-finite Newton iterate")
        # relative size of the update per field (and per real/imaginary part)
        rel = []
        for sl in fs.values():
            for part in ((np.real,) if not np.iscomplexobj(U) else (np.real, np.imag)):
                du = np.abs(part(dU[:, sl])).max()
                un = np.abs(part(U[:, sl])).max()
                rel.append(du / un if un > 0 else du)
        worst = max(rel)
        # converged, or stagnating at the round-off floor after reaching the
        # quadratic regime (the update no longer shrinks tenfold)
        if worst <= rtol or (prev is not None and worst <= 1e-6 and worst > 0.1 * prev):
            if stats is not None:
                stats.append(it)
            return U
        prev = worst
    raise NewtonFailure(f"Newton did not converge in {maxit} iterations at t={t_new}")


def _jac_params(disc, U, Uo, t, k, theta, params):
    real = {kk: np.real(v) for kk, v in params.items()}
    saved = dict(disc.p)
    disc.p.update(real)
    try:
        return disc.jacobian(U, Uo, t, k, theta=theta)
    finally:
        disc.p.clear()
        disc.p.update(saved)


def propagate(disc, U_in, t0, slice_len, nsteps, rtol=1e-10, params=None, trajectory=None,
              stats=None):
    """Take nsteps uniform steps of size slice_len / nsteps from t0 (Section 3)."""
    k = slice_len / nsteps
    U = np.array(U_in)
    for n in range(1, nsteps + 1):
        t = t0 + n * k
        U = newton_step(disc, U, t, k, rtol=rtol, params=params, stats=stats)
        if trajectory is not None:
            trajectory.append(U)
    return U


def fine_propagate(disc, p, U_in, t0, **kw):
    return propagate(disc, U_in, t0, p["slice_len"], p["m"], **kw)


def coarse_propagate(disc, p, U_in, t0, **kw):
    return propagate(disc, U_in, t0, p["slice_len"], p["M"], **kw)


def sequential(disc, p, U0, n_slices=None, rtol=1e-10):
    """Slice-boundary states of the sequential fine solution, [N+1, nodes, comp]."""
    N = p["N"] if n_slices is None else n_slices
    out = [np.array(U0)]
    for l in range(N):
        out.append(fine_propagate(disc, p, out[-1], l * p["slice_len"], rtol=rtol))
    return np.stack(out)


def relative_change(Unew, Uold, dim):
    """max over slice boundaries l and fields v, u of ||Unew_l,f - Uold_l,f|| / ||Unew_l,f||."""
    r = 0.0
    for l in range(Unew.shape[0]):
        for key, sl in field_slices(dim).items():
            if key == "p":
                continue
            num = np.linalg.norm(Unew[l][:, sl] - Uold[l][:, sl])
            den = np.linalg.norm(Unew[l][:, sl])
            r = max(r, num / den if den > 0 else num)
    return r


def theta_weight(F, C, dim, mode):
    """Weight of the coarse terms in theta-Parareal (eq. (thetaparareal:iteration)).

    The paper fits theta so that theta C(U^{i+1}_l) matches F(U^i_l): the least
    squares value <F, C> / <C, C>, or the variant it uses, read here as the
    cosine <F, C> / (|F| |C|) (<= 1 by Cauchy-Schwarz, which is what the paper
    states for its choice; the printed denominator lacks the square roots).
    Both are computed per solution component (the 2d velocity and displacement
    components) and averaged; components with a zero norm are left out, and
    with none left theta = 1 (plain Parareal).
    """
    if mode in (None, "plain"):
        return 1.0
    vals = []
    for c in range(2 * dim):
        f, g = F[:, c], C[:, c]
        fg, gg, ff = float(f @ g), float(g @ g), float(f @ f)
        if mode == "lsq":
            if gg > 0.0:
                vals.append(fg / gg)
        elif mode == "cosine":
            if gg > 0.0 and ff > 0.0:
                vals.append(fg / np.sqrt(gg * ff))
        else:
            raise ValueError(mode)
    return float(np.mean(vals)) if vals else 1.0


def parareal(disc, p, U0, tol=None, max_iter=None, rtol=1e-10, history=None, theta=None, thetas=None):
    """Parareal predictor-corrector of eq. (parareal:iteration); with theta =
    "cosine" or "lsq" the weighted variant of eq. (thetaparareal:iteration),
    U^{i+1}_{l+1} = th C(U^{i+1}_l) + F(U^i_l) - th C(U^i_l), th from
    theta_weight(F(U^i_l), C(U^{i+1}_l)).

    U^0_0 = U0, U^0_{l+1} = C(U^0_l); iteration i computes F(U^i_l) for the
    slices l >= i (earlier slices are already exact), then sweeps
    l = 0..N-1: Cn = C(U^{i+1}_l), U^{i+1}_{l+1} = Cn + F_l - Cold_l,
    Cold_l = Cn.  The full vector (v, u, p) is updated; p only seeds Newton.
    Stops when the largest relative change of v and u over the slice
    boundaries is below tol, or after N iterations.  Returns the boundary
    states [N+1, nodes, comp] and the number of iterations.
    """
    N = p["N"]
    tol = p.get("parareal_tol", 1e-8) if tol is None else tol
    max_iter = N if max_iter is None else min(max_iter, N)
    dl = p["slice_len"]
    U = [np.array(U0)]
    Cold = []
    for l in range(N):
        c = coarse_propagate(disc, p, U[l], l * dl, rtol=rtol)
        Cold.append(c)
        U.append(c.copy())
    Fv = [None] * N
    it = 0
    for i in range(max_iter):
        for l in range(i, N):
            Fv[l] = fine_propagate(disc, p, U[l], l * dl, rtol=rtol)
        Unew = [U[0]]
        for l in range(N):
            if l < i:
                # slice l started from an exact state: its coarse value is unchanged
                cn = Cold[l]
                th = 1.0
            else:
                cn = coarse_propagate(disc, p, Unew[l], l * dl, rtol=rtol)
                th = theta_weight(Fv[l], cn, disc.dim, theta)
            if thetas is not None:
                thetas.append((i, l, th))
            Unew.append(th * cn + Fv[l] - th * Cold[l])
            Cold[l] = cn
        it = i + 1
        change = relative_change(np.stack(Unew), np.stack(U), disc.dim)
        if history is not None:
            history.append((np.stack(Unew), change))
        U = Unew
        if change < tol:
            break
    return np.stack(U), it


def speedup_model(r, K, N):
    """Theoretical Parareal speedup of eq. (eq:speedup): 1 / (r + K/N (1 + r))."""
    return 1.0 / (r + (K / N) * (1.0 + r))
