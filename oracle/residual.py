"""One shifted Crank-Nicolson step of the monolithic ALE-FSI system.

The unknown of a step t_{n-1} -> t_n is the nodal vector U = (v, u, p)
(2d+1 values per node, order v_1..v_d, u_1..u_d, p); the old state is
Uo = (v°, u°, .).  Notation (Section 2.3): k step size, theta = 1/2 +
theta0 k, F = I + grad u, J = det F, the same with ° for the old state, and
the mean values F̄ = I + (grad u + grad u°)/2, J̄ = (J + J°)/2,
grad v̄ = (grad v + grad v°)/2 on the step.  (grad v)_{ij} = d_j v_i.

Residual rows, each integrated with the 2-point Gauss rule per direction for
Q1 cells and the 3-point rule for Q2 cells (Section 2.3 time-step equation
with the forms of eq. (semiforms)):

  momentum, fluid cells   rho_f J̄ ((v - v°) - grad v̄ F̄^{-1} (u - u°)) . phi
                          + k theta     [rho_f J  (grad v  F^{-1}  v ) . phi + J  sigma(v , p; F ) F^{-T}  : grad phi]
                          + k (1-theta) [rho_f J° (grad v° F°^{-1} v°) . phi + J° sigma(v°, p; F°) F°^{-T} : grad phi]
                          with sigma(v, p; F) = rho_f nu_f (grad v F^{-1} + F^{-T} grad v^T) - p I
                          (eq. (ALE:stress)); the pressure is the new one in
                          both parts, as the time-step equation writes it.
  momentum, outflow face  - k theta rho_f nu_f J (F^{-T} grad v^T F^{-T} n) . phi
                          - k (1-theta) (same with °)     (do-nothing correction, eq. (variational))
  momentum, solid cells   rho_s (v - v°) . phi + k theta F Sigma(u) : grad phi
                          + k (1-theta) F° Sigma(u°) : grad phi,
                          Sigma = 2 mu_s E + lambda_s tr(E) I, E = (F^T F - I)/2 (eq. (stress))
  pressure, fluid cells   k J tr(grad v F^{-1}) xi  (+ k s_h(p, xi), see lps.py)
  displacement, nodes of solid cells (interface included), solid cells only:
                          ((u - u°) - k (theta v + (1-theta) v°)) . psi
  displacement, other nodes, fluid cells only:
                          k (theta grad u + (1-theta) grad u°) : grad psi   (harmonic extension)
  Dirichlet data          v = inflow profile at x = 0, v = 0 on the walls,
                          u = 0 on the whole outer boundary; the row becomes
                          U_i - g_i(t_n).
  pressure at nodes that touch no fluid cell: p_i = 0.

Readings of the paper taken here (the paper is silent or garbled):
  * the second kinematic term of the time-step equation is read with the old
    velocity, k (1-theta) (v_{n-1}, psi_s);
  * "J_{n-1/2}", "F_{n-1/2}" are means of J and of F over the step;
  * pressure in strictly solid nodes is fixed to zero (p enters no solid
    equation);
  * the kinematic rows own the interface nodes (psi_f vanishes on the
    interface, eq. (test)).

All routines are plain NumPy and accept complex states, so that the
complex-step derivative gives the exact Jacobian.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fe import gauss_rule, q1_basis, q2_basis
from .mesh import Mesh
from . import lps as _lps


def det_inv(F):
    """Determinant and inverse of stacked 2x2 / 3x3 matrices (cofactor formulas)."""
    d = F.shape[-1]
    if d == 2:
        a, b, c, e = F[..., 0, 0], F[..., 0, 1], F[..., 1, 0], F[..., 1, 1]
        J = a * e - b * c
        inv = np.empty_like(F)
        inv[..., 0, 0] = e / J
        inv[..., 0, 1] = -b / J
        inv[..., 1, 0] = -c / J
        inv[..., 1, 1] = a / J
        return J, inv
    cof = np.empty_like(F)
    for i in range(3):
        for j in range(3):
            i1, i2 = (i + 1) % 3, (i + 2) % 3
            j1, j2 = (j + 1) % 3, (j + 2) % 3
            cof[..., i, j] = F[..., i1, j1] * F[..., i2, j2] - F[..., i1, j2] * F[..., i2, j1]
    J = np.einsum("...j,...j->...", F[..., 0, :], cof[..., 0, :])
    inv = np.swapaxes(cof, -1, -2) / J[..., None, None]
    return J, inv


def ramp(t: float, ramp_time: float) -> float:
    """Inflow ramp s(t) = (1 - cos(pi t / t_r)) / 2 for t < t_r, then 1.

    Same shape as the paper's s(t) (Section 4), switched on once.
    """
    if t >= ramp_time:
        return 1.0
    return 0.5 * (1.0 - np.cos(np.pi * t / ramp_time))


class Discretization:
    """Mesh, quadrature, masks and the constant stabilisation of one level.

    degree (default p.get("degree", 1)): 1 for Q1 cells (2-point Gauss rule), 2 for
    the Q2 cells of Section 2.2 (3-point rule, exact for the products of Q2 functions
    and their gradients on the affine cells), 2d."""

    def __init__(self, p: dict, level: int | None = None, degree: int | None = None):
        self.p = p
        self.degree = deg = p.get("degree", 1) if degree is None else degree
        if deg not in (1, 2) or (deg == 2 and p["dim"] != 2):
            raise ValueError("degree 1 (2d, 3d) or 2 (2d)")
        self.mesh = m = Mesh(p, level, deg)
        self.dim = d = m.dim
        self.nc = 2 * d + 1
        self.nloc = m.nloc
        npts = deg + 1
        basis = q1_basis if deg == 1 else q2_basis
        xq, wq = gauss_rule(d, npts)
        self.Nq, self.dNq = basis(d, xq)                      # [nq, a], [nq, a, r]
        self.wq = wq
        # physical gradients and weights per cell: G [cells, nq, a, r], W [cells, nq]
        self.G = self.dNq[None, :, :, :] / m.h[:, None, None, :]
        self.W = np.prod(m.h, axis=1)[:, None] * wq[None, :]
        # outflow face quadrature: reference points (1, eta[, zeta])
        xf, wf = gauss_rule(d - 1, npts)
        xf_full = np.concatenate([np.ones((xf.shape[0], 1)), xf], axis=1)
        self.Nf, dNf = basis(d, xf_full)
        oc = m.outflow_cells
        self.Gf = dNf[None, :, :, :] / m.h[oc][:, None, None, :]
        self.Wf = np.prod(m.h[oc][:, 1:], axis=1)[:, None] * wf[None, :]
        # row masks for displacement rows inside fluid cells (nodes not in N_S)
        self.fluid_urow = ~m.in_NS[m.conn]                    # [cells, a]
        # Dirichlet masks [nodes, comp]
        D = np.zeros((m.n_nodes, self.nc), dtype=bool)
        D[:, :d] = (m.on_inflow | m.on_wall)[:, None]
        D[:, d:2 * d] = (m.on_inflow | m.on_outflow | m.on_wall)[:, None]
        D[:, 2 * d] = ~m.in_NF
        self.dirichlet = D
        # scatter matrix: element-local rows -> global rows
        ne = m.n_cells * self.nloc * self.nc
        rows = (m.conn[:, :, None] * self.nc + np.arange(self.nc)[None, None, :]).ravel()
        self.scatter = sp.csr_matrix((np.ones(ne), (rows, np.arange(ne))),
                                     shape=(m.n_nodes * self.nc, ne))
        if deg == 2:
            self.S = _lps.lps_matrix_q2(self)
        else:
            self.S = _lps.lps_matrix(self) if m.level >= 1 else None

    def theta(self, k):
        """theta = 1/2 + theta0 k (Section 2.3); a fixed theta may be forced.

        With theta_ref_k = k_r > 0: the damping theta = 1/2 + alpha(k) k that the
        paper proposes (Section 4, fsi-3 discussion) so that large and small
        steps dissipate alike.  For y' = i w y the theta-scheme damps by
        ln|R| = -(theta - 1/2) w^2 k^2 + O((w k)^4) per step, i.e. by
        alpha(k) w^2 k^2 per unit time; equal damping per unit time for steps
        k and k_r gives alpha(k) = theta0 (k_r / k)^2, so steps of size k_r keep
        theta = 1/2 + theta0 k_r.
        """
        if self.p.get("theta_fixed") is not None:
            return self.p["theta_fixed"]
        kr = self.p.get("theta_ref_k") or 0.0
        if kr > 0.0:
            return 0.5 + self.p["theta0"] * kr * kr / k
        return 0.5 + self.p["theta0"] * k

    # ------------------------------------------------------------------ data
    def dirichlet_values(self, t: float, peak=None) -> np.ndarray:
        """g(t) on every Dirichlet dof (zero elsewhere), [nodes, comp]."""
        m, p, d = self.mesh, self.p, self.dim
        peak = p["inflow_peak"] if peak is None else peak
        g = np.zeros((m.n_nodes, self.nc), dtype=np.result_type(peak, np.float64))
        s = ramp(t, p["ramp_time"])
        X = m.X
        prof = np.ones(m.n_nodes)
        for q in range(1, d):
            H = m.L[q]
            prof = prof * 4.0 * X[:, q] * (H - X[:, q]) / H ** 2
        inflow_only = m.on_inflow & ~m.on_wall
        g[inflow_only, 0] = s * peak * prof[inflow_only]
        return g

    def apply_dirichlet(self, U: np.ndarray, t: float, peak=None) -> np.ndarray:
        g = self.dirichlet_values(t, peak=peak)
        U = U.astype(np.result_type(U, g))
        U[self.dirichlet] = g[self.dirichlet]
        return U

    # ----------------------------------------------------------- element form
    def element_residual(self, Ue, Uoe, k, theta, params=None):
        """Element residual vectors [cells, a, comp] (Dirichlet rows not yet replaced).

        Ue, Uoe: cell-local new/old states [cells, a, comp] (real or complex).
        params: optional dict overriding mu_s, lambda_s (complex allowed).
        """
        p = dict(self.p)
        if params:
            p.update(params)
        d, m = self.dim, self.mesh
        rf, nuf, rs = p["rho_f"], p["nu_f"], p["rho_s"]
        mu, lam = p["mu_s"], p["lambda_s"]
        dtype = np.result_type(Ue, Uoe, np.asarray(mu), np.asarray(lam))
        Re = np.zeros(Ue.shape, dtype=dtype)
        I = np.eye(d)
        N, G, W = self.Nq, self.G, self.W

        def fields(Uc, Nv, Gv):
            v = np.einsum("qa,caj->cqj", Nv, Uc[:, :, :d])
            gv = np.einsum("cqar,cai->cqir", Gv, Uc[:, :, :d])
            u = np.einsum("qa,caj->cqj", Nv, Uc[:, :, d:2 * d])
            gu = np.einsum("cqar,cai->cqir", Gv, Uc[:, :, d:2 * d])
            pr = np.einsum("qa,ca->cq", Nv, Uc[:, :, 2 * d])
            return v, gv, u, gu, pr

        v, gv, u, gu, pr = fields(Ue, N, G)
        vo, gvo, uo, guo, _ = fields(Uoe, N, G)
        F = I + gu
        Fo = I + guo
        J, Fi = det_inv(F)
        Jo, Foi = det_inv(Fo)

        fl = m.fluid
        sl = m.solid
        # ---------------- fluid cells
        if fl.any():
            Fb = I + 0.5 * (gu + guo)
            Jb = 0.5 * (J + Jo)
            _, Fbi = det_inv(Fb)
            gvb = 0.5 * (gv + gvo)
            du = u - uo
            w_ale = np.einsum("cqij,cqjk,cqk->cqi", gvb, Fbi, du)
            mvec = rf * Jb[..., None] * ((v - vo) - w_ale)
            conv = np.einsum("cqij,cqjk,cqk->cqi", gv, Fi, v)
            convo = np.einsum("cqij,cqjk,cqk->cqi", gvo, Foi, vo)
            mvec = mvec + k * theta * rf * J[..., None] * conv \
                + k * (1 - theta) * rf * Jo[..., None] * convo

            def piola(gvx, Fix, Jx):
                A = np.einsum("cqij,cqjk->cqik", gvx, Fix)
                sig = rf * nuf * (A + np.swapaxes(A, -1, -2)) - pr[..., None, None] * I
                return Jx[..., None, None] * np.einsum("cqij,cqkj->cqik", sig, Fix)

            P = k * theta * piola(gv, Fi, J) + k * (1 - theta) * piola(gvo, Foi, Jo)
            div = k * J * np.einsum("cqij,cqji->cq", gv, Fi)
            ug = k * (theta * gu + (1 - theta) * guo)

            Wf = W[fl]
            Nv = N[None]
            Re[fl, :, :d] += np.einsum("cq,qa,cqi->cai", Wf, N, mvec[fl]) \
                + np.einsum("cq,cqir,cqar->cai", Wf, P[fl], G[fl])
            Re[fl, :, 2 * d] += np.einsum("cq,qa,cq->ca", Wf, N, div[fl])
            urow = np.einsum("cq,cqir,cqar->cai", Wf, ug[fl], G[fl])
            Re[fl, :, d:2 * d] += urow * self.fluid_urow[fl][:, :, None]
            del Nv

        # ---------------- solid cells
        if sl.any():
            def first_piola(Fx):
                E = 0.5 * (np.einsum("cqji,cqjk->cqik", Fx, Fx) - I)
                trE = np.einsum("cqii->cq", E)
                Sig = 2.0 * mu * E + lam * trE[..., None, None] * I
                return np.einsum("cqij,cqjk->cqik", Fx, Sig)

            Ps = k * theta * first_piola(F[sl]) + k * (1 - theta) * first_piola(Fo[sl])
            Ws = W[sl]
            Re[sl, :, :d] += np.einsum("cq,qa,cqi->cai", Ws, N, rs * (v[sl] - vo[sl])) \
                + np.einsum("cq,cqir,cqar->cai", Ws, Ps, G[sl])
            kin = (u[sl] - uo[sl]) - k * (theta * v[sl] + (1 - theta) * vo[sl])
            Re[sl, :, d:2 * d] += np.einsum("cq,qa,cqi->cai", Ws, N, kin)

        # ---------------- outflow faces (x = L, outward normal e_x)
        oc = m.outflow_cells
        if oc.size:
            Uf, Uof = Ue[oc], Uoe[oc]
            _, gvf, _, guf, _ = fields(Uf, self.Nf, self.Gf)
            _, gvof, _, guof, _ = fields(Uof, self.Nf, self.Gf)
            Jf, Fif = det_inv(I + guf)
            Jof, Foif = det_inv(I + guof)
            n = np.zeros(d)
            n[0] = 1.0

            def corr(gvx, Fix, Jx):
                FiT = np.swapaxes(Fix, -1, -2)
                gvT = np.swapaxes(gvx, -1, -2)
                t1 = np.einsum("cqij,j->cqi", FiT, n)
                t2 = np.einsum("cqij,cqj->cqi", gvT, t1)
                t3 = np.einsum("cqij,cqj->cqi", FiT, t2)
                return rf * nuf * Jx[..., None] * t3

            bvec = k * theta * corr(gvf, Fif, Jf) + k * (1 - theta) * corr(gvof, Foif, Jof)
            Re[oc, :, :d] -= np.einsum("cq,qa,cqi->cai", self.Wf, self.Nf, bvec)
        return Re

    # -------------------------------------------------------------- assembly
    def gather(self, U):
        return U[self.mesh.conn]

    def residual(self, U, Uo, t, k, theta=None, params=None, with_dirichlet=True):
        """Global residual [nodes, comp] of one step t-k -> t at new state U."""
        if theta is None:
            theta = self.theta(k)
        Re = self.element_residual(self.gather(U), self.gather(Uo), k, theta, params)
        R = (self.scatter @ Re.reshape(-1)).reshape(U.shape[0], self.nc)
        if self.S is not None:
            R[:, 2 * self.dim] += k * (self.S @ U[:, 2 * self.dim])
        if with_dirichlet:
            g = self.dirichlet_values(t, peak=(params or {}).get("inflow_peak"))
            D = self.dirichlet
            if np.iscomplexobj(g) and not np.iscomplexobj(R):
                R = R.astype(np.complex128)
            R[D] = U[D] - g[D]
        return R

    def element_jacobian(self, U, Uo, k, theta, wrt="new", h=1e-30):
        """Element matrices d Re / d U_local [cells, a, comp, b, comp'] by complex step."""
        Ue = self.gather(U).astype(np.complex128)
        Uoe = self.gather(Uo).astype(np.complex128)
        nl, nc = self.nloc, self.nc
        Ke = np.zeros((Ue.shape[0], nl, nc, nl, nc))
        for b in range(nl):
            for c in range(nc):
                if wrt == "new":
                    Up = Ue.copy()
                    Up[:, b, c] += 1j * h
                    Re = self.element_residual(Up, Uoe, k, theta)
                else:
                    Up = Uoe.copy()
                    Up[:, b, c] += 1j * h
                    Re = self.element_residual(Ue, Up, k, theta)
                Ke[:, :, :, b, c] = Re.imag / h
        return Ke

    def assemble(self, Ke):
        m, nc, nl = self.mesh, self.nc, self.nloc
        gi = m.conn[:, :, None] * nc + np.arange(nc)[None, None, :]     # [cells, a, comp]
        rows = np.broadcast_to(gi[:, :, :, None, None], Ke.shape).ravel()
        cols = np.broadcast_to(gi[:, None, None, :, :], Ke.shape).ravel()
        n = m.n_nodes * nc
        return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))

    def jacobian(self, U, Uo, t, k, theta=None):
        """Exact d R / d U (CSR), Dirichlet rows replaced by identity rows."""
        if theta is None:
            theta = self.theta(k)
        A = self.assemble(self.element_jacobian(U, Uo, k, theta, "new"))
        if self.S is not None:
            A = A + k * self.p_block(self.S)
        return self.replace_dirichlet_rows(A, identity=True)

    def jacobian_old(self, U, Uo, t, k, theta=None):
        """d R / d Uo (CSR); Dirichlet rows are zero (they do not depend on Uo)."""
        if theta is None:
            theta = self.theta(k)
        A = self.assemble(self.element_jacobian(U, Uo, k, theta, "old"))
        return self.replace_dirichlet_rows(A, identity=False)

    def p_block(self, S):
        """Embed a pressure-pressure operator into the full dof space."""
        nn, nc, d = self.mesh.n_nodes, self.nc, self.dim
        E = sp.csr_matrix((np.ones(nn), (np.arange(nn) * nc + 2 * d, np.arange(nn))),
                          shape=(nn * nc, nn))
        return E @ S @ E.T

    def replace_dirichlet_rows(self, A, identity=True):
        D = self.dirichlet.ravel()
        keep = sp.diags((~D).astype(np.float64))
        A = keep @ A
        if identity:
            A = A + sp.diags(D.astype(np.float64))
        return A.tocsr()
