"""Seeded synthetic workloads for the ALE-FSI fine propagator.

This module holds *inputs only*: geometry breakpoints, physical constants,
time-grid choices and seeded random draws.  It contains none of the
method's arithmetic (no basis functions, no residual, no solver), so both
the CPU oracle and the GPU path may take their inputs from here without
sharing any code of the method.

The workloads stand in for the paper's 2d/3d wall-mounted elastic obstacle
problems (Section 4, Figure "geometry", Table "parameters"), whose geometry
figure is not available: a channel with an elastic bar standing on the
bottom wall, parabolic inflow, equal fluid/solid densities 1e3 and Poisson
ratio 0.4 as in Table "parameters".
"""
from __future__ import annotations

import copy
import math

import numpy as np

# ---------------------------------------------------------------------------
# Level-0 tensor meshes.  Each axis is a list of (lo, hi, cells) segments; a
# level-l mesh refines every level-0 cell 2**l times per axis.  The bar faces
# lie on segment ends, so the fluid-solid interface is resolved by the mesh on
# every level (Section 2.2 requires an interface-fitted mesh).
# ---------------------------------------------------------------------------
SEGMENTS_2D = (
    ((0.0, 0.4, 3), (0.4, 0.5, 1), (0.5, 2.0, 12)),
    ((0.0, 0.25, 2), (0.25, 0.5, 2)),
)
SEGMENTS_3D = (
    ((0.0, 0.4, 3), (0.4, 0.5, 1), (0.5, 2.0, 12)),
    ((0.0, 0.2, 2), (0.2, 0.4, 2)),
    ((0.0, 0.1, 1), (0.1, 0.3, 2), (0.3, 0.4, 1)),
)


def lame_lambda(mu_s: float, nu_s: float) -> float:
    """Lame's first parameter from shear modulus and Poisson ratio (plane strain)."""
    return 2.0 * mu_s * nu_s / (1.0 - 2.0 * nu_s)


def base_params(dim: int = 2) -> dict:
    """Physical and discretisation parameters common to the 2d workloads."""
    if dim == 2:
        p = dict(dim=2, segments=SEGMENTS_2D,
                 domain_hi=(2.0, 0.5, 0.0),
                 solid_lo=(0.4, 0.0, 0.0), solid_hi=(0.5, 0.25, 0.0),
                 mu_s=5e5)
    else:
        p = dict(dim=3, segments=SEGMENTS_3D,
                 domain_hi=(2.0, 0.4, 0.4),
                 solid_lo=(0.4, 0.0, 0.1), solid_hi=(0.5, 0.2, 0.3),
                 mu_s=1e6)
    p.update(rho_f=1e3, nu_f=1e-3, rho_s=1e3, nu_s=0.4,
             inflow_peak=0.3, ramp_time=0.1,
             theta0=1.0, lps_alpha0=0.1)
    p["lambda_s"] = lame_lambda(p["mu_s"], p["nu_s"])
    return p


def time_grid(slice_len: float, dt_req: float) -> tuple[int, float]:
    """Number of uniform steps covering one slice with step <= dt_req.

    Section 3 asks for T/L = m k = M K; requested steps that do not divide the
    slice are rounded down to the next step that does.
    """
    m = int(math.ceil(slice_len / dt_req - 1e-12))
    return m, slice_len / m


# Workloads: name -> dict.  level is the refinement level of the level-0 mesh.
_WORKLOADS = {
    # 2d, 32x8 cells, FP64, 8 slices on [0,1]
    "c1": dict(dim=2, level=1, T=1.0, N=8, dt_fine=0.01, dt_coarse=0.1,
               precision="fp64", parareal_tol=1e-8, mu_s=5e5),
    # 2d, 128x32 cells, FP64, 32 slices on [0,2], stiffer bar
    "c2": dict(dim=2, level=3, T=2.0, N=32, dt_fine=0.002, dt_coarse=0.02,
               precision="fp64", parareal_tol=1e-8, mu_s=2e6),
    # 2d, 256x64 cells, mixed precision, 64 slices on [0,2]
    "c3": dict(dim=2, level=4, T=2.0, N=64, dt_fine=0.001, dt_coarse=0.01,
               precision="mixed", parareal_tol=1e-8, mu_s=5e5),
    # 2d adjoint workload, 128x32 cells, 32 slices on [0,1]
    "c4": dict(dim=2, level=3, T=1.0, N=32, dt_fine=0.002, dt_coarse=0.02,
               precision="fp64", parareal_tol=1e-8, mu_s=5e5),
    # Q2 cells (the paper's element) on the nodes of c1 and of c2: 16x4 and 64x16 cells
    "c1q2": dict(dim=2, level=0, degree=2, T=1.0, N=8, dt_fine=0.01, dt_coarse=0.1,
                 precision="fp64", parareal_tol=1e-8, mu_s=5e5),
    "c2q2": dict(dim=2, level=2, degree=2, T=2.0, N=32, dt_fine=0.002, dt_coarse=0.02,
                 precision="fp64", parareal_tol=1e-8, mu_s=2e6),
    # Q2 cells on the nodes of c3 (128x32 cells), mixed precision
    "c3q2": dict(dim=2, level=3, degree=2, T=2.0, N=64, dt_fine=0.001, dt_coarse=0.01,
                 precision="mixed", parareal_tol=1e-8, mu_s=5e5),
    # 3d, 64x16x16 hexahedra, 16 slices on [0,0.8]
    "c5": dict(dim=3, level=2, T=0.8, N=16, dt_fine=0.005, dt_coarse=0.05,
               precision="mixed", parareal_tol=1e-8, mu_s=1e6),
}


def workload(name: str, seed: int = 0, **overrides) -> dict:
    """Return the full parameter dict of a named workload for one seed.

    The seed perturbs the inflow peak: c1, c2, c4 (and c1q2, c2q2) draw peak = 0.3 (1 + u),
    u ~ U(-0.05, 0.05); c3 (and c3q2) draws peak ~ U(0.2, 1.0); c5 keeps 0.3.
    """
    w = copy.deepcopy(_WORKLOADS[name])
    p = base_params(w["dim"])
    p.update(w)
    p["lambda_s"] = lame_lambda(p["mu_s"], p["nu_s"])
    rng = np.random.default_rng(seed)
    if name in ("c1", "c2", "c4", "c1q2", "c2q2"):
        p["inflow_peak"] = 0.3 * (1.0 + rng.uniform(-0.05, 0.05))
    elif name in ("c3", "c3q2"):
        p["inflow_peak"] = float(rng.uniform(0.2, 1.0))
    p.update(overrides)
    p["name"] = name
    p["seed"] = seed
    slice_len = p["T"] / p["N"]
    p["slice_len"] = slice_len
    p["m"], p["k_fine"] = time_grid(slice_len, p["dt_fine"])
    p["M"], p["k_coarse"] = time_grid(slice_len, p["dt_coarse"])
    return p


def mesh_shape(p: dict) -> tuple[int, ...]:
    """Cells per axis of the level-l mesh (pure bookkeeping on the segments)."""
    return tuple(sum(s[2] for s in ax) * 2 ** p["level"] for ax in p["segments"])


def node_level(p: dict) -> int:
    """Refinement level of the node grid: the cells' level for Q1, one more for Q2
    (a Q2 cell carries the 3^d nodes of 2^d cells of the next level)."""
    return p["level"] + (p.get("degree", 1) - 1)


def n_nodes(p: dict) -> int:
    return int(np.prod([sum(s[2] for s in ax) * 2 ** node_level(p) + 1 for ax in p["segments"]]))


def n_comp(p: dict) -> int:
    """Unknowns per node: velocity (d), displacement (d), pressure."""
    return 2 * p["dim"] + 1


def random_state(p: dict, seed: int, grad_u_max: float = 0.1) -> np.ndarray:
    """A random admissible nodal state [nodes, comp] (float64).

    v ~ peak * U(-1, 1), p ~ N(0, 10^2) and u a smooth random field (a few
    low Fourier modes) scaled so that the largest nodal difference quotient of
    u stays below grad_u_max, which keeps det(I + grad u) > 0.
    """
    from numpy import pi
    rng = np.random.default_rng(seed)
    d = p["dim"]
    lv = node_level(p)
    shape = tuple(sum(s[2] for s in ax) * 2 ** lv for ax in p["segments"])
    axes = []
    for ax in p["segments"][:d]:
        pts = []
        for (lo, hi, n) in ax:
            nl = n * 2 ** lv
            pts.extend(lo + (hi - lo) * np.arange(nl) / nl)
        pts.append(ax[-1][1])
        axes.append(np.asarray(pts))
    grids = np.meshgrid(*axes, indexing="ij")
    # node index i + (nx+1) j (+ ...): x fastest -> Fortran-order flatten
    X = [g.ravel(order="F") for g in grids]
    nn = X[0].size
    c = 2 * d + 1
    U = np.zeros((nn, c))
    U[:, :d] = p["inflow_peak"] * rng.uniform(-1.0, 1.0, size=(nn, d))
    L = [ax[-1][1] for ax in p["segments"][:d]]
    u = np.zeros((nn, d))
    for comp in range(d):
        for _ in range(3):
            kv = rng.integers(1, 4, size=d)
            ph = rng.uniform(0, 2 * pi, size=d)
            amp = rng.normal()
            f = np.ones(nn)
            for a in range(d):
                f = f * np.sin(kv[a] * pi * X[a] / L[a] + ph[a])
            u[:, comp] += amp * f
    # scale by the largest nodal difference quotient
    h_min = min(np.min(np.diff(a)) for a in axes)
    gmax = 0.0
    strides = [1]
    for a in range(d - 1):
        strides.append(strides[-1] * (shape[a] + 1))
    for a in range(d):
        idx = np.arange(nn)
        ia = (idx // strides[a]) % (shape[a] + 1)
        ok = ia < shape[a]
        du = np.abs(u[idx[ok] + strides[a]] - u[idx[ok]])
        gmax = max(gmax, du.max() / h_min)
    u *= grad_u_max / max(gmax, 1e-300)
    U[:, d:2 * d] = u
    U[:, 2 * d] = rng.normal(0.0, 10.0, size=nn)
    return U


def smooth_state(p: dict, seed: int, v_scale: float = 0.5, grad_u_max: float = 0.02) -> np.ndarray:
    """A smooth random nodal state [nodes, comp] (float64) for whole propagator
    steps at full size: velocity and displacement are smooth random fields (the
    low Fourier modes of random_state), |v| up to v_scale * peak, the largest
    nodal difference quotient of u below grad_u_max, pressure zero (it only
    seeds Newton).  Dirichlet data is not applied here.
    """
    d = p["dim"]
    a = random_state(p, seed, grad_u_max=grad_u_max)
    b = random_state(p, seed + 100000, grad_u_max=1.0)
    U = np.zeros_like(a)
    U[:, d:2 * d] = a[:, d:2 * d]
    vb = b[:, d:2 * d]
    U[:, :d] = vb * (v_scale * p["inflow_peak"] / max(np.abs(vb).max(), 1e-300))
    return U

