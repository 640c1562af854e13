"""ctypes binding of the C ABI in include/fsi.h (argument marshalling only).

Device arrays are torch tensors on a HIP device (float64, contiguous); their
data pointers and torch's current stream are passed to the library.  Every
numerical step runs in the HIP library; if libfsi.so is missing the import of
this module's loader raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsi.so")

FSI_OK, FSI_ERR_ARG, FSI_ERR_HIP, FSI_ERR_OOM = 0, -1, -2, -3
FSI_ERR_NEWTON, FSI_ERR_LINEAR, FSI_ERR_NONFINITE, FSI_ERR_PARAREAL = -4, -5, -6, -7
FSI_FP64, FSI_MIXED = 0, 1
MAX_SLICES = 1024

# entry points declared in include/fsi.h
EXPORTS = ("fsi_setup", "fsi_sizes", "fsi_initial_state", "fine_propagate", "coarse_propagate",
           "parareal_run", "adjoint_gradient", "fsi_debug_residual", "fsi_debug_jacobian_apply", "fsi_debug_vcycle",
           "fsi_residual_noalloc",
           "fsi_profile_enable", "fsi_profile_query", "fsi_destroy", "fsi_status_string")


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("level", C.c_int32),
        ("nseg", C.c_int32 * 3), ("seg_pts", (C.c_double * 5) * 3), ("seg_cells", (C.c_int32 * 4) * 3),
        ("solid_lo", C.c_double * 3), ("solid_hi", C.c_double * 3),
        ("rho_f", C.c_double), ("nu_f", C.c_double), ("rho_s", C.c_double), ("mu_s", C.c_double),
        ("lambda_s", C.c_double), ("inflow_peak", C.c_double), ("ramp_time", C.c_double),
        ("theta0", C.c_double), ("lps_alpha0", C.c_double), ("cip_gamma", C.c_double),
        ("precision", C.c_int32), ("gmres_restart", C.c_int32), ("gmres_maxit", C.c_int32),
        ("newton_maxit", C.c_int32), ("vanka_sweeps", C.c_int32), ("vanka_omega", C.c_double),
        ("newton_rtol", C.c_double), ("lin_rtol", C.c_double), ("max_batch", C.c_int32),
        ("vanka_sweeps_coarse", C.c_int32), ("precond_lag", C.c_int32),
        ("lin_rtol_first", C.c_double), ("parareal_theta", C.c_int32), ("theta_ref_k", C.c_double),
        ("parareal_pipeline", C.c_int32), ("batch_split", C.c_int32), ("newton_res_rtol", C.c_double),
        ("spmv_slice_fast", C.c_int32), ("vanka_slice_fast", C.c_int32), ("vanka_wide_cells", C.c_int32),
        ("degree", C.c_int32), ("newton_res_accept", C.c_double), ("newton_guess", C.c_int32),
        ("precond_lps_scale", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("newton_its", C.c_int32 * MAX_SLICES), ("krylov_its", C.c_int32 * MAX_SLICES),
        ("slice_status", C.c_int32 * MAX_SLICES), ("stage_ms", C.c_double * 8),
        ("parareal_iters", C.c_int32), ("newton_total", C.c_int32), ("krylov_total", C.c_int32),
    ]


_lib = None


def load():
    """Load libfsi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1907_01252_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    dp = C.POINTER(C.c_double)
    lib.fsi_setup.argtypes = [C.POINTER(Params), C.POINTER(vp)]
    lib.fsi_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.fsi_initial_state.argtypes = [vp, vp, vp]
    for f in (lib.fine_propagate, lib.coarse_propagate):
        f.argtypes = [vp, i32, dp, dbl, i32, vp, vp, C.POINTER(Stats), vp]
    lib.parareal_run.argtypes = [vp, dbl, i32, i32, i32, dbl, i32, vp, vp, C.POINTER(Stats), vp]
    lib.adjoint_gradient.argtypes = [vp, dbl, i32, i32, vp, dp, dp, C.POINTER(Stats), vp]
    lib.fsi_debug_residual.argtypes = [vp, i32, vp, vp, dp, dbl, vp, vp]
    lib.fsi_residual_noalloc.argtypes = [vp, i32, vp, vp, dp, dbl, vp, vp]
    lib.fsi_debug_jacobian_apply.argtypes = [vp, i32, vp, vp, dp, dbl, vp, vp, vp]
    lib.fsi_debug_vcycle.argtypes = [vp, i32, vp, vp, dp, dbl, vp, vp, vp]
    lib.fsi_profile_enable.argtypes = [vp, i32]
    lib.fsi_profile_query.argtypes = [vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.fsi_destroy.argtypes = [vp]
    lib.fsi_destroy.restype = None
    lib.fsi_status_string.argtypes = [i32]
    lib.fsi_status_string.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("fsi_destroy", "fsi_status_string"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


class FsiError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {load().fsi_status_string(code).decode()} ({code})")
        self.code = code


def _check(code, where):
    if code != FSI_OK:
        raise FsiError(code, where)


# batch_split = 3: three concurrent slice groups, the default where the autotuned table
# (tuned.json, by problem size and hardware-queue count) has no entry; four groups need
# more hardware queues than the 4 a process gets by default (GPU_MAX_HW_QUEUES)
# lin_rtol: floor of the relative tolerance of every linear solve after a step's first (the
# forcing term min(1e-2, max(lin_rtol, 0.1 newton_rtol / update size))).  With the
# extrapolated guesses, solving each Newton correction to fewer digits is faster (more Newton
# iterations, fewer Krylov ones), but the steps' error against the oracle follows the last
# correction's accuracy (2d 32x8 cells, six steps: 3e-12 at 1e-6 and 1e-5, 5e-11 to
# 8e-11 at 1e-4, 1e-9 at 1e-3, whatever the residual test): FP64 1e-5 (128x32 cells 4%
# faster than 1e-6); mixed precision, whose tolerance is 1e-6, 1e-3 in 2d (256x64 cells 28%
# faster) and 1e-4 in 3d (64x16x16 cells 13% faster)
# precond_lps_scale = 2: with Q2 cells the Q1 preconditioner's stabilisation constant is
# doubled (Krylov iterations per sweep: 64x16 Q2 cells 77,364 -> 70,793, 128x32 mixed
# 145,728 -> 133,036; 8-9% faster; 2.5 within 1%, 4 and 0.5 slower)
# newton_guess = 3: Newton starts from the cubic extrapolation of the last four states
# (against the linear one: 2d mixed 256x64 cells 13% fewer Krylov iterations and 13% faster,
# 2d FP64 128x32 cells 6% faster; the 3d 64x16x16 sweep is equal within 0.6% for degrees
# 1-3 and keeps the linear guess)
# newton_res_accept = 1e-12: a step whose scaled FP64 residual is already at 1e-12 of the
# state at the top of a Newton iteration ends there (2d c2: 30% fewer Newton and 25% fewer
# Krylov iterations, 1.84e7 instead of 1.46e7 dof*steps/s; oracle parity still 1e-12)
SOLVER_DEFAULTS = dict(cip_gamma=1e-4, gmres_restart=30, gmres_maxit=300, newton_maxit=30,
                       vanka_sweeps=2, vanka_omega=0.9, newton_rtol=1e-10, lin_rtol=1e-5,
                       vanka_sweeps_coarse=1, precond_lag=1, lin_rtol_first=1e-3, parareal_theta=0,
                       theta_ref_k=0.0, parareal_pipeline=0, batch_split=3, newton_res_rtol=1e-10,
                       spmv_slice_fast=-1, vanka_slice_fast=-1, vanka_wide_cells=0, newton_res_accept=1e-12,
                       newton_guess=3, precond_lps_scale=2.0)
# 3d: the multiplicative 8-colour Vanka sweep is stable only with more damping
# (a sweep with omega 0.9 amplifies errors at the 64x16x16 level), and the
# level-0 gradient-jump penalty needs a larger weight for the coarse correction
# to contract; a Newton step ends early only at a residual 1e-13 of the state
# (at 1e-12 the FP64 32x8x8-cell steps kept 5e-11 of the oracle's, at 1e-13
# no faster in 3d)
SOLVER_DEFAULTS_3D = dict(vanka_omega=0.6, cip_gamma=3e-4, newton_res_accept=1e-13, newton_guess=1)
# Q2 cells: one smoothing sweep on the finest Q1 level of the preconditioner (the Q2 nodes), where
# Q1 takes two (64x16 Q2 cells 10% faster, 128x32 mixed 22%: more Krylov iterations, cheaper cycles)
SOLVER_DEFAULTS_Q2 = dict(vanka_sweeps=1)
# mixed precision (the FP32 inner solve; tolerance 1e-6 after the FP64 refinement), by dimension:
# the forcing floor, and with it a lighter V-cycle: one finest-level sweep (2d: two on the coarser
# levels; 3d with the damping of 0.6: omega 0.8 was 28% faster at 64x16x16 but gave a non-finite
# state at 32x8x8, and 0.9 diverged at 64x16x16).  2d 256x64 cells 3.59e7 -> 4.16e7 dof*steps/s,
# 3d 64x16x16 3.40e6 -> 3.78e6, Q2 128x32 cells 8% faster.
MIXED_DEFAULTS = {2: dict(lin_rtol=1e-3, vanka_sweeps=1, vanka_sweeps_coarse=2),
                  3: dict(lin_rtol=1e-4, vanka_sweeps=1)}


def tuned_choice(dim, level, precision, max_batch):
    """Launch choices the autotuner stored for this problem size (autotune.py) and this process's
    hardware queue count, else those of the default count (4), else {}."""
    from . import autotune
    table = autotune.load_table()
    e = table.get(autotune.table_key(dim, level, precision, max_batch, autotune.hw_queues())) or \
        table.get(autotune.table_key(dim, level, precision, max_batch))
    return dict(e["choice"]) if e else {}


def make_params(d: dict, precision=None, max_batch=None, tuned=True, **solver) -> Params:
    """fsi_params from a workload dict (geometry segments, physics, time grid keys).

    With tuned=True the launch choices the autotuner stored for a problem of this
    dimension, level, precision and batch size are applied, except those the
    caller sets explicitly."""
    s = dict(SOLVER_DEFAULTS)
    if d["dim"] == 3:
        s.update(SOLVER_DEFAULTS_3D)
    if int(d.get("degree", 1)) == 2:
        s.update(SOLVER_DEFAULTS_Q2)
    s.update({k: v for k, v in d.items() if k in SOLVER_DEFAULTS})
    if tuned and int(d.get("degree", 1)) == 1:
        prec_name = "mixed" if (precision if precision is not None else d.get("precision", "fp64")) in \
            ("mixed", FSI_MIXED) else "fp64"
        mb = int(max_batch if max_batch is not None else d.get("N", 1))
        s.update({k: v for k, v in tuned_choice(d["dim"], d["level"], prec_name, mb).items() if k not in solver})
    s.update(solver)
    p = Params()
    p.dim = d["dim"]
    p.level = d["level"]
    p.degree = int(d.get("degree", 1))
    for a, ax in enumerate(d["segments"]):
        p.nseg[a] = len(ax)
        for q, (lo, hi, n) in enumerate(ax):
            p.seg_pts[a][q] = lo
            p.seg_pts[a][q + 1] = hi
            p.seg_cells[a][q] = n
    for a in range(3):
        p.solid_lo[a] = d["solid_lo"][a]
        p.solid_hi[a] = d["solid_hi"][a]
    for key in ("rho_f", "nu_f", "rho_s", "mu_s", "lambda_s", "inflow_peak", "ramp_time", "theta0",
                "lps_alpha0"):
        setattr(p, key, float(d[key]))
    prec = precision if precision is not None else d.get("precision", "fp64")
    p.precision = FSI_MIXED if prec in ("mixed", FSI_MIXED) else FSI_FP64
    if p.precision == FSI_MIXED:
        s.update({k: v for k, v in MIXED_DEFAULTS[d["dim"]].items() if k not in solver and k not in d})
    p.max_batch = int(max_batch if max_batch is not None else d.get("N", 1))
    if "batch_split" not in solver and p.max_batch < s["batch_split"]:
        s["batch_split"] = p.max_batch if p.max_batch >= 2 else 0   # no more groups than slices
    for key, v in s.items():
        setattr(p, key, type(getattr(p, key))(v))
    return p


def _ptr(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "expected a contiguous float64 device tensor"
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dvec(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """Owns an fsi_problem handle (fsi_setup / fsi_destroy)."""

    def __init__(self, params: Params):
        lib = load()
        self.params = params
        h = C.c_void_p()
        _check(lib.fsi_setup(C.byref(params), C.byref(h)), "fsi_setup")
        self.h = h
        nn, nd = C.c_int64(), C.c_int64()
        _check(lib.fsi_sizes(h, C.byref(nn), C.byref(nd)), "fsi_sizes")
        self.n_nodes, self.n_dofs = nn.value, nd.value

    def close(self):
        if getattr(self, "h", None):
            load().fsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def initial_state(self, U0):
        _check(load().fsi_initial_state(self.h, _ptr(U0), _stream()), "fsi_initial_state")

    def _prop(self, fn, B, t0, slice_len, nsteps, U_in, U_out, raise_on_error=True):
        st = Stats()
        arr, ptr = _dvec(t0)
        assert arr.size == B
        code = fn(self.h, B, ptr, float(slice_len), int(nsteps), _ptr(U_in), _ptr(U_out), C.byref(st), _stream())
        if raise_on_error:
            _check(code, fn.__name__)
        return code, st

    def fine_propagate(self, B, t0, slice_len, m, U_in, U_out, raise_on_error=True):
        return self._prop(load().fine_propagate, B, t0, slice_len, m, U_in, U_out, raise_on_error)

    def coarse_propagate(self, B, t0, slice_len, M, U_in, U_out, raise_on_error=True):
        return self._prop(load().coarse_propagate, B, t0, slice_len, M, U_in, U_out, raise_on_error)

    def parareal_run(self, T, N, m, M, tol, max_iter, U0, U_bnd, raise_on_error=True):
        st = Stats()
        code = load().parareal_run(self.h, float(T), int(N), int(m), int(M), float(tol), int(max_iter),
                                   _ptr(U0), _ptr(U_bnd), C.byref(st), _stream())
        if raise_on_error:
            _check(code, "parareal_run")
        return code, st

    def adjoint_gradient(self, T, N, m, U0):
        """(J, dJ/d(peak, mu_s, lambda_s), stats) of the time-integrated drag (FP64 path)."""
        st = Stats()
        J = C.c_double()
        g = (C.c_double * 3)()
        _check(load().adjoint_gradient(self.h, float(T), int(N), int(m), _ptr(U0), C.byref(J), g, C.byref(st),
                                       _stream()), "adjoint_gradient")
        return J.value, np.array(g[:]), st

    def debug_residual(self, B, U, Uo, t, k, R):
        arr, ptr = _dvec(t)
        _check(load().fsi_debug_residual(self.h, B, _ptr(U), _ptr(Uo), ptr, float(k), _ptr(R), _stream()),
               "fsi_debug_residual")

    def residual_noalloc(self, B, U, Uo, t, k, R, raise_on_error=True):
        """fsi_residual_noalloc: the residual of fsi_debug_residual, with its scratch in the
        library's static device array (the call allocates nothing)."""
        arr, ptr = _dvec(t)
        code = load().fsi_residual_noalloc(self.h, B, _ptr(U), _ptr(Uo), ptr, float(k), _ptr(R), _stream())
        if raise_on_error:
            _check(code, "fsi_residual_noalloc")
        return code

    def debug_jacobian_apply(self, B, U, Uo, t, k, X, Y):
        arr, ptr = _dvec(t)
        _check(load().fsi_debug_jacobian_apply(self.h, B, _ptr(U), _ptr(Uo), ptr, float(k), _ptr(X), _ptr(Y),
                                               _stream()), "fsi_debug_jacobian_apply")

    def debug_vcycle(self, B, U, Uo, t, k, X, Y):
        arr, ptr = _dvec(t)
        _check(load().fsi_debug_vcycle(self.h, B, _ptr(U), _ptr(Uo), ptr, float(k), _ptr(X), _ptr(Y), _stream()),
               "fsi_debug_vcycle")

    def profile_enable(self, on=True):
        _check(load().fsi_profile_enable(self.h, 1 if on else 0), "fsi_profile_enable")

    def profile_query(self, which):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        _check(load().fsi_profile_query(self.h, int(which), C.byref(n), C.byref(ms), C.byref(by)),
               "fsi_profile_query")
        return n.value, ms.value, by.value


def drag_objective(workload: dict, **solver):
    """torch.autograd.Function factory: J(peak, mu_s, lambda_s) = time-integrated drag.

    forward() builds a problem with the given parameters, runs adjoint_gradient
    (sequential fine solve, batched recompute, backward sweep) and returns J;
    backward() returns grad_output * dJ/dq from the same call.
    """
    import torch

    class DragObjective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, peak, mu_s, lambda_s):
            d = dict(workload)
            d.update(inflow_peak=float(peak), mu_s=float(mu_s), lambda_s=float(lambda_s))
            prob = Problem(make_params(d, precision="fp64", max_batch=d["N"], **solver))
            U0 = torch.zeros(prob.n_nodes, 5, dtype=torch.float64, device="cuda")
            prob.initial_state(U0)
            J, grad, _ = prob.adjoint_gradient(d["T"], d["N"], d["m"], U0)
            prob.close()
            ctx.save_for_backward(torch.as_tensor(grad, dtype=torch.float64))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout * grad[0], gout * grad[1], gout * grad[2]

    return DragObjective
