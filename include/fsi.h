/*
 * fsi.h -- C ABI of the MI355X fine propagator for monolithic ALE
 * fluid-structure interaction (Margenberg & Richter, "Parallel time-stepping
 * for fluid-structure interactions").
 *
 * The library integrates the semi-discrete ALE-FSI system of eqs. (ALE),
 * (ALE:stress), discretised as in eqs. (variational), (test) with equal-order
 * Q1 elements on an interface-fitted quadrilateral mesh (Section 2.2), by the
 * shifted Crank-Nicolson step of Section 2.3 with theta = 1/2 + theta0 k.
 * Each step is solved by Newton's method with an exact Jacobian; the linear
 * systems are solved by restarted FGMRES preconditioned with a geometric
 * multigrid V-cycle (colored multiplicative Vanka smoother).  The propagators
 * and the Parareal iteration follow Section 3, eq. (parareal:iteration).
 *
 * Conventions (all entry points):
 *   - Every call returns fsi_status (FSI_OK = 0, errors < 0).  No C++
 *     exception crosses the ABI.
 *   - State vectors are device arrays of float64 in node-major layout
 *     U[b][node][comp], comp = (v_x, v_y, u_x, u_y, p) in 2d, node index
 *     i + (nx+1) j.  The caller owns every array it passes; the library keeps
 *     no caller pointer after a call returns.
 *   - The library owns the fsi_problem handle and all device workspace; it is
 *     sized in fsi_setup for up to params.max_batch slices per call.
 *   - Work is enqueued on the given HIP stream; calls return after
 *     completion because the host needs the convergence status.
 *   - Host arrays (t0_host, stats) are read/written synchronously.
 *   - Calls on one fsi_problem must not overlap (the workspace is shared).
 */
#ifndef FSI_H
#define FSI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSI_OK = 0,
  FSI_ERR_ARG = -1,        /* invalid argument (null pointer, size out of range, bad params) */
  FSI_ERR_HIP = -2,        /* a HIP runtime call failed */
  FSI_ERR_OOM = -3,        /* device allocation failed */
  FSI_ERR_NEWTON = -4,     /* Newton did not converge within newton_maxit in some slice */
  FSI_ERR_LINEAR = -5,     /* FGMRES did not reach its tolerance within gmres_maxit */
  FSI_ERR_NONFINITE = -6,  /* non-finite input or iterate */
  FSI_ERR_PARAREAL = -7    /* Parareal did not reach its tolerance within max_iter */
} fsi_status;

enum { FSI_FP64 = 0, FSI_MIXED = 1 };

typedef struct fsi_problem fsi_problem;

/* Problem description.  SI units as in Table "parameters" of Section 4. */
typedef struct {
  int32_t dim;               /* 2 (quadrilaterals, 5 unknowns per node) or 3 (hexahedra, 7) */
  int32_t level;             /* refinement level l >= 1 of the level-0 mesh */
  /* level-0 tensor mesh: per axis nseg segments, breakpoints seg_pts[a][0..nseg],
     seg_cells[a][s] level-0 cells in segment s; the bar faces must be breakpoints */
  int32_t nseg[3];
  double seg_pts[3][5];
  int32_t seg_cells[3][4];
  double solid_lo[3], solid_hi[3];   /* elastic bar: cells whose centre lies inside */
  double rho_f, nu_f, rho_s, mu_s, lambda_s;
  double inflow_peak;        /* peak of the parabolic inflow profile */
  double ramp_time;          /* s(t) = (1 - cos(pi t / ramp_time)) / 2 for t < ramp_time, then 1 */
  double theta0;             /* theta = 1/2 + theta0 k */
  double lps_alpha0;         /* local-projection constant: alpha_K = alpha0 h_K^2 / (rho_f nu_f) */
  double cip_gamma;          /* coarsest multigrid level only: gradient-jump pressure penalty */
  int32_t precision;         /* FSI_FP64 or FSI_MIXED (FP32 FGMRES/multigrid, FP64 Newton residual) */
  int32_t gmres_restart;     /* Krylov basis size (<= 64) */
  int32_t gmres_maxit;       /* total FGMRES iterations per linear solve */
  int32_t newton_maxit;
  int32_t vanka_sweeps;      /* pre- and post-smoothing sweeps per level */
  double vanka_omega;        /* Vanka damping */
  double newton_rtol;        /* stop when every field's update <= rtol * |field|_inf */
  double lin_rtol;           /* smallest FGMRES relative tolerance (row-scaled residual); the
                                tolerance of Newton iteration j > 1 of a slice is
                                min(1e-2, max(lin_rtol, 0.1 newton_rtol / e)), e the error
                                estimate after iteration j - 1 */
  int32_t max_batch;         /* largest number of slices per call */
  int32_t vanka_sweeps_coarse; /* pre- and post-smoothing sweeps on the levels below the finest */
  int32_t precond_lag;       /* 0: rebuild the multigrid preconditioner (coarse operators, Vanka
                                inverses, coarsest factorisation) at every Newton iteration;
                                1: only at the first Newton iteration of each time step (the
                                Krylov operator is the exact Jacobian either way) */
  double lin_rtol_first;     /* FGMRES relative tolerance of the first Newton iteration of a step
                                (0 < lin_rtol_first < 1) */
  int32_t parareal_theta;    /* parareal_run correction (eq. (thetaparareal:iteration)):
                                0 plain Parareal (theta = 1);
                                1 theta = mean over the velocity and displacement components c of
                                  <F_c, C_c> / (|F_c| |C_c|);
                                2 theta = mean over c of <F_c, C_c> / <C_c, C_c>;
                                F = F(U^i_l), C = C(U^{i+1}_l); components with a zero norm are
                                left out, and with none left theta = 1 */
  double theta_ref_k;        /* 0: every step of size k uses theta = 1/2 + theta0 k (Section 2.3).
                                k_r > 0: theta = 1/2 + theta0 k_r^2 / k, the damping
                                theta = 1/2 + alpha(k) k with equal dissipation per unit time
                                for all step sizes (Section 4, fsi-3 discussion); steps of
                                size k_r keep 1/2 + theta0 k_r */
  int32_t parareal_pipeline; /* parareal_run schedule (Section 3, task-based implementation):
                                0: each iteration runs one batched fine sweep, then the
                                sequential correction sweep;
                                G in [1, max_batch]: the fine propagations run in chunks of G
                                consecutive slices on a second workspace and stream, each
                                starting as soon as the correction sweep has written its
                                inputs, overlapped with the rest of the sweep.  Same iterates
                                as 0.  The second workspace (max_batch G) is created on the
                                first such call and kept with the problem. */
  int32_t batch_split;       /* fine_propagate / coarse_propagate with B >= 2 slices:
                                0 or 1: one batch on the library stream;
                                S in [2, 8] (and <= max_batch): the slices are cut into S
                                consecutive groups of (nearly) equal size, each run by its
                                own host thread on its own workspace and stream, so that
                                one group's latency-bound phases (coarse levels, Krylov
                                scalars, host synchronisation) overlap another group's
                                bandwidth-bound passes on the same GPU.  Every slice's
                                arithmetic is that of the single batch (same results, bit
                                for bit).  The S - 1 extra workspaces (max_batch
                                ceil(max_batch / S) each) are created on the first call
                                that splits (FSI_ERR_OOM from that call if they do not
                                fit) and kept with the problem.  Calls made while
                                per-kernel timing is enabled, and the adjoint's recompute,
                                run as one batch.  Each group's stream takes a hardware
                                queue: S = 3 leaves one for the caller's stream. */
  double newton_res_rtol;    /* FP64 residual test of Newton's method (in the mixed path the test
                                of the iterative refinement): a slice's step is done when, after
                                an iteration whose linear solve reached its tolerance, the update
                                test (newton_rtol) holds and then the residual R of the time-step
                                equation (Section 2.3) at the new state satisfies, per field f,
                                max |D R_f| <= newton_res_rtol max |U_f|, D the row scaling
                                1 / max_j |J_ij| of the step Jacobian (0 < newton_res_rtol < 1) */
  /* launch choices (results do not depend on them; the binding takes them from its
     autotuner table): */
  int32_t spmv_slice_fast;   /* SpMV grid with the slices as the fast dimension: 1 yes, 0 no,
                                -1 the built-in default (yes for 2d FP64) */
  int32_t vanka_slice_fast;  /* the same for the fused Vanka pass (-1: yes for 3d and 2d FP64) */
  int32_t vanka_wide_cells;  /* 3d: a level whose colours hold at least this many cells over
                                the batch runs the fused Vanka pass with 32 cells per block,
                                others with 8 (0: 8192) */
  int32_t degree;            /* polynomial degree of the equal-order elements (Section 2.2):
                                1 (Q1, every mode) or 2 (Q2, the paper's choice; 2d, FP64 or
                                mixed precision, no adjoint).  With degree 2 the cells are
                                those of `level` (which may then be 0) and the nodes those of
                                level + 1 (9 per cell); the Krylov operator is the Q2 step
                                Jacobian (stored in the linear solve's type) and the
                                preconditioner the Q1 multigrid V-cycle on the same nodes */
  double newton_res_accept;  /* 0: off.  > 0: a slice whose residual at the top of a Newton
                                iteration (after at least one update) meets the residual test
                                with this tolerance ends its step there, without a further
                                linear solve (round-off level, below newton_res_rtol) */
  int32_t newton_guess;      /* Newton's starting point at step n: 0: U^{n-1}; q in [1, 3]:
                                the polynomial of degree q through the last q + 1 states of
                                the slice, evaluated at t_n (degree min(q, n - 1) at the
                                first steps; the Dirichlet values of t_n replace it on the
                                boundary).  The converged step does not depend on it */
  double precond_lps_scale;  /* degree 2 only: factor on the local-projection constant of the
                                Q1 levels that precondition the Q2 system (0: 1, the Q1
                                discretisation's own; > 0: the factor).  Only the
                                preconditioner changes, not the Q2 step */
} fsi_params;

#define FSI_MAX_SLICES 1024
typedef struct {
  int32_t newton_its[FSI_MAX_SLICES];   /* Newton iterations summed over the steps, per slice */
  int32_t krylov_its[FSI_MAX_SLICES];   /* FGMRES iterations summed over the steps, per slice */
  int32_t slice_status[FSI_MAX_SLICES]; /* fsi_status of the slice */
  double stage_ms[8];                   /* propagators: milliseconds summed over the call's Newton
                                           iterations, from HIP events on the call's stream (with
                                           concurrent slice groups the largest group's figure):
                                           0 residual, 1 Jacobian + multigrid setup, 2 linear
                                           solve, 3 update and convergence tests; 4 wall time of
                                           the call (host clock).  parareal_run: 4 wall time,
                                           5 coarse propagations, 6 fine sweeps (host clock) */
  int32_t parareal_iters;               /* completed Parareal iterations (also when a later one failed) */
  int32_t newton_total, krylov_total;   /* totals over all slices of the call */
} fsi_stats;

/* Build the mesh hierarchy, node classes, constant stabilisation operators and
   device workspace for params->max_batch slices.  *out receives the handle.
   The mesh is the tensor mesh of params->seg_* refined `level` times, with the
   elastic bar resolved by cell faces on every level (Section 2.2 asks for an
   interface-fitted mesh); the node classes and the Dirichlet data follow the
   ALE system of eqs. (ALE), (ALE:stress) and the test spaces of eq. (test);
   the pressure stabilisation is the local projection named in Section 2.2.
   Errors: FSI_ERR_ARG (bad params: a size or count out of range, a non-finite
   constant, rho_f, nu_f, rho_s, mu_s or ramp_time not positive, lambda_s,
   theta0, lps_alpha0 or cip_gamma negative, vanka_omega outside (0, 2),
   newton_rtol not positive, lin_rtol or lin_rtol_first outside (0, 1),
   batch_split outside [0, 8] or above max_batch, newton_guess outside [0, 3]),
   FSI_ERR_OOM, FSI_ERR_HIP. */
fsi_status fsi_setup(const fsi_params* params, fsi_problem** out);

/* Number of mesh nodes and of unknowns on the finest level: the equal-order
   nodal unknowns (v, u, p) of Section 2.2, 5 per node in 2d and 7 in 3d.
   FSI_ERR_ARG if pb is NULL; either output pointer may be NULL. */
fsi_status fsi_sizes(const fsi_problem* pb, int64_t* n_nodes, int64_t* n_dofs);

/* U0_dev[n_dofs] := the initial value of eq. (ALE) used by the workloads: the
   fluid and the bar at rest (v = u = p = 0) with the Dirichlet data of t = 0
   (the inflow profile of Section 4 scaled by the ramp s(0) = 0, so also zero).
   Device array of the caller, written on `stream`; returns after completion.
   FSI_ERR_ARG for NULL arguments. */
fsi_status fsi_initial_state(fsi_problem* pb, double* U0_dev, hipStream_t stream);

/* Fine propagator F of Section 3: for each of B slices b, m uniform steps of
   size k = slice_len / m from t0_host[b] (host array), starting from
   U_in_dev[b] and writing the final state to U_out_dev[b] (both [B][n_dofs],
   may alias).  The pressure of U_in only seeds Newton.  Per-slice status and
   iteration counts go to stats (host, may be NULL).  FSI_ERR_ARG if B is not
   in [1, max_batch], m < 1, slice_len is not positive or a pointer is NULL;
   non-finite input gives FSI_ERR_NONFINITE before any work (U_out is then not
   written); a slice that fails keeps its last iterate.  Per-slice statuses
   (stats->slice_status; the call returns one of the failing ones):
   FSI_ERR_NEWTON (the update and residual tests, newton_rtol and
   newton_res_rtol, not met within newton_maxit iterations), FSI_ERR_LINEAR
   (the same, and the last linear solve of the slice missed its tolerance
   within gmres_maxit iterations; an update from such a solve is never
   accepted), FSI_ERR_NONFINITE (a Newton iterate was not finite).  A failed
   slice stops; the others go on. */
fsi_status fine_propagate(fsi_problem* pb, int32_t B, const double* t0_host, double slice_len,
                          int32_t m, const double* U_in_dev, double* U_out_dev,
                          fsi_stats* stats, hipStream_t stream);

/* Coarse propagator C of Section 3: the same scheme with M steps of size
   K = slice_len / M (theta = 1/2 + theta0 K).  Arguments as fine_propagate. */
fsi_status coarse_propagate(fsi_problem* pb, int32_t B, const double* t0_host, double slice_len,
                            int32_t M, const double* U_in_dev, double* U_out_dev,
                            fsi_stats* stats, hipStream_t stream);

/* Parareal, eq. (parareal:iteration): N slices of length T/N on [0, T], fine
   propagator with m steps, coarse with M steps per slice.  Writes the slice
   boundary states U_bnd_dev[N+1][n_dofs] (U_bnd[0] = U0).  Stops when the
   largest relative change over the boundaries of v and u is below tol or after
   max_iter (<= N) iterations; the last fine sweep batches all unconverged
   slices in one call.  Returns FSI_ERR_PARAREAL if tol was not met. */
fsi_status parareal_run(fsi_problem* pb, double T, int32_t N, int32_t m, int32_t M, double tol,
                        int32_t max_iter, const double* U0_dev, double* U_bnd_dev,
                        fsi_stats* stats, hipStream_t stream);

/* Discrete adjoint of the time-integrated drag on the bar (FP64 path only).
   The functional is J = k sum_{n=1}^{N m} D(U^n) over the sequential fine
   trajectory on [0, T] (N slices of m steps from U0_dev), D = x-component of
   the fluid traction J sigma F^{-T} n_s on the bar faces shared with fluid
   cells (sigma of eq. (ALE:stress)).  The forward pass stores the N + 1
   slice-boundary states, recomputes all steps in one batched call from them,
   then sweeps backward solving (dR_n/dU^n)^T lambda_n = -k dD/dU(U^n)
   - (dR_{n+1}/dU^n)^T lambda_{n+1} with the transposed multigrid/FGMRES
   solver (relative tolerance 1e-12).  Outputs (host): J_out, and grad_out[3]
   = dJ/d(inflow peak), dJ/d(mu_s) at fixed lambda_s, dJ/d(lambda_s) at fixed
   mu_s.  Errors: FSI_ERR_ARG (bad sizes, mixed precision), solver errors as
   in fine_propagate. */
fsi_status adjoint_gradient(fsi_problem* pb, double T, int32_t N, int32_t m, const double* U0_dev, double* J_out,
                            double grad_out[3], fsi_stats* stats, hipStream_t stream);

/* Test and benchmark entry points (same conventions).
   fsi_debug_residual: R_out[b] = residual of one step t_host[b]-k -> t_host[b]
     at the new state U[b] with old state Uo[b] (Dirichlet rows included).
   fsi_debug_jacobian_apply: assemble the Jacobian at (U[b], Uo[b]) on the
     finest level and return Y[b] = J X[b] (FP64 path), or the FP32 copy's
     product in the mixed path.
   fsi_debug_vcycle: one V-cycle of the multigrid built at (U, Uo): Y = M^{-1} X. */
fsi_status fsi_debug_residual(fsi_problem* pb, int32_t B, const double* U, const double* Uo,
                              const double* t_host, double k, double* R_out, hipStream_t stream);
fsi_status fsi_debug_jacobian_apply(fsi_problem* pb, int32_t B, const double* U, const double* Uo,
                                    const double* t_host, double k, const double* X, double* Y,
                                    hipStream_t stream);
fsi_status fsi_debug_vcycle(fsi_problem* pb, int32_t B, const double* U, const double* Uo,
                            const double* t_host, double k, const double* X, double* Y,
                            hipStream_t stream);

/* Allocation-free variant of fsi_debug_residual, for callers that cannot
   allocate device memory during the call (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc).  Same arguments, layout and
   result as fsi_debug_residual: R_out[b] = residual of the step
   t_host[b] - k -> t_host[b] at U[b] with old state Uo[b].  The element
   residuals and the slice times go to a static device array of 32 MiB that the
   library holds on each GPU until the process ends, not to the problem's
   workspace; the call allocates nothing.  Limit: B * (NE * n_cells) + B
   doubles (NE = 20 in 2d, 56 in 3d; n_cells of the finest level, the first
   term rounded up to 32) must fit in 32 MiB, else FSI_ERR_ARG with a message
   on stderr (e.g. 51 slices of 128x32 cells, 4 of 64x16x16).  Every call on a
   GPU shares that GPU's array: calls that overlap on one GPU (any problem,
   any stream) race and must be serialised by the caller.  Nothing in the
   array has to start at zero (every value read is written earlier in the
   same call).  Also FSI_ERR_ARG as fsi_debug_residual. */
fsi_status fsi_residual_noalloc(fsi_problem* pb, int32_t B, const double* U, const double* Uo,
                                const double* t_host, double k, double* R_out, hipStream_t stream);

/* Per-kernel timing over the calls made while enabled (HIP events on the
   caller's stream around every launch of the named kernel family).
   fsi_profile_enable(pb, 1) starts collecting (and clears), 0 stops.
   fsi_profile_query returns the launch count and summed milliseconds of
   kernel family `which` and the algorithmic bytes those launches moved:
   0 = fused Vanka colour pass on the finest level, 1 = Jacobian product of
   the Krylov iteration, 2 = element Jacobian (all levels), 3 = residual,
   4 = residual before restriction on the finest level, 5 = every smoother
   and residual kernel of the coarser levels, 6 = coarsest-level solve. */
fsi_status fsi_profile_enable(fsi_problem* pb, int32_t on);
fsi_status fsi_profile_query(const fsi_problem* pb, int32_t which, int64_t* launches, double* ms,
                             double* bytes);

void fsi_destroy(fsi_problem* pb);
const char* fsi_status_string(fsi_status s);

#ifdef __cplusplus
}
#endif
#endif /* FSI_H */
