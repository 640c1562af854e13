// Declarations of the HIP kernels (defined and instantiated in assemble.hip and
// solver.hip) for the host driver.  D is the space dimension (2 or 3), S the
// storage type of the linear solve, CJ the Jacobian block layout (compressed
// or full).
#pragma once
#include "fsi_internal.h"

namespace fsi {

// threads of the coarsest-level factorisation and inverse kernels (one block per
// slice, or per slice and super-column): the dense block work of a slice is
// spread over all of them
constexpr int CF_THREADS = 1024;

template <int D>
__global__ void k_elem_residual(Geom g, StepPar sp, const double* U, const double* Uo, double* Re, const int* active);
template <int D, bool OLD>
__global__ void k_elem_jacobian(Geom g, StepPar sp, const double* U, const double* Uo, double* Ke, const int* active);
template <int D>
__global__ void k_apply_dirichlet(Geom g, StepPar sp, double* U, const double* t, const int* active);
template <int D>
__global__ void k_gather_residual(Geom g, StepPar sp, const double* Re, const double* U, const double* t, double* R,
                                  const int* active);
template <int D, class S, bool CJ>
__global__ void k_gather_jacobian(Geom g, double k, const double* Ke, S* J, double* Dsc, const int* active,
                                  int dir_identity);
template <int D>
__global__ void k_inject(Geom gc, Geom gf, const double* Uf, double* Uc);

// Q2 cells (2d): gc the cells' level, gn the node grid (the next level)
__global__ void k_elem_residual_q2(Geom gc, Geom gn, StepPar sp, const double* U, const double* Uo, double* Re,
                                   const int* active);
__global__ void k_elem_jacobian_q2(Geom gc, Geom gn, StepPar sp, const double* U, const double* Uo, double* Ke,
                                   const int* active);
__global__ void k_gather_residual_q2(Geom gc, Geom gn, StepPar sp, const double* pst2, const double* Re,
                                     const double* U, const double* t, double* R, const int* active);
template <class S>
__global__ void k_gather_jacobian_q2(Geom gc, Geom gn, double k, const double* pst2, const double* Ke, S* J2,
                                     double* Dsc, const int* active);
template <class S>
__global__ void k_spmv_q2(Geom gn, double k, const double* pst2, const S* J2, const S* x, const S* bv,
                          const double* Dsc, S* y, const int* active);
constexpr int Q2_JAC_CELLS = 64, Q2_JAC_THREADS = 256;   // k_elem_jacobian_q2 launch shape

// 2d adjoint
__global__ void k_drag_values(Geom g, double rn, const DragFace* faces, int nf, const double* U, size_t stride,
                              int nstates, double* vals);
__global__ void k_drag_gradient(Geom g, double rn, const DragFace* faces, int nf, const double* U, double scale,
                                double* grad);
__global__ void k_param_sens(Geom g, StepPar sp, const double* U, const double* Uo, const double* lam, double t,
                             double* out);
template <class S>
__global__ void k_transpose_J(Geom g, double k, const S* J, S* Jt, double* Dsc);
template <class S>
__global__ void k_spmv_T(Geom g, double k, const S* J, const S* x, S* y, int with_pst);
__global__ void k_fix_dirichlet(Geom g, double* lam, const double* rhs, const double* y);
__global__ void k_adjoint_rhs(Geom g, const double* rhs, double* Res);
__global__ void k_daxpy(size_t n, double a, const double* x, double* y);

template <int D, class S, bool CJ>
__global__ void k_spmv(Geom g, double k, const S* J, const S* x, const S* b, const double* Dsc, S* y,
                       const int* active, int slice_fast);
template <int D, class S, bool CJ>
__global__ void k_vanka_factor(Geom g, double k, const S* J, S* Ainv, S* Yu, int vc, const int* active);
template <int D, class S, int VC, bool CJ>
__global__ void k_vanka_color(Geom g, double k, int color, S omega, int zero_in, const S* J, const S* Ainv,
                              const S* Yu, const S* b, const S* xo, S* xn, const int* active, int slice_fast);
template <int D, class S>
__global__ void k_restrict(Geom gc, Geom gf, const S* rf, S* bc, const int* active);
template <int D, class S>
__global__ void k_prolong_add(Geom gf, Geom gc, const S* xc, S* xf, const int* active);
// 2d coarsest level
template <class S, bool CJ>
__global__ void k_coarse_factor(Geom g, double k, const S* J, int bsz, int nsb, double* Dinv, double* W, double* Lb,
                                const int* active);
template <class S>
__global__ void k_coarse_inverse(Geom g, int bsz, int nsb, const double* Dinv, const double* W, const double* Lb,
                                 double* Ysc, S* AinvS, const int* active);
template <class S>
__global__ void k_coarse_gemv(Geom g, const S* AinvS, const S* bvec, S* xvec, const int* active);

template <class S>
__global__ void k_multidot(int n, int nv, const S* X, size_t sxb, const S* Y, size_t syb, size_t syi, int chunk,
                           double* partial, int nchunk, const int* active);
__global__ void k_reduce_partials(int nv, int nchunk, const double* partial, double* out, int ostride,
                                  const int* active);
template <class S>
__global__ void k_multiaxpy(int n, int nv, S* X, size_t sxb, const S* Y, size_t syb, size_t syi, const double* h,
                            int hstride, double sign, const int* active);
template <class S>
__global__ void k_scale(int n, const S* X, size_t sxb, S* Y, size_t syb, const double* alpha, int astride,
                        int invert_sqrt, const int* active);
template <class S>
__global__ void k_unscale(int n, const S* X, size_t sxb, const double* D, S* Y, const int* active);
template <class S>
__global__ void k_scale_rhs(int n, const double* X, const double* D, S* Y, size_t syb, const int* active);
__global__ void k_givens(int j, int R, double* H, const double* hcol, double* cs, double* sn, double* gv, double* res,
                         const double* beta0, const double* tolv, int* state, int* ncol, const int* active, int B);
__global__ void k_init_cycle(int R, int cycle, const double* beta2, double* beta0, double* gv, int* state, int* ncol,
                             const double* tolv, const int* gact, int B);
__global__ void k_cgs_combine(int j, double* hcol, const double* hcol2, const double* hn2, const int* active, int B);
__global__ void k_update_gact(const int* nact, const int* state, int* gact, int* ord, int B, int* hout = nullptr);
__global__ void k_trisolve(int R, const double* H, const double* gv, const int* ncol, double* y, const int* active,
                           int B);
template <int D, class S>
__global__ void k_newton_update(int nn, double* U, const S* dx, int chunk, double* part, int nchunk,
                                const int* active);
template <int D>
__global__ void k_residual_norms(int nn, const double* R, const double* Dsc, const double* U, int chunk, double* part,
                                 int nchunk, const int* active);
__global__ void k_max_partials(int nchunk, const double* part, double* out, int B);
__global__ void k_nonfinite(size_t n, const double* X, int* flag);
__global__ void k_extrapolate(size_t n, int q, double* U, const double* U1, const double* U2, const double* U3,
                              const double* U4, const int* active);
__global__ void k_parareal_update(size_t n, const double* Cn, const double* Fv, const double* Cold, double* out,
                                  double th);
template <int D>
__global__ void k_theta_dots(int nn, const double* F, const double* Cv, int chunk, double* part, int nchunk);
template <int D>
__global__ void k_change_norms(int nn, const double* A, const double* Bv, int chunk, double* part, int nchunk);
template <class S>
__global__ void k_fill(size_t n, S* X, S v);
template <class A, class B2>
__global__ void k_convert(size_t n, const A* X, B2* Y);

}  // namespace fsi
