// Batched linear-solver kernels: block-stencil SpMV, transposed products of the
// adjoint, multigrid transfers, the coarsest-level block-tridiagonal direct
// solve (2d) and the FGMRES building blocks (the Vanka kernels are in
// vanka.hip and vanka_factor.hip).  Every kernel takes the slice index from
// blockIdx.y (the SpMV from blockIdx.x when its slices are the fast grid
// dimension) and skips slices whose active flag is 0.  S is the storage and
// arithmetic type of the linear solve (double, or float in the mixed-precision
// path); D the space dimension.
#include "stencil.h"
#include "kernels.h"

namespace fsi {

using D2 = Dm<2>;

// ------------------------------------------------------------------ SpMV
// y = D (A x)            (b == nullptr)
// y = D (b - A x)        (b != nullptr)
// with A = J (3^D block stencil of NC x NC blocks) + k * S_p (pressure stencil).
// D = Dsc (row scaling) when given, else identity.
// One thread per (node, row): a block of NC waves takes 64 lanes of nodes of
// the Jacobian storage (one tile in 2d, two tiles of copy 0 in 3d), wave r
// forming row r, so the rows of a node read its neighbours' x through the same
// CU's cache, and a wave streams whole runs of each coefficient.  The slice is
// blockIdx.y, or blockIdx.x when slice_fast is set (slices as the fast grid
// dimension, so the blocks of one tile in all slices run together).
template <int D, class S, bool CJ>
__global__ void __launch_bounds__(Dm<D>::NC * 64) k_spmv(Geom g, double k, const S* __restrict__ J,
                                                         const S* __restrict__ x, const S* __restrict__ b,
                                                         const double* __restrict__ Dsc, S* __restrict__ y,
                                                         const int* __restrict__ active, int slice_fast) {
  FSI_DIM(D);
  // slice_fast = 2: active is the ordered list of working slices (k_update_gact)
  const int bs = slice_fast == 2 ? active[blockIdx.x] : (slice_fast ? blockIdx.x : blockIdx.y);
  const int bx = slice_fast ? blockIdx.y : blockIdx.x;
  const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int n, i, row;
  if (!jrowtiles<D, S>()) {
    n = bx * 64 + lane;
    row = n / (g.nx + 1);
    i = n - row * (g.nx + 1);
    if (n >= g.nn) return;
  } else {
    constexpr int TX = jtx<D, S>();
    const int ntx = jntx<D, S>(g, 0);
    const int t = bx * (64 / TX) + lane / TX;
    row = t / ntx;
    i = (t - row * ntx) * TX + lane % TX;
    if (row >= jrows<D>(g) || i > g.nx) return;
    n = i + (g.nx + 1) * row;
  }
  if (slice_fast == 2 ? bs < 0 : (active && !active[bs])) return;
  const int j = row % (g.ny + 1), kk = row / (g.ny + 1);
  const S* jn = J + jslice_row<D, S, CJ>(g, bs, r) + jnode<D, S, CJ>(g, i, row, 0);
  const S* xb = x + (size_t)bs * g.nn * NC;
  S acc = stencil_row<D, S, CJ>(jn, xb, n, r, nbr_offsets<D>(g, i, j, kk));
  if (r == PC) acc += pst_row<D, S>(g, k, n, i, j, kk, xb);
  const size_t o = ((size_t)bs * g.nn + n) * NC + r;
  S v = b ? b[o] - acc : acc;
  y[o] = Dsc ? (S)(Dsc[o] * (double)v) : v;
}

// ------------------------------------------------------------ transposes (2d adjoint)
// Jt = J^T with the Dirichlet rows of Jt replaced by identity rows (the
// transposed system of the free unknowns), and the row scaling of Jt.
// (J^T)_{(i,r),(j,c)} = J_{(j,c),(i,r)}: node j = i + offset(s) stores it in the
// slot of offset -offset(s), entry (c, r).
template <class S>
__global__ void k_transpose_J(Geom g, double k, const S* __restrict__ J, S* __restrict__ Jt, double* __restrict__ Dsc) {
  const int bs = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const int i = n % (g.nx + 1), j = n / (g.nx + 1);
  const S* jb = J + (size_t)bs * jslice<2, S, false>(g);
  S* jt = Jt + (size_t)bs * jslice<2, S, false>(g);
  S* jt0 = jt + jnode<2, S, false>(g, i, j, 0);
  const uint8_t m = g.dmask[n];
  double rmax[D2::NC] = {0, 0, 0, 0, 0};
  for (int s = 0; s < D2::NSLOT; ++s) {
    const int dx = s % 3 - 1, dy = s / 3 - 1;
    const int ii = i + dx, jj = j + dy;
    const bool ok = ii >= 0 && jj >= 0 && ii <= g.nx && jj <= g.ny;
    const S* jnb = jb + (ok ? jnode<2, S, false>(g, ii, jj, 0) : 0);
    const int so = slot_of<2>(-dx, -dy, 0);
    for (int r = 0; r < D2::NC; ++r)
      for (int c = 0; c < D2::NC; ++c) {
        double v = ok ? (double)jnb[jent<2, S, false>(so, D2::NC * c + r)] : 0.0;
        if (m & (1u << r)) v = (s == 4 && c == r) ? 1.0 : 0.0;
        jt0[jent<2, S, false>(s, D2::NC * r + c)] = (S)v;
        rmax[r] = fmax(rmax[r], fabs(v));
      }
  }
  if (!(m & dm_p<2>()))
    for (int q = 0; q < D2::NPST; ++q) rmax[4] = fmax(rmax[4], fabs(k * g.pst[(size_t)q * g.nn + n]));
  if (Dsc)
    for (int r = 0; r < D2::NC; ++r) Dsc[((size_t)bs * g.nn + n) * D2::NC + r] = rmax[r] > 0.0 ? 1.0 / rmax[r] : 1.0;
}

// y = J^T x for the stored block stencil (no Dirichlet modification) plus, when
// with_pst, k S x_p (S is symmetric).
template <class S>
__global__ void k_spmv_T(Geom g, double k, const S* __restrict__ J, const S* __restrict__ x, S* __restrict__ y,
                         int with_pst) {
  const int bs = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const int i = n % (g.nx + 1), j = n / (g.nx + 1);
  const S* jb = J + (size_t)bs * jslice<2, S, false>(g);
  const S* xb = x + (size_t)bs * g.nn * D2::NC;
  S acc[D2::NC] = {0, 0, 0, 0, 0};
  for (int s = 0; s < D2::NSLOT; ++s) {
    // row node m = n - offset(s) holds the entry in slot s
    const int dx = s % 3 - 1, dy = s / 3 - 1;
    const int ii = i - dx, jj = j - dy;
    if (ii < 0 || jj < 0 || ii > g.nx || jj > g.ny) continue;
    const int mr = ii + (g.nx + 1) * jj;
    for (int r = 0; r < D2::NC; ++r) {
      const S xr = xb[(size_t)mr * D2::NC + r];
      const S* jm = jb + jnode<2, S, false>(g, ii, jj, 0);
      for (int c = 0; c < D2::NC; ++c) acc[c] += jm[jent<2, S, false>(s, D2::NC * r + c)] * xr;
    }
  }
  if (with_pst && !(g.dmask[n] & dm_p<2>())) {
    S ap = 0;
    for (int q = 0; q < D2::NPST; ++q) {
      const int dx = q % 5 - 2, dy = q / 5 - 2;
      const int ii = i + dx, jj = j + dy;
      if (ii < 0 || jj < 0 || ii > g.nx || jj > g.ny) continue;
      ap += (S)g.pst[(size_t)q * g.nn + n] * xb[(size_t)(ii + (g.nx + 1) * jj) * D2::NC + 4];
    }
    acc[4] += (S)k * ap;
  }
  for (int c = 0; c < D2::NC; ++c) y[((size_t)bs * g.nn + n) * D2::NC + c] = acc[c];
}

// Dirichlet unknowns of the adjoint: lam_D = rhs_D - (J^T lam)_D with lam_D = 0 in y.
__global__ void k_fix_dirichlet(Geom g, double* __restrict__ lam, const double* __restrict__ rhs,
                                const double* __restrict__ y) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const uint8_t m = g.dmask[n];
  for (int c = 0; c < D2::NC; ++c)
    if (m & (1u << c)) lam[(size_t)n * D2::NC + c] = rhs[(size_t)n * D2::NC + c] - y[(size_t)n * D2::NC + c];
}

// y += a x (FP64)
__global__ void k_daxpy(size_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

// rhs_reduced = rhs with the Dirichlet entries set to zero; Res = -rhs_reduced
__global__ void k_adjoint_rhs(Geom g, const double* __restrict__ rhs, double* __restrict__ Res) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const uint8_t m = g.dmask[n];
  for (int c = 0; c < D2::NC; ++c) Res[(size_t)n * D2::NC + c] = (m & (1u << c)) ? 0.0 : -rhs[(size_t)n * D2::NC + c];
}

// --------------------------------------------------------- grid transfers
// b_c = P^T r_f ((bi/tri)linear weights), zero on coarse Dirichlet components
// and ignoring fine Dirichlet components (P has zero rows there).
template <int D, class S>
__global__ void k_restrict(Geom gc, Geom gf, const S* __restrict__ rf, S* __restrict__ bc,
                           const int* __restrict__ active) {
  FSI_DIM(D);
  const int bs = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gc.nn || (active && !active[bs])) return;
  int I, Jc, K;
  node_ijk<D>(gc, n, I, Jc, K);
  const uint8_t mc = gc.dmask[n];
  S acc[NC];
  for (int c = 0; c < NC; ++c) acc[c] = 0;
  for (int s = 0; s < NSLOT; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = D == 3 ? s / 9 - 1 : 0;
    const int fi = 2 * I + dx, fj = 2 * Jc + dy, fk = 2 * K + dz;
    if (fi < 0 || fj < 0 || fk < 0 || fi > gf.nx || fj > gf.ny || fk > gf.nz) continue;
    const S w = (S)((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
    const int nf = node_at(gf, fi, fj, fk);
    const uint8_t mf = gf.dmask[nf];
    const S* rv = rf + ((size_t)bs * gf.nn + nf) * NC;
    for (int c = 0; c < NC; ++c)
      if (!(mf & (1u << c))) acc[c] += w * rv[c];
  }
  S* o = bc + ((size_t)bs * gc.nn + n) * NC;
  for (int c = 0; c < NC; ++c) o[c] = (mc & (1u << c)) ? (S)0 : acc[c];
}

// x_f += P x_c on non-Dirichlet fine components (coarse Dirichlet values are zero).
template <int D, class S>
__global__ void k_prolong_add(Geom gf, Geom gc, const S* __restrict__ xc, S* __restrict__ xf,
                              const int* __restrict__ active) {
  FSI_DIM(D);
  const int bs = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gf.nn || (active && !active[bs])) return;
  int fi, fj, fk;
  node_ijk<D>(gf, n, fi, fj, fk);
  const int lo[3] = {fi >> 1, fj >> 1, fk >> 1};
  const int odd[3] = {fi & 1, fj & 1, fk & 1};
  const uint8_t mf = gf.dmask[n];
  S add[NC];
  for (int c = 0; c < NC; ++c) add[c] = 0;
  for (int q = 0; q < NL; ++q) {
    bool skip = false;
    double w = 1.0;
    int cc[3] = {lo[0], lo[1], lo[2]};
    for (int ax = 0; ax < D; ++ax) {
      const int bit = (q >> ax) & 1;
      if (bit && !odd[ax]) skip = true;   // even fine index: one coarse node on this axis
      if (odd[ax]) w *= 0.5;
      cc[ax] += bit;
    }
    if (skip) continue;
    const int nc = node_at(gc, cc[0], cc[1], D == 3 ? cc[2] : 0);
    const uint8_t mc = gc.dmask[nc];
    const S* xv = xc + ((size_t)bs * gc.nn + nc) * NC;
    for (int c = 0; c < NC; ++c)
      if (!(mc & (1u << c))) add[c] += (S)w * xv[c];
  }
  S* xo = xf + ((size_t)bs * gf.nn + n) * NC;
  for (int c = 0; c < NC; ++c)
    if (!(mf & (1u << c))) xo[c] += add[c];
}

// ------------------------------------------- coarsest level: direct solve (2d)
// Unknowns ordered by super-columns of two x-node columns (bs = 2 (ny+1) 5);
// the 3x3 block stencil plus the 5x5 pressure stencil make the matrix block
// tridiagonal.  Factor: Delta_0 = D_0, Delta_K = D_K - L_K W_{K-1},
// W_K = Delta_K^{-1} U_K.  Stored per slice: Dinv_K, W_K, L_K (bs x bs each).
// From the factors the explicit inverse is formed once per factorisation, so
// each coarse solve of a V-cycle is one dense matrix-vector product.
template <class S, bool CJ>
__device__ inline double coarse_entry(const Geom& g, double k, const S* jb, int K, int l, int K2, int l2) {
  // row: super-column K local l; column: super-column K2 local l2
  const int r = l % D2::NC, nl = l / D2::NC, colx = nl / (g.ny + 1), jr = nl % (g.ny + 1);
  const int c = l2 % D2::NC, nl2 = l2 / D2::NC, colx2 = nl2 / (g.ny + 1), jc = nl2 % (g.ny + 1);
  const int ir = 2 * K + colx, ic = 2 * K2 + colx2;
  if (ir > g.nx || ic > g.nx) return (K == K2 && l == l2) ? 1.0 : 0.0;   // padding: identity
  const int dx = ic - ir, dy = jc - jr;
  const int n = ir + (g.nx + 1) * jr;
  double v = 0.0;
  const int e = jentry<2, CJ>(r, c);
  if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && e >= 0)
    v = (double)jb[jnode<2, S, CJ>(g, ir, jr, 0) + jent<2, S, CJ>(slot_of<2>(dx, dy, 0), e)];
  if (r == 4 && c == 4 && dx >= -2 && dx <= 2 && dy >= -2 && dy <= 2 && !(g.dmask[n] & dm_p<2>()))
    v += k * g.pst[(size_t)pslot_of<2>(dx, dy, 0) * g.nn + n];
  return v;
}

// global dof index of local unknown l of super-column K, or -1 for padding
__device__ inline int coarse_gidx(const Geom& g, int K, int l) {
  const int c = l % D2::NC, nl = l / D2::NC, colx = nl / (g.ny + 1), jn = nl % (g.ny + 1);
  const int i = 2 * K + colx;
  if (i > g.nx) return -1;
  return (i + (g.nx + 1) * jn) * D2::NC + c;
}

// C = alpha A B for bs x bs row-major tiles in LDS (all threads of the block)
__device__ inline void tile_gemm(int bsz, const double* A, const double* Bm, double* C, double alpha) {
  for (int e = threadIdx.x; e < bsz * bsz; e += blockDim.x) {
    const int r = e / bsz, c = e % bsz;
    double s = 0.0;
    for (int q = 0; q < bsz; ++q) s += A[r * bsz + q] * Bm[q * bsz + c];
    C[e] = alpha * s;
  }
}

// One workgroup per slice.  LDS: [Delta | I] (bs x 2bs), L_K, U_K and W_{K-1}
// (bs x bs each).  Gauss-Jordan with partial pivoting: wave 0 finds the pivot and
// the row factors, then every thread owns columns of [Delta | I] for the update.
template <class S, bool CJ>
__global__ void __launch_bounds__(CF_THREADS) k_coarse_factor(Geom g, double k, const S* __restrict__ J, int bsz, int nsb,
                                                       double* __restrict__ Dinv, double* __restrict__ W,
                                                       double* __restrict__ Lb, const int* __restrict__ active) {
  extern __shared__ double lds[];
  const int bs = blockIdx.x;
  if (active && !active[bs]) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const S* jb = J + (size_t)bs * jslice<2, S, CJ>(g);
  const int w2 = 2 * bsz;
  const int B2i = bsz * bsz;
  double* M = lds;                  // bsz x 2bsz
  double* Lt = M + bsz * w2;        // bsz x bsz
  double* Ut = Lt + B2i;
  double* Wp = Ut + B2i;
  __shared__ double fac[64];
  __shared__ double prow[128];
  __shared__ int colmap[64];
  __shared__ int usedf[64];
  __shared__ int piv_row;
  __shared__ double piv_val;
  const size_t B2 = (size_t)B2i;
  double* dinv = Dinv + (size_t)bs * nsb * B2;
  double* w = W + (size_t)bs * nsb * B2;
  double* lb = Lb + (size_t)bs * nsb * B2;
  for (int K = 0; K < nsb; ++K) {
    for (int e = tid; e < B2i; e += nt) {
      const int r = e / bsz, c = e % bsz;
      M[r * w2 + c] = coarse_entry<S, CJ>(g, k, jb, K, r, K, c);
      M[r * w2 + bsz + c] = (r == c) ? 1.0 : 0.0;
      if (K > 0) Lt[e] = coarse_entry<S, CJ>(g, k, jb, K, r, K - 1, c);
      if (K < nsb - 1) Ut[e] = coarse_entry<S, CJ>(g, k, jb, K, r, K + 1, c);
    }
    for (int e = tid; e < bsz; e += nt) usedf[e] = 0;
    __syncthreads();
    if (K > 0) {
      for (int e = tid; e < B2i; e += nt) {
        lb[K * B2 + e] = Lt[e];
        const int r = e / bsz, c = e % bsz;
        double s = 0.0;
        for (int q = 0; q < bsz; ++q) s += Lt[r * bsz + q] * Wp[q * bsz + c];
        M[r * w2 + c] -= s;
      }
      __syncthreads();
    }
    for (int jc = 0; jc < bsz; ++jc) {
      if (tid < 64) {
        double best = -1.0;
        int bi = 0;
        if (tid < bsz && !usedf[tid]) { best = fabs(M[tid * w2 + jc]); bi = tid; }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        double pv = M[bi * w2 + jc];
        if (pv == 0.0) pv = 1.0;
        if (tid < bsz) fac[tid] = (tid == bi) ? 0.0 : M[tid * w2 + jc] / pv;
        if (tid == 0) { usedf[bi] = 1; colmap[jc] = bi; piv_row = bi; piv_val = pv; }
      }
      __syncthreads();
      const int pr = piv_row;
      const double pv = piv_val;
      // the pivot row, then every (row, column) pair in parallel: columns left of
      // jc are already eliminated in all rows but their pivot rows, so only
      // columns >= jc change (and the identity half)
      for (int c = tid; c < w2; c += nt) prow[c] = M[pr * w2 + c];
      __syncthreads();
      const int wc = w2 - jc;
      for (int e = tid; e < bsz * wc; e += nt) {
        const int r = e / wc, c = jc + (e - r * wc);
        const double pc = prow[c];
        M[r * w2 + c] = r == pr ? pc / pv : M[r * w2 + c] - fac[r] * pc;
      }
      __syncthreads();
    }
    // Dinv_K (row jc of the inverse sits in the row that pivoted column jc), kept in Lt for W
    for (int e = tid; e < B2i; e += nt) {
      const int jr = e / bsz, c = e % bsz;
      const double v = M[colmap[jr] * w2 + bsz + c];
      dinv[K * B2 + e] = v;
      Lt[e] = v;
    }
    __syncthreads();
    if (K < nsb - 1) {
      tile_gemm(bsz, Lt, Ut, Wp, 1.0);   // W_K = Dinv_K U_K
      __syncthreads();
      for (int e = tid; e < B2i; e += nt) w[K * B2 + e] = Wp[e];
    }
    __syncthreads();
  }
}

// Explicit inverse from the block factors, one workgroup per (column super-block
// Kc, slice): the columns of block Kc solve A X = E_Kc.  Forward: Y_K = 0 (K < Kc),
// Y_Kc = Dinv_Kc, Y_K = -Dinv_K L_K Y_{K-1}; backward: X_K = Y_K - W_K X_{K+1}.
// Block products run on LDS tiles; Y blocks go through a global scratch.
// The result is written in dof order, column-major: AinvS[b][j][i].
template <class S>
__global__ void __launch_bounds__(CF_THREADS) k_coarse_inverse(Geom g, int bsz, int nsb, const double* __restrict__ Dinv,
                                                        const double* __restrict__ W, const double* __restrict__ Lb,
                                                        double* __restrict__ Ysc, S* __restrict__ AinvS,
                                                        const int* __restrict__ active) {
  extern __shared__ double lds[];
  const int Kc = blockIdx.x, bs = blockIdx.y;
  if (active && !active[bs]) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int B2i = bsz * bsz;
  const size_t B2 = (size_t)B2i;
  double* At = lds;
  double* Y = At + B2i;
  double* T = Y + B2i;
  const double* dinv = Dinv + (size_t)bs * nsb * B2;
  const double* w = W + (size_t)bs * nsb * B2;
  const double* lb = Lb + (size_t)bs * nsb * B2;
  double* ys = Ysc + ((size_t)bs * nsb + Kc) * nsb * B2;
  const int n0 = g.nn * D2::NC;
  S* out = AinvS + (size_t)bs * n0 * n0;
  for (int e = tid; e < B2i; e += nt) { Y[e] = dinv[Kc * B2 + e]; ys[Kc * B2 + e] = Y[e]; }
  __syncthreads();
  for (int K = Kc + 1; K < nsb; ++K) {
    for (int e = tid; e < B2i; e += nt) At[e] = lb[K * B2 + e];
    __syncthreads();
    tile_gemm(bsz, At, Y, T, 1.0);          // T = L_K Y_{K-1}
    __syncthreads();
    for (int e = tid; e < B2i; e += nt) At[e] = dinv[K * B2 + e];
    __syncthreads();
    tile_gemm(bsz, At, T, Y, -1.0);         // Y_K = -Dinv_K T
    __syncthreads();
    for (int e = tid; e < B2i; e += nt) ys[K * B2 + e] = Y[e];
    __syncthreads();
  }
  // backward: Y holds X_{nsb-1}
  for (int K = nsb - 1; K >= 0; --K) {
    if (K < nsb - 1) {
      for (int e = tid; e < B2i; e += nt) At[e] = w[K * B2 + e];
      __syncthreads();
      tile_gemm(bsz, At, Y, T, 1.0);        // T = W_K X_{K+1}
      __syncthreads();
      for (int e = tid; e < B2i; e += nt) Y[e] = (K >= Kc ? ys[K * B2 + e] : 0.0) - T[e];
      __syncthreads();
    }
    for (int e = tid; e < B2i; e += nt) {
      const int l = e / bsz, c = e % bsz;
      const int i = coarse_gidx(g, K, l), j = coarse_gidx(g, Kc, c);
      if (i >= 0 && j >= 0) out[(size_t)j * n0 + i] = (S)Y[e];
    }
    __syncthreads();
  }
}

// x = A^{-1} b on the coarsest level: a block owns 64 rows; its waves split
// the columns (coalesced column-major reads) and reduce through LDS.
template <class S>
__global__ void __launch_bounds__(CG_THREADS) k_coarse_gemv(Geom g, const S* __restrict__ AinvS,
                                                            const S* __restrict__ bvec, S* __restrict__ xvec,
                                                            const int* __restrict__ active) {
  // 64 rows per block; wave w takes the columns j = w (mod CG_WAVES) with four
  // independent partial sums, so each lane keeps four loads in flight
  constexpr int W = CG_THREADS / 64;
  const int bs = blockIdx.y;
  if (active && !active[bs]) return;
  const int n0 = g.nn * D2::NC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  __shared__ S part[W][64];
  const S* bb = bvec + (size_t)bs * n0;
  const S* A = AinvS + (size_t)bs * n0 * n0;
  S a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (i < n0) {
    int j = wv;
    for (; j + 3 * W < n0; j += 4 * W) {
      a0 += A[(size_t)j * n0 + i] * bb[j];
      a1 += A[(size_t)(j + W) * n0 + i] * bb[j + W];
      a2 += A[(size_t)(j + 2 * W) * n0 + i] * bb[j + 2 * W];
      a3 += A[(size_t)(j + 3 * W) * n0 + i] * bb[j + 3 * W];
    }
    for (; j < n0; j += W) a0 += A[(size_t)j * n0 + i] * bb[j];
  }
  part[wv][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (wv == 0 && i < n0) {
    S x = part[0][lane];
#pragma unroll
    for (int w = 1; w < W; ++w) x += part[w][lane];
    xvec[(size_t)bs * n0 + i] = x;
  }
}

// ------------------------------------------------------------ FGMRES pieces
__device__ inline double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// partial[b][i][chunk] = sum over the chunk of X[b] . Y_i[b] for i < nv (nv <= 64):
// every thread accumulates all nv products of its elements in one pass, then a
// wave-shuffle and an LDS stage reduce them (fixed order, deterministic).
template <class S>
__global__ void __launch_bounds__(RED_T) k_multidot(int n, int nv, const S* __restrict__ X, size_t sxb,
                                                    const S* __restrict__ Y, size_t syb, size_t syi, int chunk,
                                                    double* __restrict__ partial, int nchunk,
                                                    const int* __restrict__ active) {
  __shared__ double sh[RED_T / 64][64];
  const int b = blockIdx.y, ch = blockIdx.x;
  if (active && !active[b]) return;
  const int lo = ch * chunk, hi = min(n, lo + chunk);
  const S* x = X + b * sxb;
  const S* yb = Y + b * syb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = 0; i0 < nv; i0 += 8) {
    const int m = min(8, nv - i0);
    S acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const S xv = x[e];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < m) acc[q] += xv * yb[(size_t)(i0 + q) * syi + e];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double v = (double)acc[q];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0 && q < m) sh[wv][i0 + q] = v;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < RED_T / 64; ++w) s += sh[w][i];
    partial[((size_t)b * 64 + i) * nchunk + ch] = s;
  }
}

// out[b][i] = sum over chunks of partial[b][i][*] (fixed order)
__global__ void k_reduce_partials(int nv, int nchunk, const double* __restrict__ partial, double* __restrict__ out,
                                  int ostride, const int* __restrict__ active) {
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += partial[((size_t)b * 64 + i) * nchunk + c];
    out[(size_t)b * ostride + i] = s;
  }
}

// X[b] -= sum_{i<nv} h[b][i] Y_i[b]
template <class S>
__global__ void k_multiaxpy(int n, int nv, S* __restrict__ X, size_t sxb, const S* __restrict__ Y, size_t syb,
                            size_t syi, const double* __restrict__ h, int hstride, double sign,
                            const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  S acc = X[b * sxb + e];
  for (int i = 0; i < nv; ++i) acc += (S)(sign * h[(size_t)b * hstride + i]) * Y[b * syb + i * syi + e];
  X[b * sxb + e] = acc;
}

// Y[b] = alpha[b] X[b]  (alpha per slice, from a device array with a stride)
template <class S>
__global__ void k_scale(int n, const S* __restrict__ X, size_t sxb, S* __restrict__ Y, size_t syb,
                        const double* __restrict__ alpha, int astride, int invert_sqrt,
                        const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double a = 1.0;   // mode 2: plain copy
  if (invert_sqrt == 0) a = alpha[(size_t)b * astride];
  if (invert_sqrt == 1) { a = alpha[(size_t)b * astride]; a = a > 0.0 ? 1.0 / sqrt(a) : 0.0; }
  Y[b * syb + e] = (S)(a * (double)X[b * sxb + e]);
}

// Y[b] = X[b] / D[b]  (undo the row scaling: preconditioner input)
template <class S>
__global__ void k_unscale(int n, const S* __restrict__ X, size_t sxb, const double* __restrict__ D, S* __restrict__ Y,
                          const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  Y[(size_t)b * n + e] = (S)((double)X[b * sxb + e] / D[(size_t)b * n + e]);
}

// Y[b] = D[b] * X[b] (scaled right-hand side), X double
template <class S>
__global__ void k_scale_rhs(int n, const double* __restrict__ X, const double* __restrict__ D, S* __restrict__ Y,
                            size_t syb, const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double d = D ? D[(size_t)b * n + e] : 1.0;
  Y[b * syb + e] = (S)(-X[(size_t)b * n + e] * d);
}

// Start of an FGMRES cycle: beta = ||r||, g = (beta, 0, ...), state and column count.
__global__ void k_init_cycle(int R, int cycle, const double* __restrict__ beta2, double* __restrict__ beta0,
                             double* __restrict__ gv, int* __restrict__ state, int* __restrict__ ncol,
                             const double* __restrict__ tolv, const int* __restrict__ gact, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  ncol[b] = 0;
  if (!gact[b]) { state[b] = 1; return; }
  const double beta = sqrt(fmax(beta2[b], 0.0));
  if (cycle == 0) beta0[b] = beta;
  for (int i = 0; i <= R; ++i) gv[(size_t)b * (R + 1) + i] = 0.0;
  gv[(size_t)b * (R + 1)] = beta;
  state[b] = (beta <= tolv[b] * beta0[b] || beta == 0.0) ? 1 : 0;
}

// hcol[b][i] += hcol2[b][i] (i <= j); hcol[b][j+1] = ||w||^2
__global__ void k_cgs_combine(int j, double* __restrict__ hcol, const double* __restrict__ hcol2,
                              const double* __restrict__ hn2, const int* __restrict__ active, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || (active && !active[b])) return;
  for (int i = 0; i <= j; ++i) hcol[(size_t)b * 64 + i] += hcol2[(size_t)b * 64 + i];
  hcol[(size_t)b * 64 + j + 1] = hn2[b];
}

// gact[b] = nact[b] && state[b] == 0 (gact = nact without state), and the working
// slices in order: ord[q] = index of the q-th slice with gact set, -1 from their
// count on.  Launches with the slices as the fast grid dimension take their slice
// from ord (slice_fast = 2), so the working slices fill the first grid columns and
// their blocks spread evenly over the XCDs (consecutive blocks go to consecutive
// XCDs); with the flags, converged slices leave their XCDs' share of the launch
// idle while the others still hold whole slices.  With hout (pinned host memory)
// set, also hout[b] = state[b], so the host reads the states once the launch has
// finished without a separate copy.  One wave.
__global__ void k_update_gact(const int* __restrict__ nact, const int* __restrict__ state, int* __restrict__ gact,
                              int* __restrict__ ord, int B, int* hout) {
  const int lane = threadIdx.x;
  int base = 0;
  for (int b0 = 0; b0 < B; b0 += 64) {
    const int b = b0 + lane;
    int f = 0;
    if (b < B) {
      const int s = state ? state[b] : 0;
      f = (nact[b] && s == 0) ? 1 : 0;
      gact[b] = f;
      if (hout) hout[b] = s;
    }
    const unsigned long long m = __ballot(f);
    if (f) ord[base + __popcll(m & ((1ull << lane) - 1ull))] = b;
    base += __popcll(m);
  }
  for (int q = base + lane; q < B; q += 64) ord[q] = -1;
}

// Arnoldi bookkeeping for column j of every active slice: Hcol = h (j+2 entries,
// the last one the squared norm of w after orthogonalisation), apply the stored
// Givens rotations, create a new one, update g and the residual estimate.
// state[b]: 0 running, 1 converged, 2 breakdown.
__global__ void k_givens(int j, int R, double* __restrict__ H, const double* __restrict__ hcol,
                         double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ gv,
                         double* __restrict__ res, const double* __restrict__ beta0, const double* __restrict__ tolv,
                         int* __restrict__ state, int* __restrict__ ncol, const int* __restrict__ active, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if ((active && !active[b]) || state[b] != 0) return;
  ncol[b] = j + 1;
  double* h = H + (size_t)b * (R + 1) * R;   // column-major: h[i + (R+1) j]
  for (int i = 0; i <= j; ++i) h[i + (R + 1) * j] = hcol[(size_t)b * 64 + i];
  double hn = sqrt(fmax(hcol[(size_t)b * 64 + j + 1], 0.0));
  h[j + 1 + (R + 1) * j] = hn;
  for (int i = 0; i < j; ++i) {
    const double c = cs[(size_t)b * R + i], s = sn[(size_t)b * R + i];
    const double a = h[i + (R + 1) * j], bb = h[i + 1 + (R + 1) * j];
    h[i + (R + 1) * j] = c * a + s * bb;
    h[i + 1 + (R + 1) * j] = -s * a + c * bb;
  }
  const double a = h[j + (R + 1) * j], bb = h[j + 1 + (R + 1) * j];
  const double r = hypot(a, bb);
  const double c = r > 0 ? a / r : 1.0, s = r > 0 ? bb / r : 0.0;
  cs[(size_t)b * R + j] = c;
  sn[(size_t)b * R + j] = s;
  h[j + (R + 1) * j] = r;
  h[j + 1 + (R + 1) * j] = 0.0;
  const double gj = gv[(size_t)b * (R + 1) + j];
  gv[(size_t)b * (R + 1) + j] = c * gj;
  gv[(size_t)b * (R + 1) + j + 1] = -s * gj;
  res[b] = fabs(gv[(size_t)b * (R + 1) + j + 1]);
  if (res[b] <= tolv[b] * beta0[b]) state[b] = 1;
  else if (hn <= 1e-300) state[b] = 2;
}

// Solve the (jmax x jmax) triangular system of each slice: y = H^{-1} g,
// using its own column count ncol[b].
__global__ void k_trisolve(int R, const double* __restrict__ H, const double* __restrict__ gv,
                           const int* __restrict__ ncol, double* __restrict__ y, const int* __restrict__ active,
                           int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (active && !active[b]) return;
  const int m = ncol[b];
  const double* h = H + (size_t)b * (R + 1) * R;
  double* yy = y + (size_t)b * 64;
  for (int i = 0; i < 64; ++i) yy[i] = 0.0;
  for (int i = m - 1; i >= 0; --i) {
    double s = gv[(size_t)b * (R + 1) + i];
    for (int q = i + 1; q < m; ++q) s -= h[i + (R + 1) * q] * yy[q];
    const double d = h[i + (R + 1) * i];
    yy[i] = d != 0.0 ? s / d : 0.0;
  }
}

// ------------------------------------------------------------ Newton update
// U[b] += dx[b] (on active slices), then per-slice maxima of |dx| and |U| per
// field (v, u, p) into part[b][6][chunk].
template <int D, class S>
__global__ void __launch_bounds__(RED_T) k_newton_update(int nn, double* __restrict__ U, const S* __restrict__ dx,
                                                         int chunk, double* __restrict__ part, int nchunk,
                                                         const int* __restrict__ active) {
  FSI_DIM(D);
  __shared__ double sh[RED_T];
  const int b = blockIdx.y, ch = blockIdx.x;
  if (active && !active[b]) return;
  const int lo = ch * chunk, hi = min(nn, lo + chunk);
  double m[6] = {0, 0, 0, 0, 0, 0};
  for (int n = lo + threadIdx.x; n < hi; n += blockDim.x) {
    double* u = U + ((size_t)b * nn + n) * NC;
    const S* d = dx + ((size_t)b * nn + n) * NC;
    for (int c = 0; c < NC; ++c) {
      const double dv = (double)d[c];
      const double un = u[c] + dv;
      u[c] = un;
      const int f = c < D ? 0 : (c < 2 * D ? 1 : 2);
      m[f] = fmax(m[f], fabs(dv));
      m[3 + f] = fmax(m[3 + f], fabs(un));
      if (!isfinite(un)) m[f] = INFINITY;
    }
  }
  for (int q = 0; q < 6; ++q) {
    const int t = threadIdx.x;
    sh[t] = m[q];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
      __syncthreads();
    }
    if (t == 0) part[((size_t)b * 6 + q) * nchunk + ch] = sh[0];
    __syncthreads();
  }
}

// max over chunks -> out[b][6]
// Newton's residual test: per slice b and field f (v, u, p), partial maxima of
// |Dsc R| (q = f) and of |U| (q = 3 + f) over chunks of nodes -> part[b][q][chunk]
// (Dsc = row scaling 1 / max_j |J_ij| of the last assembly); non-finite R gives infinity.
template <int D>
__global__ void __launch_bounds__(RED_T) k_residual_norms(int nn, const double* __restrict__ R,
                                                          const double* __restrict__ Dsc,
                                                          const double* __restrict__ U, int chunk,
                                                          double* __restrict__ part, int nchunk,
                                                          const int* __restrict__ active) {
  FSI_DIM(D);
  __shared__ double sh[RED_T];
  const int b = blockIdx.y, ch = blockIdx.x;
  if (active && !active[b]) return;
  const int lo = ch * chunk, hi = min(nn, lo + chunk);
  double m[6] = {0, 0, 0, 0, 0, 0};
  for (int n = lo + threadIdx.x; n < hi; n += blockDim.x) {
    const size_t o = ((size_t)b * nn + n) * NC;
    for (int c = 0; c < NC; ++c) {
      const double r = Dsc[o + c] * R[o + c];
      const int f = c < D ? 0 : (c < 2 * D ? 1 : 2);
      m[f] = isfinite(r) ? fmax(m[f], fabs(r)) : INFINITY;
      m[3 + f] = fmax(m[3 + f], fabs(U[o + c]));
    }
  }
  for (int q = 0; q < 6; ++q) {
    const int t = threadIdx.x;
    sh[t] = m[q];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
      __syncthreads();
    }
    if (t == 0) part[((size_t)b * 6 + q) * nchunk + ch] = sh[0];
    __syncthreads();
  }
}

__global__ void k_max_partials(int nchunk, const double* __restrict__ part, double* __restrict__ out, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  for (int q = 0; q < 6; ++q) {
    double m = 0.0;
    for (int c = 0; c < nchunk; ++c) m = fmax(m, part[((size_t)b * 6 + q) * nchunk + c]);
    out[(size_t)b * 6 + q] = m;
  }
}

// Parareal correction of one boundary, FP64: out = th Cn + Fv - th Cold
// (eq. (parareal:iteration) for th = 1, eq. (thetaparareal:iteration) otherwise).
__global__ void k_parareal_update(size_t n, const double* __restrict__ Cn, const double* __restrict__ Fv,
                                  const double* __restrict__ Cold, double* __restrict__ out, double th) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    out[e] = th * Cn[e] + Fv[e] - th * Cold[e];
}

// Per boundary b: sums of squares of (A - B) and of A for the velocity and the
// displacement components -> part[b][4][chunk].
template <int D>
__global__ void __launch_bounds__(RED_T) k_change_norms(int nn, const double* __restrict__ A,
                                                        const double* __restrict__ Bv, int chunk,
                                                        double* __restrict__ part, int nchunk) {
  FSI_DIM(D);
  __shared__ double sh[RED_T];
  const int b = blockIdx.y, ch = blockIdx.x;
  const int lo = ch * chunk, hi = min(nn, lo + chunk);
  double s[4] = {0, 0, 0, 0};
  for (int n = lo + threadIdx.x; n < hi; n += blockDim.x) {
    const double* a = A + ((size_t)b * nn + n) * NC;
    const double* o = Bv + ((size_t)b * nn + n) * NC;
    for (int c = 0; c < 2 * D; ++c) {
      const double d = a[c] - o[c];
      const int f = c < D ? 0 : 1;
      s[2 * f] += d * d;
      s[2 * f + 1] += a[c] * a[c];
    }
  }
  for (int q = 0; q < 4; ++q) {
    const double r = block_sum(s[q], sh);
    if (threadIdx.x == 0) part[((size_t)b * 4 + q) * nchunk + ch] = r;
  }
}

// theta-Parareal inner products: per velocity/displacement component c, the
// chunk sums of F_c F_c, F_c C_c and C_c C_c -> part[3 c + {0, 1, 2}][chunk].
template <int D>
__global__ void __launch_bounds__(RED_T) k_theta_dots(int nn, const double* __restrict__ F,
                                                      const double* __restrict__ Cv, int chunk,
                                                      double* __restrict__ part, int nchunk) {
  FSI_DIM(D);
  __shared__ double sh[RED_T];
  const int ch = blockIdx.x;
  const int lo = ch * chunk, hi = min(nn, lo + chunk);
  double s[3 * 2 * D];
  for (int q = 0; q < 3 * 2 * D; ++q) s[q] = 0.0;
  for (int n = lo + threadIdx.x; n < hi; n += blockDim.x)
    for (int c = 0; c < 2 * D; ++c) {
      const double f = F[(size_t)n * NC + c], g = Cv[(size_t)n * NC + c];
      s[3 * c] += f * f;
      s[3 * c + 1] += f * g;
      s[3 * c + 2] += g * g;
    }
  for (int q = 0; q < 3 * 2 * D; ++q) {
    const double r = block_sum(s[q], sh);
    if (threadIdx.x == 0) part[(size_t)q * nchunk + ch] = r;
  }
}

// Newton initial guess of step n: the polynomial of degree q (1 to 3) through the
// states at t_{n-1}, ..., t_{n-1-q} (equal steps) evaluated at t_n, i.e. the
// binomial weights U = sum_j (-1)^j C(q+1, j+1) U^{n-1-j}:
//   q = 1: 2 U^{n-1} - U^{n-2};  q = 2: 3 U^{n-1} - 3 U^{n-2} + U^{n-3};
//   q = 3: 4 U^{n-1} - 6 U^{n-2} + 4 U^{n-3} - U^{n-4}.
__global__ void k_extrapolate(size_t n, int q, double* __restrict__ U, const double* __restrict__ U1,
                              const double* __restrict__ U2, const double* __restrict__ U3,
                              const double* __restrict__ U4, const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t o = (size_t)b * n + e;
    double u;
    if (q == 1)
      u = 2.0 * U1[o] - U2[o];
    else if (q == 2)
      u = 3.0 * (U1[o] - U2[o]) + U3[o];
    else
      u = 4.0 * (U1[o] + U3[o]) - 6.0 * U2[o] - U4[o];
    U[o] = u;
  }
}

// flag[b] = 1 if any entry of X[b] is not finite
__global__ void k_nonfinite(size_t n, const double* __restrict__ X, int* __restrict__ flag) {
  const int b = blockIdx.y;
  for (size_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(X[(size_t)b * n + e])) flag[b] = 1;
}

template <class S>
__global__ void k_fill(size_t n, S* __restrict__ X, S v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) X[e] = v;
}

template <class A, class B2>
__global__ void k_convert(size_t n, const A* __restrict__ X, B2* __restrict__ Y) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    Y[e] = (B2)X[e];
}

// explicit instantiations
#define FSI_INST_DS(D, S)                                                                                         \
  template __global__ void k_spmv<D, S, true>(Geom, double, const S*, const S*, const S*, const double*, S*,     \
                                              const int*, int);                                                  \
  template __global__ void k_restrict<D, S>(Geom, Geom, const S*, S*, const int*);                               \
  template __global__ void k_prolong_add<D, S>(Geom, Geom, const S*, S*, const int*);                            \
  template __global__ void k_newton_update<D, S>(int, double*, const S*, int, double*, int, const int*);
#define FSI_INST_S(S)                                                                                             \
  FSI_INST_DS(2, S)                                                                                               \
  FSI_INST_DS(3, S)                                                                                               \
  template __global__ void k_coarse_factor<S, true>(Geom, double, const S*, int, int, double*, double*, double*, \
                                                    const int*);                                                 \
  template __global__ void k_coarse_inverse<S>(Geom, int, int, const double*, const double*, const double*,      \
                                               double*, S*, const int*);                                          \
  template __global__ void k_coarse_gemv<S>(Geom, const S*, const S*, S*, const int*);                           \
  template __global__ void k_multidot<S>(int, int, const S*, size_t, const S*, size_t, size_t, int, double*, int, \
                                         const int*);                                                            \
  template __global__ void k_multiaxpy<S>(int, int, S*, size_t, const S*, size_t, size_t, const double*, int,    \
                                          double, const int*);                                                   \
  template __global__ void k_scale<S>(int, const S*, size_t, S*, size_t, const double*, int, int, const int*);   \
  template __global__ void k_unscale<S>(int, const S*, size_t, const double*, S*, const int*);                   \
  template __global__ void k_scale_rhs<S>(int, const double*, const double*, S*, size_t, const int*);            \
  template __global__ void k_fill<S>(size_t, S*, S);
FSI_INST_S(double)
FSI_INST_S(float)
// full-layout operators of the (2d, FP64) transposed adjoint system
template __global__ void k_spmv<2, double, false>(Geom, double, const double*, const double*, const double*,
                                                  const double*, double*, const int*, int);
template __global__ void k_coarse_factor<double, false>(Geom, double, const double*, int, int, double*, double*,
                                                        double*, const int*);
template __global__ void k_residual_norms<2>(int, const double*, const double*, const double*, int, double*, int,
                                             const int*);
template __global__ void k_residual_norms<3>(int, const double*, const double*, const double*, int, double*, int,
                                             const int*);
template __global__ void k_change_norms<2>(int, const double*, const double*, int, double*, int);
template __global__ void k_change_norms<3>(int, const double*, const double*, int, double*, int);
template __global__ void k_theta_dots<2>(int, const double*, const double*, int, double*, int);
template __global__ void k_theta_dots<3>(int, const double*, const double*, int, double*, int);
template __global__ void k_transpose_J<double>(Geom, double, const double*, double*, double*);
template __global__ void k_spmv_T<double>(Geom, double, const double*, const double*, double*, int);
template __global__ void k_convert<double, float>(size_t, const double*, float*);
template __global__ void k_convert<float, double>(size_t, const float*, double*);
template __global__ void k_convert<double, double>(size_t, const double*, double*);
template __global__ void k_convert<float, float>(size_t, const float*, float*);

}  // namespace fsi
