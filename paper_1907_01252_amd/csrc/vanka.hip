// The fused colored multiplicative Vanka pass: patch residuals from the block
// stencil and the patch update in one kernel (the patch inverses it applies
// are formed in vanka_factor.hip).  The kernel takes the slice index from
// blockIdx.y (blockIdx.x when slice_fast is set, the slices then being the
// fast grid dimension) and skips slices whose active flag is 0; with
// slice_fast = 2 active lists the working slices in order and blockIdx.x
// indexes that list (-1: nothing to do).  S is the
// storage type of the linear solve, D the space dimension, CJ the Jacobian
// block layout.
#include "stencil.h"

namespace fsi {

// ------------------------------------------------------ colored Vanka pass
// One multiplicative pass over the cells of one colour, residual and patch
// update fused: every cell P of the colour forms r_P = b_P - (A x_old)_P on its
// nodes and writes x_new[P] = x_old[P] + omega Ainv_P r_P.  The cells of one
// colour do not share nodes, so each node is written by at most one patch;
// the nodes no patch of the colour covers are copied.  x_old and x_new are
// different buffers (other patches read x_old at the shared neighbours).
// zero_in: x_old is taken as zero (first pass of a cycle): r_P = b_P and the
// uncovered nodes get zero.
// Thread mapping: a block of VC consecutive cells of the colour has NC waves,
// wave r forming row r of every patch node.  A lane group of 2 VC lanes takes
// one node pair (a, a + 1) of the VC cells, so within one cell row a wave
// reads runs of 2 VC consecutive nodes and the inverses in VC-cell runs.
// 2d uses VC = 16 (two groups: pairs (0,1) and (2,3)).  3d uses VC = 32 on
// large levels (one group; each thread loops over the four pairs) and VC = 8
// on small ones (four groups, one pair each: more blocks for few cells).  The
// NE patch residuals meet in LDS; the same thread then forms patch rows
// NC a + r of Ainv_P r_P.  Extra blocks past the patch blocks copy the
// uncovered nodes.
//
// Minimum waves per SIMD requested for the fused pass: in 2d FP32 the register
// budget of 6 waves (85 VGPRs) keeps enough waves resident to hide latency; in 2d
// FP64 4 waves with the compressed Jacobian (128 VGPRs: three blocks of five waves per CU;
// the full-layout variant of the transposed adjoint operator keeps the compiler's choice).
template <int D, class S, bool CJ>
constexpr int vanka_waves_per_simd() {
  return D == 2 ? (sizeof(S) == 4 ? 6 : (CJ ? 4 : 1)) : 1;
}
template <int D, class S, int VC, bool CJ>
__global__ void __launch_bounds__(Dm<D>::NC * 64, (vanka_waves_per_simd<D, S, CJ>()))
    k_vanka_color(Geom g, double k, int color, S omega, int zero_in,
                                                                const S* __restrict__ J, const S* __restrict__ Ainv,
                                                                const S* __restrict__ Yu,
                                                                const S* __restrict__ b, const S* __restrict__ xo,
                                                                S* __restrict__ xn, const int* __restrict__ active,
                                                                int slice_fast) {
  FSI_DIM(D);
  static_assert(VC == 8 || VC == 16 || VC == 32, "cells per block");
  // the pressure-stabilisation row of a node is spread over the D
  // displacement-row waves, which have the fewest block-stencil loads (in 2d
  // FP64 the pressure wave keeps it: measured as fast, and one barrier fewer)
  constexpr bool SPLIT = !(D == 2 && sizeof(S) == 8);
  __shared__ S rs[NE][VC];
  __shared__ S pp[SPLIT ? NL : 1][D][VC];   // parts of the pressure rows' stabilisation terms
  // staged x around the block's nodes: all components within one node (box
  // RX1 x RY1 x RZ1), the pressure within two (box RX2 x RY2 x RZ2)
  constexpr int RX1 = 2 * VC + 2, RY1 = 4, RZ1 = D == 3 ? 4 : 1;
  constexpr int RX2 = 2 * VC + 4, RY2 = 6, RZ2 = D == 3 ? 6 : 1;
  __shared__ S xr[RX1 * RY1 * RZ1 * NC];
  __shared__ S pr[RX2 * RY2 * RZ2];
  constexpr bool SP = patch_split<D, S, CJ>();   // split patch solve (see ainv_rows)
  __shared__ S dv[SP ? NL * D : 1][VC];        // velocity part of the patch update
  // 2d FP64 split solve: the displacement-row waves, which have the fewest stencil loads,
  // copy the block's inverse rows (one contiguous region) to LDS while the other waves
  // load the Jacobian, so the inverse is not fetched only after the residual barrier
  // (in 2d FP32 those waves also form the pressure stabilisation, and the copy made
  // the 256x64-cell pass 1.6 times slower)
  constexpr bool AL = D == 2 && SP && sizeof(S) == 8;
  constexpr int NR = ainv_rows<D, SP>();
  __shared__ S ainvL[AL ? NR * NE * VC : 1];
  // slice_fast = 2: active is the ordered list of working slices (k_update_gact)
  const int bs = slice_fast == 2 ? active[blockIdx.x] : (slice_fast ? blockIdx.x : blockIdx.y);
  const int bx = slice_fast ? blockIdx.y : blockIdx.x;
  if (slice_fast == 2 ? bs < 0 : (active && !active[bs])) return;   // uniform over the block
  const ColorInfo L = color_info<D>(g, color, VC);
  const int nc = L.nc;
  const int npb = (nc + VC - 1) / VC;
  const S* xob = xo + (size_t)bs * g.nn * NC;
  S* xnb = xn + (size_t)bs * g.nn * NC;
  const int cx = color & 1, cy = (color >> 1) & 1, cz = (color >> 2) & 1;
  if (bx >= npb) {
    const int t = (bx - npb) * (NC * 64) + threadIdx.x;
    if (t >= g.nn) return;
    int ni, nj, nk;
    node_ijk<D>(g, t, ni, nj, nk);
    const int ci = ni - ((ni - cx) & 1), cj = nj - ((nj - cy) & 1), ck = nk - ((nk - cz) & 1);
    const bool covered = ci >= 0 && cj >= 0 && ci < g.nx && cj < g.ny && (D == 2 || (ck >= 0 && ck < g.nz));
    if (!covered)
      for (int c = 0; c < NC; ++c) xnb[(size_t)t * NC + c] = zero_in ? (S)0 : xob[(size_t)t * NC + c];
    return;
  }
  // lane -> (cell jc of the block, node-pair group gp); the G = 64 / (2 VC)
  // groups of a wave take the node pairs (2 gp, 2 gp + 1), and each thread
  // loops over the NQ = NL / (2 G) pairs gp + G q
  const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int G = 64 / (2 * VC), NQ = NL / (2 * G), QS = 2 * G;
  const int jc = (lane % (2 * VC)) >> 1;
  const int a0 = (lane & 1) + 2 * (lane / (2 * VC));
  const int idx = bx * VC + jc;
  const bool live = idx < nc;
  // The block's cells lie in one cell row when the colour's rows hold whole
  // blocks: then the x values its stencils read are staged in LDS once
  // (block-uniform), instead of every wave loading every neighbour's vector.
  const bool stage = !zero_in && L.ncx % VC == 0;
  int X1 = 0, Y1 = 0, Z1 = 0;
  if (stage) {
    const int idx0 = bx * VC, rest0 = idx0 / L.ncx;
    X1 = 2 * (idx0 % L.ncx) + cx - 1;
    Y1 = 2 * (rest0 % L.ncy) + cy - 1;
    Z1 = D == 3 ? 2 * (rest0 / L.ncy) + cz - 1 : 0;
    const int W = g.nx + 1, P = W * (g.ny + 1);
    for (int e = threadIdx.x; e < RX1 * RY1 * RZ1 * NC; e += NC * 64) {
      const int c = e % NC, t = e / NC;
      const int gx = min(max(X1 + t % RX1, 0), g.nx), gy = min(max(Y1 + (t / RX1) % RY1, 0), g.ny);
      const int gz = D == 3 ? min(max(Z1 + t / (RX1 * RY1), 0), g.nz) : 0;
      xr[e] = xob[(size_t)(gx + W * gy + P * gz) * NC + c];
    }
    for (int e = threadIdx.x; e < RX2 * RY2 * RZ2; e += NC * 64) {
      const int gx = min(max(X1 - 1 + e % RX2, 0), g.nx), gy = min(max(Y1 - 1 + (e / RX2) % RY2, 0), g.ny);
      const int gz = D == 3 ? min(max(Z1 - 1 + e / (RX2 * RY2), 0), g.nz) : 0;
      pr[e] = xob[(size_t)(gx + W * gy + P * gz) * NC + PC];
    }
    __syncthreads();
  }
  if constexpr (AL) {
    if (r >= D && r < 2 * D) {
      // whole region of the block (colours are padded to whole blocks, so it is allocated)
      const S* src = Ainv + (size_t)bs * ainv_slice<D>(g.ncell) + ((size_t)L.off + (size_t)bx * VC) * NR * NE;
      constexpr int NT = D * 64, NV = NR * NE * VC / NT;
      static_assert(NR * NE * VC % NT == 0, "inverse region per copying thread");
      const int t0 = (r - D) * 64 + lane;
      constexpr int CH = 10;   // loads in flight per chunk (registers)
      static_assert(NV % CH == 0, "chunks");
#pragma unroll 1
      for (int q0 = 0; q0 < NV; q0 += CH) {
        S tmp[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) tmp[q] = src[t0 + (q0 + q) * NT];
#pragma unroll
        for (int q = 0; q < CH; ++q) ainvL[t0 + (q0 + q) * NT] = tmp[q];
      }
    }
  }
  int ci = 0, cj = 0, ck = 0;
  if (live) {
    const int ix = idx % L.ncx, rest = idx / L.ncx;
    ci = 2 * ix + cx;
    cj = 2 * (rest % L.ncy) + cy;
    ck = D == 3 ? 2 * (rest / L.ncy) + cz : 0;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      const int a = a0 + q * QS;
      const int n = node_at(g, ci + (a & 1), cj + ((a >> 1) & 1), ck + ((a >> 2) & 1));
      S acc = 0;
      if (!zero_in) {
        int i, j, kk;
        node_ijk<D>(g, n, i, j, kk);
        // (3d: the copy whose tiles start where this colour's node runs start)
        const S* jn = J + jslice_row<D, S, CJ>(g, bs, r) + jnode<D, S, CJ>(g, i, j + (g.ny + 1) * kk, cx);
        constexpr int NROW = D == 3 ? 25 : 5;
        const int part = r - D, p0 = part * NROW / D, p1 = (part + 1) * NROW / D;
        if (stage) {
          const int ln = (i - X1) + RX1 * ((j - Y1) + RY1 * (kk - Z1));
          acc = stencil_row<D, S, CJ>(jn, xr, ln, r, nbr_offsets<D>(g, i, j, kk, RX1, RX1 * RY1));
          if (!SPLIT && r == PC)
            acc += pst_rows_staged<D, S>(g, k, n, i, j, kk, pr, X1 - 1, Y1 - 1, Z1 - 1, RX2, RY2, 0, NROW);
          if (SPLIT && r >= D && r < 2 * D)
            pp[a][part][jc] = pst_rows_staged<D, S>(g, k, n, i, j, kk, pr, X1 - 1, Y1 - 1, Z1 - 1, RX2, RY2, p0, p1);
        } else {
          acc = stencil_row<D, S, CJ>(jn, xob, n, r, nbr_offsets<D>(g, i, j, kk));
          if (!SPLIT && r == PC) acc += pst_row<D, S>(g, k, n, i, j, kk, xob);
          if (SPLIT && r >= D && r < 2 * D) pp[a][part][jc] = pst_rows<D, S>(g, k, n, i, j, kk, xob, p0, p1);
        }
      }
      rs[NC * a + r][jc] = b[((size_t)bs * g.nn + n) * NC + r] - acc;
    }
  }
  __syncthreads();
  if (SPLIT && !zero_in) {   // uniform over the block: every thread meets the barrier
    if (live && r == PC) {
#pragma unroll 1
      for (int q = 0; q < NQ; ++q) {
        const int a = a0 + q * QS;
        S s = pp[a][0][jc];
        for (int part = 1; part < D; ++part) s += pp[a][part][jc];
        rs[NC * a + PC][jc] -= s;
      }
    }
    __syncthreads();
  }
  // patch update: rows of the stored inverse first (in the split solve the
  // non-displacement unknowns), then the displacements from Y1, Y2 and the
  // velocity update
  const bool urow = SP && r >= D && r < 2 * D;
  if (live && !urow) {
    const S* ai = AL ? ainvL + jc
                     : Ainv + (size_t)bs * ainv_slice<D>(g.ncell) + ((size_t)L.off + (size_t)bx * VC) * NR * NE + jc;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      const int a = a0 + q * QS;
      const int wr = ainv_row<D, SP>(a, r);
      S z = 0;
      constexpr int EU = NQ == 1 ? NE : 8;   // looping threads: bounded loads in flight (registers)
#pragma unroll EU
      for (int e = 0; e < NE; ++e) z += ai[(NE * wr + e) * VC] * rs[e][jc];
      if (SP && r < D) dv[D * a + r][jc] = z;
      const int n = node_at(g, ci + (a & 1), cj + ((a >> 1) & 1), ck + ((a >> 2) & 1));
      const size_t o = (size_t)n * NC + r;
      xnb[o] = (zero_in ? (S)0 : xob[o]) + omega * z;
    }
  }
  if constexpr (SP) {
    __syncthreads();   // every thread of the block: dv is complete
    if (live && urow) {
      const int i = r - D;
      const S* y1 = Yu + ((size_t)L.off + (size_t)bx * VC) * yu_cell<D>() + jc + (size_t)(2 * i) * NL * NL * VC;
      const S* y2 = y1 + (size_t)NL * NL * VC;
#pragma unroll 1
      for (int q = 0; q < NQ; ++q) {
        const int a = a0 + q * QS;
        S z = 0;
#pragma unroll
        for (int bb = 0; bb < NL; ++bb)
          z += y1[(NL * a + bb) * VC] * rs[NC * bb + r][jc] - y2[(NL * a + bb) * VC] * dv[D * bb + i][jc];
        const int n = node_at(g, ci + (a & 1), cj + ((a >> 1) & 1), ck + ((a >> 2) & 1));
        const size_t o = (size_t)n * NC + r;
        xnb[o] = (zero_in ? (S)0 : xob[o]) + omega * z;
      }
    }
  }
}

#define FSI_INST_VANKA(D, S)                                                                                      \
  template __global__ void k_vanka_color<D, S, (D == 2 ? 16 : 32), true>(Geom, double, int, S, int, const S*,   \
                                                                         const S*, const S*, const S*, const S*,  \
                                                                         S*, const int*, int);
FSI_INST_VANKA(2, double)
FSI_INST_VANKA(2, float)
FSI_INST_VANKA(3, double)
FSI_INST_VANKA(3, float)
template __global__ void k_vanka_color<3, double, 8, true>(Geom, double, int, double, int, const double*,
                                                           const double*, const double*, const double*,
                                                           const double*, double*, const int*, int);
template __global__ void k_vanka_color<3, float, 8, true>(Geom, double, int, float, int, const float*, const float*,
                                                          const float*, const float*, const float*, float*,
                                                          const int*, int);
// full-layout operators of the (2d, FP64) transposed adjoint system
template __global__ void k_vanka_color<2, double, 16, false>(Geom, double, int, double, int, const double*,
                                                             const double*, const double*, const double*,
                                                             const double*, double*, const int*, int);

}  // namespace fsi
