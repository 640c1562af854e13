// Vanka patch inverses: the NE x NE matrix of every cell patch, gathered from
// the block-stencil Jacobian (and the pressure stabilisation), inverted by
// Gauss-Jordan in LDS and stored by colour and block of the fused pass.
#include "stencil.h"

namespace fsi {

// ------------------------------------------------------- Vanka patch inverse
// One lane group (vf_lanes lanes) inverts the NE x NE patch matrix of one cell
// (rows = local unknowns NC a + c) by Gauss-Jordan with partial pivoting, in
// place and in registers: lane r holds row r.  Per column the pivot row is
// found by a shuffle reduction; the pivot lane scales its row and publishes it
// in LDS, and every other row eliminates the column with it.  Each step also
// rotates the rows left by one and appends the eliminated column, the column
// of the inverse that belongs to the pivot row, at the end, so that the column
// to eliminate is always entry 0 and every register index is static.  After NE
// steps entry j of a row is again column j; the lane that pivoted column m
// holds row m of the inverse, with column j of the pivot order at the place of
// the pivot row of column j.  Ainv is stored by colour and block of vc cells
// of the fused pass (ainv_slice in fsi_internal.h).
template <int D, class S, bool CJ>
__global__ void __launch_bounds__(vf_lanes<D>() * vf_patches<D>()) k_vanka_factor(Geom g, double k,
                                                                                  const S* __restrict__ J,
                                                                                  S* __restrict__ Ainv,
                                                                                  S* __restrict__ Yu, int vc,
                                                                                  const int* __restrict__ active) {
  FSI_DIM(D);
  constexpr int GL = vf_lanes<D>(), NP = vf_patches<D>();
  __shared__ double Q[2][NP][NE];   // published pivot row, one buffer per step parity
  __shared__ int colmap[NP][NE];    // pivot row of each column
  // [A_uu,i | A_uv,i | I] of every displacement component i (slice 0 only)
  constexpr bool SP = patch_split<D, S, CJ>();
  __shared__ double Mu[SP ? NP : 1][SP ? D : 1][SP ? NL : 1][SP ? 3 * NL : 1];
  const int bs = blockIdx.y;
  if (active && !active[bs]) return;   // uniform over the block
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int cell = blockIdx.x * NP + grp;
  const bool live = cell < g.ncell;
  int ci = 0, cj = 0, ck = 0;
  if (live) cell_ijk<D>(g, cell, ci, cj, ck);
  double row[NE];
#pragma unroll
  for (int c = 0; c < NE; ++c) row[c] = c == lane ? 1.0 : 0.0;
  if (live && lane < NE) {
    const int a = lane / NC, rc = lane % NC;
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const int na = node_at(g, ci + ax, cj + ay, ck + az);
    const S* jn = J + (size_t)bs * jslice<D, S, CJ>(g) + jnode_n<D, S, CJ>(g, na, 0);
    const bool pst_row = (rc == PC) && !(g.dmask[na] & dm_p<D>());
#pragma unroll
    for (int bb = 0; bb < NL; ++bb) {
      const int dx = (bb & 1) - ax, dy = ((bb >> 1) & 1) - ay, dz = ((bb >> 2) & 1) - az;
      const int s = slot_of<D>(dx, dy, dz);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int e = jentry<D, CJ>(rc, c);
        row[NC * bb + c] = e >= 0 ? (double)jn[jent<D, S, CJ>(s, e)] : 0.0;
      }
      if (pst_row) row[NC * bb + PC] += k * g.pst[(size_t)pslot_of<D>(dx, dy, dz) * g.nn + na];
    }
  }
  if constexpr (SP) {
    // Y1_i = A_uu,i^{-1} and Y2_i = Y1_i A_uv,i of the patch, the same in every
    // slice: slice 0 writes them (block-uniform branch)
    if (bs == 0) {
      const int rc = lane % NC, a = lane / NC;
      if (lane < NE && rc >= D && rc < 2 * D) {
        const int i = rc - D;
#pragma unroll
        for (int c = 0; c < NE; ++c) {
          const int cb = c / NC, cc = c % NC;
          if (cc == D + i) Mu[grp][i][a][cb] = row[c];
          else if (cc == i) Mu[grp][i][a][NL + cb] = row[c];
        }
        for (int b = 0; b < NL; ++b) Mu[grp][i][a][2 * NL + b] = a == b ? 1.0 : 0.0;
      }
      __syncthreads();
      if (lane < D) {
        // Gauss-Jordan with partial pivoting on the NL x 3 NL system of component lane
        double(*m)[3 * NL] = Mu[grp][lane];
#pragma unroll 1
        for (int pc = 0; pc < NL; ++pc) {
          int pr = pc;
#pragma unroll 1
          for (int rr = pc + 1; rr < NL; ++rr)
            if (fabs(m[rr][pc]) > fabs(m[pr][pc])) pr = rr;
          if (pr != pc)
#pragma unroll 1
            for (int c = 0; c < 3 * NL; ++c) {
              const double t = m[pc][c];
              m[pc][c] = m[pr][c];
              m[pr][c] = t;
            }
          const double inv = m[pc][pc] == 0.0 ? 1.0 : 1.0 / m[pc][pc];
#pragma unroll 1
          for (int c = 0; c < 3 * NL; ++c) m[pc][c] *= inv;
#pragma unroll 1
          for (int rr = 0; rr < NL; ++rr) {
            if (rr == pc) continue;
            const double f = m[rr][pc];
            if (f != 0.0)
#pragma unroll 1
              for (int c = 0; c < 3 * NL; ++c) m[rr][c] -= f * m[pc][c];
          }
        }
        if (live) {
          int col, idx;
          ColorInfo L;
          cell_colour<D>(g, ci, cj, ck, vc, col, idx, L);
          const int q = idx / vc, t = idx - q * vc;
          S* y = Yu + ((size_t)L.off + (size_t)q * vc) * yu_cell<D>() + t;
#pragma unroll 1
          for (int a2 = 0; a2 < NL; ++a2)
#pragma unroll 1
            for (int b = 0; b < NL; ++b) {
              y[(size_t)((2 * lane) * NL * NL + a2 * NL + b) * vc] = (S)m[a2][2 * NL + b];       // Y1
              y[(size_t)((2 * lane + 1) * NL * NL + a2 * NL + b) * vc] = (S)m[a2][NL + b];      // Y2
            }
        }
      }
    }
  }
  bool used = lane >= NE;
  int mycol = 0;
#pragma unroll 1
  for (int jc = 0; jc < NE; ++jc) {
    double v = row[0];
    double cand = used ? -1.0 : fabs(v);
    int idx = lane;
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
      const double oc = __shfl_xor(cand, off, GL);
      const int oi = __shfl_xor(idx, off, GL);
      if (oc > cand || (oc == cand && oi < idx)) { cand = oc; idx = oi; }
    }
    double* q = Q[jc & 1][grp];
    if (lane == idx) {
      // scaled pivot row in rotated order; this lane then takes it over as its
      // new row through the common update with a zero row and v = -1
      const double inv = v == 0.0 ? 1.0 : 1.0 / v;   // singular patch: no pivot for this column
#pragma unroll
      for (int c = 0; c + 1 < NE; ++c) { q[c] = row[c + 1] * inv; row[c + 1] = 0.0; }
      q[NE - 1] = inv;
      v = -1.0;
      used = true;
      mycol = jc;
      colmap[grp][jc] = lane;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c + 1 < NE; ++c) row[c] = fma(-v, q[c], row[c + 1]);
    row[NE - 1] = -v * q[NE - 1];
  }
  const int mrc = mycol % NC;
  if (live && lane < NE && !(SP && mrc >= D && mrc < 2 * D)) {
    // row mycol of the inverse: entry (mycol, pivot row of j) is held in entry j
    // (in the split patch solve only the rows of the non-displacement unknowns are stored)
    int col, idx;
    ColorInfo L;
    cell_colour<D>(g, ci, cj, ck, vc, col, idx, L);
    const int q = idx / vc, t = idx - q * vc;
    constexpr int NR = ainv_rows<D, SP>();
    const int wr = ainv_row<D, SP>(mycol / NC, mrc);
    S* out = Ainv + (size_t)bs * ainv_slice<D>(g.ncell) + ((size_t)L.off + (size_t)q * vc) * NR * NE + t;
#pragma unroll
    for (int j = 0; j < NE; ++j) out[(size_t)(NE * wr + colmap[grp][j]) * vc] = (S)row[j];
  }
}

template __global__ void k_vanka_factor<2, double, true>(Geom, double, const double*, double*, double*, int, const int*);
template __global__ void k_vanka_factor<2, float, true>(Geom, double, const float*, float*, float*, int, const int*);
template __global__ void k_vanka_factor<3, double, true>(Geom, double, const double*, double*, double*, int, const int*);
template __global__ void k_vanka_factor<3, float, true>(Geom, double, const float*, float*, float*, int, const int*);
template __global__ void k_vanka_factor<2, double, false>(Geom, double, const double*, double*, double*, int, const int*);

}  // namespace fsi
