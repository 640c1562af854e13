// Vanka patch inverses: the NE x NE matrix of every cell patch, gathered from
// the block-stencil Jacobian (and the pressure stabilisation), inverted by
// Gauss-Jordan in LDS and stored by colour and block of the fused pass.
#include "stencil.h"

namespace fsi {

// ------------------------------------------------------- Vanka patch inverse
// One lane group (vf_lanes lanes) inverts the NE x NE patch matrix of one cell
// (rows = local unknowns NC a + c) by Gauss-Jordan with partial pivoting, in
// place: A lives in LDS, lane r owning row r; per column the pivot row is
// found by a shuffle reduction, every other row eliminates the column with the
// unscaled pivot row and stores its multiplier there, then the pivot row
// scales itself.  Column j ends up holding the column of the inverse that
// belongs to the pivot row of j, and the row a lane pivoted gives the row of
// the inverse it holds.  Ainv is stored by colour and
// block of vc cells of the fused pass (ainv_slice in fsi_internal.h).
template <int D, class S, bool CJ>
__global__ void __launch_bounds__(vf_lanes<D>() * vf_patches<D>()) k_vanka_factor(Geom g, double k,
                                                                                  const S* __restrict__ J,
                                                                                  S* __restrict__ Ainv, int vc,
                                                                                  const int* __restrict__ active) {
  FSI_DIM(D);
  constexpr int GL = vf_lanes<D>(), NP = vf_patches<D>(), LD = NE + 1;
  __shared__ double M[NP][NE][LD];
  __shared__ int colmap[NP][NE];   // pivot row of each column
  const int bs = blockIdx.y;
  if (active && !active[bs]) return;   // uniform over the block
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int cell = blockIdx.x * NP + grp;
  const bool live = cell < g.ncell;
  int ci = 0, cj = 0, ck = 0;
  if (live) cell_ijk<D>(g, cell, ci, cj, ck);
  double(*Mp)[LD] = M[grp];
  if (lane < NE) {
    const int a = lane / NC, rc = lane % NC;
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const int na = node_at(g, ci + ax, cj + ay, ck + az);
    if (live) {
      const S* jn = J + (size_t)bs * jslice<D, S, CJ>(g) + jnode_n<D, S, CJ>(g, na, 0);
      const bool pst_row = (rc == PC) && !(g.dmask[na] & dm_p<D>());
      for (int bb = 0; bb < NL; ++bb) {
        const int dx = (bb & 1) - ax, dy = ((bb >> 1) & 1) - ay, dz = ((bb >> 2) & 1) - az;
        const int s = slot_of<D>(dx, dy, dz);
        for (int c = 0; c < NC; ++c) {
          const int e = jentry<D, CJ>(rc, c);
          Mp[lane][NC * bb + c] = e >= 0 ? (double)jn[jent<D, S, CJ>(s, e)] : 0.0;
        }
        if (pst_row) Mp[lane][NC * bb + PC] += k * g.pst[(size_t)pslot_of<D>(dx, dy, dz) * g.nn + na];
      }
    } else {
      for (int c = 0; c < NE; ++c) Mp[lane][c] = (c == lane) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  // in-place Gauss-Jordan: after the step of column jc, column jc holds the
  // column of the inverse that belongs to the pivot row of jc
  bool used = lane >= NE;
  int mycol = 0;
  for (int jc = 0; jc < NE; ++jc) {
    const double v = lane < NE ? Mp[lane][jc] : 0.0;
    double cand = used ? -1.0 : fabs(v);
    int idx = lane;
#pragma unroll
    for (int off = GL / 2; off > 0; off >>= 1) {
      const double oc = __shfl_xor(cand, off, GL);
      const int oi = __shfl_xor(idx, off, GL);
      if (oc > cand || (oc == cand && oi < idx)) { cand = oc; idx = oi; }
    }
    double pv = Mp[idx][jc];
    if (pv == 0.0) pv = 1.0;   // singular patch: no pivot for this column
    if (lane == idx) { used = true; mycol = jc; }
    if (lane == 0) colmap[grp][jc] = idx;
    // the other rows eliminate column jc with the unscaled pivot row
    const double f = (lane < NE && lane != idx) ? v / pv : 0.0;
    if (f != 0.0) {
#pragma unroll 8
      for (int c = 0; c < NE; ++c)
        if (c != jc) Mp[lane][c] -= f * Mp[idx][c];
      Mp[lane][jc] = -f;
    }
    __syncthreads();
    // then the pivot row scales itself
    if (lane == idx) {
      const double inv = 1.0 / pv;
#pragma unroll 8
      for (int c = 0; c < NE; ++c) Mp[lane][c] = c == jc ? inv : Mp[lane][c] * inv;
    }
    __syncthreads();
  }
  if (live && lane < NE) {
    // row mycol of the inverse: entry (mycol, pivot row of j) is held in column j
    int col, idx;
    ColorInfo L;
    cell_colour<D>(g, ci, cj, ck, vc, col, idx, L);
    const int q = idx / vc, t = idx - q * vc;
    S* out = Ainv + (size_t)bs * ainv_slice<D>(g.ncell) + ((size_t)L.off + (size_t)q * vc) * NE * NE + t;
    for (int j = 0; j < NE; ++j) out[(size_t)(NE * mycol + colmap[grp][j]) * vc] = (S)Mp[lane][j];
  }
}

template __global__ void k_vanka_factor<2, double, true>(Geom, double, const double*, double*, int, const int*);
template __global__ void k_vanka_factor<2, float, true>(Geom, double, const float*, float*, int, const int*);
template __global__ void k_vanka_factor<3, double, true>(Geom, double, const double*, double*, int, const int*);
template __global__ void k_vanka_factor<3, float, true>(Geom, double, const float*, float*, int, const int*);
template __global__ void k_vanka_factor<2, double, false>(Geom, double, const double*, double*, int, const int*);

}  // namespace fsi
