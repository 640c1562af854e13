// Device helpers of the block-stencil operator, shared by the SpMV and the
// fused Vanka pass: neighbour offsets, the pressure-stabilisation row and one
// row of the block stencil times a vector.
#pragma once
#include "fsi_internal.h"

namespace fsi {

// Neighbour node offsets of the 3^D block stencil of node (i, j, k), per axis
// (offset index 0, 1, 2 for -1, 0, +1), without branches: an out-of-mesh
// neighbour maps onto the node itself.  The Jacobian stores zeros in those
// slots (and the pressure stencil for such pairs), so the product adds exactly
// nothing and every load of a row can be in flight at once.
struct Nbr {
  int ox[3], oy[3], oz[3];
};
// W, P: the strides of y and z in the indexing of x (the mesh's own, or those of
// a block's staged copy of its neighbourhood)
template <int D>
__device__ inline Nbr nbr_offsets(const Geom& g, int i, int j, int k, int W, int P) {
  Nbr o;
  o.ox[0] = i > 0 ? -1 : 0;
  o.ox[1] = 0;
  o.ox[2] = i < g.nx ? 1 : 0;
  o.oy[0] = j > 0 ? -W : 0;
  o.oy[1] = 0;
  o.oy[2] = j < g.ny ? W : 0;
  o.oz[0] = D == 3 && k > 0 ? -P : 0;
  o.oz[1] = 0;
  o.oz[2] = D == 3 && k < g.nz ? P : 0;
  return o;
}
template <int D>
__device__ inline Nbr nbr_offsets(const Geom& g, int i, int j, int k) {
  return nbr_offsets<D>(g, i, j, k, g.nx + 1, (g.nx + 1) * (g.ny + 1));
}

// k * sum_q pst[q][n] x_p(neighbour q) over the 5^D pressure stencil (clamped
// neighbours, zero coefficients outside the mesh and on Dirichlet pressure rows).
template <int D, class S>
__device__ inline S pst_row(const Geom& g, double k, int n, int i, int j, int kk, const S* __restrict__ xb) {
  FSI_DIM(D);
  int cx[5], cy[5], cz[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    cx[d] = min(max(i + d - 2, 0), g.nx);
    cy[d] = (g.nx + 1) * min(max(j + d - 2, 0), g.ny);
    cz[d] = D == 3 ? (g.nx + 1) * (g.ny + 1) * min(max(kk + d - 2, 0), g.nz) : 0;
  }
  S ap = 0;
#pragma unroll
  for (int q = 0; q < NPST; ++q)
    ap += (S)g.pst[(size_t)q * g.nn + n] * xb[(size_t)(cx[q % 5] + cy[(q / 5) % 5] + cz[q / 25]) * NC + PC];
  return (S)k * ap;
}

// Part of the pressure-stabilisation row: k * sum of pst[q][n] x_p(neighbour q)
// over the stencil rows [r0, r1) (a row is one (dy, dz) offset, its five dx
// offsets unrolled).  The fused Vanka pass spreads the rows over the waves of
// the displacement rows, which have the fewest block-stencil loads.
template <int D, class S>
__device__ inline S pst_rows(const Geom& g, double k, int n, int i, int j, int kk, const S* __restrict__ xb, int r0,
                             int r1) {
  FSI_DIM(D);
  int cx[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) cx[d] = min(max(i + d - 2, 0), g.nx);
  S ap = 0;
  for (int rr = r0; rr < r1; ++rr) {
    const int dy = rr % 5, dz = rr / 5;
    const int oy = (g.nx + 1) * min(max(j + dy - 2, 0), g.ny);
    const int oz = D == 3 ? (g.nx + 1) * (g.ny + 1) * min(max(kk + dz - 2, 0), g.nz) : 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx)
      ap += (S)g.pst[(size_t)(5 * rr + dx) * g.nn + n] * xb[(size_t)(cx[dx] + oy + oz) * NC + PC];
  }
  return (S)k * ap;
}

// The same from a staged copy of the pressure values of a box of nodes: xp
// holds p at (x, y, z) = (X0 + lx, Y0 + ly, Z0 + lz) at lx + RX (ly + RY lz);
// the box contains every clamped stencil neighbour of node (i, j, kk).
template <int D, class S>
__device__ inline S pst_rows_staged(const Geom& g, double k, int n, int i, int j, int kk, const S* xp, int X0,
                                    int Y0, int Z0, int RX, int RY, int r0, int r1) {
  int cx[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) cx[d] = min(max(i + d - 2, 0), g.nx) - X0;
  S ap = 0;
  for (int rr = r0; rr < r1; ++rr) {
    const int dy = rr % 5, dz = rr / 5;
    const int oy = RX * (min(max(j + dy - 2, 0), g.ny) - Y0);
    const int oz = D == 3 ? RX * RY * (min(max(kk + dz - 2, 0), g.nz) - Z0) : 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) ap += (S)g.pst[(size_t)(5 * rr + dx) * g.nn + n] * xp[cx[dx] + oy + oz];
  }
  return (S)k * ap;
}

// Row r of the block stencil at node n times x: the sum over the slots of the
// stored entries of row r (jn: the node's position in the tiled Jacobian).  In
// the compressed layout a displacement row holds (v_i, u_i) only; the row kind
// is uniform over a wave and tested once, outside the slot loops, so that the
// loads of all slots (3d: of one plane of slots) are in flight together.
template <int D, class S, bool CJ>
__device__ inline S stencil_row(const S* __restrict__ jn, const S* __restrict__ xb, int n, int r, const Nbr& nb) {
  FSI_DIM(D);
  S acc = 0;
  const int e0 = jrow_off<D, CJ>(r);
  constexpr int NZ = D == 3 ? 3 : 1;
  if (CJ && r >= D && r < 2 * D) {
#pragma unroll 1
    for (int sz = 0; sz < NZ; ++sz) {
      const int oz = sz == 0 ? nb.oz[0] : (sz == 1 ? 0 : nb.oz[2]);
#pragma unroll
      for (int sy = 0; sy < 3; ++sy)
#pragma unroll
        for (int sx = 0; sx < 3; ++sx) {
          const int s = sx + 3 * sy + 9 * sz;
          const S* xv = xb + (size_t)(n + nb.ox[sx] + nb.oy[sy] + oz) * NC;
          acc += jn[jent<D, S, CJ>(s, e0)] * xv[r - D];
          acc += jn[jent<D, S, CJ>(s, e0 + 1)] * xv[r];
        }
    }
  } else {
#pragma unroll 1
    for (int sz = 0; sz < NZ; ++sz) {
      const int oz = sz == 0 ? nb.oz[0] : (sz == 1 ? 0 : nb.oz[2]);
#pragma unroll
      for (int sy = 0; sy < 3; ++sy)
#pragma unroll
        for (int sx = 0; sx < 3; ++sx) {
          const int s = sx + 3 * sy + 9 * sz;
          const S* xv = xb + (size_t)(n + nb.ox[sx] + nb.oy[sy] + oz) * NC;
#pragma unroll
          for (int c = 0; c < NC; ++c) acc += jn[jent<D, S, CJ>(s, e0 + c)] * xv[c];
        }
    }
  }
  return acc;
}

}  // namespace fsi
