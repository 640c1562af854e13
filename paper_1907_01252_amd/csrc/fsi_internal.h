// Internal definitions shared by the HIP kernels and the host driver of the
// ALE-FSI fine propagator.  Q1 elements on tensor-product meshes in 2d
// (quadrilaterals, 5 unknowns per node: v_x, v_y, u_x, u_y, p) and 3d
// (hexahedra, 7 unknowns per node: v_x, v_y, v_z, u_x, u_y, u_z, p).  Every
// kernel and driver routine that depends on the dimension takes it as the
// template parameter D and reads its sizes from Dm<D>.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "../../include/fsi.h"

namespace fsi {

template <int D>
struct Dm;
template <>
struct Dm<2> {
  static constexpr int NC = 5;      // unknowns per node
  static constexpr int NL = 4;      // nodes per cell
  static constexpr int NE = 20;     // unknowns per cell
  static constexpr int NSLOT = 9;   // block-stencil slots (3x3 neighbourhood)
  static constexpr int NPST = 25;   // pressure-stencil slots (5x5 neighbourhood)
  static constexpr int BLK = 25;    // entries of a 5x5 block
  static constexpr int NCOL = 4;    // cell colours of the Vanka sweep
};
template <>
struct Dm<3> {
  static constexpr int NC = 7;
  static constexpr int NL = 8;
  static constexpr int NE = 56;
  static constexpr int NSLOT = 27;  // 3x3x3
  static constexpr int NPST = 125;  // 5x5x5
  static constexpr int BLK = 49;    // 7x7
  static constexpr int NCOL = 8;
};

// Local copies of the sizes of dimension D inside a templated function.
#define FSI_DIM(D)                                      \
  [[maybe_unused]] constexpr int NC = Dm<D>::NC;       \
  [[maybe_unused]] constexpr int NL = Dm<D>::NL;       \
  [[maybe_unused]] constexpr int NE = Dm<D>::NE;       \
  [[maybe_unused]] constexpr int NSLOT = Dm<D>::NSLOT; \
  [[maybe_unused]] constexpr int NPST = Dm<D>::NPST;   \
  [[maybe_unused]] constexpr int BLK = Dm<D>::BLK;     \
  [[maybe_unused]] constexpr int PC = 2 * D   // component index of p

constexpr int RED_T = 256;  // threads of the reduction kernels

// component bits of the Dirichlet mask: v = bits 0..D-1, u = bits D..2D-1, p = bit 2D
template <int D>
__host__ __device__ constexpr uint8_t dm_v() { return (uint8_t)((1u << D) - 1u); }
template <int D>
__host__ __device__ constexpr uint8_t dm_u() { return (uint8_t)(((1u << D) - 1u) << D); }
template <int D>
__host__ __device__ constexpr uint8_t dm_p() { return (uint8_t)(1u << (2 * D)); }
// node class bits
constexpr uint8_t CL_NS = 0x01;     // node of a solid cell
constexpr uint8_t CL_NF = 0x02;     // node of a fluid cell
constexpr uint8_t CL_INFLOW = 0x04; // inflow node carrying the parabolic profile

// Device view of one mesh level (all pointers device memory).  Node (i, j, k)
// has index i + (nx+1) (j + (ny+1) k), cell (i, j, k) index i + nx (j + ny k);
// in 2d nz = 0, k = 0 and z is unused.
struct Geom {
  int nx, ny, nz, nn, ncell;
  const double* x;          // [nx+1] node x-coordinates
  const double* y;          // [ny+1]
  const double* z;          // [nz+1] (3d)
  const uint8_t* solid;     // [ncell] 1 = solid cell
  const uint8_t* cls;       // [nn] node class bits
  const uint8_t* dmask;     // [nn] Dirichlet component mask (bit c -> component c)
  const double* pst;        // [NPST][nn] constant pressure stencil (LPS or CIP), zero on Dirichlet p rows
};

template <int D>
__host__ __device__ inline void node_ijk(const Geom& g, int n, int& i, int& j, int& k) {
  const int W = g.nx + 1;
  if constexpr (D == 2) {
    k = 0;
    j = n / W;
    i = n - j * W;
  } else {
    const int P = W * (g.ny + 1);
    k = n / P;
    const int r = n - k * P;
    j = r / W;
    i = r - j * W;
  }
}
template <int D>
__host__ __device__ inline void cell_ijk(const Geom& g, int c, int& i, int& j, int& k) {
  if constexpr (D == 2) {
    k = 0;
    j = c / g.nx;
    i = c - j * g.nx;
  } else {
    const int P = g.nx * g.ny;
    k = c / P;
    const int r = c - k * P;
    j = r / g.nx;
    i = r - j * g.nx;
  }
}
__host__ __device__ inline int node_at(const Geom& g, int i, int j, int k) {
  return i + (g.nx + 1) * (j + (g.ny + 1) * k);
}
__host__ __device__ inline int cell_at(const Geom& g, int i, int j, int k) { return i + g.nx * (j + g.ny * k); }

// Neighbour slot of offset (dx, dy, dz) in the 3x3(x3) block stencil, and of
// the 5x5(x5) pressure stencil.
template <int D>
__host__ __device__ inline int slot_of(int dx, int dy, int dz) {
  return (dx + 1) + 3 * (dy + 1) + (D == 3 ? 9 * (dz + 1) : 0);
}
template <int D>
__host__ __device__ inline int pslot_of(int dx, int dy, int dz) {
  return (dx + 2) + 5 * (dy + 2) + (D == 3 ? 25 * (dz + 2) : 0);
}

// Jacobian storage (block-stencil coefficients of the NSLOT neighbours of each
// node), per slice, as runs of jtx() values of one coefficient over
// consecutive nodes, so that a wave reads whole runs.  Two tilings, chosen by
// dimension and storage type S:
//  - compact (2d FP64): tiles of 64 consecutive node indices (row-major node
//    order), one copy.  The working set of the finest level over the slice
//    batch is a few hundred MB, and compact storage keeps a large part of the
//    repeated passes inside the GPU's last-level cache.
//  - row tiles (3d, and 2d FP32): tiles of 32 consecutive x-positions within
//    one mesh row (fixed j, k), rows padded to whole tiles (the padding is
//    never read), in two copies, with tile origins at x = 0 (copy 0) and x = 1
//    (copy 1): a block of the fused Vanka pass takes the cells of one colour,
//    whose nodes start at x = 0 or x = 1 (by the colour's x-parity), and reads
//    the copy whose runs it covers exactly, in whole 128-byte lines.
//
// Two block layouts (CJ):
//  - full: all NC x NC entries, row-major (the transposed adjoint system);
//  - compressed: the structural nonzeros of the step Jacobian only.  A
//    displacement row (harmonic extension in the fluid, kinematic equation in
//    the solid, identity when Dirichlet) depends on v_i and u_i of its own
//    component i only, so it stores 2 entries (v_i, u_i); velocity and
//    pressure rows store all NC.  2d: 19 of 25 entries, 3d: 34 of 49.
template <int D, class S>
__host__ __device__ constexpr bool jrowtiles() {
  return D == 3 || sizeof(S) == 4;
}
template <int D, class S>
__host__ __device__ constexpr int jtx() {
  return jrowtiles<D, S>() ? 32 : 64;
}
template <int D, class S>
__host__ __device__ constexpr int jcopies() {
  return jrowtiles<D, S>() ? 2 : 1;
}
template <int D, bool CJ>
__host__ __device__ constexpr int jblk() {
  return CJ ? D * (2 * D + 1) + 2 * D + (2 * D + 1) : (2 * D + 1) * (2 * D + 1);
}
// first stored entry of row r
template <int D, bool CJ>
__host__ __device__ constexpr int jrow_off(int r) {
  return !CJ ? r * (2 * D + 1)
             : (r < D ? r * (2 * D + 1) : (r < 2 * D ? D * (2 * D + 1) + 2 * (r - D) : D * (2 * D + 1) + 2 * D));
}
// stored index of entry (r, c) of a block, -1 for a structural zero of the compressed layout
template <int D, bool CJ>
__host__ __device__ inline int jentry(int r, int c) {
  if (!CJ || r < D || r == 2 * D) return jrow_off<D, CJ>(r) + c;
  if (c == r - D) return jrow_off<D, CJ>(r);
  if (c == r) return jrow_off<D, CJ>(r) + 1;
  return -1;
}
// mesh rows (j, k), and tiles per row of copy sh (row tiles)
template <int D>
__host__ __device__ inline int jrows(const Geom& g) {
  return (g.ny + 1) * (D == 3 ? g.nz + 1 : 1);
}
template <int D, class S>
__host__ __device__ inline int jntx(const Geom& g, int sh) {
  return (g.nx + 1 + sh * (jtx<D, S>() - 1) + jtx<D, S>() - 1) / jtx<D, S>();
}
template <int D, class S, bool CJ>
__host__ __device__ constexpr int jtile() {
  return Dm<D>::NSLOT * jblk<D, CJ>() * jtx<D, S>();
}
// tiles per slice
template <int D, class S>
__host__ __device__ inline size_t jtiles(const Geom& g) {
  if (!jrowtiles<D, S>()) return (size_t)(g.nn + jtx<D, S>() - 1) / jtx<D, S>();
  return (size_t)(jntx<D, S>(g, 0) + jntx<D, S>(g, 1)) * jrows<D>(g);
}
// values per slice
template <int D, class S, bool CJ>
__host__ __device__ inline size_t jslice(const Geom& g) {
  return jtiles<D, S>(g) * jtile<D, S, CJ>();
}
// position of node (x, row) (in copy sh of the row tiles); entry e of slot s
// sits jent(s, e) further
template <int D, class S, bool CJ>
__host__ __device__ inline size_t jnode(const Geom& g, int x, int row, int sh) {
  constexpr int TX = jtx<D, S>();
  if (!jrowtiles<D, S>()) {
    const int n = x + (g.nx + 1) * row;
    return (size_t)(n / TX) * jtile<D, S, CJ>() + n % TX;
  }
  const int p = x + sh * (TX - 1);
  const size_t t = (sh ? (size_t)jntx<D, S>(g, 0) * jrows<D>(g) : 0) + (size_t)row * jntx<D, S>(g, sh) + p / TX;
  return t * jtile<D, S, CJ>() + p % TX;
}
template <int D, class S, bool CJ>
__host__ __device__ constexpr int jent(int s, int e) {
  return (s * jblk<D, CJ>() + e) * jtx<D, S>();
}
// Offset of the slice whose Jacobian values row r of slice bs reads in the
// SpMV and the fused Vanka pass.  The displacement rows of the step Jacobian
// (harmonic extension, kinematic equation, Dirichlet identity) are linear in
// (v, u) with coefficients fixed by the mesh, k and theta, so every slice of a
// call assembles the same values (bit for bit) for them; in the compressed
// layout all slices read them from slice 0, which every call assembles at its
// first Newton iteration, and that one copy stays in cache.
template <int D, class S, bool CJ>
__host__ __device__ inline size_t jslice_row(const Geom& g, int bs, int r) {
  return (CJ && r >= D && r < 2 * D) ? 0 : (size_t)bs * jslice<D, S, CJ>(g);
}
// stored entries of a block that all slices read from slice 0 (the displacement rows)
template <int D, bool CJ>
__host__ __device__ constexpr int jblk_shared() {
  return CJ ? 2 * D : 0;
}
// Jacobian bytes one SpMV or fused-pass launch over B slices reads from memory
template <int D, class S, bool CJ>
inline double jbytes_launch(const Geom& g, int B) {
  return ((double)B * (jblk<D, CJ>() - jblk_shared<D, CJ>()) + jblk_shared<D, CJ>()) * Dm<D>::NSLOT * g.nn * sizeof(S);
}
// position of node n (in copy sh of the row tiles)
template <int D, class S, bool CJ>
__host__ __device__ inline size_t jnode_n(const Geom& g, int n, int sh) {
  return jnode<D, S, CJ>(g, n % (g.nx + 1), n / (g.nx + 1), sh);
}

// Launch shapes: the SpMV and the fused Vanka pass run one wave per row of a
// node (NC waves), the Vanka factor one lane group per patch row set.
template <int D>
__host__ __device__ constexpr int spmv_threads() { return Dm<D>::NC * 64; }

template <int D>
__host__ __device__ constexpr int vf_lanes() { return D == 2 ? 32 : 64; }    // lanes per patch (>= NE)
template <int D>
__host__ __device__ constexpr int vf_patches() { return D == 2 ? 8 : 1; }    // patches per factor block
// coarsest-level dense product (2d): threads per block of 64 rows
constexpr int CG_THREADS = 512;
// element Jacobian: blocks of jac_cells cells, jac_waves threads per cell
template <int D>
__host__ __device__ constexpr int jac_cells() { return 64; }
template <int D>
__host__ __device__ constexpr int jac_waves() { return D == 2 ? 4 : 2; }

// ------------------------------------------------------------ colour helpers
// Cells of colour c = (i mod 2) + 2 (j mod 2) + 4 (k mod 2): ncx per row, ncy
// rows per plane, nc in total.  The fused Vanka pass takes the cells of a
// colour in blocks of vc consecutive ones; off is the first cell slot of the
// colour in the Vanka inverse storage, where every colour is padded to a
// multiple of vc cells (colours stored in order).  Computed without arrays, so
// a colour only known at run time costs no private memory.
struct ColorInfo {
  int ncx, ncy, nc, off;
};
template <int D>
__host__ __device__ inline ColorInfo color_info(const Geom& g, int c, int vc) {
  ColorInfo ci;
  ci.off = 0;
#pragma unroll
  for (int q = 0; q < Dm<D>::NCOL; ++q) {
    const int nq = ((g.nx - (q & 1) + 1) / 2) * ((g.ny - ((q >> 1) & 1) + 1) / 2) *
                   (D == 3 ? (g.nz - ((q >> 2) & 1) + 1) / 2 : 1);
    if (q < c) ci.off += (nq + vc - 1) / vc * vc;
  }
  ci.ncx = (g.nx - (c & 1) + 1) / 2;
  ci.ncy = (g.ny - ((c >> 1) & 1) + 1) / 2;
  ci.nc = ci.ncx * ci.ncy * (D == 3 ? (g.nz - ((c >> 2) & 1) + 1) / 2 : 1);
  return ci;
}
// Colour and index within the colour of cell (i, j, k).
template <int D>
__host__ __device__ inline void cell_colour(const Geom& g, int i, int j, int k, int vc, int& col, int& idx,
                                            ColorInfo& L) {
  col = (i & 1) + 2 * (j & 1) + (D == 3 ? 4 * (k & 1) : 0);
  L = color_info<D>(g, col, vc);
  idx = (i >> 1) + L.ncx * ((j >> 1) + L.ncy * (k >> 1));
}

// Vanka inverses: per slice, the NE x NE inverse of every cell patch, stored by
// colour and, within a colour, by block of vc cells: entry (r, e) of cell
// idx = vc q + t sits at ((off + vc q) NE^2 + (NE r + e) vc + t).  A block of the
// fused pass so reads one contiguous region.  VC_MAX bounds vc (padding).
constexpr int VC_MAX = 32;
template <int D>
__host__ __device__ inline size_t ainv_slice(int ncell) {
  return ((size_t)ncell + (size_t)Dm<D>::NCOL * VC_MAX) * Dm<D>::NE * Dm<D>::NE;
}
// Patch solves with the compressed Jacobian (CJ) split the patch unknowns into
// the displacements u (D NL of them) and the rest w = (v, p) (NW).  The patch
// matrix's displacement rows touch only v_i and u_i of their own component i
// and do not depend on the state, so with Y1_i = A_uu,i^{-1} and
// Y2_i = Y1_i A_uv,i (NL x NL per component, the same in every slice) the
// patch update is delta_w = (A^{-1} r)_w from the NW rows of the inverse that
// belong to w (stored per slice), then delta_u,i = Y1_i r_u,i - Y2_i delta_v,i.
// Rows of the full layout (the transposed adjoint system) are all stored.
// the split patch solve is used with the compressed layout in FP64 and in 2d FP32
// (in 3d FP32 one slice of the mixed-precision step on 32x8x8 cells no longer
// converged with it)
template <int D, class S, bool CJ>
__host__ __device__ constexpr bool patch_split() {
  return CJ && (sizeof(S) == 8 || D == 2);
}
template <int D, bool CJ>
__host__ __device__ constexpr int ainv_rows() {
  return CJ ? (D + 1) * Dm<D>::NL : Dm<D>::NE;
}
// stored row of local unknown NC a + c (c not a displacement in CJ)
template <int D, bool CJ>
__host__ __device__ constexpr int ainv_row(int a, int c) {
  return CJ ? (D + 1) * a + (c < D ? c : D) : Dm<D>::NC * a + c;
}
// values of Y1 and Y2 per cell, and per level (slot layout as the inverses)
template <int D>
__host__ __device__ constexpr int yu_cell() {
  return 2 * D * Dm<D>::NL * Dm<D>::NL;
}
template <int D>
__host__ __device__ inline size_t yu_level(int ncell) {
  return ((size_t)ncell + (size_t)Dm<D>::NCOL * VC_MAX) * yu_cell<D>();
}

// A bar face shared with a fluid cell (2d): fluid cell index, face axis (0: x,
// 1: y), side of the face in the fluid cell (0: low, 1: high) and the sign of
// the solid's outward normal n_s = sign e_axis.
struct DragFace {
  int cell, axis, side, sign;
};

// Ramp of the inflow: (1 - cos(pi t / t_r)) / 2 for t < t_r, then 1.
__host__ __device__ inline double inflow_ramp(double t, double tr) {
  return t >= tr ? 1.0 : 0.5 * (1.0 - cos(M_PI * t / tr));
}

// Physical and step constants of one time step.
struct StepPar {
  double k, theta;
  double rho_f, nu_f, rho_s, mu_s, lambda_s;
  double peak, ramp_time;
};

}  // namespace fsi
