// Internal definitions shared by the HIP kernels and the host driver of the
// ALE-FSI fine propagator.  2d, Q1 elements, 5 unknowns per node
// (v_x, v_y, u_x, u_y, p).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "../../include/fsi.h"

namespace fsi {

constexpr int NC = 5;      // unknowns per node
constexpr int NL = 4;      // nodes per cell
constexpr int NE = 20;     // unknowns per cell
constexpr int NSLOT = 9;   // block-stencil slots (3x3 neighbourhood)
constexpr int NPST = 25;   // pressure-stencil slots (5x5 neighbourhood)
constexpr int BLK = 25;    // entries of a 5x5 block
constexpr int RED_T = 256; // threads of the reduction kernels

// component bits of the Dirichlet mask
constexpr uint8_t DM_V = 0x03, DM_U = 0x0c, DM_P = 0x10;
// node class bits
constexpr uint8_t CL_NS = 0x01;     // node of a solid cell
constexpr uint8_t CL_NF = 0x02;     // node of a fluid cell
constexpr uint8_t CL_INFLOW = 0x04; // inflow node carrying the parabolic profile

// Device view of one mesh level (all pointers device memory).
struct Geom {
  int nx, ny, nn, ncell;
  const double* x;          // [nx+1] node x-coordinates
  const double* y;          // [ny+1] node y-coordinates
  const uint8_t* solid;     // [ncell] 1 = solid cell
  const uint8_t* cls;       // [nn] node class bits
  const uint8_t* dmask;     // [nn] Dirichlet component mask (bit c -> component c)
  const double* pst;        // [25][nn] constant pressure stencil (LPS or CIP), zero on Dirichlet p rows
};

// Physical and step constants of one time step.
struct StepPar {
  double k, theta;
  double rho_f, nu_f, rho_s, mu_s, lambda_s;
  double peak, ramp_time;
};

// Neighbour slot of offset (dx, dy) in the 3x3 block stencil.
__host__ __device__ inline int slot_of(int dx, int dy) { return (dx + 1) + 3 * (dy + 1); }

// Jacobian storage: per slice, nodes are grouped in tiles of 64; a tile holds its
// 9 x 25 block-stencil coefficients as 225 runs of 64 consecutive values, so one
// wave streams one contiguous 225 x 64 array.
constexpr int JT = 64;
constexpr int SPMV_THREADS = 5 * 64;   // row-variant SpMV block: five waves over 64 nodes
constexpr int VC_CELLS = 16;           // cells per block of the fused Vanka pass
constexpr int VC_THREADS = 5 * 64;     // its five waves (one per row of a patch node)
constexpr int VF_PATCHES = 8;          // patches per block of the Vanka factor kernel (32 lanes each)
__host__ __device__ inline int nn_pad(int nn) { return (nn + JT - 1) / JT * JT; }
__host__ __device__ inline size_t jslice(int nn) { return (size_t)NSLOT * BLK * nn_pad(nn); }
__host__ __device__ inline size_t jidx(int node, int s, int e) {
  return (size_t)(node / JT) * (NSLOT * BLK * JT) + (size_t)(s * BLK + e) * JT + (node % JT);
}
__host__ __device__ inline int pslot_of(int dx, int dy) { return (dx + 2) + 5 * (dy + 2); }

// ------------------------------------------------------------ colour helpers
// Cells of colour c = (i mod 2) + 2 (j mod 2): ncx per row, nc in total, and
// the offset of the colour's block in the per-colour Vanka inverse storage
// (colours stored in order 0..3).  Computed without arrays, so a colour that
// is only known at run time costs no private memory.
struct ColorInfo {
  int ncx, nc, off;
};
__host__ __device__ inline ColorInfo color_info(int nx, int ny, int c) {
  ColorInfo ci;
  ci.off = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int nq = ((nx - (q & 1) + 1) / 2) * ((ny - (q >> 1) + 1) / 2);
    if (q < c) ci.off += nq;
  }
  ci.ncx = (nx - (c & 1) + 1) / 2;
  ci.nc = ci.ncx * ((ny - (c >> 1) + 1) / 2);
  return ci;
}

// A bar face shared with a fluid cell: fluid cell index, face axis (0: x, 1: y),
// side of the face in the fluid cell (0: low, 1: high) and the sign of the solid's
// outward normal n_s = sign e_axis.
struct DragFace {
  int cell, axis, side, sign;
};

// Ramp of the inflow: (1 - cos(pi t / t_r)) / 2 for t < t_r, then 1.
__host__ __device__ inline double inflow_ramp(double t, double tr) {
  return t >= tr ? 1.0 : 0.5 * (1.0 - cos(M_PI * t / tr));
}

}  // namespace fsi
