// Element-batched assembly of the shifted Crank-Nicolson step residual and of
// its exact Jacobian (Section 2.3, time-step equation with eq. (semiforms)).
//
// One thread owns one (cell, slice).  The element residual is written once as
// a template over the scalar type; the Jacobian evaluates it in forward-mode
// dual arithmetic, one local unknown at a time, which gives the exact
// derivative of every term (J, F^{-1}, the step means, the outflow correction)
// without hand-derived linearisations.  Element vectors/matrices go to a
// cell-major scratch array; node-centred gather kernels then sum the (at most
// four) cell contributions per node, deterministically and without atomics.
#include "fsi_internal.h"

namespace fsi {

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  __device__ Dual() = default;
  __device__ constexpr Dual(double a) : v(a), d(0.0) {}
  __device__ constexpr Dual(double a, double b) : v(a), d(b) {}
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(Dual a, Dual b) {
  double iv = 1.0 / b.v;
  return Dual(a.v * iv, (a.d - a.v * iv * b.d) * iv);
}
__device__ inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__device__ inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__device__ inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ inline Dual operator/(Dual a, double b) { double i = 1.0 / b; return Dual(a.v * i, a.d * i); }
__device__ inline Dual& operator+=(Dual& a, Dual b) { a.v += b.v; a.d += b.d; return a; }
__device__ inline Dual& operator-=(Dual& a, Dual b) { a.v -= b.v; a.d -= b.d; return a; }

__device__ inline double val(double a) { return a; }
__device__ inline double val(Dual a) { return a.v; }

// two-point Gauss-Legendre abscissae on [0, 1]
constexpr double GA = 0.21132486540518711775;  // 1/2 - 1/(2 sqrt 3)
constexpr double GB = 0.78867513459481288225;  // 1/2 + 1/(2 sqrt 3)

struct Cell {
  double hx, hy;
  bool solid, outflow;
  bool urow[NL];   // fluid cell: harmonic-extension row of local node a is owned here
};

// Field values and gradients at one point: v, grad v (gv[i][r] = d_r v_i), u, grad u, p.
template <class T>
struct Pt {
  T v[2], gv[2][2], u[2], gu[2][2], p;
};

template <class T, class S>
__device__ inline void eval_point(const S (&U)[NE], const double (&N)[NL], const double (&Gx)[NL],
                                  const double (&Gy)[NL], Pt<T>& f) {
  for (int i = 0; i < 2; ++i) {
    f.v[i] = T(0.0); f.u[i] = T(0.0);
    for (int r = 0; r < 2; ++r) { f.gv[i][r] = T(0.0); f.gu[i][r] = T(0.0); }
  }
  f.p = T(0.0);
  for (int a = 0; a < NL; ++a) {
    for (int i = 0; i < 2; ++i) {
      T va = U[NC * a + i], ua = U[NC * a + 2 + i];
      f.v[i] += N[a] * va;
      f.u[i] += N[a] * ua;
      f.gv[i][0] += Gx[a] * va; f.gv[i][1] += Gy[a] * va;
      f.gu[i][0] += Gx[a] * ua; f.gu[i][1] += Gy[a] * ua;
    }
    f.p += N[a] * T(U[NC * a + 4]);
  }
}

// F = I + grad u: determinant and inverse.
template <class T>
__device__ inline void def_grad(const T (&gu)[2][2], T (&F)[2][2], T& J, T (&Fi)[2][2]) {
  F[0][0] = 1.0 + gu[0][0]; F[0][1] = gu[0][1];
  F[1][0] = gu[1][0];       F[1][1] = 1.0 + gu[1][1];
  J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  Fi[0][0] = F[1][1] / J;  Fi[0][1] = -F[0][1] / J;
  Fi[1][0] = -F[1][0] / J; Fi[1][1] = F[0][0] / J;
}

// C = grad v F^{-1}
template <class T, class U2>
__device__ inline void mat_mul(const T (&A)[2][2], const U2 (&B)[2][2], T (&C)[2][2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) C[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j];
}

// Element residual R[5a+c] of one step (Dirichlet rows are replaced later).
template <class T>
__device__ void elem_residual(const Cell& c, const StepPar& sp, const T (&U)[NE], const T (&Uo)[NE],
                              T (&R)[NE]) {
  const double k = sp.k, th = sp.theta;
  const double kth = k * th, k1th = k * (1.0 - th);
  const double rf = sp.rho_f, rn = sp.rho_f * sp.nu_f;
  for (int e = 0; e < NE; ++e) R[e] = T(0.0);
  const double w = 0.25 * c.hx * c.hy;
  const double gq[2] = {GA, GB};
  for (int q = 0; q < 4; ++q) {
    const double xi = gq[q & 1], eta = gq[q >> 1];
    const double N[NL] = {(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta};
    const double Gx[NL] = {-(1 - eta) / c.hx, (1 - eta) / c.hx, -eta / c.hx, eta / c.hx};
    const double Gy[NL] = {-(1 - xi) / c.hy, -xi / c.hy, (1 - xi) / c.hy, xi / c.hy};
    Pt<T> f, o;
    eval_point<T, T>(U, N, Gx, Gy, f);
    eval_point<T, T>(Uo, N, Gx, Gy, o);
    T F[2][2], J, Fi[2][2];
    T Fo[2][2], Jo, Foi[2][2];
    def_grad(f.gu, F, J, Fi);
    def_grad(o.gu, Fo, Jo, Foi);
    if (!c.solid) {
      // ALE time derivative with the means of the step
      T gub[2][2], Fb[2][2], Jbd, Fbi[2][2], gvb[2][2];
      for (int i = 0; i < 2; ++i)
        for (int r = 0; r < 2; ++r) {
          gub[i][r] = 0.5 * (f.gu[i][r] + o.gu[i][r]);
          gvb[i][r] = 0.5 * (f.gv[i][r] + o.gv[i][r]);
        }
      def_grad(gub, Fb, Jbd, Fbi);
      T Jb = 0.5 * (J + Jo);
      T A[2][2];
      mat_mul(gvb, Fbi, A);
      T du0 = f.u[0] - o.u[0], du1 = f.u[1] - o.u[1];
      T m[2];
      for (int i = 0; i < 2; ++i) m[i] = rf * Jb * ((f.v[i] - o.v[i]) - (A[i][0] * du0 + A[i][1] * du1));
      // convection, new and old
      T C[2][2], Co[2][2];
      mat_mul(f.gv, Fi, C);
      mat_mul(o.gv, Foi, Co);
      for (int i = 0; i < 2; ++i) {
        m[i] += kth * rf * J * (C[i][0] * f.v[0] + C[i][1] * f.v[1]);
        m[i] += k1th * rf * Jo * (Co[i][0] * o.v[0] + Co[i][1] * o.v[1]);
      }
      // Piola-transformed Cauchy stress J sigma F^{-T}; the pressure is the new one in both parts
      T s[2][2], so[2][2];
      s[0][0] = 2.0 * rn * C[0][0] - f.p; s[1][1] = 2.0 * rn * C[1][1] - f.p;
      s[0][1] = rn * (C[0][1] + C[1][0]); s[1][0] = s[0][1];
      so[0][0] = 2.0 * rn * Co[0][0] - f.p; so[1][1] = 2.0 * rn * Co[1][1] - f.p;
      so[0][1] = rn * (Co[0][1] + Co[1][0]); so[1][0] = so[0][1];
      T P[2][2];
      for (int i = 0; i < 2; ++i)
        for (int r = 0; r < 2; ++r) {
          T pn = J * (s[i][0] * Fi[r][0] + s[i][1] * Fi[r][1]);
          T po = Jo * (so[i][0] * Foi[r][0] + so[i][1] * Foi[r][1]);
          P[i][r] = kth * pn + k1th * po;
        }
      T div = k * J * (C[0][0] + C[1][1]);
      T ug[2][2];
      for (int i = 0; i < 2; ++i)
        for (int r = 0; r < 2; ++r) ug[i][r] = k * (th * f.gu[i][r] + (1.0 - th) * o.gu[i][r]);
      for (int a = 0; a < NL; ++a) {
        for (int i = 0; i < 2; ++i) R[NC * a + i] += w * (m[i] * N[a] + P[i][0] * Gx[a] + P[i][1] * Gy[a]);
        R[NC * a + 4] += w * div * N[a];
        if (c.urow[a])
          for (int i = 0; i < 2; ++i) R[NC * a + 2 + i] += w * (ug[i][0] * Gx[a] + ug[i][1] * Gy[a]);
      }
    } else {
      // St. Venant-Kirchhoff first Piola stress F Sigma(E), E = (F^T F - I)/2
      const double mu = sp.mu_s, lam = sp.lambda_s;
      T E00 = 0.5 * (F[0][0] * F[0][0] + F[1][0] * F[1][0] - 1.0);
      T E01 = 0.5 * (F[0][0] * F[0][1] + F[1][0] * F[1][1]);
      T E11 = 0.5 * (F[0][1] * F[0][1] + F[1][1] * F[1][1] - 1.0);
      T trE = E00 + E11;
      T S00 = 2.0 * mu * E00 + lam * trE, S01 = 2.0 * mu * E01, S11 = 2.0 * mu * E11 + lam * trE;
      T Eo00 = 0.5 * (Fo[0][0] * Fo[0][0] + Fo[1][0] * Fo[1][0] - 1.0);
      T Eo01 = 0.5 * (Fo[0][0] * Fo[0][1] + Fo[1][0] * Fo[1][1]);
      T Eo11 = 0.5 * (Fo[0][1] * Fo[0][1] + Fo[1][1] * Fo[1][1] - 1.0);
      T trEo = Eo00 + Eo11;
      T So00 = 2.0 * mu * Eo00 + lam * trEo, So01 = 2.0 * mu * Eo01, So11 = 2.0 * mu * Eo11 + lam * trEo;
      T Ps[2][2];
      Ps[0][0] = kth * (F[0][0] * S00 + F[0][1] * S01) + k1th * (Fo[0][0] * So00 + Fo[0][1] * So01);
      Ps[0][1] = kth * (F[0][0] * S01 + F[0][1] * S11) + k1th * (Fo[0][0] * So01 + Fo[0][1] * So11);
      Ps[1][0] = kth * (F[1][0] * S00 + F[1][1] * S01) + k1th * (Fo[1][0] * So00 + Fo[1][1] * So01);
      Ps[1][1] = kth * (F[1][0] * S01 + F[1][1] * S11) + k1th * (Fo[1][0] * So01 + Fo[1][1] * So11);
      for (int a = 0; a < NL; ++a)
        for (int i = 0; i < 2; ++i) {
          R[NC * a + i] += w * (sp.rho_s * (f.v[i] - o.v[i]) * N[a] + Ps[i][0] * Gx[a] + Ps[i][1] * Gy[a]);
          T kin = (f.u[i] - o.u[i]) - k * (th * f.v[i] + (1.0 - th) * o.v[i]);
          R[NC * a + 2 + i] += w * kin * N[a];
        }
    }
  }
  if (c.outflow) {
    // do-nothing correction on the face x = L (outward normal e_x), points (1, eta)
    const double wf = 0.5 * c.hy;
    for (int q = 0; q < 2; ++q) {
      const double eta = gq[q];
      const double N[NL] = {0.0, 1.0 - eta, 0.0, eta};
      const double Gx[NL] = {-(1 - eta) / c.hx, (1 - eta) / c.hx, -eta / c.hx, eta / c.hx};
      const double Gy[NL] = {0.0, -1.0 / c.hy, 0.0, 1.0 / c.hy};
      Pt<T> f, o;
      eval_point<T, T>(U, N, Gx, Gy, f);
      eval_point<T, T>(Uo, N, Gx, Gy, o);
      T F[2][2], J, Fi[2][2];
      T Fo[2][2], Jo, Foi[2][2];
      def_grad(f.gu, F, J, Fi);
      def_grad(o.gu, Fo, Jo, Foi);
      // F^{-T} grad v^T F^{-T} n with n = e_x
      T t2[2], t2o[2];
      for (int i = 0; i < 2; ++i) {
        t2[i] = f.gv[0][i] * Fi[0][0] + f.gv[1][i] * Fi[0][1];
        t2o[i] = o.gv[0][i] * Foi[0][0] + o.gv[1][i] * Foi[0][1];
      }
      for (int i = 0; i < 2; ++i) {
        T t3 = Fi[0][i] * t2[0] + Fi[1][i] * t2[1];
        T t3o = Foi[0][i] * t2o[0] + Foi[1][i] * t2o[1];
        T b = kth * rn * J * t3 + k1th * rn * Jo * t3o;
        for (int a = 0; a < NL; ++a) R[NC * a + i] -= wf * b * N[a];
      }
    }
  }
}

struct CellIn {
  Cell c;
  int nodes[NL];
};

__device__ inline CellIn load_cell(const Geom& g, int cell) {
  CellIn ci;
  const int i = cell % g.nx, j = cell / g.nx;
  ci.c.hx = g.x[i + 1] - g.x[i];
  ci.c.hy = g.y[j + 1] - g.y[j];
  ci.c.solid = g.solid[cell] != 0;
  ci.c.outflow = (i == g.nx - 1) && !ci.c.solid;
  const int n0 = i + (g.nx + 1) * j;
  ci.nodes[0] = n0; ci.nodes[1] = n0 + 1; ci.nodes[2] = n0 + g.nx + 1; ci.nodes[3] = n0 + g.nx + 2;
  for (int a = 0; a < NL; ++a) ci.c.urow[a] = !(g.cls[ci.nodes[a]] & CL_NS);
  return ci;
}

// Re[b][e][cell], e = local row 5a + c
__global__ void k_elem_residual(Geom g, StepPar sp, const double* __restrict__ U, const double* __restrict__ Uo,
                                double* __restrict__ Re, const int* __restrict__ active) {
  const int b = blockIdx.y;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell || (active && !active[b])) return;
  CellIn ci = load_cell(g, cell);
  const size_t so = (size_t)b * g.nn * NC;
  double Ue[NE], Uoe[NE], R[NE];
  for (int a = 0; a < NL; ++a)
    for (int c = 0; c < NC; ++c) {
      Ue[NC * a + c] = U[so + (size_t)ci.nodes[a] * NC + c];
      Uoe[NC * a + c] = Uo[so + (size_t)ci.nodes[a] * NC + c];
    }
  elem_residual<double>(ci.c, sp, Ue, Uoe, R);
  double* out = Re + (size_t)b * NE * g.ncell;
  for (int e = 0; e < NE; ++e) out[(size_t)e * g.ncell + cell] = R[e];
}

// Ke[b][20*row + col][cell]: d Re_row / d U_col (new state) or / d Uo_col (old state).
template <bool OLD>
__global__ void __launch_bounds__(128) k_elem_jacobian(Geom g, StepPar sp, const double* __restrict__ U,
                                                       const double* __restrict__ Uo, double* __restrict__ Ke,
                                                       const int* __restrict__ active) {
  const int b = blockIdx.y;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell || (active && !active[b])) return;
  CellIn ci = load_cell(g, cell);
  const size_t so = (size_t)b * g.nn * NC;
  double Ue[NE], Uoe[NE];
  for (int a = 0; a < NL; ++a)
    for (int c = 0; c < NC; ++c) {
      Ue[NC * a + c] = U[so + (size_t)ci.nodes[a] * NC + c];
      Uoe[NC * a + c] = Uo[so + (size_t)ci.nodes[a] * NC + c];
    }
  double* out = Ke + (size_t)b * NE * NE * g.ncell;
  for (int d = 0; d < NE; ++d) {
    Dual Un[NE], Uold[NE], R[NE];
    for (int e = 0; e < NE; ++e) {
      Un[e] = Dual(Ue[e], (!OLD && e == d) ? 1.0 : 0.0);
      Uold[e] = Dual(Uoe[e], (OLD && e == d) ? 1.0 : 0.0);
    }
    elem_residual<Dual>(ci.c, sp, Un, Uold, R);
    for (int e = 0; e < NE; ++e) out[(size_t)(NE * e + d) * g.ncell + cell] = R[e].d;
  }
}

// Dirichlet value of component c at node n at time t.
__device__ inline double dirichlet_value(const Geom& g, const StepPar& sp, int n, int c, double t) {
  if (c != 0 || !(g.cls[n] & CL_INFLOW)) return 0.0;
  const int j = n / (g.nx + 1);
  const double H = g.y[g.ny], y = g.y[j];
  return inflow_ramp(t, sp.ramp_time) * sp.peak * 4.0 * y * (H - y) / (H * H);
}

// U[b] Dirichlet components := g(t_b)
__global__ void k_apply_dirichlet(Geom g, StepPar sp, double* __restrict__ U, const double* __restrict__ t,
                                  const int* __restrict__ active) {
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn || (active && !active[b])) return;
  const uint8_t m = g.dmask[n];
  if (!m) return;
  double* u = U + ((size_t)b * g.nn + n) * NC;
  for (int c = 0; c < NC; ++c)
    if (m & (1u << c)) u[c] = dirichlet_value(g, sp, n, c, t[b]);
}

// Sum the element residuals of the cells around each node, add k * S p, and
// replace the Dirichlet rows by U - g(t).
__global__ void k_gather_residual(Geom g, StepPar sp, const double* __restrict__ Re, const double* __restrict__ U,
                                  const double* __restrict__ t, double* __restrict__ R,
                                  const int* __restrict__ active) {
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn || (active && !active[b])) return;
  const int i = n % (g.nx + 1), j = n / (g.nx + 1);
  const double* re = Re + (size_t)b * NE * g.ncell;
  double r[NC] = {0, 0, 0, 0, 0};
  for (int a = 0; a < NL; ++a) {
    const int ci = i - (a & 1), cj = j - (a >> 1);
    if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
    const int cell = ci + g.nx * cj;
    for (int c = 0; c < NC; ++c) r[c] += re[(size_t)(NC * a + c) * g.ncell + cell];
  }
  const double* u = U + (size_t)b * g.nn * NC;
  double sp_ = 0.0;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      const int ii = i + dx, jj = j + dy;
      if (ii < 0 || jj < 0 || ii > g.nx || jj > g.ny) continue;
      sp_ += g.pst[(size_t)pslot_of(dx, dy) * g.nn + n] * u[(size_t)(ii + (g.nx + 1) * jj) * NC + 4];
    }
  r[4] += sp.k * sp_;
  const uint8_t m = g.dmask[n];
  double* out = R + ((size_t)b * g.nn + n) * NC;
  for (int c = 0; c < NC; ++c)
    out[c] = (m & (1u << c)) ? u[(size_t)n * NC + c] - dirichlet_value(g, sp, n, c, t[b]) : r[c];
}

// Gather the element matrices into the block stencil J[b][slot][25][node]
// (Dirichlet rows become identity rows) and compute the row scaling
// Dsc[b][node][c] = 1 / max_j |J_row,j| (including k S on pressure rows).
template <class S>
__global__ void k_gather_jacobian(Geom g, double k, const double* __restrict__ Ke, S* __restrict__ J,
                                  double* __restrict__ Dsc, const int* __restrict__ active, int dir_identity) {
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn || (active && !active[b])) return;
  const int i = n % (g.nx + 1), j = n / (g.nx + 1);
  const double* ke = Ke + (size_t)b * NE * NE * g.ncell;
  S* jb = J + (size_t)b * jslice(g.nn);
  const uint8_t m = g.dmask[n];
  double rmax[NC] = {0, 0, 0, 0, 0};
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      double blk[BLK];
      for (int e = 0; e < BLK; ++e) blk[e] = 0.0;
      const int ii = i + dx, jj = j + dy;
      if (ii >= 0 && jj >= 0 && ii <= g.nx && jj <= g.ny) {
        // cells containing both n and its neighbour
        for (int a = 0; a < NL; ++a) {
          const int ci = i - (a & 1), cj = j - (a >> 1);
          if (ci < 0 || cj < 0 || ci >= g.nx || cj >= g.ny) continue;
          const int bx = ii - ci, by = jj - cj;
          if (bx < 0 || bx > 1 || by < 0 || by > 1) continue;
          const int bl = bx + 2 * by;
          const int cell = ci + g.nx * cj;
          for (int r = 0; r < NC; ++r)
            for (int c = 0; c < NC; ++c)
              blk[NC * r + c] += ke[(size_t)(NE * (NC * a + r) + NC * bl + c) * g.ncell + cell];
        }
      }
      for (int r = 0; r < NC; ++r) {
        if (m & (1u << r))
          for (int c = 0; c < NC; ++c) blk[NC * r + c] = (dir_identity && dx == 0 && dy == 0 && c == r) ? 1.0 : 0.0;
        for (int c = 0; c < NC; ++c) rmax[r] = fmax(rmax[r], fabs(blk[NC * r + c]));
      }
      const int s = slot_of(dx, dy);
      for (int e = 0; e < BLK; ++e) jb[jidx(n, s, e)] = (S)blk[e];
    }
  if (!(m & DM_P)) {
    double pm = 0.0;
    for (int q = 0; q < NPST; ++q) pm = fmax(pm, fabs(k * g.pst[(size_t)q * g.nn + n]));
    rmax[4] = fmax(rmax[4], pm);
  }
  if (!Dsc) return;
  double* d = Dsc + ((size_t)b * g.nn + n) * NC;
  for (int r = 0; r < NC; ++r) d[r] = rmax[r] > 0.0 ? 1.0 / rmax[r] : 1.0;
}

template __global__ void k_gather_jacobian<double>(Geom, double, const double*, double*, double*, const int*, int);
template __global__ void k_gather_jacobian<float>(Geom, double, const double*, float*, double*, const int*, int);
template __global__ void k_elem_jacobian<false>(Geom, StepPar, const double*, const double*, double*, const int*);
template __global__ void k_elem_jacobian<true>(Geom, StepPar, const double*, const double*, double*, const int*);

// ------------------------------------------------------------------ drag

// x-component of the fluid traction J sigma(v, p; F) F^{-T} n_s integrated over one face
template <class T>
__device__ T face_drag(const Geom& g, double rn, const DragFace& f, const T (&U)[NE]) {
  const int i = f.cell % g.nx, j = f.cell / g.nx;
  const double hx = g.x[i + 1] - g.x[i], hy = g.y[j + 1] - g.y[j];
  const double len = f.axis == 0 ? hy : hx;
  const double gq[2] = {GA, GB};
  T tot = T(0.0);
  for (int q = 0; q < 2; ++q) {
    const double xi = f.axis == 0 ? (double)f.side : gq[q];
    const double eta = f.axis == 0 ? gq[q] : (double)f.side;
    const double N[NL] = {(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta};
    const double Gx[NL] = {-(1 - eta) / hx, (1 - eta) / hx, -eta / hx, eta / hx};
    const double Gy[NL] = {-(1 - xi) / hy, -xi / hy, (1 - xi) / hy, xi / hy};
    Pt<T> pt;
    eval_point<T, T>(U, N, Gx, Gy, pt);
    T F[2][2], J, Fi[2][2], A[2][2];
    def_grad(pt.gu, F, J, Fi);
    mat_mul(pt.gv, Fi, A);
    T s00 = 2.0 * rn * A[0][0] - pt.p, s01 = rn * (A[0][1] + A[1][0]);
    // (J sigma F^{-T} n_s)_x = J sign sum_j sigma_0j Fi[axis][j]
    T tr = J * (double)f.sign * (s00 * Fi[f.axis][0] + s01 * Fi[f.axis][1]);
    tot += 0.5 * len * tr;
  }
  return tot;
}

__device__ inline void load_cell_state(const Geom& g, const double* U, int cell, double (&Ue)[NE]) {
  const int i = cell % g.nx, j = cell / g.nx;
  const int n0 = i + (g.nx + 1) * j;
  const int nodes[NL] = {n0, n0 + 1, n0 + g.nx + 1, n0 + g.nx + 2};
  for (int a = 0; a < NL; ++a)
    for (int c = 0; c < NC; ++c) Ue[NC * a + c] = U[(size_t)nodes[a] * NC + c];
}

// vals[s] = D(U_s) for nstates states spaced by stride doubles (one thread per state, faces in order)
__global__ void k_drag_values(Geom g, double rn, const DragFace* __restrict__ faces, int nf,
                              const double* __restrict__ U, size_t stride, int nstates, double* __restrict__ vals) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nstates) return;
  const double* u = U + (size_t)s * stride;
  double tot = 0.0;
  for (int q = 0; q < nf; ++q) {
    double Ue[NE];
    load_cell_state(g, u, faces[q].cell, Ue);
    tot += face_drag<double>(g, rn, faces[q], Ue);
  }
  vals[s] = tot;
}

// grad += scale * dD/dU at U (single thread: faces and local unknowns in a fixed order)
__global__ void k_drag_gradient(Geom g, double rn, const DragFace* __restrict__ faces, int nf,
                                const double* __restrict__ U, double scale, double* __restrict__ grad) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int q = 0; q < nf; ++q) {
    double Ue[NE];
    load_cell_state(g, U, faces[q].cell, Ue);
    const int i = faces[q].cell % g.nx, j = faces[q].cell / g.nx;
    const int n0 = i + (g.nx + 1) * j;
    const int nodes[NL] = {n0, n0 + 1, n0 + g.nx + 1, n0 + g.nx + 2};
    for (int d = 0; d < NE; ++d) {
      Dual Ud[NE];
      for (int e = 0; e < NE; ++e) Ud[e] = Dual(Ue[e], e == d ? 1.0 : 0.0);
      const Dual v = face_drag<Dual>(g, rn, faces[q], Ud);
      grad[(size_t)nodes[d / NC] * NC + d % NC] += scale * v.d;
    }
  }
}

// out[0..2] += lam^T dR/dq for q = (inflow peak, mu_s, lambda_s) at the step (U, Uo) of time t.
// One workgroup; Dirichlet rows are excluded except the inflow rows (which carry the peak).
__global__ void __launch_bounds__(256) k_param_sens(Geom g, StepPar sp, const double* __restrict__ U,
                                                    const double* __restrict__ Uo, const double* __restrict__ lam,
                                                    double t, double* __restrict__ out) {
  __shared__ double sh[3][256];
  double acc[3] = {0.0, 0.0, 0.0};
  // inflow peak: R_i = U_i - s(t) peak prof(y_i) on the inflow rows
  const double H = g.y[g.ny], ramp = inflow_ramp(t, sp.ramp_time);
  for (int n = threadIdx.x; n < g.nn; n += blockDim.x)
    if (g.cls[n] & CL_INFLOW) {
      const double y = g.y[n / (g.nx + 1)];
      acc[0] -= lam[(size_t)n * NC] * ramp * 4.0 * y * (H - y) / (H * H);
    }
  // solid stress: d/dmu and d/dlambda of k theta F Sigma(E) + k (1-theta) F° Sigma(E°)
  const double k = sp.k, th = sp.theta;
  const double gq[2] = {GA, GB};
  for (int cell = threadIdx.x; cell < g.ncell; cell += blockDim.x) {
    if (!g.solid[cell]) continue;
    CellIn ci = load_cell(g, cell);
    double Ue[NE], Uoe[NE], le[NE];
    for (int a = 0; a < NL; ++a)
      for (int c = 0; c < NC; ++c) {
        const size_t o = (size_t)ci.nodes[a] * NC + c;
        Ue[NC * a + c] = U[o];
        Uoe[NC * a + c] = Uo[o];
        le[NC * a + c] = (g.dmask[ci.nodes[a]] & (1u << c)) ? 0.0 : lam[o];
      }
    const double w = 0.25 * ci.c.hx * ci.c.hy;
    for (int q = 0; q < 4; ++q) {
      const double xi = gq[q & 1], eta = gq[q >> 1];
      const double N[NL] = {(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta};
      const double Gx[NL] = {-(1 - eta) / ci.c.hx, (1 - eta) / ci.c.hx, -eta / ci.c.hx, eta / ci.c.hx};
      const double Gy[NL] = {-(1 - xi) / ci.c.hy, -xi / ci.c.hy, (1 - xi) / ci.c.hy, xi / ci.c.hy};
      Pt<double> f, o;
      eval_point<double, double>(Ue, N, Gx, Gy, f);
      eval_point<double, double>(Uoe, N, Gx, Gy, o);
      double F[2][2], J, Fi[2][2], Fo[2][2], Jo, Foi[2][2];
      def_grad(f.gu, F, J, Fi);
      def_grad(o.gu, Fo, Jo, Foi);
      double dmu[2][2], dla[2][2];
      for (int pass = 0; pass < 2; ++pass) {
        const double (*Fx)[2] = pass == 0 ? F : Fo;
        const double wt = pass == 0 ? k * th : k * (1.0 - th);
        const double E00 = 0.5 * (Fx[0][0] * Fx[0][0] + Fx[1][0] * Fx[1][0] - 1.0);
        const double E01 = 0.5 * (Fx[0][0] * Fx[0][1] + Fx[1][0] * Fx[1][1]);
        const double E11 = 0.5 * (Fx[0][1] * Fx[0][1] + Fx[1][1] * Fx[1][1] - 1.0);
        const double trE = E00 + E11;
        // F (2E) and F (tr E I)
        const double m00 = Fx[0][0] * 2 * E00 + Fx[0][1] * 2 * E01, m01 = Fx[0][0] * 2 * E01 + Fx[0][1] * 2 * E11;
        const double m10 = Fx[1][0] * 2 * E00 + Fx[1][1] * 2 * E01, m11 = Fx[1][0] * 2 * E01 + Fx[1][1] * 2 * E11;
        if (pass == 0) {
          dmu[0][0] = wt * m00; dmu[0][1] = wt * m01; dmu[1][0] = wt * m10; dmu[1][1] = wt * m11;
          for (int a2 = 0; a2 < 2; ++a2)
            for (int b2 = 0; b2 < 2; ++b2) dla[a2][b2] = wt * Fx[a2][b2] * trE;
        } else {
          dmu[0][0] += wt * m00; dmu[0][1] += wt * m01; dmu[1][0] += wt * m10; dmu[1][1] += wt * m11;
          for (int a2 = 0; a2 < 2; ++a2)
            for (int b2 = 0; b2 < 2; ++b2) dla[a2][b2] += wt * Fx[a2][b2] * trE;
        }
      }
      for (int a = 0; a < NL; ++a)
        for (int i2 = 0; i2 < 2; ++i2) {
          acc[1] += w * le[NC * a + i2] * (dmu[i2][0] * Gx[a] + dmu[i2][1] * Gy[a]);
          acc[2] += w * le[NC * a + i2] * (dla[i2][0] * Gx[a] + dla[i2][1] * Gy[a]);
        }
    }
  }
  for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) out[q] += sh[q][0];
}

// Coarse state by injection: coarse node (I, J) takes fine node (2I, 2J).
__global__ void k_inject(Geom gc, Geom gf, const double* __restrict__ Uf, double* __restrict__ Uc, int B) {
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gc.nn) return;
  const int I = n % (gc.nx + 1), Jj = n / (gc.nx + 1);
  const int nf = 2 * I + (gf.nx + 1) * 2 * Jj;
  const double* s = Uf + ((size_t)b * gf.nn + nf) * NC;
  double* d = Uc + ((size_t)b * gc.nn + n) * NC;
  for (int c = 0; c < NC; ++c) d[c] = s[c];
  (void)B;
}

}  // namespace fsi
