// Element-batched assembly of the shifted Crank-Nicolson step residual and of
// its exact Jacobian (Section 2.3, time-step equation with eq. (semiforms)),
// for Q1 quadrilaterals (D = 2) and hexahedra (D = 3).
//
// One thread owns one (cell, slice).  The element residual is written once as
// a template over the scalar types of the new and the old state; the Jacobian
// evaluates it in forward-mode dual arithmetic, one local unknown at a time,
// which gives the exact derivative of every term (J, F^{-1}, the step means,
// the outflow correction) without hand-derived linearisations.  Element
// vectors/matrices go to a cell-major scratch array; node-centred gather
// kernels then sum the (at most 2^D) cell contributions per node,
// deterministically and without atomics.
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
__device__ inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
__device__ inline Dual& operator+=(Dual& a, Dual b) { a.v += b.v; a.d += b.d; return a; }
__device__ inline Dual& operator-=(Dual& a, Dual b) { a.v -= b.v; a.d -= b.d; return a; }

// two-point Gauss-Legendre abscissae on [0, 1]
constexpr double GA = 0.21132486540518711775;  // 1/2 - 1/(2 sqrt 3)
constexpr double GB = 0.78867513459481288225;  // 1/2 + 1/(2 sqrt 3)

template <int D, int NLoc = Dm<D>::NL>
struct Cell {
  double h[D];
  bool solid, outflow;
  bool urow[NLoc];   // fluid cell: harmonic-extension row of local node a is owned here
};

// Q1 shape functions and their physical gradients at reference point xi of a
// box cell with edge lengths h; local node a sits at offset bit r of a on axis r.
template <int D>
__device__ inline void q1_at(const double (&xi)[D], const double (&h)[D], double (&N)[Dm<D>::NL],
                             double (&G)[Dm<D>::NL][D]) {
#pragma unroll
  for (int a = 0; a < Dm<D>::NL; ++a) {
    double n = 1.0;
#pragma unroll
    for (int r = 0; r < D; ++r) n *= ((a >> r) & 1) ? xi[r] : 1.0 - xi[r];
    N[a] = n;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      double gr = (((a >> r) & 1) ? 1.0 : -1.0) / h[r];
#pragma unroll
      for (int s = 0; s < D; ++s)
        if (s != r) gr *= ((a >> s) & 1) ? xi[s] : 1.0 - xi[s];
      G[a][r] = gr;
    }
  }
}

// Field values and gradients at one point: v, grad v (gv[i][r] = d_r v_i), u,
// grad u, p, with scalar types per field (velocity TV, displacement TD,
// pressure TP; one type T for all by default).
template <int D, class TV, class TD = TV, class TP = TV>
struct Pt {
  TV v[D], gv[D][D];
  TD u[D], gu[D][D];
  TP p;
};

// Scalar type of a product of the given types (Dual if any is Dual).
template <class... T>
using Pr = decltype((T() * ...));

template <int D, class T, int NLoc = Dm<D>::NL>
__device__ inline void eval_point(const T (&U)[NLoc * (2 * D + 1)], const double (&N)[NLoc],
                                  const double (&G)[NLoc][D], Pt<D, T>& f) {
  FSI_DIM(D);
  for (int i = 0; i < D; ++i) {
    f.v[i] = T(0.0); f.u[i] = T(0.0);
    for (int r = 0; r < D; ++r) { f.gv[i][r] = T(0.0); f.gu[i][r] = T(0.0); }
  }
  f.p = T(0.0);
  for (int a = 0; a < NLoc; ++a) {
    for (int i = 0; i < D; ++i) {
      const T va = U[NC * a + i], ua = U[NC * a + D + i];
      f.v[i] += N[a] * va;
      f.u[i] += N[a] * ua;
      for (int r = 0; r < D; ++r) {
        f.gv[i][r] += G[a][r] * va;
        f.gu[i][r] += G[a][r] * ua;
      }
    }
    f.p += N[a] * U[NC * a + PC];
  }
}

// F = I + grad u: determinant and inverse (cofactor formulas).
template <int D, class T>
__device__ inline void def_grad(const T (&gu)[D][D], T (&F)[D][D], T& J, T (&Fi)[D][D]) {
  for (int i = 0; i < D; ++i)
    for (int r = 0; r < D; ++r) F[i][r] = (i == r ? 1.0 : 0.0) + gu[i][r];
  if constexpr (D == 2) {
    J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
    Fi[0][0] = F[1][1] / J;  Fi[0][1] = -F[0][1] / J;
    Fi[1][0] = -F[1][0] / J; Fi[1][1] = F[0][0] / J;
  } else {
    T cof[D][D];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        const int i1 = (i + 1) % D, i2 = (i + 2) % D, j1 = (j + 1) % D, j2 = (j + 2) % D;
        cof[i][j] = F[i1][j1] * F[i2][j2] - F[i1][j2] * F[i2][j1];
      }
    J = F[0][0] * cof[0][0] + F[0][1] * cof[0][1] + F[0][2] * cof[0][2];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) Fi[i][j] = cof[j][i] / J;
  }
}

// C = A B
template <int D, class TA, class TB, class TC>
__device__ inline void mat_mul(const TA (&A)[D][D], const TB (&B)[D][D], TC (&C)[D][D]) {
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      TC s = A[i][0] * B[0][j];
      for (int r = 1; r < D; ++r) s += A[i][r] * B[r][j];
      C[i][j] = s;
    }
}

// Pointwise coefficients of the element residual at one quadrature point: the
// residual of local row (a, i) is the quadrature sum of w times
//   momentum row i:      am[i] N_a + sum_r bm[i][r] d_r N_a
//   pressure row:        ap N_a
//   displacement row i:  au[i] N_a + sum_r bu[i][r] d_r N_a  (bu only on rows owned by the cell)
// (the outflow face adds its own term).  Fluid cells: ALE momentum, divergence
// and harmonic extension; solid cells: St. Venant-Kirchhoff momentum and the
// kinematic equation.
template <int D, class T>
struct Flux {
  T am[D], bm[D][D], ap, au[D], bu[D][D];
};

// f, o: new state (field types TV, TD, TP) and old state (TO) at the point; TR
// the result type.  Every intermediate carries only the types it depends on,
// so a derivative in one field's direction skips the parts that do not see it.
template <int D, class TV, class TD, class TP, class TO, class TR, int NLoc>
__device__ void point_flux(const Cell<D, NLoc>& c, const StepPar& sp, const Pt<D, TV, TD, TP>& f,
                           const Pt<D, TO>& o, Flux<D, TR>& fl) {
  using TVo = Pr<TV, TO>;
  using TDo = Pr<TD, TO>;
  using TVD = Pr<TV, TD>;
  using TA = Pr<TV, TD, TO>;
  using TS = Pr<TV, TD, TP>;
  using TPo = Pr<TP, TO>;
  const double k = sp.k, th = sp.theta;
  const double kth = k * th, k1th = k * (1.0 - th);
  const double rf = sp.rho_f, rn = sp.rho_f * sp.nu_f;
  TD F[D][D], J, Fi[D][D];
  TO Fo[D][D], Jo, Foi[D][D];
  def_grad<D, TD>(f.gu, F, J, Fi);
  def_grad<D, TO>(o.gu, Fo, Jo, Foi);
  if (!c.solid) {
    // ALE time derivative with the means of the step
    TDo gub[D][D], Fb[D][D], Jbd, Fbi[D][D];
    TVo gvb[D][D];
    for (int i = 0; i < D; ++i)
      for (int r = 0; r < D; ++r) {
        gub[i][r] = 0.5 * (f.gu[i][r] + o.gu[i][r]);
        gvb[i][r] = 0.5 * (f.gv[i][r] + o.gv[i][r]);
      }
    def_grad<D, TDo>(gub, Fb, Jbd, Fbi);
    const TDo Jb = 0.5 * (J + Jo);
    TA A[D][D];
    mat_mul<D, TVo, TDo, TA>(gvb, Fbi, A);
    for (int i = 0; i < D; ++i) {
      TA adv = A[i][0] * (f.u[0] - o.u[0]);
      for (int r = 1; r < D; ++r) adv += A[i][r] * (f.u[r] - o.u[r]);
      fl.am[i] = rf * Jb * ((f.v[i] - o.v[i]) - adv);
    }
    // convection, new and old
    TVD C[D][D];
    TO Co[D][D];
    mat_mul<D, TV, TD, TVD>(f.gv, Fi, C);
    mat_mul<D, TO, TO, TO>(o.gv, Foi, Co);
    for (int i = 0; i < D; ++i) {
      TVD cn = C[i][0] * f.v[0];
      TO co = Co[i][0] * o.v[0];
      for (int r = 1; r < D; ++r) { cn += C[i][r] * f.v[r]; co += Co[i][r] * o.v[r]; }
      fl.am[i] += kth * rf * J * cn;
      fl.am[i] += k1th * rf * Jo * co;
    }
    // Piola-transformed Cauchy stress J sigma F^{-T}; the pressure is the new one in both parts
    for (int i = 0; i < D; ++i)
      for (int r = 0; r < D; ++r) {
        TS pn = TS(0.0);
        TPo po = TPo(0.0);
        for (int cc = 0; cc < D; ++cc) {
          const TS s = rn * (C[i][cc] + C[cc][i]) - (i == cc ? f.p : TP(0.0));
          const TPo so = rn * (Co[i][cc] + Co[cc][i]) - (i == cc ? f.p : TP(0.0));
          pn += s * Fi[r][cc];
          po += so * Foi[r][cc];
        }
        fl.bm[i][r] = kth * (J * pn) + k1th * (Jo * po);
      }
    TVD trc = C[0][0];
    for (int i = 1; i < D; ++i) trc += C[i][i];
    fl.ap = k * J * trc;
    for (int i = 0; i < D; ++i) {
      fl.au[i] = TR(0.0);
      for (int r = 0; r < D; ++r) fl.bu[i][r] = k * (th * f.gu[i][r] + (1.0 - th) * o.gu[i][r]);
    }
  } else {
    // St. Venant-Kirchhoff first Piola stress F Sigma(E), E = (F^T F - I)/2
    const double mu = sp.mu_s, lam = sp.lambda_s;
    TD E[D][D], S[D][D];
    TO Eo[D][D], So[D][D];
    for (int r = 0; r < D; ++r)
      for (int s = 0; s < D; ++s) {
        TD e = F[0][r] * F[0][s];
        TO eo = Fo[0][r] * Fo[0][s];
        for (int i = 1; i < D; ++i) { e += F[i][r] * F[i][s]; eo += Fo[i][r] * Fo[i][s]; }
        E[r][s] = 0.5 * (e - (r == s ? 1.0 : 0.0));
        Eo[r][s] = 0.5 * (eo - (r == s ? 1.0 : 0.0));
      }
    TD trE = E[0][0];
    TO trEo = Eo[0][0];
    for (int r = 1; r < D; ++r) { trE += E[r][r]; trEo += Eo[r][r]; }
    for (int r = 0; r < D; ++r)
      for (int s = 0; s < D; ++s) {
        S[r][s] = 2.0 * mu * E[r][s] + (r == s ? lam * trE : TD(0.0));
        So[r][s] = 2.0 * mu * Eo[r][s] + (r == s ? lam * trEo : TO(0.0));
      }
    for (int i = 0; i < D; ++i)
      for (int r = 0; r < D; ++r) {
        TD pn = F[i][0] * S[0][r];
        TO po = Fo[i][0] * So[0][r];
        for (int s = 1; s < D; ++s) { pn += F[i][s] * S[s][r]; po += Fo[i][s] * So[s][r]; }
        fl.bm[i][r] = kth * pn + k1th * po;
      }
    fl.ap = TR(0.0);
    for (int i = 0; i < D; ++i) {
      fl.am[i] = sp.rho_s * (f.v[i] - o.v[i]);
      fl.au[i] = (f.u[i] - o.u[i]) - k * (th * f.v[i] + (1.0 - th) * o.v[i]);
      for (int r = 0; r < D; ++r) fl.bu[i][r] = TR(0.0);
    }
  }
}

// R[NC a + c] += w (coefficients of fl against the test functions of local node a)
template <int D, class T, int NLoc>
__device__ inline void add_flux(const Cell<D, NLoc>& c, const Flux<D, T>& fl, const double (&N)[NLoc],
                                const double (&G)[NLoc][D], double w, T (&R)[NLoc * (2 * D + 1)]) {
  FSI_DIM(D);
  for (int a = 0; a < NLoc; ++a) {
    for (int i = 0; i < D; ++i) {
      T s = fl.am[i] * N[a];
      for (int r = 0; r < D; ++r) s += fl.bm[i][r] * G[a][r];
      R[NC * a + i] += w * s;
    }
    R[NC * a + PC] += w * fl.ap * N[a];
    for (int i = 0; i < D; ++i) {
      T s = fl.au[i] * N[a];
      if (c.urow[a])
        for (int r = 0; r < D; ++r) s += fl.bu[i][r] * G[a][r];
      R[NC * a + D + i] += w * s;
    }
  }
}

// Outflow (do-nothing) correction at a point of the face x = L, outward normal
// e_x: bt[i] = k theta rho nu J (F^{-T} grad v^T F^{-T} n)_i + the old-state part;
// momentum row (a, i) gets - w bt[i] N_a.
template <int D, class TV, class TD, class TP, class TO, class TR>
__device__ void face_flux(const StepPar& sp, const Pt<D, TV, TD, TP>& f, const Pt<D, TO>& o, TR (&bt)[D]) {
  using TVD = Pr<TV, TD>;
  const double k = sp.k, th = sp.theta;
  const double kth = k * th, k1th = k * (1.0 - th);
  const double rn = sp.rho_f * sp.nu_f;
  TD F[D][D], J, Fi[D][D];
  TO Fo[D][D], Jo, Foi[D][D];
  def_grad<D, TD>(f.gu, F, J, Fi);
  def_grad<D, TO>(o.gu, Fo, Jo, Foi);
  TVD t2[D];
  TO t2o[D];
  for (int i = 0; i < D; ++i) {
    t2[i] = f.gv[0][i] * Fi[0][0];
    t2o[i] = o.gv[0][i] * Foi[0][0];
    for (int j = 1; j < D; ++j) { t2[i] += f.gv[j][i] * Fi[0][j]; t2o[i] += o.gv[j][i] * Foi[0][j]; }
  }
  for (int i = 0; i < D; ++i) {
    TVD t3 = Fi[0][i] * t2[0];
    TO t3o = Foi[0][i] * t2o[0];
    for (int j = 1; j < D; ++j) { t3 += Fi[j][i] * t2[j]; t3o += Foi[j][i] * t2o[j]; }
    bt[i] = kth * rn * J * t3 + k1th * rn * Jo * t3o;
  }
}

// A value of scalar type T with derivative der (dropped for double).
template <class T>
__device__ inline T seeded(double val, double der);
template <>
__device__ inline double seeded<double>(double val, double) { return val; }
template <>
__device__ inline Dual seeded<Dual>(double val, double der) { return Dual(val, der); }

// State at a point in FP64 (value) with the derivative in the direction of
// local unknown (node bn, component cc): N_bn on that component's value, grad
// N_bn on its gradient, zero elsewhere.  Only the field of cc is dual-typed.
template <int D, class TV, class TD, class TP, int NLoc>
__device__ inline void seed_point(const double (&U)[NLoc * (2 * D + 1)], const double (&N)[NLoc],
                                  const double (&G)[NLoc][D], int bn, int cc, Pt<D, TV, TD, TP>& f) {
  FSI_DIM(D);
  Pt<D, double> v;
  eval_point<D, double, NLoc>(U, N, G, v);
  double Nb = 0.0, Gb[D];
  for (int r = 0; r < D; ++r) Gb[r] = 0.0;
#pragma unroll
  for (int a = 0; a < NLoc; ++a)
    if (a == bn) {
      Nb = N[a];
      for (int r = 0; r < D; ++r) Gb[r] = G[a][r];
    }
  for (int i = 0; i < D; ++i) {
    f.v[i] = seeded<TV>(v.v[i], cc == i ? Nb : 0.0);
    f.u[i] = seeded<TD>(v.u[i], cc == D + i ? Nb : 0.0);
    for (int r = 0; r < D; ++r) {
      f.gv[i][r] = seeded<TV>(v.gv[i][r], cc == i ? Gb[r] : 0.0);
      f.gu[i][r] = seeded<TD>(v.gu[i][r], cc == D + i ? Gb[r] : 0.0);
    }
  }
  f.p = seeded<TP>(v.p, cc == PC ? Nb : 0.0);
}

// K[NC a + c] += w (derivatives of the coefficients fl against the test functions)
template <int D, int NLoc>
__device__ inline void add_flux_tangent(const Cell<D, NLoc>& c, const Flux<D, Dual>& fl, const double (&N)[NLoc],
                                        const double (&G)[NLoc][D], double w, double (&K)[NLoc * (2 * D + 1)]) {
  FSI_DIM(D);
  for (int a = 0; a < NLoc; ++a) {
    for (int i = 0; i < D; ++i) {
      double s = fl.am[i].d * N[a];
      for (int r = 0; r < D; ++r) s += fl.bm[i][r].d * G[a][r];
      K[NC * a + i] += w * s;
    }
    K[NC * a + PC] += w * fl.ap.d * N[a];
    for (int i = 0; i < D; ++i) {
      double s = fl.au[i].d * N[a];
      if (c.urow[a])
        for (int r = 0; r < D; ++r) s += fl.bu[i][r].d * G[a][r];
      K[NC * a + D + i] += w * s;
    }
  }
}

// Column (bn, cc) of the element Jacobian dR/dU^n: K[e] = dR_e / dU_{NC bn + cc}.
// TV, TD, TP: Dual for the field of cc (or all Dual), double for the others.
template <int D, class TV, class TD, class TP>
__device__ inline void jac_column(const Cell<D>& c, const StepPar& sp, const double (&Ue)[Dm<D>::NE],
                                  const double (&Uoe)[Dm<D>::NE], int bn, int cc, double (&K)[Dm<D>::NE]) {
  FSI_DIM(D);
  const double gq[2] = {GA, GB};
  double wq = 1.0;
  for (int r = 0; r < D; ++r) wq *= 0.5 * c.h[r];
  for (int e = 0; e < NE; ++e) K[e] = 0.0;
  for (int q = 0; q < (1 << D); ++q) {
    double xi[D];
    for (int r = 0; r < D; ++r) xi[r] = gq[(q >> r) & 1];
    double N[NL], G[NL][D];
    q1_at<D>(xi, c.h, N, G);
    Pt<D, TV, TD, TP> f;
    Pt<D, double> o;
    seed_point<D, TV, TD, TP>(Ue, N, G, bn, cc, f);
    eval_point<D, double>(Uoe, N, G, o);
    Flux<D, Dual> fl;
    point_flux<D, TV, TD, TP, double, Dual>(c, sp, f, o, fl);
    add_flux_tangent<D>(c, fl, N, G, wq, K);
  }
  if (c.outflow) {
    double wf = 1.0;
    for (int r = 1; r < D; ++r) wf *= 0.5 * c.h[r];
    for (int q = 0; q < (1 << (D - 1)); ++q) {
      double xi[D];
      xi[0] = 1.0;
      for (int r = 1; r < D; ++r) xi[r] = gq[(q >> (r - 1)) & 1];
      double N[NL], G[NL][D];
      q1_at<D>(xi, c.h, N, G);
      Pt<D, TV, TD, TP> f;
      Pt<D, double> o;
      seed_point<D, TV, TD, TP>(Ue, N, G, bn, cc, f);
      eval_point<D, double>(Uoe, N, G, o);
      Dual bt[D];
      face_flux<D, TV, TD, TP, double, Dual>(sp, f, o, bt);
      for (int i = 0; i < D; ++i)
        for (int a = 0; a < NL; ++a) K[NC * a + i] -= wf * bt[i].d * N[a];
    }
  }
}

// The same as a called function: the three field-typed variants of a 3d
// element then share one stack frame instead of three inlined ones.
template <int D, class TV, class TD, class TP>
__device__ __noinline__ void jac_column_call(const Cell<D>& c, const StepPar& sp, const double (&Ue)[Dm<D>::NE],
                                             const double (&Uoe)[Dm<D>::NE], int bn, int cc,
                                             double (&K)[Dm<D>::NE]) {
  jac_column<D, TV, TD, TP>(c, sp, Ue, Uoe, bn, cc, K);
}

// Element residual R[NC a + c] of one step (Dirichlet rows are replaced later).
// TU, TO: scalar types of the new and the old state; R has the common type.
template <int D, class TU, class TO, class TR>
__device__ void elem_residual(const Cell<D>& c, const StepPar& sp, const TU (&U)[Dm<D>::NE],
                              const TO (&Uo)[Dm<D>::NE], TR (&R)[Dm<D>::NE]) {
  FSI_DIM(D);
  for (int e = 0; e < NE; ++e) R[e] = TR(0.0);
  double w = 1.0;
  for (int r = 0; r < D; ++r) w *= 0.5 * c.h[r];
  const double gq[2] = {GA, GB};
  for (int q = 0; q < (1 << D); ++q) {
    double xi[D];
    for (int r = 0; r < D; ++r) xi[r] = gq[(q >> r) & 1];
    double N[NL], G[NL][D];
    q1_at<D>(xi, c.h, N, G);
    Pt<D, TU> f;
    Pt<D, TO> o;
    eval_point<D, TU>(U, N, G, f);
    eval_point<D, TO>(Uo, N, G, o);
    Flux<D, TR> fl;
    point_flux<D, TU, TU, TU, TO, TR>(c, sp, f, o, fl);
    add_flux<D, TR>(c, fl, N, G, w, R);
  }
  if (c.outflow) {
    // do-nothing correction on the face x = L (outward normal e_x), points (1, eta[, zeta])
    double wf = 1.0;
    for (int r = 1; r < D; ++r) wf *= 0.5 * c.h[r];
    for (int q = 0; q < (1 << (D - 1)); ++q) {
      double xi[D];
      xi[0] = 1.0;
      for (int r = 1; r < D; ++r) xi[r] = gq[(q >> (r - 1)) & 1];
      double N[NL], G[NL][D];
      q1_at<D>(xi, c.h, N, G);
      Pt<D, TU> f;
      Pt<D, TO> o;
      eval_point<D, TU>(U, N, G, f);
      eval_point<D, TO>(Uo, N, G, o);
      TR bt[D];
      face_flux<D, TU, TU, TU, TO, TR>(sp, f, o, bt);
      for (int i = 0; i < D; ++i)
        for (int a = 0; a < NL; ++a) R[NC * a + i] -= wf * bt[i] * N[a];
    }
  }
}

template <int D>
struct CellIn {
  Cell<D> c;
  int nodes[Dm<D>::NL];
};

template <int D>
__device__ inline CellIn<D> load_cell(const Geom& g, int cell) {
  FSI_DIM(D);
  CellIn<D> ci;
  int i, j, kk;
  cell_ijk<D>(g, cell, i, j, kk);
  ci.c.h[0] = g.x[i + 1] - g.x[i];
  ci.c.h[1] = g.y[j + 1] - g.y[j];
  if constexpr (D == 3) ci.c.h[2] = g.z[kk + 1] - g.z[kk];
  ci.c.solid = g.solid[cell] != 0;
  ci.c.outflow = (i == g.nx - 1) && !ci.c.solid;
  for (int a = 0; a < NL; ++a) {
    ci.nodes[a] = node_at(g, i + (a & 1), j + ((a >> 1) & 1), kk + ((a >> 2) & 1));
    ci.c.urow[a] = !(g.cls[ci.nodes[a]] & CL_NS);
  }
  return ci;
}

// Re[b][e][cell], e = local row NC a + c
template <int D>
__global__ void k_elem_residual(Geom g, StepPar sp, const double* __restrict__ U, const double* __restrict__ Uo,
                                double* __restrict__ Re, const int* __restrict__ active) {
  FSI_DIM(D);
  const int b = blockIdx.y;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell || (active && !active[b])) return;
  CellIn<D> ci = load_cell<D>(g, cell);
  const size_t so = (size_t)b * g.nn * NC;
  double Ue[NE], Uoe[NE], R[NE];
  for (int a = 0; a < NL; ++a)
    for (int c = 0; c < NC; ++c) {
      Ue[NC * a + c] = U[so + (size_t)ci.nodes[a] * NC + c];
      Uoe[NC * a + c] = Uo[so + (size_t)ci.nodes[a] * NC + c];
    }
  elem_residual<D, double, double, double>(ci.c, sp, Ue, Uoe, R);
  double* out = Re + (size_t)b * NE * g.ncell;
  for (int e = 0; e < NE; ++e) out[(size_t)e * g.ncell + cell] = R[e];
}

// Ke[b][NE*row + col][cell]: d Re_row / d U_col (new state) or / d Uo_col (old state).
// A block takes jac_cells<D> consecutive cells (one per thread of a group) and
// jac_waves<D> such groups; group w evaluates the dual-number residual for the
// directions d = w, w + groups, ..., so the element matrices are written in
// coalesced cell runs; the work of one cell is spread over 4 groups in 2d and 2
// in 3d (3d, 16 slices of 64x16x16 cells: one group 34.9 ms for the element
// matrices of all levels, two 31.9, four 34.3, eight 43.9; the outputs are the
// same bit for bit).
template <int D, bool OLD>
__global__ void __launch_bounds__(jac_cells<D>() * jac_waves<D>()) k_elem_jacobian(Geom g, StepPar sp,
                                                                      const double* __restrict__ U,
                                                                      const double* __restrict__ Uo,
                                                                      double* __restrict__ Ke,
                                                                      const int* __restrict__ active) {
  FSI_DIM(D);
  const int b = blockIdx.y;
  const int cell = blockIdx.x * jac_cells<D>() + (int)threadIdx.x % jac_cells<D>();
  const int w = (int)threadIdx.x / jac_cells<D>();
  if (cell >= g.ncell || (active && !active[b])) return;
  CellIn<D> ci = load_cell<D>(g, cell);
  const size_t so = (size_t)b * g.nn * NC;
  double Ue[NE], Uoe[NE];
  for (int a = 0; a < NL; ++a)
    for (int c = 0; c < NC; ++c) {
      Ue[NC * a + c] = U[so + (size_t)ci.nodes[a] * NC + c];
      Uoe[NC * a + c] = Uo[so + (size_t)ci.nodes[a] * NC + c];
    }
  double* out = Ke + (size_t)b * NE * NE * g.ncell;
  if constexpr (OLD) {
    for (int d = w; d < NE; d += jac_waves<D>()) {
      Dual R[NE];
      Dual Uold[NE];
      for (int e = 0; e < NE; ++e) Uold[e] = Dual(Uoe[e], e == d ? 1.0 : 0.0);
      elem_residual<D, double, Dual, Dual>(ci.c, sp, Ue, Uold, R);
      for (int e = 0; e < NE; ++e) out[(size_t)(NE * e + d) * g.ncell + cell] = R[e].d;
    }
  } else {
    // column d = (node bn, component cc): at each quadrature point the state is
    // interpolated in FP64 and only its derivative in direction d is seeded
    // (N_bn on the value, grad N_bn on the gradient of component cc); the
    // pointwise coefficients are differentiated in dual numbers, with only the
    // field of cc dual-typed, and only their derivatives are integrated
    for (int d = w; d < NE; d += jac_waves<D>()) {
      const int bn = d / NC, cc = d % NC;
      double K[NE];
      if constexpr (D == 2) {
        // 2d: one all-dual variant, inlined (it fits the registers; the typed,
        // called variants measured slower here)
        jac_column<D, Dual, Dual, Dual>(ci.c, sp, Ue, Uoe, bn, cc, K);
      } else {
        // 3d: only the field of cc is dual-typed (half the time of the all-dual form)
        if (cc < D)
          jac_column_call<D, Dual, double, double>(ci.c, sp, Ue, Uoe, bn, cc, K);
        else if (cc < 2 * D)
          jac_column_call<D, double, Dual, double>(ci.c, sp, Ue, Uoe, bn, cc, K);
        else
          jac_column_call<D, double, double, Dual>(ci.c, sp, Ue, Uoe, bn, cc, K);
      }
      for (int e = 0; e < NE; ++e) out[(size_t)(NE * e + d) * g.ncell + cell] = K[e];
    }
  }
}

// Inflow profile at node n: prod over the cross-stream axes of 4 s (H - s) / H^2.
template <int D>
__device__ inline double inflow_profile(const Geom& g, int n) {
  int i, j, kk;
  node_ijk<D>(g, n, i, j, kk);
  const double H = g.y[g.ny], y = g.y[j];
  double prof = 4.0 * y * (H - y) / (H * H);
  if constexpr (D == 3) {
    const double W = g.z[g.nz], z = g.z[kk];
    prof *= 4.0 * z * (W - z) / (W * W);
  }
  return prof;
}

// Dirichlet value of component c at node n at time t.
template <int D>
__device__ inline double dirichlet_value(const Geom& g, const StepPar& sp, int n, int c, double t) {
  if (c != 0 || !(g.cls[n] & CL_INFLOW)) return 0.0;
  return inflow_ramp(t, sp.ramp_time) * sp.peak * inflow_profile<D>(g, n);
}

// U[b] Dirichlet components := g(t_b)
template <int D>
__global__ void k_apply_dirichlet(Geom g, StepPar sp, double* __restrict__ U, const double* __restrict__ t,
                                  const int* __restrict__ active) {
  FSI_DIM(D);
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn || (active && !active[b])) return;
  const uint8_t m = g.dmask[n];
  if (!m) return;
  double* u = U + ((size_t)b * g.nn + n) * NC;
  for (int c = 0; c < NC; ++c)
    if (m & (1u << c)) u[c] = dirichlet_value<D>(g, sp, n, c, t[b]);
}

// Sum the element residuals of the cells around each node, add k * S p, and
// replace the Dirichlet rows by U - g(t).
template <int D>
__global__ void k_gather_residual(Geom g, StepPar sp, const double* __restrict__ Re, const double* __restrict__ U,
                                  const double* __restrict__ t, double* __restrict__ R,
                                  const int* __restrict__ active) {
  FSI_DIM(D);
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn || (active && !active[b])) return;
  int i, j, kk;
  node_ijk<D>(g, n, i, j, kk);
  const double* re = Re + (size_t)b * NE * g.ncell;
  double r[NC];
  for (int c = 0; c < NC; ++c) r[c] = 0.0;
  for (int a = 0; a < NL; ++a) {
    const int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = kk - ((a >> 2) & 1);
    if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || (D == 3 && ck >= g.nz)) continue;
    const int cell = cell_at(g, ci, cj, ck);
    for (int c = 0; c < NC; ++c) r[c] += re[(size_t)(NC * a + c) * g.ncell + cell];
  }
  const double* u = U + (size_t)b * g.nn * NC;
  double sp_ = 0.0;
  for (int q = 0; q < NPST; ++q) {
    const int dx = q % 5 - 2, dy = (q / 5) % 5 - 2, dz = D == 3 ? q / 25 - 2 : 0;
    const int ii = i + dx, jj = j + dy, kz = kk + dz;
    if (ii < 0 || jj < 0 || kz < 0 || ii > g.nx || jj > g.ny || kz > g.nz) continue;
    sp_ += g.pst[(size_t)q * g.nn + n] * u[(size_t)node_at(g, ii, jj, kz) * NC + PC];
  }
  r[PC] += sp.k * sp_;
  const uint8_t m = g.dmask[n];
  double* out = R + ((size_t)b * g.nn + n) * NC;
  for (int c = 0; c < NC; ++c)
    out[c] = (m & (1u << c)) ? u[(size_t)n * NC + c] - dirichlet_value<D>(g, sp, n, c, t[b]) : r[c];
}

// Gather the element matrices into the block stencil J[b][slot][BLK][node]
// (Dirichlet rows become identity rows) and compute the row scaling
// Dsc[b][node][c] = 1 / max_j |J_row,j| (including k S on pressure rows).
// Slots whose neighbour lies outside the mesh are written as zeros.
template <int D, class S, bool CJ>
__global__ void k_gather_jacobian(Geom g, double k, const double* __restrict__ Ke, S* __restrict__ J,
                                  double* __restrict__ Dsc, const int* __restrict__ active, int dir_identity) {
  FSI_DIM(D);
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nn || (active && !active[b])) return;
  int i, j, kk;
  node_ijk<D>(g, n, i, j, kk);
  const double* ke = Ke + (size_t)b * NE * NE * g.ncell;
  S* jb = J + (size_t)b * jslice<D, S, CJ>(g);
  const int row = n / (g.nx + 1);
  S* j0 = jb + jnode<D, S, CJ>(g, i, row, 0);   // every copy of the tiled storage
  S* j1 = jb + jnode<D, S, CJ>(g, i, row, jcopies<D, S>() - 1);
  const uint8_t m = g.dmask[n];
  double rmax[NC];
  for (int c = 0; c < NC; ++c) rmax[c] = 0.0;
  for (int s = 0; s < NSLOT; ++s) {
    const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = D == 3 ? s / 9 - 1 : 0;
    double blk[BLK];
    for (int e = 0; e < BLK; ++e) blk[e] = 0.0;
    const int ii = i + dx, jj = j + dy, kz = kk + dz;
    if (ii >= 0 && jj >= 0 && kz >= 0 && ii <= g.nx && jj <= g.ny && kz <= g.nz) {
      // cells containing both n and its neighbour
      for (int a = 0; a < NL; ++a) {
        const int ci = i - (a & 1), cj = j - ((a >> 1) & 1), ck = kk - ((a >> 2) & 1);
        if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || (D == 3 && ck >= g.nz)) continue;
        const int bx = ii - ci, by = jj - cj, bz = kz - ck;
        if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
        const int bl = bx + 2 * by + 4 * bz;
        const int cell = cell_at(g, ci, cj, ck);
        for (int r = 0; r < NC; ++r)
          for (int c = 0; c < NC; ++c)
            blk[NC * r + c] += ke[(size_t)(NE * (NC * a + r) + NC * bl + c) * g.ncell + cell];
      }
    }
    const bool centre = dx == 0 && dy == 0 && dz == 0;
    for (int r = 0; r < NC; ++r) {
      if (m & (1u << r))
        for (int c = 0; c < NC; ++c) blk[NC * r + c] = (dir_identity && centre && c == r) ? 1.0 : 0.0;
      for (int c = 0; c < NC; ++c) rmax[r] = fmax(rmax[r], fabs(blk[NC * r + c]));
    }
    for (int r = 0; r < NC; ++r)
      for (int c = 0; c < NC; ++c) {
        const int e = jentry<D, CJ>(r, c);   // compressed layout: structural zeros are not stored
        if (e >= 0) {
          j0[jent<D, S, CJ>(s, e)] = (S)blk[NC * r + c];
          if (jcopies<D, S>() == 2) j1[jent<D, S, CJ>(s, e)] = (S)blk[NC * r + c];
        }
      }
  }
  if (!(m & dm_p<D>())) {
    double pm = 0.0;
    for (int q = 0; q < NPST; ++q) pm = fmax(pm, fabs(k * g.pst[(size_t)q * g.nn + n]));
    rmax[PC] = fmax(rmax[PC], pm);
  }
  if (!Dsc) return;
  double* d = Dsc + ((size_t)b * g.nn + n) * NC;
  for (int r = 0; r < NC; ++r) d[r] = rmax[r] > 0.0 ? 1.0 / rmax[r] : 1.0;
}

// Coarse state by injection: coarse node (I, J, K) takes fine node (2I, 2J, 2K).
template <int D>
__global__ void k_inject(Geom gc, Geom gf, const double* __restrict__ Uf, double* __restrict__ Uc) {
  FSI_DIM(D);
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gc.nn) return;
  int I, Jj, K;
  node_ijk<D>(gc, n, I, Jj, K);
  const int nf = node_at(gf, 2 * I, 2 * Jj, 2 * K);
  const double* s = Uf + ((size_t)b * gf.nn + nf) * NC;
  double* d = Uc + ((size_t)b * gc.nn + n) * NC;
  for (int c = 0; c < NC; ++c) d[c] = s[c];
}

// ------------------------------------------------------------------ drag (2d)
// Drag, its gradient and the parameter sensitivities of the adjoint are built
// for the 2d channel-with-bar workloads.
using D2 = Dm<2>;

// x-component of the fluid traction J sigma(v, p; F) F^{-T} n_s integrated over one face
template <class T>
__device__ T face_drag(const Geom& g, double rn, const DragFace& f, const T (&U)[D2::NE]) {
  const int i = f.cell % g.nx, j = f.cell / g.nx;
  const double h[2] = {g.x[i + 1] - g.x[i], g.y[j + 1] - g.y[j]};
  const double len = f.axis == 0 ? h[1] : h[0];
  const double gq[2] = {GA, GB};
  T tot = T(0.0);
  for (int q = 0; q < 2; ++q) {
    const double xi[2] = {f.axis == 0 ? (double)f.side : gq[q], f.axis == 0 ? gq[q] : (double)f.side};
    double N[D2::NL], G[D2::NL][2];
    q1_at<2>(xi, h, N, G);
    Pt<2, T> pt;
    eval_point<2, T>(U, N, G, pt);
    T F[2][2], J, Fi[2][2], A[2][2];
    def_grad<2, T>(pt.gu, F, J, Fi);
    mat_mul<2, T, T>(pt.gv, Fi, A);
    T s00 = 2.0 * rn * A[0][0] - pt.p, s01 = rn * (A[0][1] + A[1][0]);
    // (J sigma F^{-T} n_s)_x = J sign sum_j sigma_0j Fi[axis][j]
    T tr = J * (double)f.sign * (s00 * Fi[f.axis][0] + s01 * Fi[f.axis][1]);
    tot += 0.5 * len * tr;
  }
  return tot;
}

__device__ inline void load_cell_state(const Geom& g, const double* U, int cell, double (&Ue)[D2::NE]) {
  const int i = cell % g.nx, j = cell / g.nx;
  const int n0 = i + (g.nx + 1) * j;
  const int nodes[D2::NL] = {n0, n0 + 1, n0 + g.nx + 1, n0 + g.nx + 2};
  for (int a = 0; a < D2::NL; ++a)
    for (int c = 0; c < D2::NC; ++c) Ue[D2::NC * a + c] = U[(size_t)nodes[a] * D2::NC + c];
}

// vals[s] = D(U_s) for nstates states spaced by stride doubles (one thread per state, faces in order)
__global__ void k_drag_values(Geom g, double rn, const DragFace* __restrict__ faces, int nf,
                              const double* __restrict__ U, size_t stride, int nstates, double* __restrict__ vals) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nstates) return;
  const double* u = U + (size_t)s * stride;
  double tot = 0.0;
  for (int q = 0; q < nf; ++q) {
    double Ue[D2::NE];
    load_cell_state(g, u, faces[q].cell, Ue);
    tot += face_drag<double>(g, rn, faces[q], Ue);
  }
  vals[s] = tot;
}

// grad += scale * dD/dU at U (single thread: faces and local unknowns in a fixed order)
__global__ void k_drag_gradient(Geom g, double rn, const DragFace* __restrict__ faces, int nf,
                                const double* __restrict__ U, double scale, double* __restrict__ grad) {
  constexpr int NC = D2::NC, NL = D2::NL, NE = D2::NE;
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
  constexpr int NC = D2::NC, NL = D2::NL, NE = D2::NE;
  __shared__ double sh[3][256];
  double acc[3] = {0.0, 0.0, 0.0};
  // inflow peak: R_i = U_i - s(t) peak prof(y_i) on the inflow rows
  const double ramp = inflow_ramp(t, sp.ramp_time);
  for (int n = threadIdx.x; n < g.nn; n += blockDim.x)
    if (g.cls[n] & CL_INFLOW) acc[0] -= lam[(size_t)n * NC] * ramp * inflow_profile<2>(g, n);
  // solid stress: d/dmu and d/dlambda of k theta F Sigma(E) + k (1-theta) F° Sigma(E°)
  const double k = sp.k, th = sp.theta;
  const double gq[2] = {GA, GB};
  for (int cell = threadIdx.x; cell < g.ncell; cell += blockDim.x) {
    if (!g.solid[cell]) continue;
    CellIn<2> ci = load_cell<2>(g, cell);
    double Ue[NE], Uoe[NE], le[NE];
    for (int a = 0; a < NL; ++a)
      for (int c = 0; c < NC; ++c) {
        const size_t o = (size_t)ci.nodes[a] * NC + c;
        Ue[NC * a + c] = U[o];
        Uoe[NC * a + c] = Uo[o];
        le[NC * a + c] = (g.dmask[ci.nodes[a]] & (1u << c)) ? 0.0 : lam[o];
      }
    const double w = 0.25 * ci.c.h[0] * ci.c.h[1];
    for (int q = 0; q < 4; ++q) {
      const double xi[2] = {gq[q & 1], gq[q >> 1]};
      double N[NL], G[NL][2];
      q1_at<2>(xi, ci.c.h, N, G);
      Pt<2, double> f, o;
      eval_point<2, double>(Ue, N, G, f);
      eval_point<2, double>(Uoe, N, G, o);
      double F[2][2], J, Fi[2][2], Fo[2][2], Jo, Foi[2][2];
      def_grad<2, double>(f.gu, F, J, Fi);
      def_grad<2, double>(o.gu, Fo, Jo, Foi);
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
          acc[1] += w * le[NC * a + i2] * (dmu[i2][0] * G[a][0] + dmu[i2][1] * G[a][1]);
          acc[2] += w * le[NC * a + i2] * (dla[i2][0] * G[a][0] + dla[i2][1] * G[a][1]);
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


// ================================================================ Q2 cells (2d)
// Biquadratic equal-order elements (Section 2.2, the paper's V_h^(2)): the cells
// of one level (geometry gc) carry the nine nodes of the next level's node grid
// (geometry gn): local node a = ox + 3 oy sits at node (2 i + ox, 2 j + oy) of cell
// (i, j).  The pointwise coefficients are those of the Q1 element (point_flux);
// basis and quadrature change: Lagrange polynomials on 0, 1/2, 1 per axis and the
// 3-point Gauss rule per direction (exact for the products of Q2 functions and
// gradients on these affine cells).
constexpr int Q2NL = 9, Q2NE = 45;
constexpr double G3X[3] = {0.11270166537925831148, 0.5, 0.88729833462074168852};   // 1/2 -+ sqrt(15)/10
constexpr double G3W[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

// Q2 shape functions and physical gradients at reference point xi of a box cell
__device__ inline void q2_at(const double (&xi)[2], const double (&h)[2], double (&N)[Q2NL], double (&G)[Q2NL][2]) {
  double L[2][3], dL[2][3];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double x = xi[r];
    L[r][0] = (2.0 * x - 1.0) * (x - 1.0);
    L[r][1] = 4.0 * x * (1.0 - x);
    L[r][2] = x * (2.0 * x - 1.0);
    dL[r][0] = (4.0 * x - 3.0) / h[r];
    dL[r][1] = (4.0 - 8.0 * x) / h[r];
    dL[r][2] = (4.0 * x - 1.0) / h[r];
  }
#pragma unroll
  for (int a = 0; a < Q2NL; ++a) {
    const int ox = a % 3, oy = a / 3;
    N[a] = L[0][ox] * L[1][oy];
    G[a][0] = dL[0][ox] * L[1][oy];
    G[a][1] = L[0][ox] * dL[1][oy];
  }
}

struct CellInQ2 {
  Cell<2, Q2NL> c;
  int nodes[Q2NL];
};

__device__ inline CellInQ2 load_cell_q2(const Geom& gc, const Geom& gn, int cell) {
  CellInQ2 ci;
  const int i = cell % gc.nx, j = cell / gc.nx;
  ci.c.h[0] = gc.x[i + 1] - gc.x[i];
  ci.c.h[1] = gc.y[j + 1] - gc.y[j];
  ci.c.solid = gc.solid[cell] != 0;
  ci.c.outflow = (i == gc.nx - 1) && !ci.c.solid;
  for (int a = 0; a < Q2NL; ++a) {
    ci.nodes[a] = (2 * i + a % 3) + (gn.nx + 1) * (2 * j + a / 3);
    ci.c.urow[a] = !(gn.cls[ci.nodes[a]] & CL_NS);
  }
  return ci;
}

// Element residual of one Q2 cell (Dirichlet rows are replaced in the gather).
template <class TU, class TO, class TR>
__device__ void elem_residual_q2(const Cell<2, Q2NL>& c, const StepPar& sp, const TU (&U)[Q2NE],
                                 const TO (&Uo)[Q2NE], TR (&R)[Q2NE]) {
  constexpr int NC = 5;
  for (int e = 0; e < Q2NE; ++e) R[e] = TR(0.0);
  for (int q = 0; q < 9; ++q) {
    const double xi[2] = {G3X[q % 3], G3X[q / 3]};
    const double w = G3W[q % 3] * G3W[q / 3] * c.h[0] * c.h[1];
    double N[Q2NL], G[Q2NL][2];
    q2_at(xi, c.h, N, G);
    Pt<2, TU> f;
    Pt<2, TO> o;
    eval_point<2, TU, Q2NL>(U, N, G, f);
    eval_point<2, TO, Q2NL>(Uo, N, G, o);
    Flux<2, TR> fl;
    point_flux<2, TU, TU, TU, TO, TR>(c, sp, f, o, fl);
    add_flux<2, TR>(c, fl, N, G, w, R);
  }
  if (c.outflow) {
    for (int q = 0; q < 3; ++q) {
      const double xi[2] = {1.0, G3X[q]};
      const double wf = G3W[q] * c.h[1];
      double N[Q2NL], G[Q2NL][2];
      q2_at(xi, c.h, N, G);
      Pt<2, TU> f;
      Pt<2, TO> o;
      eval_point<2, TU, Q2NL>(U, N, G, f);
      eval_point<2, TO, Q2NL>(Uo, N, G, o);
      TR bt[2];
      face_flux<2, TU, TU, TU, TO, TR>(sp, f, o, bt);
      for (int i = 0; i < 2; ++i)
        for (int a = 0; a < Q2NL; ++a) R[NC * a + i] -= wf * bt[i] * N[a];
    }
  }
}

// Column (bn, cc) of the Q2 element Jacobian dR/dU^n (all fields dual-typed).
__device__ inline void jac_column_q2(const Cell<2, Q2NL>& c, const StepPar& sp, const double (&Ue)[Q2NE],
                                     const double (&Uoe)[Q2NE], int bn, int cc, double (&K)[Q2NE]) {
  constexpr int NC = 5;
  for (int e = 0; e < Q2NE; ++e) K[e] = 0.0;
  for (int q = 0; q < 9; ++q) {
    const double xi[2] = {G3X[q % 3], G3X[q / 3]};
    const double w = G3W[q % 3] * G3W[q / 3] * c.h[0] * c.h[1];
    double N[Q2NL], G[Q2NL][2];
    q2_at(xi, c.h, N, G);
    Pt<2, Dual> f;
    Pt<2, double> o;
    seed_point<2, Dual, Dual, Dual, Q2NL>(Ue, N, G, bn, cc, f);
    eval_point<2, double, Q2NL>(Uoe, N, G, o);
    Flux<2, Dual> fl;
    point_flux<2, Dual, Dual, Dual, double, Dual>(c, sp, f, o, fl);
    add_flux_tangent<2, Q2NL>(c, fl, N, G, w, K);
  }
  if (c.outflow) {
    for (int q = 0; q < 3; ++q) {
      const double xi[2] = {1.0, G3X[q]};
      const double wf = G3W[q] * c.h[1];
      double N[Q2NL], G[Q2NL][2];
      q2_at(xi, c.h, N, G);
      Pt<2, Dual> f;
      Pt<2, double> o;
      seed_point<2, Dual, Dual, Dual, Q2NL>(Ue, N, G, bn, cc, f);
      eval_point<2, double, Q2NL>(Uoe, N, G, o);
      Dual bt[2];
      face_flux<2, Dual, Dual, Dual, double, Dual>(sp, f, o, bt);
      for (int i = 0; i < 2; ++i)
        for (int a = 0; a < Q2NL; ++a) K[NC * a + i] -= wf * bt[i].d * N[a];
    }
  }
}

// Re[b][e][cell] of every Q2 cell
__global__ void k_elem_residual_q2(Geom gc, Geom gn, StepPar sp, const double* __restrict__ U,
                                   const double* __restrict__ Uo, double* __restrict__ Re,
                                   const int* __restrict__ active) {
  constexpr int NC = 5;
  const int b = blockIdx.y;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= gc.ncell || (active && !active[b])) return;
  const CellInQ2 ci = load_cell_q2(gc, gn, cell);
  const size_t so = (size_t)b * gn.nn * NC;
  double Ue[Q2NE], Uoe[Q2NE], R[Q2NE];
  for (int a = 0; a < Q2NL; ++a)
    for (int c = 0; c < NC; ++c) {
      Ue[NC * a + c] = U[so + (size_t)ci.nodes[a] * NC + c];
      Uoe[NC * a + c] = Uo[so + (size_t)ci.nodes[a] * NC + c];
    }
  elem_residual_q2<double, double, double>(ci.c, sp, Ue, Uoe, R);
  double* out = Re + (size_t)b * Q2NE * gc.ncell;
  for (int e = 0; e < Q2NE; ++e) out[(size_t)e * gc.ncell + cell] = R[e];
}

// Ke[b][45 row + col][cell]: a block takes Q2_JC cells and Q2_JW groups of them;
// group w forms the columns w, w + Q2_JW, ...
constexpr int Q2_JC = 64, Q2_JW = 4;
__global__ void __launch_bounds__(Q2_JC * Q2_JW) k_elem_jacobian_q2(Geom gc, Geom gn, StepPar sp,
                                                                   const double* __restrict__ U,
                                                                   const double* __restrict__ Uo,
                                                                   double* __restrict__ Ke,
                                                                   const int* __restrict__ active) {
  constexpr int NC = 5;
  const int b = blockIdx.y;
  const int cell = blockIdx.x * Q2_JC + (int)threadIdx.x % Q2_JC;
  const int w = (int)threadIdx.x / Q2_JC;
  if (cell >= gc.ncell || (active && !active[b])) return;
  const CellInQ2 ci = load_cell_q2(gc, gn, cell);
  const size_t so = (size_t)b * gn.nn * NC;
  double Ue[Q2NE], Uoe[Q2NE];
  for (int a = 0; a < Q2NL; ++a)
    for (int c = 0; c < NC; ++c) {
      Ue[NC * a + c] = U[so + (size_t)ci.nodes[a] * NC + c];
      Uoe[NC * a + c] = Uo[so + (size_t)ci.nodes[a] * NC + c];
    }
  double* out = Ke + (size_t)b * Q2NE * Q2NE * gc.ncell;
  for (int d = w; d < Q2NE; d += Q2_JW) {
    double K[Q2NE];
    jac_column_q2(ci.c, sp, Ue, Uoe, d / NC, d % NC, K);
    for (int e = 0; e < Q2NE; ++e) out[(size_t)(Q2NE * e + d) * gc.ncell + cell] = K[e];
  }
}

// The Q2 cells containing node coordinate I of an axis with nc cells: cell index and
// local offset (0, 1, 2) of the node in it; returns their number (1 or 2).
__device__ inline int q2_cells_of(int I, int nc, int (&cell)[2], int (&off)[2]) {
  if (I & 1) {
    cell[0] = I >> 1;
    off[0] = 1;
    return 1;
  }
  int n = 0;
  if (I / 2 - 1 >= 0) { cell[n] = I / 2 - 1; off[n] = 2; ++n; }
  if (I / 2 < nc) { cell[n] = I / 2; off[n] = 0; ++n; }
  return n;
}

// Sum the Q2 element residuals of the cells around each node, add k S2 p (the Q2
// pressure stabilisation, 5 x 5 node stencil pst2), replace the Dirichlet rows by U - g(t).
__global__ void k_gather_residual_q2(Geom gc, Geom gn, StepPar sp, const double* __restrict__ pst2,
                                     const double* __restrict__ Re, const double* __restrict__ U,
                                     const double* __restrict__ t, double* __restrict__ R,
                                     const int* __restrict__ active) {
  constexpr int NC = 5;
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gn.nn || (active && !active[b])) return;
  const int I = n % (gn.nx + 1), Jn = n / (gn.nx + 1);
  int cxs[2], oxs[2], cys[2], oys[2];
  const int ncx = q2_cells_of(I, gc.nx, cxs, oxs), ncy = q2_cells_of(Jn, gc.ny, cys, oys);
  const double* re = Re + (size_t)b * Q2NE * gc.ncell;
  double r[NC] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int qy = 0; qy < ncy; ++qy)
    for (int qx = 0; qx < ncx; ++qx) {
      const int cell = cxs[qx] + gc.nx * cys[qy], a = oxs[qx] + 3 * oys[qy];
      for (int c = 0; c < NC; ++c) r[c] += re[(size_t)(NC * a + c) * gc.ncell + cell];
    }
  const double* u = U + (size_t)b * gn.nn * NC;
  double sp_ = 0.0;
  for (int q = 0; q < 25; ++q) {
    const int ii = I + q % 5 - 2, jj = Jn + q / 5 - 2;
    if (ii < 0 || jj < 0 || ii > gn.nx || jj > gn.ny) continue;
    sp_ += pst2[(size_t)q * gn.nn + n] * u[(size_t)(ii + (gn.nx + 1) * jj) * NC + 4];
  }
  r[4] += sp.k * sp_;
  const uint8_t m = gn.dmask[n];
  double* out = R + ((size_t)b * gn.nn + n) * NC;
  for (int c = 0; c < NC; ++c)
    out[c] = (m & (1u << c)) ? u[(size_t)n * NC + c] - dirichlet_value<2>(gn, sp, n, c, t[b]) : r[c];
}

// Gather the Q2 element matrices into the 5 x 5 node stencil of full 5 x 5 blocks,
// J2[b][25 slot + 5 r + c][node] (slot (dx + 2) + 5 (dy + 2)), stored in the linear
// solve's type S (summed in FP64); Dirichlet rows become identity rows;
// Dsc[b][node][r] = 1 / max_j |J_rj| (with k S2 on pressure rows).
template <class S>
__global__ void k_gather_jacobian_q2(Geom gc, Geom gn, double k, const double* __restrict__ pst2,
                                     const double* __restrict__ Ke, S* __restrict__ J2,
                                     double* __restrict__ Dsc, const int* __restrict__ active) {
  constexpr int NC = 5;
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gn.nn || (active && !active[b])) return;
  const int I = n % (gn.nx + 1), Jn = n / (gn.nx + 1);
  int cxs[2], oxs[2], cys[2], oys[2];
  const int ncx = q2_cells_of(I, gc.nx, cxs, oxs), ncy = q2_cells_of(Jn, gc.ny, cys, oys);
  const double* ke = Ke + (size_t)b * Q2NE * Q2NE * gc.ncell;
  S* jb = J2 + (size_t)b * 625 * gn.nn + n;
  const uint8_t m = gn.dmask[n];
  double rmax[NC] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < 25; ++s) {
    const int dx = s % 5 - 2, dy = s / 5 - 2;
    double blk[25];
    for (int e = 0; e < 25; ++e) blk[e] = 0.0;
    for (int qy = 0; qy < ncy; ++qy) {
      const int by = oys[qy] + dy;
      if (by < 0 || by > 2) continue;
      for (int qx = 0; qx < ncx; ++qx) {
        const int bx = oxs[qx] + dx;
        if (bx < 0 || bx > 2) continue;
        const int cell = cxs[qx] + gc.nx * cys[qy], a = oxs[qx] + 3 * oys[qy], bl = bx + 3 * by;
        for (int r = 0; r < NC; ++r)
          for (int c = 0; c < NC; ++c)
            blk[NC * r + c] += ke[(size_t)(Q2NE * (NC * a + r) + NC * bl + c) * gc.ncell + cell];
      }
    }
    for (int r = 0; r < NC; ++r) {
      if (m & (1u << r))
        for (int c = 0; c < NC; ++c) blk[NC * r + c] = (s == 12 && c == r) ? 1.0 : 0.0;
      for (int c = 0; c < NC; ++c) rmax[r] = fmax(rmax[r], fabs(blk[NC * r + c]));
    }
    for (int e = 0; e < 25; ++e) jb[(size_t)(25 * s + e) * gn.nn] = (S)blk[e];
  }
  if (!(m & dm_p<2>())) {
    double pm = 0.0;
    for (int q = 0; q < 25; ++q) pm = fmax(pm, fabs(k * pst2[(size_t)q * gn.nn + n]));
    rmax[4] = fmax(rmax[4], pm);
  }
  if (!Dsc) return;
  double* d = Dsc + ((size_t)b * gn.nn + n) * NC;
  for (int r = 0; r < NC; ++r) d[r] = rmax[r] > 0.0 ? 1.0 / rmax[r] : 1.0;
}

// Product with the Q2 Jacobian, y = D (bv - J2 x) (or D J2 x without bv; D = 1 without
// Dsc), the stabilisation k S2 included on the pressure rows, in the linear solve's
// type S (FP32 accumulation in the mixed-precision path).  One thread per node; a
// neighbour slot outside the mesh reads the node itself (J2 and pst2 hold zeros there).
template <class S>
__global__ void k_spmv_q2(Geom gn, double k, const double* __restrict__ pst2, const S* __restrict__ J2,
                          const S* __restrict__ x, const S* __restrict__ bv,
                          const double* __restrict__ Dsc, S* __restrict__ y,
                          const int* __restrict__ active) {
  constexpr int NC = 5;
  const int b = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= gn.nn || (active && !active[b])) return;
  const int I = n % (gn.nx + 1), Jn = n / (gn.nx + 1);
  const S* jb = J2 + (size_t)b * 625 * gn.nn + n;
  const S* xb = x + (size_t)b * gn.nn * NC;
  S acc[NC] = {0, 0, 0, 0, 0};
  for (int s = 0; s < 25; ++s) {
    const int ii = I + s % 5 - 2, jj = Jn + s / 5 - 2;
    const int nb = (ii < 0 || jj < 0 || ii > gn.nx || jj > gn.ny) ? n : ii + (gn.nx + 1) * jj;
    S xn[NC];
    for (int c = 0; c < NC; ++c) xn[c] = xb[(size_t)nb * NC + c];
    for (int r = 0; r < NC; ++r) {
      S a = acc[r];
      for (int c = 0; c < NC; ++c) a = fma(jb[(size_t)(25 * s + NC * r + c) * gn.nn], xn[c], a);
      acc[r] = a;
    }
    acc[4] = fma((S)(k * pst2[(size_t)s * gn.nn + n]), xn[4], acc[4]);
  }
  const size_t o = ((size_t)b * gn.nn + n) * NC;
  for (int r = 0; r < NC; ++r) {
    const S v = bv ? bv[o + r] - acc[r] : acc[r];
    y[o + r] = Dsc ? (S)(Dsc[o + r] * v) : v;
  }
}
template __global__ void k_gather_jacobian_q2<double>(Geom, Geom, double, const double*, const double*, double*,
                                                      double*, const int*);
template __global__ void k_gather_jacobian_q2<float>(Geom, Geom, double, const double*, const double*, float*,
                                                     double*, const int*);
template __global__ void k_spmv_q2<double>(Geom, double, const double*, const double*, const double*, const double*,
                                           const double*, double*, const int*);
template __global__ void k_spmv_q2<float>(Geom, double, const double*, const float*, const float*, const float*,
                                          const double*, float*, const int*);

#define FSI_INST_ASM(D)                                                                                           \
  template __global__ void k_elem_residual<D>(Geom, StepPar, const double*, const double*, double*, const int*); \
  template __global__ void k_elem_jacobian<D, false>(Geom, StepPar, const double*, const double*, double*,       \
                                                     const int*);                                                \
  template __global__ void k_apply_dirichlet<D>(Geom, StepPar, double*, const double*, const int*);              \
  template __global__ void k_gather_residual<D>(Geom, StepPar, const double*, const double*, const double*,      \
                                                double*, const int*);                                            \
  template __global__ void k_gather_jacobian<D, double, true>(Geom, double, const double*, double*, double*,     \
                                                              const int*, int);                                  \
  template __global__ void k_gather_jacobian<D, float, true>(Geom, double, const double*, float*, double*,       \
                                                             const int*, int);                                   \
  template __global__ void k_inject<D>(Geom, Geom, const double*, double*);
FSI_INST_ASM(2)
FSI_INST_ASM(3)
template __global__ void k_elem_jacobian<2, true>(Geom, StepPar, const double*, const double*, double*, const int*);
template __global__ void k_gather_jacobian<2, double, false>(Geom, double, const double*, double*, double*, const int*,
                                                             int);

}  // namespace fsi
