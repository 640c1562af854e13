// Host driver: mesh hierarchy and constant operators (setup), Newton's method
// per time step with a multigrid-preconditioned FGMRES inner solve, the fine
// and coarse propagators, Parareal, and the C ABI of include/fsi.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "kernels.h"

using namespace fsi;

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) {                         \
      std::fprintf(stderr, "fsi: %s failed: %s (%s:%d)\n", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      return FSI_ERR_HIP;                           \
    }                                               \
  } while (0)

#define CHK(...)                      \
  do {                                \
    fsi_status s_ = (__VA_ARGS__);    \
    if (s_ != FSI_OK) return s_;      \
  } while (0)

namespace {

constexpr int TPB = 256;
constexpr int MAXLEV = 8;
// elements per block of the Krylov dot products (one partial sum per block and
// vector): at least KDOT_CHUNK, and about KDOT_BLOCKS blocks per slice, so a
// slice batch fills the GPU and the partial sums stay few
constexpr int KDOT_CHUNK = 512;
constexpr int KDOT_BLOCKS = 48;

struct Level {
  int nx = 0, ny = 0, nz = 0, nn = 0, ncell = 0;   // nz = 0 in 2d
  std::vector<double> x, y, z, pst;
  std::vector<uint8_t> solid, cls, dmask;
  double *d_x = nullptr, *d_y = nullptr, *d_z = nullptr, *d_pst = nullptr;
  uint8_t *d_solid = nullptr, *d_cls = nullptr, *d_dmask = nullptr;
  // batch workspace
  double *U = nullptr, *Uo = nullptr, *Dsc = nullptr;
  void *J = nullptr, *Ainv = nullptr, *Yu = nullptr, *x_ = nullptr, *b_ = nullptr, *r_ = nullptr, *t_ = nullptr;
  Geom geom() const {
    Geom g;
    g.nx = nx; g.ny = ny; g.nz = nz; g.nn = nn; g.ncell = ncell;
    g.x = d_x; g.y = d_y; g.z = d_z; g.solid = d_solid; g.cls = d_cls; g.dmask = d_dmask; g.pst = d_pst;
    return g;
  }
};

// profiled kernel families (HIP events around each launch while enabled)
enum Fam {
  F_SMOOTH = 0,        // fused Vanka colour pass (residual + patch update), finest level
  F_GMRES_SPMV = 1,    // Jacobian product of the Krylov iteration, finest level
  F_JAC = 2,           // element Jacobian, all levels
  F_RES = 3,           // residual assembly
  F_LEVEL_RES = 4,     // residual before restriction, finest level
  F_COARSE_LEV = 5,    // smoother kernels on the coarser levels
  F_COARSE_SOLVE = 6,  // coarsest-level dense solve
  F_NFAM = 7
};
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[F_NFAM];
  double bytes[F_NFAM] = {};
  int64_t launches[F_NFAM] = {};
  // slices the timed launches work on (the kernels return at once for the others):
  // the algorithmic bytes are charged for these only
  int pact = 0;
};

}  // namespace

struct fsi_problem {
  fsi_params p;
  int nlev = 0;          // levels 0..nlev-1, nlev-1 finest
  Level lev[MAXLEV];
  int Bmax = 0;
  bool mixed = false;
  size_t ssz = 8;        // sizeof(S)
  int R = 30;
  // finest-level Newton data (double)
  double *Uprev2 = nullptr, *Uprev3 = nullptr;   // U^{n-3}, U^{n-4} (higher-degree Newton guesses)
  double *U = nullptr, *Uold = nullptr, *Uprev = nullptr, *Res = nullptr, *Re = nullptr, *Ke = nullptr,
         *tdev = nullptr;
  // V-cycle replay graph (captured per batch size and step size)
  hipGraphExec_t vc_exec = nullptr;
  int vc_B = -1;
  double vc_k = -1.0;
  bool vc_mixed = false;
  bool vc_cj = true;
  bool use_graphs = true;
  bool verbose = false;   // FSI_VERBOSE=1: Newton progress of slice 0 on stderr
  // library-owned stream for the propagators (capturable; ordered after the caller's stream)
  hipStream_t ist = nullptr;
  hipEvent_t iev = nullptr;
  int *nact = nullptr;   // Newton-active slices (device)
  int *gact = nullptr;   // FGMRES-active slices (device)
  int *gord = nullptr;   // the FGMRES-active slices in order, then -1 (device; k_update_gact)
  int *flag = nullptr;
  // device address of the static scratch array on this problem's device (allocation-free residual)
  double* scratch = nullptr;
  // Q2 cells (degree 2, 2d FP64): the cells are those of level nlev - 2, the nodes those of
  // the finest level; the Q1 hierarchy on the same nodes is the preconditioner
  int deg = 1;
  double *pst2 = nullptr, *Ke2 = nullptr, *Re2 = nullptr;
  void *J2 = nullptr;   // Q2 step Jacobian in the linear solve's type
  // FGMRES: Arnoldi step j replayed from a captured graph (V-cycle included) per (B, k, type,
  // layout); a few configurations are kept.  Each step writes the slices' Krylov states to
  // pinned host memory (one buffer per step parity) and records an event.
  struct StepGraphs {
    int B;
    double k;
    bool mixed, cj;
    std::vector<hipGraphExec_t> ex;
    uint64_t used;
  };
  std::vector<StepGraphs> sg;
  uint64_t sg_clock = 0;
  int* hst_pin = nullptr;   // [2][Bmax], hipHostMalloc
  hipEvent_t step_ev[2] = {nullptr, nullptr};
  // FGMRES workspace
  void *V = nullptr, *Z = nullptr, *w = nullptr, *xs = nullptr, *tmp = nullptr;
  double *H = nullptr, *hcol = nullptr, *hcol2 = nullptr, *cs = nullptr, *sn = nullptr, *gv = nullptr,
         *res = nullptr, *beta0 = nullptr, *beta = nullptr, *ycoef = nullptr, *partial = nullptr;
  int *gstate = nullptr, *ncol = nullptr;
  double* ltol = nullptr;              // per-slice FGMRES tolerance (device)
  std::vector<double> ltol_h;
  // coarsest level block LU and explicit inverse
  double *cDinv = nullptr, *cW = nullptr, *cL = nullptr, *cY = nullptr;
  // adjoint scratch (allocated on the first adjoint call)
  double *Jtmp = nullptr, *Jcopy = nullptr, *Jold = nullptr, *traj = nullptr, *abnd = nullptr, *lam = nullptr,
         *lamn = nullptr, *arhs = nullptr, *ay = nullptr, *dvals = nullptr, *agrad = nullptr;
  double *aout = nullptr, *traj_out = nullptr;
  double adj_rtol = 1e-12;
  DragFace* faces = nullptr;
  int nfaces = 0;
  size_t traj_cap = 0;
  void* cAinv = nullptr;
  int cbs = 0, cnsb = 0;
  // Newton norms
  double *npart = nullptr, *nmax = nullptr;
  int nchunk_n = 1, chunk_n = 1;
  Prof prof;
  // stage events of the Newton iterations (pool reused by every call)
  struct StageEv {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> spool;
  size_t sused = 0;
  std::vector<StageEv> sev;
  std::vector<void*> allocs;
  // pipelined Parareal: workspace of the fine-sweep worker (created on first use)
  fsi_problem* pipe = nullptr;
  // concurrent slice groups of a propagator call: workspaces of groups 1 .. S-1
  std::vector<fsi_problem*> sub;
};

namespace {

// ------------------------------------------------------------------ helpers
// Runs an entry point's body; a C++ exception (host allocation, thread start)
// becomes a status instead of crossing the C ABI.
template <class F>
fsi_status guarded(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return FSI_ERR_OOM;
  } catch (...) {
    return FSI_ERR_HIP;
  }
}

template <class T>
fsi_status dalloc(fsi_problem* pb, T** p, size_t n) {
  void* q = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) return FSI_ERR_OOM;
  if (hipMemset(q, 0, n * sizeof(T)) != hipSuccess) return FSI_ERR_HIP;
  pb->allocs.push_back(q);
  *p = (T*)q;
  return FSI_OK;
}
fsi_status dalloc_bytes(fsi_problem* pb, void** p, size_t bytes) {
  void* q = nullptr;
  if (bytes == 0) bytes = 1;
  if (hipMalloc(&q, bytes) != hipSuccess) return FSI_ERR_OOM;
  if (hipMemset(q, 0, bytes) != hipSuccess) return FSI_ERR_HIP;
  pb->allocs.push_back(q);
  *p = q;
  return FSI_OK;
}
template <class T>
fsi_status upload(fsi_problem* pb, T** d, const std::vector<T>& h) {
  CHK(dalloc(pb, d, h.size()));
  HIPCHK(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return FSI_OK;
}

inline dim3 grid1(int n, int B) { return dim3((n + TPB - 1) / TPB, B); }

// ---------------------------------------------------------------- setup
// Axis coordinates of level l: every level-0 segment split into cells*2^l equal parts.
std::vector<double> axis_points(const fsi_params& p, int a, int l) {
  std::vector<double> pts;
  for (int s = 0; s < p.nseg[a]; ++s) {
    const double lo = p.seg_pts[a][s], hi = p.seg_pts[a][s + 1];
    const int n = p.seg_cells[a][s] << l;
    for (int q = 0; q < n; ++q) pts.push_back(lo + (hi - lo) * q / n);
  }
  pts.push_back(p.seg_pts[a][p.nseg[a]]);
  return pts;
}

// host view of a level's geometry (host arrays), for the setup loops
Geom host_geom(const Level& L) {
  Geom g{};
  g.nx = L.nx; g.ny = L.ny; g.nz = L.nz; g.nn = L.nn; g.ncell = L.ncell;
  return g;
}

// Q1 Laplace stiffness of a box cell with edge lengths h (2-point Gauss rule per
// axis, exact); local node a at offset bit r of a on axis r.
template <int D>
void q1_stiffness(const double (&h)[D], double (&K)[Dm<D>::NL][Dm<D>::NL]) {
  FSI_DIM(D);
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  double w = 1.0;
  for (int r = 0; r < D; ++r) w *= 0.5 * h[r];
  for (int a = 0; a < NL; ++a)
    for (int b = 0; b < NL; ++b) K[a][b] = 0.0;
  for (int q = 0; q < (1 << D); ++q) {
    double xi[D], G[NL][D];
    for (int r = 0; r < D; ++r) xi[r] = g[(q >> r) & 1];
    for (int a = 0; a < NL; ++a)
      for (int r = 0; r < D; ++r) {
        double v = (((a >> r) & 1) ? 1.0 : -1.0) / h[r];
        for (int s = 0; s < D; ++s)
          if (s != r) v *= ((a >> s) & 1) ? xi[s] : 1.0 - xi[s];
        G[a][r] = v;
      }
    for (int a = 0; a < NL; ++a)
      for (int b = 0; b < NL; ++b) {
        double s = 0.0;
        for (int r = 0; r < D; ++r) s += G[a][r] * G[b][r];
        K[a][b] += w * s;
      }
  }
}

template <int D>
void add_pst(Level& L, int nr, int nc, double v) {
  const Geom g = host_geom(L);
  int ir, jr, kr, ic, jc, kc;
  node_ijk<D>(g, nr, ir, jr, kr);
  node_ijk<D>(g, nc, ic, jc, kc);
  L.pst[(size_t)pslot_of<D>(ic - ir, jc - jr, kc - kr) * L.nn + nr] += v;
}

template <int D>
void cell_h(const Level& L, int i, int j, int k, double (&h)[D]) {
  h[0] = L.x[i + 1] - L.x[i];
  h[1] = L.y[j + 1] - L.y[j];
  if constexpr (D == 3) h[2] = L.z[k + 1] - L.z[k];
}

// Two-level local projection: alpha_K (grad(p - i2h p), grad(q - i2h q))_K over fluid cells,
// i2h = Q1 interpolation on the parent (2^D cells) of K, alpha_K = alpha0 |K|^(2/D) / (rho nu).
template <int D>
void build_lps(Level& L, const fsi_params& p) {
  FSI_DIM(D);
  // with Q2 cells these levels only precondition the Q2 system: their constant may differ
  const double lps_scale = (p.degree == 2 && p.precond_lps_scale > 0.0) ? p.precond_lps_scale : 1.0;
  constexpr int NP = D == 2 ? 9 : 27;   // nodes of the parent patch
  const Geom g = host_geom(L);
  for (int cell = 0; cell < L.ncell; ++cell) {
    if (L.solid[cell]) continue;
    int i, j, k;
    cell_ijk<D>(g, cell, i, j, k);
    double h[D];
    cell_h<D>(L, i, j, k, h);
    double vol = 1.0;
    for (int r = 0; r < D; ++r) vol *= h[r];
    const double alpha = lps_scale * p.lps_alpha0 * std::pow(vol, 2.0 / D) / (p.rho_f * p.nu_f);
    double K[NL][NL];
    q1_stiffness<D>(h, K);
    const int org[3] = {i - (i & 1), j - (j & 1), k - (k & 1)};   // parent patch origin node
    const int ch[3] = {i & 1, j & 1, k & 1};
    // kap[a][q]: fluctuation at fine node a in terms of the NP patch nodes
    double kap[NL][NP];
    for (int a = 0; a < NL; ++a) {
      for (int q = 0; q < NP; ++q) kap[a][q] = 0.0;
      int pq = 0, mul = 1;
      double s[3];
      for (int r = 0; r < D; ++r) {
        const int pr = ch[r] + ((a >> r) & 1);
        pq += mul * pr;
        mul *= 3;
        s[r] = 0.5 * pr;
      }
      kap[a][pq] += 1.0;
      for (int b = 0; b < NL; ++b) {
        double w = 1.0;
        int pb2 = 0, m2 = 1;
        for (int r = 0; r < D; ++r) {
          const int br = (b >> r) & 1;
          w *= br ? s[r] : 1.0 - s[r];
          pb2 += m2 * 2 * br;
          m2 *= 3;
        }
        kap[a][pb2] -= w;
      }
    }
    for (int q = 0; q < NP; ++q)
      for (int r = 0; r < NP; ++r) {
        double s = 0.0;
        for (int a = 0; a < NL; ++a)
          for (int b = 0; b < NL; ++b) s += kap[a][q] * K[a][b] * kap[b][r];
        if (s == 0.0) continue;
        const int nq = node_at(g, org[0] + q % 3, org[1] + (q / 3) % 3, D == 3 ? org[2] + q / 9 : 0);
        const int nr = node_at(g, org[0] + r % 3, org[1] + (r / 3) % 3, D == 3 ? org[2] + r / 9 : 0);
        add_pst<D>(L, nq, nr, alpha * s);
      }
  }
}

// Coarsest level: gradient-jump penalty gamma h_n^3 / (rho nu) int_F [d_n p][d_n q] over
// interior faces F between fluid cells (a preconditioner-only stabilisation; level 0 has
// no parents), 2-point Gauss per face direction.
template <int D>
void build_cip(Level& L, const fsi_params& p) {
  FSI_DIM(D);
  const double gq[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const Geom g = host_geom(L);
  for (int c1 = 0; c1 < L.ncell; ++c1) {
    int i, j, k;
    cell_ijk<D>(g, c1, i, j, k);
    for (int dir = 0; dir < D; ++dir) {
      const int i2 = i + (dir == 0), j2 = j + (dir == 1), k2 = k + (dir == 2);
      if (i2 >= L.nx || j2 >= L.ny || (D == 3 && k2 >= L.nz)) continue;
      const int c2 = cell_at(g, i2, j2, k2);
      if (L.solid[c1] || L.solid[c2]) continue;
      double h1[D], h2[D];
      cell_h<D>(L, i, j, k, h1);
      cell_h<D>(L, i2, j2, k2, h2);
      double area = 1.0;
      for (int r = 0; r < D; ++r)
        if (r != dir) area *= h1[r];
      const double hn = 0.5 * (h1[dir] + h2[dir]);
      int nodes[2 * NL];
      for (int a = 0; a < NL; ++a) {
        nodes[a] = node_at(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
        nodes[NL + a] = node_at(g, i2 + (a & 1), j2 + ((a >> 1) & 1), k2 + ((a >> 2) & 1));
      }
      for (int q = 0; q < (1 << (D - 1)); ++q) {
        // face point: tangential coordinates from q, normal coordinate 1 in cell 1 and 0 in cell 2
        double t[3];
        for (int r = 0, b = 0; r < D; ++r)
          if (r != dir) t[r] = gq[(q >> b++) & 1];
        double c[2 * NL];
        for (int a = 0; a < NL; ++a) {
          double tang = 1.0;
          for (int r = 0; r < D; ++r)
            if (r != dir) tang *= ((a >> r) & 1) ? t[r] : 1.0 - t[r];
          const double sgn = ((a >> dir) & 1) ? 1.0 : -1.0;
          c[a] = sgn * tang / h1[dir];
          c[NL + a] = -sgn * tang / h2[dir];
        }
        const double w = p.cip_gamma * area / (1 << (D - 1)) * hn * hn * hn / (p.rho_f * p.nu_f);
        for (int a = 0; a < 2 * NL; ++a)
          for (int b = 0; b < 2 * NL; ++b) add_pst<D>(L, nodes[a], nodes[b], w * c[a] * c[b]);
      }
    }
  }
}

template <int D>
fsi_status build_level(fsi_problem* pb, int l) {
  FSI_DIM(D);
  const fsi_params& p = pb->p;
  Level& L = pb->lev[l];
  L.x = axis_points(p, 0, l);
  L.y = axis_points(p, 1, l);
  L.nx = (int)L.x.size() - 1;
  L.ny = (int)L.y.size() - 1;
  if (D == 3) {
    L.z = axis_points(p, 2, l);
    L.nz = (int)L.z.size() - 1;
  } else {
    L.z.assign(1, 0.0);
    L.nz = 0;
  }
  L.nn = (L.nx + 1) * (L.ny + 1) * (L.nz + 1);
  L.ncell = L.nx * L.ny * (D == 3 ? L.nz : 1);
  const Geom g = host_geom(L);
  L.solid.assign(L.ncell, 0);
  for (int c = 0; c < L.ncell; ++c) {
    int i, j, k;
    cell_ijk<D>(g, c, i, j, k);
    const double ctr[3] = {0.5 * (L.x[i] + L.x[i + 1]), 0.5 * (L.y[j] + L.y[j + 1]),
                           D == 3 ? 0.5 * (L.z[k] + L.z[k + 1]) : 0.0};
    bool in = true;
    for (int r = 0; r < D; ++r) in = in && ctr[r] > p.solid_lo[r] && ctr[r] < p.solid_hi[r];
    L.solid[c] = in;
  }
  L.cls.assign(L.nn, 0);
  for (int c = 0; c < L.ncell; ++c) {
    int i, j, k;
    cell_ijk<D>(g, c, i, j, k);
    const uint8_t bit = L.solid[c] ? CL_NS : CL_NF;
    for (int a = 0; a < NL; ++a) L.cls[node_at(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1))] |= bit;
  }
  L.dmask.assign(L.nn, 0);
  for (int n = 0; n < L.nn; ++n) {
    int i, j, k;
    node_ijk<D>(g, n, i, j, k);
    const bool inflow = i == 0, outflow = i == L.nx;
    const bool wall = j == 0 || j == L.ny || (D == 3 && (k == 0 || k == L.nz));
    uint8_t m = 0;
    if (inflow || wall) m |= dm_v<D>();
    if (inflow || outflow || wall) m |= dm_u<D>();
    if (!(L.cls[n] & CL_NF)) m |= dm_p<D>();
    L.dmask[n] = m;
    if (inflow && !wall) L.cls[n] |= CL_INFLOW;
  }
  L.pst.assign((size_t)NPST * L.nn, 0.0);
  if (l >= 1)
    build_lps<D>(L, p);
  else
    build_cip<D>(L, p);
  CHK(upload(pb, &L.d_x, L.x));
  CHK(upload(pb, &L.d_y, L.y));
  CHK(upload(pb, &L.d_z, L.z));
  CHK(upload(pb, &L.d_pst, L.pst));
  CHK(upload(pb, &L.d_solid, L.solid));
  CHK(upload(pb, &L.d_cls, L.cls));
  CHK(upload(pb, &L.d_dmask, L.dmask));
  // batch workspace
  const int B = pb->Bmax;
  const size_t ss = pb->ssz;
  CHK(dalloc(pb, &L.U, (size_t)B * L.nn * NC));
  CHK(dalloc(pb, &L.Uo, (size_t)B * L.nn * NC));
  CHK(dalloc(pb, &L.Dsc, (size_t)B * L.nn * NC));
  const size_t jvals = std::max(jslice<D, double, false>(L.geom()), jslice<D, float, false>(L.geom()));
  CHK(dalloc_bytes(pb, &L.J, (size_t)B * jvals * ss));
  // Vanka inverses: every smoothed level (in 3d level 0 is smoothed too)
  if (l >= 1 || D == 3) {
    CHK(dalloc_bytes(pb, &L.Ainv, (size_t)B * ainv_slice<D>(L.ncell) * ss));
    CHK(dalloc_bytes(pb, &L.Yu, yu_level<D>(L.ncell) * ss));   // shared by the slices
  }
  CHK(dalloc_bytes(pb, &L.x_, (size_t)B * L.nn * NC * ss));
  CHK(dalloc_bytes(pb, &L.b_, (size_t)B * L.nn * NC * ss));
  CHK(dalloc_bytes(pb, &L.r_, (size_t)B * L.nn * NC * ss));
  CHK(dalloc_bytes(pb, &L.t_, (size_t)B * L.nn * NC * ss));
  return FSI_OK;
}

// Pressure stabilisation of Q2 cells (one-level local projection): over every fluid
// Q2 cell K, alpha_K (grad(p - i_h p), grad(q - i_h q))_K with i_h the bilinear
// interpolation on K from its vertices, alpha_K = alpha0 |K| / (rho_f nu_f); the Q2
// Laplace stiffness of the box cell is the tensor form of the 1d quadratic element
// matrices (mass h/30 [4 2 -1; 2 16 2; -1 2 4], stiffness 1/(3h) [7 -8 1; -8 16 -8;
// 1 -8 7]).  Returned as the 5 x 5 node stencil [25][nn] of the node grid N (the cells'
// nodes: local node a = ox + 3 oy of cell (i, j) is node (2 i + ox, 2 j + oy)).
std::vector<double> q2_lps_stencil(const Level& C, const Level& N, const fsi_params& p) {
  std::vector<double> pst((size_t)25 * N.nn, 0.0);
  const int W = N.nx + 1;
  for (int j = 0; j < C.ny; ++j)
    for (int i = 0; i < C.nx; ++i) {
      if (C.solid[i + C.nx * j]) continue;
      const double hx = C.x[i + 1] - C.x[i], hy = C.y[j + 1] - C.y[j];
      double M[2][3][3], Ks[2][3][3];
      const double Mr[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}}, Kr[3][3] = {{7, -8, 1}, {-8, 16, -8}, {1, -8, 7}};
      const double hh[2] = {hx, hy};
      for (int r = 0; r < 2; ++r)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            M[r][a][b] = Mr[a][b] * hh[r] / 30.0;
            Ks[r][a][b] = Kr[a][b] / (3.0 * hh[r]);
          }
      double K[9][9], kap[9][9];
      for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b)
          K[a][b] = Ks[0][a % 3][b % 3] * M[1][a / 3][b / 3] + M[0][a % 3][b % 3] * Ks[1][a / 3][b / 3];
      // kap = I - i_h: node a at (ox/2, oy/2) minus the bilinear combination of the vertex values
      for (int a = 0; a < 9; ++a) {
        const double sx = (a % 3) * 0.5, sy = (a / 3) * 0.5;
        for (int b = 0; b < 9; ++b) {
          double v = a == b ? 1.0 : 0.0;
          const int bx = b % 3, by = b / 3;
          if (bx != 1 && by != 1) v -= (bx == 2 ? sx : 1.0 - sx) * (by == 2 ? sy : 1.0 - sy);
          kap[a][b] = v;
        }
      }
      const double alpha = p.lps_alpha0 * hx * hy / (p.rho_f * p.nu_f);
      for (int q = 0; q < 9; ++q)
        for (int r = 0; r < 9; ++r) {
          double v = 0.0;
          for (int a = 0; a < 9; ++a)
            for (int b = 0; b < 9; ++b) v += kap[a][q] * K[a][b] * kap[b][r];
          if (v == 0.0) continue;
          const int nq = (2 * i + q % 3) + W * (2 * j + q / 3);
          const int slot = (r % 3 - q % 3 + 2) + 5 * (r / 3 - q / 3 + 2);
          pst[(size_t)slot * N.nn + nq] += alpha * v;
        }
    }
  return pst;
}

// ------------------------------------------------------------ profiling
// The timing events carry no system-scope fence: they only measure, and a fence at
// every event would write back and invalidate the caches between the timed launches.
void prof_rec(fsi_problem* pb, hipEvent_t* e, hipStream_t st) {
  Prof& P = pb->prof;
  if (P.used >= P.pool.size()) {
    hipEvent_t ev;
    (void)hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
    P.pool.push_back(ev);
  }
  *e = P.pool[P.used++];
  (void)hipEventRecord(*e, st);
}
struct ProfScope {
  fsi_problem* pb;
  int fam;
  hipStream_t st;
  hipEvent_t e0{}, e1{};
  double bytes;
  ProfScope(fsi_problem* p, int f, hipStream_t s, double by) : pb(p), fam(f), st(s), bytes(by) {
    if (pb->prof.on) prof_rec(pb, &e0, st);
  }
  ~ProfScope() {
    if (!pb->prof.on) return;
    prof_rec(pb, &e1, st);
    pb->prof.ev[fam].push_back({e0, e1});
    pb->prof.bytes[fam] += bytes;
    pb->prof.launches[fam] += 1;
  }
};

// slices whose bytes a profiled launch over a batch of B is charged for
inline int prof_nb(const fsi_problem* pb, int B) { return pb->prof.on ? std::min(pb->prof.pact, B) : B; }
inline int count_active(const std::vector<int>& a) {
  int n = 0;
  for (int v : a) n += v != 0;
  return n;
}

StepPar step_par(const fsi_problem* pb, double k) {
  StepPar sp;
  sp.k = k;
  // shifted Crank-Nicolson damping; with a reference step k_r the dissipation-matched
  // theta = 1/2 + theta0 k_r^2 / k (equal damping per unit time for every step size)
  const double kr = pb->p.theta_ref_k;
  sp.theta = kr > 0.0 ? 0.5 + pb->p.theta0 * kr * kr / k : 0.5 + pb->p.theta0 * k;
  sp.rho_f = pb->p.rho_f; sp.nu_f = pb->p.nu_f; sp.rho_s = pb->p.rho_s;
  sp.mu_s = pb->p.mu_s; sp.lambda_s = pb->p.lambda_s;
  sp.peak = pb->p.inflow_peak; sp.ramp_time = pb->p.ramp_time;
  return sp;
}

// ------------------------------------------------------------ assembly
template <int D>
fsi_status residual(fsi_problem* pb, int B, const StepPar& sp, const double* U, const double* Uo, double* R,
                    const int* act, hipStream_t st) {
  FSI_DIM(D);
  Level& F = pb->lev[pb->nlev - 1];
  const Geom g = F.geom();
  if constexpr (D == 2) {
    if (pb->deg == 2) {
      const Geom gc = pb->lev[pb->nlev - 2].geom();
      ProfScope ps(pb, F_RES, st, (double)prof_nb(pb, B) * (F.nn * NC * 8.0 * 3 + gc.ncell * 45 * 8.0 * 2));
      k_elem_residual_q2<<<grid1(gc.ncell, B), TPB, 0, st>>>(gc, g, sp, U, Uo, pb->Re2, act);
      k_gather_residual_q2<<<grid1(g.nn, B), TPB, 0, st>>>(gc, g, sp, pb->pst2, pb->Re2, U, pb->tdev, R, act);
      HIPCHK(hipGetLastError());
      return FSI_OK;
    }
  }
  {
    ProfScope ps(pb, F_RES, st, (double)prof_nb(pb, B) * (F.nn * NC * 8.0 * 3 + F.ncell * NE * 8.0 * 2));
    k_elem_residual<D><<<grid1(g.ncell, B), TPB, 0, st>>>(g, sp, U, Uo, pb->Re, act);
    k_gather_residual<D><<<grid1(g.nn, B), TPB, 0, st>>>(g, sp, pb->Re, U, pb->tdev, R, act);
  }
  HIPCHK(hipGetLastError());
  return FSI_OK;
}

// Cells per block of the fused Vanka pass on a level (and the block width of its
// Vanka inverse storage): 16 in 2d; in 3d 32 where a colour has cells enough
// over the batch to fill the GPU with wide blocks (fsi_params.vanka_wide_cells,
// 8192 by default), else 8.
template <int D>
int vanka_vc(const fsi_problem* pb, const Geom& g, int B) {
  if (D == 2) return 16;
  const long long th = pb->p.vanka_wide_cells > 0 ? pb->p.vanka_wide_cells : 8192;
  return (long long)(g.ncell / Dm<D>::NCOL) * B >= th ? 32 : 8;
}

// Launch order of the SpMV and of the fused Vanka pass: slices as the fast grid
// dimension (1) or the slow one (0).  fsi_params.spmv_slice_fast /
// vanka_slice_fast choose; -1 keeps the measured defaults: slices fast for the
// 2d FP64 SpMV (the 128x32-cell, 32-slice one 4% faster; the 3d 64x16x16 one was
// 8% slower) and for the 3d and 2d FP64 Vanka passes (the 2d FP32 pass was 6%
// slower that way).
template <int D, class S>
int spmv_slice_fast(const fsi_problem* pb) {
  const int f = pb->p.spmv_slice_fast;
  return f >= 0 ? f : ((D == 2 && sizeof(S) == 8) ? 1 : 0);
}
template <int D, class S>
int vanka_slice_fast(const fsi_problem* pb) {
  const int f = pb->p.vanka_slice_fast;
  return f >= 0 ? f : ((D == 3 || sizeof(S) == 8) ? 1 : 0);
}

// Jacobian of the finest level (always) and, when precond is set, the multigrid
// hierarchy: injected coarse states, coarse-level Jacobians, Vanka inverses and
// the coarsest-level solver (2d: explicit inverse; 3d: Vanka inverses, the
// level is smoothed).  CJ selects the compressed block layout (the step
// Jacobian) or the full one (the transposed adjoint operator).
template <int D, class S, bool CJ>
fsi_status assemble_levels(fsi_problem* pb, int B, const StepPar& sp, const int* act, hipStream_t st,
                           bool precond = true, bool transpose = false, double* save_fine = nullptr) {
  FSI_DIM(D);
  if (CJ && transpose) return FSI_ERR_ARG;   // a transposed block needs the full layout
  const int L = pb->nlev - 1;
  // Q2: the Q1 hierarchy is only the preconditioner, so without precond nothing of it is rebuilt
  const int lstop = precond ? 0 : (pb->deg == 2 ? L + 1 : L);
  for (int l = L; l >= lstop; --l) {
    Level& lv = pb->lev[l];
    const Geom g = lv.geom();
    const double* U = (l == L) ? pb->U : lv.U;
    const double* Uo = (l == L) ? pb->Uold : lv.Uo;
    if (l < L) {
      const Level& f = pb->lev[l + 1];
      const double* Uf = (l + 1 == L) ? pb->U : f.U;
      const double* Uof = (l + 1 == L) ? pb->Uold : f.Uo;
      k_inject<D><<<grid1(g.nn, B), TPB, 0, st>>>(g, f.geom(), Uf, lv.U);
      k_inject<D><<<grid1(g.nn, B), TPB, 0, st>>>(g, f.geom(), Uof, lv.Uo);
    }
    {
      ProfScope ps(pb, F_JAC, st, (double)prof_nb(pb, B) * (g.ncell * NE * NE * 8.0 + 2.0 * g.nn * NC * 8));
      k_elem_jacobian<D, false><<<dim3((g.ncell + jac_cells<D>() - 1) / jac_cells<D>(), B),
                                  jac_cells<D>() * jac_waves<D>(), 0, st>>>(g, sp, U, Uo, pb->Ke, act);
    }
    k_gather_jacobian<D, S, CJ><<<grid1(g.nn, B), TPB, 0, st>>>(g, sp.k, pb->Ke, (S*)lv.J, lv.Dsc, act, 1);
    if (transpose) {
      // adjoint (2d): the operator of every level becomes the transpose of the free block (B = 1)
      const size_t bytes = jslice<D, S, false>(g) * sizeof(S);
      if (l == L && save_fine) HIPCHK(hipMemcpyAsync(save_fine, lv.J, bytes, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(pb->Jtmp, lv.J, bytes, hipMemcpyDeviceToDevice, st));
      k_transpose_J<double><<<grid1(g.nn, 1), TPB, 0, st>>>(g, sp.k, (const double*)pb->Jtmp, (double*)lv.J, lv.Dsc);
    }
    if (!precond) break;
    if (l >= 1 || D == 3) {
      k_vanka_factor<D, S, CJ><<<dim3((g.ncell + vf_patches<D>() - 1) / vf_patches<D>(), B),
                                 vf_lanes<D>() * vf_patches<D>(), 0, st>>>(g, sp.k, (const S*)lv.J, (S*)lv.Ainv,
                                                                          (S*)lv.Yu, vanka_vc<D>(pb, g, B), act);
    } else {
      const size_t lds_f = (size_t)5 * pb->cbs * pb->cbs * sizeof(double);
      const size_t lds_i = (size_t)3 * pb->cbs * pb->cbs * sizeof(double);
      k_coarse_factor<S, CJ><<<B, CF_THREADS, lds_f, st>>>(g, sp.k, (const S*)lv.J, pb->cbs, pb->cnsb, pb->cDinv,
                                                           pb->cW, pb->cL, act);
      k_coarse_inverse<S><<<dim3(pb->cnsb, B), CF_THREADS, lds_i, st>>>(g, pb->cbs, pb->cnsb, pb->cDinv, pb->cW,
                                                                        pb->cL, pb->cY, (S*)pb->cAinv, act);
    }
    HIPCHK(hipGetLastError());
  }
  if constexpr (D == 2) {
    if (pb->deg == 2) {
      // the Krylov operator: the exact Jacobian of the Q2 step (and its row scaling)
      const Level& F = pb->lev[L];
      const Geom gc = pb->lev[L - 1].geom(), gn = F.geom();
      {
        ProfScope ps(pb, F_JAC, st, (double)prof_nb(pb, B) * (gc.ncell * 45.0 * 45.0 * 8.0 + 2.0 * gn.nn * NC * 8));
        k_elem_jacobian_q2<<<dim3((gc.ncell + Q2_JAC_CELLS - 1) / Q2_JAC_CELLS, B), Q2_JAC_THREADS, 0, st>>>(
            gc, gn, sp, pb->U, pb->Uold, pb->Ke2, act);
      }
      k_gather_jacobian_q2<S><<<grid1(gn.nn, B), TPB, 0, st>>>(gc, gn, sp.k, pb->pst2, pb->Ke2, (S*)pb->J2, F.Dsc,
                                                                act);
      HIPCHK(hipGetLastError());
    }
  }
  return FSI_OK;
}

// Blocks per slice of a launch with the slices as the slow grid dimension, rounded up
// to a multiple of the 8 XCDs: consecutive blocks go to consecutive XCDs, so block x
// of every slice then runs on XCD x mod 8, and the values every slice shares (the
// displacement rows of slice 0, the stabilisation stencil) are fetched by one XCD and
// reused from its cache by the following slices.  The extra blocks return at once.
inline int xcd_pad(int nb) { return (nb + 7) / 8 * 8; }

// Grid mode of a launch with the slices as the fast grid dimension: under the
// FGMRES mask the kernel takes its slice from the ordered list of the working
// slices (mode 2, act replaced by that list), else from its column (mode 1,
// act the per-slice flags or null).
inline int slice_mode(const fsi_problem* pb, int sf, const int*& act) {
  if (sf && act && act == pb->gact) {
    act = pb->gord;
    return 2;
  }
  return sf;
}

// y = D (b - A x) (or D A x)
template <int D, class S, bool CJ>
void spmv(const fsi_problem* pb, const Geom& g, int B, double k, const S* J, const S* x, const S* b, const double* Dv,
          S* y, const int* act, hipStream_t st) {
  const int nb =
      !jrowtiles<D, S>() ? (g.nn + 63) / 64 : (jntx<D, S>(g, 0) * jrows<D>(g) * jtx<D, S>() + 63) / 64;
  const int sf = slice_mode(pb, spmv_slice_fast<D, S>(pb) && nb <= 65535 ? 1 : 0, act);
  k_spmv<D, S, CJ><<<sf ? dim3(B, nb) : dim3(xcd_pad(nb), B), spmv_threads<D>(), 0, st>>>(g, k, J, x, b, Dv, y, act,
                                                                                      sf);
}

// The Krylov operator's product y = D (b - J x) (or D J x): the Q1 step Jacobian of the
// finest level, or with Q2 cells their Jacobian (in the linear solve's type).
template <int D, class S, bool CJ>
void krylov_spmv(const fsi_problem* pb, int B, double k, const S* x, const S* b, const double* Dv, S* y,
                 const int* act, hipStream_t st) {
  const Level& F = pb->lev[pb->nlev - 1];
  if constexpr (D == 2 && CJ) {
    if (pb->deg == 2) {
      k_spmv_q2<S><<<grid1(F.nn, B), TPB, 0, st>>>(F.geom(), k, pb->pst2, (const S*)pb->J2, x, b, Dv, y, act);
      return;
    }
  }
  spmv<D, S, CJ>(pb, F.geom(), B, k, (const S*)F.J, x, b, Dv, y, act, st);
}

// ------------------------------------------------------------ multigrid
template <int D, class S, bool CJ>
void smooth(fsi_problem* pb, int l, int B, double k, int sweeps, bool zero_first, S* x, const S* b, const int* act,
            hipStream_t st) {
  FSI_DIM(D);
  Level& lv = pb->lev[l];
  const Geom g = lv.geom();
  const S om = (S)pb->p.vanka_omega;
  const bool fine = l == pb->nlev - 1;
  constexpr int NCOL = Dm<D>::NCOL;
  // the passes alternate between x and the level's residual buffer; an even
  // number of colours per sweep leaves the result in x
  S* buf[2] = {x, (S*)lv.r_};
  int cur = 0;
  for (int s = 0; s < sweeps; ++s)
    for (int c = 0; c < NCOL; ++c) {
      const bool zero = zero_first && s == 0 && c == 0;
      const int vc = vanka_vc<D>(pb, g, B);
      const int nc = color_info<D>(g, c, vc).nc;
      const double vec = 3.0 * g.nn * NC * sizeof(S);
      // inverse rows per slice; in the split patch solve Y1, Y2 once per launch
      constexpr bool SP = patch_split<D, S, CJ>();
      const double inv = (double)ainv_rows<D, SP>() * NE * nc * sizeof(S);
      const double ysh = SP ? (double)yu_cell<D>() * nc * sizeof(S) : 0.0;
      const int nb = prof_nb(pb, B);
      const double by = zero ? (double)nb * (inv + 2.0 * g.nn * NC * sizeof(S)) + ysh
                             : jbytes_launch<D, S, CJ>(g, nb) + (double)nb * (inv + vec) + ysh + (double)NPST * g.nn * 8.0;
      ProfScope ps(pb, fine ? F_SMOOTH : F_COARSE_LEV, st, by);
      const int ncopy = (g.nn + NC * 64 - 1) / (NC * 64);
      const S *J = (const S*)lv.J, *Ai = (const S*)lv.Ainv, *Yu = (const S*)lv.Yu;
      // blocks of the colour (vc cells each) and of the copy of the other nodes, per slice.
      // Slices as the fast grid dimension: the blocks of one tile in all slices are dispatched
      // together, so the values every slice shares (displacement rows of slice 0, the
      // stabilisation stencil) are fetched once per XCD cache and reused (the 2d FP64 pass on
      // 128x32 cells and 32 slices 4% faster, the 3d one on 64x16x16 cells and 16 slices 13%);
      // the 2d FP32 pass (row tiles, six waves per SIMD) was 6% slower that way.
      const int nbx = (nc + vc - 1) / vc + ncopy;
      const int* sel = act;
      const int sf = slice_mode(pb, vanka_slice_fast<D, S>(pb) && nbx <= 65535 ? 1 : 0, sel);
      const dim3 grid = sf ? dim3(B, nbx) : dim3(xcd_pad(nbx), B);
      if constexpr (D == 2) {
        k_vanka_color<D, S, 16, CJ><<<grid, NC * 64, 0, st>>>(g, k, c, om, zero ? 1 : 0, J, Ai, Yu, b, buf[cur],
                                                              buf[cur ^ 1], sel, sf);
      } else if (vc == 32) {
        k_vanka_color<D, S, 32, CJ><<<grid, NC * 64, 0, st>>>(g, k, c, om, zero ? 1 : 0, J, Ai, Yu, b, buf[cur],
                                                              buf[cur ^ 1], sel, sf);
      } else {
        k_vanka_color<D, S, 8, CJ><<<grid, NC * 64, 0, st>>>(g, k, c, om, zero ? 1 : 0, J, Ai, Yu, b, buf[cur],
                                                             buf[cur ^ 1], sel, sf);
      }
      cur ^= 1;
    }
}

// Sweeps of the Vanka smoother that stand in for a direct solve on the 3d
// coarsest level (17 x 5 x 5 nodes at the workloads' level-0 mesh).
constexpr int COARSEST_SWEEPS_3D = 4;

template <int D, class S, bool CJ>
void vcycle(fsi_problem* pb, int B, double k, const S* rhs, S* out, const int* act, hipStream_t st) {
  FSI_DIM(D);
  const int L = pb->nlev - 1;
  // level L uses rhs/out directly; lower levels their own b_/x_
  for (int l = L; l >= 1; --l) {
    Level& lv = pb->lev[l];
    Level& lc = pb->lev[l - 1];
    const S* b = (l == L) ? rhs : (const S*)lv.b_;
    S* x = (l == L) ? out : (S*)lv.x_;
    smooth<D, S, CJ>(pb, l, B, k, l == L ? pb->p.vanka_sweeps : pb->p.vanka_sweeps_coarse, true, x, b, act, st);
    const Geom g = lv.geom();
    {
      const int nb = prof_nb(pb, B);
      const double by = jbytes_launch<D, S, CJ>(g, nb) + (double)nb * 3.0 * g.nn * NC * sizeof(S) + (double)NPST * g.nn * 8.0;
      ProfScope ps(pb, l == L ? F_LEVEL_RES : F_COARSE_LEV, st, by);
      spmv<D, S, CJ>(pb, g, B, k, (const S*)lv.J, x, b, nullptr, (S*)lv.r_, act, st);
    }
    k_restrict<D, S><<<grid1(lc.nn, B), TPB, 0, st>>>(lc.geom(), g, (const S*)lv.r_, (S*)lc.b_, act);
  }
  {
    Level& l0 = pb->lev[0];
    const int n0 = l0.nn * NC;
    if constexpr (D == 2) {
      ProfScope ps(pb, F_COARSE_SOLVE, st, (double)prof_nb(pb, B) * ((double)n0 * n0 + 2.0 * n0) * sizeof(S));
      k_coarse_gemv<S><<<dim3((n0 + 63) / 64, B), CG_THREADS, 0, st>>>(l0.geom(), (const S*)pb->cAinv,
                                                                       (const S*)l0.b_, (S*)l0.x_, act);
    } else {
      smooth<D, S, CJ>(pb, 0, B, k, COARSEST_SWEEPS_3D, true, (S*)l0.x_, (const S*)l0.b_, act, st);
    }
  }
  for (int l = 1; l <= L; ++l) {
    Level& lv = pb->lev[l];
    Level& lc = pb->lev[l - 1];
    const S* b = (l == L) ? rhs : (const S*)lv.b_;
    S* x = (l == L) ? out : (S*)lv.x_;
    k_prolong_add<D, S><<<grid1(lv.nn, B), TPB, 0, st>>>(lv.geom(), lc.geom(), (const S*)lc.x_, x, act);
    smooth<D, S, CJ>(pb, l, B, k, l == L ? pb->p.vanka_sweeps : pb->p.vanka_sweeps_coarse, false, x, b, act, st);
  }
}

// One V-cycle on the finest-level buffers (rhs = pb->tmp, out = pb->w), replayed
// from a captured graph when no per-kernel profiling is requested.  The graph
// depends on the batch size and the step size; pointers are fixed per problem.
template <int D, class S, bool CJ>
fsi_status vcycle_run(fsi_problem* pb, int B, double k, hipStream_t st) {
  const bool mixed = sizeof(S) == 4;
  if (!pb->use_graphs || pb->prof.on) {
    vcycle<D, S, CJ>(pb, B, k, (const S*)pb->tmp, (S*)pb->w, pb->gact, st);
    HIPCHK(hipGetLastError());
    return FSI_OK;
  }
  if (!pb->vc_exec || pb->vc_B != B || pb->vc_k != k || pb->vc_mixed != mixed || pb->vc_cj != CJ) {
    if (pb->vc_exec) {
      HIPCHK(hipGraphExecDestroy(pb->vc_exec));
      pb->vc_exec = nullptr;
    }
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    vcycle<D, S, CJ>(pb, B, k, (const S*)pb->tmp, (S*)pb->w, pb->gact, st);
    HIPCHK(hipStreamEndCapture(st, &graph));
    HIPCHK(hipGraphInstantiate(&pb->vc_exec, graph, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(graph));
    pb->vc_B = B;
    pb->vc_k = k;
    pb->vc_mixed = mixed;
    pb->vc_cj = CJ;
  }
  HIPCHK(hipGraphLaunch(pb->vc_exec, st));
  return FSI_OK;
}

// ------------------------------------------------------------ FGMRES
// Classical Gram-Schmidt twice against V_0..V_j for the new Arnoldi vector a (in
// pb->tmp), its norm, V_{j+1} = a / |a|, and the Givens update of column j.
template <int D, class S>
void arnoldi_tail(fsi_problem* pb, int B, int j, int n, hipStream_t st) {
  Level& F = pb->lev[pb->nlev - 1];
  (void)F;
  const int R = pb->R;
  const size_t vb = (size_t)(R + 1) * n;
  S* V = (S*)pb->V;
  S* a = (S*)pb->tmp;
  const int chunk = std::max(KDOT_CHUNK, (n + KDOT_BLOCKS * 256 - 1) / (KDOT_BLOCKS * 256) * 256);
  const int nchunk = (n + chunk - 1) / chunk;
  const dim3 gb((B + 63) / 64), tb(64);
  k_multidot<S><<<dim3(nchunk, B), RED_T, 0, st>>>(n, j + 1, a, (size_t)n, V, vb, (size_t)n, chunk, pb->partial,
                                                     nchunk, pb->gact);
  k_reduce_partials<<<B, 64, 0, st>>>(j + 1, nchunk, pb->partial, pb->hcol, 64, pb->gact);
  k_multiaxpy<S><<<grid1(n, B), TPB, 0, st>>>(n, j + 1, a, (size_t)n, V, vb, (size_t)n, pb->hcol, 64, -1.0, pb->gact);
  k_multidot<S><<<dim3(nchunk, B), RED_T, 0, st>>>(n, j + 1, a, (size_t)n, V, vb, (size_t)n, chunk, pb->partial,
                                                     nchunk, pb->gact);
  k_reduce_partials<<<B, 64, 0, st>>>(j + 1, nchunk, pb->partial, pb->hcol2, 64, pb->gact);
  k_multiaxpy<S><<<grid1(n, B), TPB, 0, st>>>(n, j + 1, a, (size_t)n, V, vb, (size_t)n, pb->hcol2, 64, -1.0, pb->gact);
  k_multidot<S><<<dim3(nchunk, B), RED_T, 0, st>>>(n, 1, a, (size_t)n, a, (size_t)n, 0, chunk, pb->partial, nchunk,
                                                     pb->gact);
  k_reduce_partials<<<B, 64, 0, st>>>(1, nchunk, pb->partial, pb->res, 1, pb->gact);
  k_cgs_combine<<<gb, tb, 0, st>>>(j, pb->hcol, pb->hcol2, pb->res, pb->gact, B);
  k_scale<S><<<grid1(n, B), TPB, 0, st>>>(n, a, (size_t)n, V + (size_t)(j + 1) * n, vb, pb->res, 1, 1, pb->gact);
  k_givens<<<gb, tb, 0, st>>>(j, R, pb->H, pb->hcol, pb->cs, pb->sn, pb->gv, pb->res, pb->beta0, pb->ltol, pb->gstate,
                              pb->ncol, pb->gact, B);
}

// Capture Arnoldi step j (Z_j = M^{-1} (V_j / D) with the V-cycle, the product
// a = D J Z_j, orthogonalisation, Givens update, the slices' new masks, and their
// states copied to pinned host memory) into one graph.
template <int D, class S, bool CJ>
fsi_status capture_step(fsi_problem* pb, int B, double k, int j, hipGraphExec_t* out, hipStream_t st) {
  FSI_DIM(D);
  Level& F = pb->lev[pb->nlev - 1];
  const int n = F.nn * NC;
  const int R = pb->R;
  const size_t vb = (size_t)(R + 1) * n, zb = (size_t)R * n;
  S* Vj = (S*)pb->V + (size_t)j * n;
  S* Zj = (S*)pb->Z + (size_t)j * n;
  S* w = (S*)pb->w;
  S* a = (S*)pb->tmp;
  hipGraph_t graph;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  k_unscale<S><<<grid1(n, B), TPB, 0, st>>>(n, Vj, vb, F.Dsc, a, pb->gact);
  vcycle<D, S, CJ>(pb, B, k, (const S*)a, w, pb->gact, st);
  k_scale<S><<<grid1(n, B), TPB, 0, st>>>(n, w, (size_t)n, Zj, zb, nullptr, 0, 2, pb->gact);
  krylov_spmv<D, S, CJ>(pb, B, k, w, nullptr, F.Dsc, a, pb->gact, st);
  arnoldi_tail<D, S>(pb, B, j, n, st);
  k_update_gact<<<1, 64, 0, st>>>(pb->nact, pb->gstate, pb->gact, pb->gord, B,
                                  pb->hst_pin + (size_t)(j & 1) * pb->Bmax);
  const hipError_t e0 = hipGetLastError();
  const hipError_t e1 = hipStreamEndCapture(st, &graph);
  if (e0 != hipSuccess || e1 != hipSuccess) return FSI_ERR_HIP;
  const hipError_t e2 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e2 == hipSuccess ? FSI_OK : FSI_ERR_HIP;
}

// The step graphs of (B, k, S, CJ): found in the cache, or a new empty entry (graphs
// are captured when first needed); the least recently used entry makes room.
template <int D, class S, bool CJ>
fsi_status step_graphs(fsi_problem* pb, int B, double k, std::vector<hipGraphExec_t>*& ex, hipStream_t st) {
  constexpr int KEEP = 4;
  const bool mixed = sizeof(S) == 4;
  for (auto& e : pb->sg)
    if (e.B == B && e.k == k && e.mixed == mixed && e.cj == CJ) {
      e.used = ++pb->sg_clock;
      ex = &e.ex;
      return FSI_OK;
    }
  if ((int)pb->sg.size() >= KEEP) {
    auto old = std::min_element(pb->sg.begin(), pb->sg.end(),
                                [](const fsi_problem::StepGraphs& a, const fsi_problem::StepGraphs& b) {
                                  return a.used < b.used;
                                });
    HIPCHK(hipStreamSynchronize(st));
    for (hipGraphExec_t x : old->ex)
      if (x) HIPCHK(hipGraphExecDestroy(x));
    pb->sg.erase(old);
  }
  pb->sg.push_back({B, k, mixed, CJ, std::vector<hipGraphExec_t>(pb->R, nullptr), ++pb->sg_clock});
  ex = &pb->sg.back().ex;
  return FSI_OK;
}

// Solve J dx = -R for the slices with nact[b] = 1 (row-scaled system D J dx = -D R),
// right-preconditioned FGMRES(R) with classical Gram-Schmidt applied twice; the
// preconditioner is one multigrid V-cycle.  The solution (type S) goes to pb->xs.
template <int D, class S, bool CJ>
fsi_status fgmres(fsi_problem* pb, int B, double k, std::vector<int>& kits, hipStream_t st,
                  std::vector<int>* failed = nullptr) {
  FSI_DIM(D);
  Level& F = pb->lev[pb->nlev - 1];
  const Geom g = F.geom();
  const int n = F.nn * NC;
  const int R = pb->R;
  const size_t vb = (size_t)(R + 1) * n;   // per-slice stride of V
  const size_t zb = (size_t)R * n;         // per-slice stride of Z
  S* V = (S*)pb->V;
  S* Z = (S*)pb->Z;
  S* w = (S*)pb->w;
  S* xs = (S*)pb->xs;
  S* tmp = (S*)pb->tmp;
  const int chunk = std::max(KDOT_CHUNK, (n + KDOT_BLOCKS * 256 - 1) / (KDOT_BLOCKS * 256) * 256);
  const int nchunk = (n + chunk - 1) / chunk;
  const dim3 gb((B + 63) / 64), tb(64);
  std::vector<int> hstate(B);
  if (failed) failed->assign(B, 0);
  HIPCHK(hipMemcpyAsync(pb->ltol, pb->ltol_h.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
  k_fill<S><<<1024, TPB, 0, st>>>((size_t)B * n, xs, (S)0);
  k_update_gact<<<1, 64, 0, st>>>(pb->nact, nullptr, pb->gact, pb->gord, B);   // gact = nact
  int total = 0;
  for (int cycle = 0;; ++cycle) {
    // V0 = D (b - J xs), b = -R
    if (cycle == 0) {
      k_scale_rhs<S><<<grid1(n, B), TPB, 0, st>>>(n, pb->Res, F.Dsc, V, vb, pb->gact);
    } else {
      k_scale_rhs<S><<<grid1(n, B), TPB, 0, st>>>(n, pb->Res, nullptr, tmp, (size_t)n, pb->gact);
      krylov_spmv<D, S, CJ>(pb, B, k, xs, tmp, F.Dsc, w, pb->gact, st);
      k_scale<S><<<grid1(n, B), TPB, 0, st>>>(n, w, (size_t)n, V, vb, nullptr, 0, 2, pb->gact);
    }
    k_multidot<S><<<dim3(nchunk, B), RED_T, 0, st>>>(n, 1, V, vb, V, vb, 0, chunk, pb->partial, nchunk, pb->gact);
    k_reduce_partials<<<B, 64, 0, st>>>(1, nchunk, pb->partial, pb->beta, 1, pb->gact);
    k_init_cycle<<<gb, tb, 0, st>>>(R, cycle, pb->beta, pb->beta0, pb->gv, pb->gstate, pb->ncol, pb->ltol, pb->gact,
                                    B);
    k_update_gact<<<1, 64, 0, st>>>(pb->nact, pb->gstate, pb->gact, pb->gord, B);
    k_scale<S><<<grid1(n, B), TPB, 0, st>>>(n, V, vb, V, vb, pb->beta, 1, 1, pb->gact);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hstate.data(), pb->gstate, B * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool any = false;
    for (int b = 0; b < B; ++b) any |= hstate[b] == 0;
    if (!any) break;
    if (pb->prof.on) {
      int na = 0;
      for (int b = 0; b < B; ++b) na += hstate[b] == 0;
      pb->prof.pact = na;
    }
    int jmax = 0;
    if (pb->use_graphs && !pb->prof.on && pb->hst_pin) {
      // Arnoldi steps from graphs, one step ahead: step j + 1 is queued before the host
      // reads the states step j wrote, so the GPU does not wait for the host between
      // steps.  A step queued after the last slice has converged finds every slice
      // masked out and changes nothing.
      std::vector<hipGraphExec_t>* ex = nullptr;
      CHK(step_graphs<D, S, CJ>(pb, B, k, ex, st));
      auto launch = [&](int j) -> fsi_status {
        if (!(*ex)[j]) CHK(capture_step<D, S, CJ>(pb, B, k, j, &(*ex)[j], st));
        HIPCHK(hipGraphLaunch((*ex)[j], st));
        HIPCHK(hipEventRecord(pb->step_ev[j & 1], st));
        return FSI_OK;
      };
      CHK(launch(0));
      for (int j = 0; j < R; ++j) {
        if (j + 1 < R && total + 1 < pb->p.gmres_maxit) CHK(launch(j + 1));
        HIPCHK(hipEventSynchronize(pb->step_ev[j & 1]));
        const int* hs = pb->hst_pin + (size_t)(j & 1) * pb->Bmax;
        any = false;
        for (int b = 0; b < B; ++b) {
          if (hstate[b] == 0) kits[b] += 1;
          hstate[b] = hs[b];
          any |= hstate[b] == 0;
        }
        ++total;
        jmax = j + 1;
        if (!any || total >= pb->p.gmres_maxit) break;
      }
      // the look-ahead step (if queued) has run before anything later on the stream
    } else {
    for (int j = 0; j < R; ++j) {
      S* Vj = V + (size_t)j * n;
      S* Zj = Z + (size_t)j * n;
      // Z_j = M^{-1} (V_j / D);  a = D J Z_j  (the new Arnoldi vector a lives in tmp)
      k_unscale<S><<<grid1(n, B), TPB, 0, st>>>(n, Vj, vb, F.Dsc, tmp, pb->gact);
      CHK(vcycle_run<D, S, CJ>(pb, B, k, st));
      k_scale<S><<<grid1(n, B), TPB, 0, st>>>(n, w, (size_t)n, Zj, zb, nullptr, 0, 2, pb->gact);
      S* a = tmp;
      {
        const int nb = prof_nb(pb, B);
        const double jb = pb->deg == 2 ? (double)nb * 625.0 * F.nn * sizeof(S) + 25.0 * F.nn * 8.0 : jbytes_launch<D, S, CJ>(g, nb);
        ProfScope ps(pb, F_GMRES_SPMV, st, jb + (double)nb * (2.0 * n * sizeof(S) + n * 8.0) + (double)NPST * F.nn * 8.0);
        krylov_spmv<D, S, CJ>(pb, B, k, w, nullptr, F.Dsc, a, pb->gact, st);
      }
      arnoldi_tail<D, S>(pb, B, j, n, st);
      HIPCHK(hipGetLastError());
      for (int b = 0; b < B; ++b)
        if (hstate[b] == 0) kits[b] += 1;
      ++total;
      jmax = j + 1;
      k_update_gact<<<1, 64, 0, st>>>(pb->nact, pb->gstate, pb->gact, pb->gord, B);
      HIPCHK(hipMemcpyAsync(hstate.data(), pb->gstate, B * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      any = false;
      int na = 0;
      for (int b = 0; b < B; ++b) {
        any |= hstate[b] == 0;
        na += hstate[b] == 0;
      }
      pb->prof.pact = na;
      if (!any || total >= pb->p.gmres_maxit) break;
    }
    }
    // xs += Z y on every slice that ran in this cycle (ncol > 0)
    k_trisolve<<<gb, tb, 0, st>>>(R, pb->H, pb->gv, pb->ncol, pb->ycoef, pb->nact, B);
    k_multiaxpy<S><<<grid1(n, B), TPB, 0, st>>>(n, jmax, xs, (size_t)n, Z, zb, (size_t)n, pb->ycoef, 64, 1.0,
                                                  pb->nact);
    HIPCHK(hipGetLastError());
    if (!any) break;
    if (total >= pb->p.gmres_maxit) {
      // the slices still running did not reach their tolerance
      if (failed)
        for (int b = 0; b < B; ++b) (*failed)[b] = hstate[b] == 0 ? 1 : 0;
      return FSI_ERR_LINEAR;
    }
    // restart the unconverged slices
    k_update_gact<<<1, 64, 0, st>>>(pb->nact, pb->gstate, pb->gact, pb->gord, B);
  }
  return FSI_OK;
}

// ------------------------------------------------------------ propagation
struct RunStats {
  std::vector<int> newton, krylov, status;
};

// Stage timing of the Newton iterations (stats->stage_ms[0..3]): HIP events on
// the call's stream at the stage boundaries, summed after the call has finished.
hipEvent_t stage_mark(fsi_problem* pb, hipStream_t st) {
  if (pb->sused >= pb->spool.size()) {
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    pb->spool.push_back(ev);
  }
  hipEvent_t ev = pb->spool[pb->sused++];
  return hipEventRecord(ev, st) == hipSuccess ? ev : nullptr;
}
void stage_span(fsi_problem* pb, int stage, hipEvent_t a, hipEvent_t b) {
  if (a && b) pb->sev.push_back({stage, a, b});
}

template <int D, class S>
fsi_status newton_solve_step(fsi_problem* pb, int B, const StepPar& sp, std::vector<int>& hact, RunStats& rs,
                             hipStream_t st) {
  FSI_DIM(D);
  Level& F = pb->lev[pb->nlev - 1];
  const int nn = F.nn;
  const int maxit = pb->p.newton_maxit;
  std::vector<double> prev((size_t)B * 3, -1.0), hm((size_t)B * 6), est_prev(B, 1e300);
  std::vector<int> nact(hact);
  // pending[b]: the update test of slice b held after an iteration whose linear solve
  // converged; the slice is done once the FP64 residual at its new state passes too
  std::vector<int> pending(B, 0), lin_failed(B, 0), last_lin_failed(B, 0);
  for (int it = 1; it <= maxit + 1; ++it) {
    // per-slice Krylov tolerance (inexact Newton): the first iteration only has to bring
    // the extrapolated guess close enough for the quadratic phase; later ones are tight
    // while the error estimate is large and loose once it is near the Newton tolerance,
    // where the update only has to be resolved to a few digits:
    // eta = clamp(0.1 rtol / est, lin_rtol, 1e-2)
    for (int b = 0; b < B; ++b)
      pb->ltol_h[b] = it == 1 ? pb->p.lin_rtol_first
                              : std::min(1e-2, std::max(pb->p.lin_rtol, 0.1 * pb->p.newton_rtol / est_prev[b]));
    const int k0 = rs.krylov[0];
    HIPCHK(hipMemcpyAsync(pb->nact, nact.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
    pb->prof.pact = count_active(nact);
    hipEvent_t e0 = stage_mark(pb, st);
    CHK(residual<D>(pb, B, sp, pb->U, pb->Uold, pb->Res, pb->nact, st));
    hipEvent_t e1 = stage_mark(pb, st);
    stage_span(pb, 0, e0, e1);
    bool anyp = false;
    for (int b = 0; b < B; ++b) anyp |= pending[b] != 0;
    // with newton_res_accept > 0 every slice updated at least once is also tested: a residual
    // at that (round-off) level ends its step without another solve
    const bool early = pb->p.newton_res_accept > 0.0 && it >= 2;
    if (anyp || early) {
      // residual test of the pending slices: per field, max |D R_f| <= res_rtol max |U_f|,
      // D the row scaling of the last Jacobian (the refinement test of the mixed path:
      // the FP64 residual of the FP64 state)
      k_residual_norms<D><<<dim3(pb->nchunk_n, B), RED_T, 0, st>>>(nn, pb->Res, F.Dsc, pb->U, pb->chunk_n, pb->npart,
                                                                  pb->nchunk_n, pb->nact);
      k_max_partials<<<(B + 63) / 64, 64, 0, st>>>(pb->nchunk_n, pb->npart, pb->nmax, B);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hm.data(), pb->nmax, (size_t)B * 6 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      hipEvent_t ec = stage_mark(pb, st);
      stage_span(pb, 3, e1, ec);
      e1 = ec;
      bool left = false;
      for (int b = 0; b < B; ++b) {
        if (pending[b] || (early && nact[b])) {
          const double tol = pending[b] ? pb->p.newton_res_rtol : pb->p.newton_res_accept;
          bool ok = true;
          for (int f = 0; f < 3; ++f) {
            const double r = hm[(size_t)b * 6 + f], un = hm[(size_t)b * 6 + 3 + f];
            if (!(r <= std::max(tol * un, 1e-300))) ok = false;
          }
          const bool was_pending = pending[b] != 0;
          pending[b] = 0;
          if (ok) {
            nact[b] = 0;
            continue;
          }
          if (pb->verbose && b == 0 && was_pending)
            std::fprintf(stderr, "fsi newton slice 0: residual test failed, iterating on\n");
        }
        left |= nact[b] != 0;
      }
      if (!left) return FSI_OK;
      HIPCHK(hipMemcpyAsync(pb->nact, nact.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
      pb->prof.pact = count_active(nact);
    }
    if (it > maxit) break;
    CHK(assemble_levels<D, S, true>(pb, B, sp, pb->nact, st, it == 1 || pb->p.precond_lag == 0));
    hipEvent_t e2 = stage_mark(pb, st);
    stage_span(pb, 1, e1, e2);
    fsi_status ls = fgmres<D, S, true>(pb, B, sp.k, rs.krylov, st, &lin_failed);
    if (ls != FSI_OK && ls != FSI_ERR_LINEAR) return ls;
    hipEvent_t e3 = stage_mark(pb, st);
    stage_span(pb, 2, e2, e3);
    k_newton_update<D, S><<<dim3(pb->nchunk_n, B), RED_T, 0, st>>>(nn, pb->U, (const S*)pb->xs, pb->chunk_n, pb->npart,
                                                                 pb->nchunk_n, pb->nact);
    k_max_partials<<<(B + 63) / 64, 64, 0, st>>>(pb->nchunk_n, pb->npart, pb->nmax, B);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hm.data(), pb->nmax, (size_t)B * 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    stage_span(pb, 3, e3, stage_mark(pb, st));
    for (int b = 0; b < B; ++b) {
      if (!nact[b]) continue;
      rs.newton[b] += 1;
      last_lin_failed[b] = lin_failed[b];
      // per field: relative size of the update just applied, and an estimate of
      // the error left after it from the observed contraction (d_k / d_{k-1}) d_k
      double worst = 0.0, est = 0.0;
      bool finite = true;
      for (int f = 0; f < 3; ++f) {
        const double du = hm[(size_t)b * 6 + f], un = hm[(size_t)b * 6 + 3 + f];
        if (!std::isfinite(du) || !std::isfinite(un)) finite = false;
        const double rel = un > 0.0 ? du / un : du;
        worst = std::max(worst, rel);
        const double pf = prev[(size_t)b * 3 + f];
        const double theta = (pf > 0.0) ? rel / pf : 1.0;
        est = std::max(est, theta < 1.0 ? theta * rel / (1.0 - theta) : 1e300);
        prev[(size_t)b * 3 + f] = rel;
      }
      if (!finite) {
        rs.status[b] = FSI_ERR_NONFINITE;
        nact[b] = 0;
        hact[b] = 0;
        continue;
      }
      if (pb->verbose && b == 0)
        std::fprintf(stderr, "fsi newton it %d slice 0: rel(v,u,p) = %.3e %.3e %.3e  est %.3e  krylov %d%s\n", it,
                     hm[3] > 0 ? hm[0] / hm[3] : hm[0], hm[4] > 0 ? hm[1] / hm[4] : hm[1],
                     hm[5] > 0 ? hm[2] / hm[5] : hm[2], est, rs.krylov[0] - k0, lin_failed[0] ? " (linear solve failed)" : "");
      est_prev[b] = est;
      // an update from a linear solve that missed its tolerance is never accepted
      if ((worst <= pb->p.newton_rtol || est <= pb->p.newton_rtol) && !lin_failed[b]) pending[b] = 1;
    }
    bool any = false;
    for (int b = 0; b < B; ++b) any |= nact[b] != 0;
    if (!any) return FSI_OK;
  }
  for (int b = 0; b < B; ++b)
    if (nact[b]) {
      rs.status[b] = last_lin_failed[b] ? FSI_ERR_LINEAR : FSI_ERR_NEWTON;
      hact[b] = 0;
    }
  return FSI_OK;
}

// FSI_ERR_NONFINITE (with the status of every slice) if any of the B input
// states holds a value that is not finite
fsi_status check_finite(fsi_problem* pb, int B, const double* U_in, fsi_stats* stats, hipStream_t st) {
  const size_t ndof = (size_t)pb->lev[pb->nlev - 1].nn * (2 * pb->p.dim + 1);
  HIPCHK(hipMemsetAsync(pb->flag, 0, B * sizeof(int), st));
  k_nonfinite<<<dim3(64, B), TPB, 0, st>>>(ndof, U_in, pb->flag);
  std::vector<int> hflag(B);
  HIPCHK(hipMemcpyAsync(hflag.data(), pb->flag, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int b = 0; b < B; ++b)
    if (hflag[b]) {
      if (stats)
        for (int q = 0; q < B && q < FSI_MAX_SLICES; ++q) stats->slice_status[q] = hflag[q] ? FSI_ERR_NONFINITE : FSI_OK;
      return FSI_ERR_NONFINITE;
    }
  return FSI_OK;
}

template <int D, class S>
fsi_status propagate(fsi_problem* pb, int B, const double* t0, double slice_len, int nsteps, const double* U_in,
                     double* U_out, fsi_stats* stats, hipStream_t st, bool check_input) {
  FSI_DIM(D);
  Level& F = pb->lev[pb->nlev - 1];
  const Geom g = F.geom();
  const size_t ndof = (size_t)F.nn * NC;
  const double k = slice_len / nsteps;
  const StepPar sp = step_par(pb, k);
  auto t_start = std::chrono::steady_clock::now();
  pb->sused = 0;
  pb->sev.clear();
  if (check_input) CHK(check_finite(pb, B, U_in, stats, st));
  HIPCHK(hipMemcpyAsync(pb->U, U_in, (size_t)B * ndof * sizeof(double), hipMemcpyDeviceToDevice, st));
  RunStats rs;
  rs.newton.assign(B, 0);
  rs.krylov.assign(B, 0);
  rs.status.assign(B, FSI_OK);
  std::vector<int> hact(B, 1);
  std::vector<double> th(B);
  for (int n = 1; n <= nsteps; ++n) {
    for (int b = 0; b < B; ++b) th[b] = t0[b] + n * k;
    HIPCHK(hipMemcpyAsync(pb->tdev, th.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(pb->nact, hact.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
    // history U^{n-1} .. U^{n-1-q} of the Newton guess (older states first)
    const int q = std::min(pb->p.newton_guess, n - 1);
    const size_t sb = (size_t)B * ndof * sizeof(double);
    if (n >= 4 && pb->p.newton_guess >= 3) HIPCHK(hipMemcpyAsync(pb->Uprev3, pb->Uprev2, sb, hipMemcpyDeviceToDevice, st));
    if (n >= 3 && pb->p.newton_guess >= 2) HIPCHK(hipMemcpyAsync(pb->Uprev2, pb->Uprev, sb, hipMemcpyDeviceToDevice, st));
    if (n >= 2) HIPCHK(hipMemcpyAsync(pb->Uprev, pb->Uold, sb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(pb->Uold, pb->U, sb, hipMemcpyDeviceToDevice, st));
    // Newton guess: the old state, or the extrapolation of degree q of the last q + 1 states
    if (q >= 1)
      k_extrapolate<<<dim3(64, B), TPB, 0, st>>>(ndof, q, pb->U, pb->Uold, pb->Uprev, pb->Uprev2, pb->Uprev3, pb->nact);
    k_apply_dirichlet<D><<<grid1(F.nn, B), TPB, 0, st>>>(g, sp, pb->U, pb->tdev, pb->nact);
    HIPCHK(hipGetLastError());
    CHK(newton_solve_step<D, S>(pb, B, sp, hact, rs, st));
    if (pb->traj_out)
      HIPCHK(hipMemcpyAsync(pb->traj_out + (size_t)(n - 1) * B * ndof, pb->U, (size_t)B * ndof * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    bool any = false;
    for (int b = 0; b < B; ++b) any |= hact[b] != 0;
    if (!any) break;
  }
  HIPCHK(hipMemcpyAsync(U_out, pb->U, (size_t)B * ndof * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  fsi_status ret = FSI_OK;
  for (int b = 0; b < B; ++b)
    if (rs.status[b] != FSI_OK) ret = (fsi_status)rs.status[b];
  if (stats) {
    int nt = 0, kt = 0;
    for (int b = 0; b < B && b < FSI_MAX_SLICES; ++b) {
      stats->newton_its[b] = rs.newton[b];
      stats->krylov_its[b] = rs.krylov[b];
      stats->slice_status[b] = rs.status[b];
      nt += rs.newton[b];
      kt += rs.krylov[b];
    }
    stats->newton_total = nt;
    stats->krylov_total = kt;
    for (const auto& e : pb->sev) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) stats->stage_ms[e.stage] += ms;
    }
    stats->stage_ms[4] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return ret;
}

// One batch of B slices on pb's workspace and stream (which already waits for the caller's work).
fsi_status propagate_batch(fsi_problem* pb, int B, const double* t0, double slice_len, int nsteps,
                           const double* U_in, double* U_out, fsi_stats* stats, bool check_input) {
  hipStream_t st = pb->ist;
  if (pb->p.dim == 3)
    return pb->mixed ? propagate<3, float>(pb, B, t0, slice_len, nsteps, U_in, U_out, stats, st, check_input)
                     : propagate<3, double>(pb, B, t0, slice_len, nsteps, U_in, U_out, stats, st, check_input);
  return pb->mixed ? propagate<2, float>(pb, B, t0, slice_len, nsteps, U_in, U_out, stats, st, check_input)
                   : propagate<2, double>(pb, B, t0, slice_len, nsteps, U_in, U_out, stats, st, check_input);
}

fsi_status run_propagate(fsi_problem* pb, int B, const double* t0, double slice_len, int nsteps, const double* U_in,
                         double* U_out, fsi_stats* stats, hipStream_t caller) {
  if (!pb || !t0 || !U_in || !U_out || B <= 0 || B > pb->Bmax || nsteps <= 0 || !(slice_len > 0.0))
    return FSI_ERR_ARG;
  if (stats) std::memset(stats, 0, sizeof(fsi_stats));
  // work on the library stream after everything already queued on the caller's stream;
  // the call returns after completion, so the caller's later work sees the results
  HIPCHK(hipEventRecord(pb->iev, caller));
  HIPCHK(hipStreamWaitEvent(pb->ist, pb->iev, 0));
  const int S = std::min(std::max(pb->p.batch_split, 1), B);
  if (S <= 1 || pb->prof.on || pb->traj_out)
    return propagate_batch(pb, B, t0, slice_len, nsteps, U_in, U_out, stats, true);
  // the groups' workspaces are made on the first call that splits (their streams then
  // exist only in a process that uses them: each stream takes a hardware queue)
  if (pb->sub.empty()) {
    fsi_params q = pb->p;
    q.max_batch = (pb->p.max_batch + pb->p.batch_split - 1) / pb->p.batch_split;
    q.batch_split = 0;
    q.parareal_pipeline = 0;
    std::vector<fsi_problem*> ws;
    for (int g = 1; g < pb->p.batch_split; ++g) {
      fsi_problem* w = nullptr;
      const fsi_status e = fsi_setup(&q, &w);
      if (e != FSI_OK) {
        for (fsi_problem* x : ws) fsi_destroy(x);
        return e;
      }
      ws.push_back(w);
    }
    pb->sub = std::move(ws);
  }
  // concurrent slice groups: the whole batch's input is checked first, so that a
  // bad slice stops the call before any group writes U_out
  CHK(check_finite(pb, B, U_in, stats, pb->ist));
  const size_t ndof = (size_t)pb->lev[pb->nlev - 1].nn * (2 * pb->p.dim + 1);
  std::vector<int> g0(S + 1);
  for (int g = 0; g <= S; ++g) g0[g] = (int)((long long)B * g / S);
  std::vector<fsi_stats> gst(S);
  std::vector<fsi_status> gret(S, FSI_OK);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  auto group = [&](int g) {
    fsi_problem* q = g == 0 ? pb : pb->sub[g - 1];
    std::memset(&gst[g], 0, sizeof(fsi_stats));
    if (g > 0 && (hipSetDevice(dev) != hipSuccess || hipEventRecord(q->iev, caller) != hipSuccess ||
                  hipStreamWaitEvent(q->ist, q->iev, 0) != hipSuccess)) {
      gret[g] = FSI_ERR_HIP;
      return;
    }
    const int b0 = g0[g], nb = g0[g + 1] - g0[g];
    gret[g] = guarded([&] {
      return propagate_batch(q, nb, t0 + b0, slice_len, nsteps, U_in + b0 * ndof, U_out + b0 * ndof, &gst[g], false);
    });
  };
  std::vector<std::thread> th;
  th.reserve(S - 1);
  int started = 1;   // groups 1 .. started-1 have a thread; a group whose thread did not start runs here
  try {
    for (int g = 1; g < S; ++g) {
      th.emplace_back(group, g);
      started = g + 1;
    }
  } catch (...) {
  }
  group(0);
  for (int g = started; g < S; ++g) group(g);
  for (std::thread& t : th) t.join();
  fsi_status ret = FSI_OK;
  for (int g = 0; g < S; ++g) {
    if (gret[g] != FSI_OK && ret == FSI_OK) ret = gret[g];
    if (!stats) continue;
    for (int b = g0[g]; b < g0[g + 1] && b < FSI_MAX_SLICES; ++b) {
      stats->newton_its[b] = gst[g].newton_its[b - g0[g]];
      stats->krylov_its[b] = gst[g].krylov_its[b - g0[g]];
      stats->slice_status[b] = gst[g].slice_status[b - g0[g]];
    }
    stats->newton_total += gst[g].newton_total;
    stats->krylov_total += gst[g].krylov_total;
    for (int i = 0; i < 8; ++i) stats->stage_ms[i] = std::max(stats->stage_ms[i], gst[g].stage_ms[i]);
  }
  return ret;
}

// ------------------------------------------------------------ adjoint
// Drag faces of the finest level: bar faces shared with a fluid cell.
std::vector<DragFace> drag_faces(const Level& L) {
  std::vector<DragFace> f;
  for (int j = 0; j < L.ny; ++j)
    for (int i = 0; i < L.nx; ++i) {
      if (!L.solid[i + L.nx * j]) continue;
      const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
      for (int q = 0; q < 4; ++q) {
        const int ii = i + di[q], jj = j + dj[q];
        if (ii < 0 || jj < 0 || ii >= L.nx || jj >= L.ny) continue;
        const int c = ii + L.nx * jj;
        if (L.solid[c]) continue;
        DragFace d;
        d.cell = c;
        d.axis = q < 2 ? 0 : 1;
        d.sign = (q % 2) ? 1 : -1;
        d.side = d.sign > 0 ? 0 : 1;
        f.push_back(d);
      }
    }
  return f;
}

fsi_status adjoint_alloc(fsi_problem* pb, size_t nstates, int N) {
  FSI_DIM(2);
  Level& F = pb->lev[pb->nlev - 1];
  const size_t nd = (size_t)F.nn * NC;
  if (!pb->Jtmp) {
    CHK(dalloc(pb, &pb->Jtmp, jslice<2, double, false>(F.geom())));
    CHK(dalloc(pb, &pb->Jcopy, jslice<2, double, false>(F.geom())));
    CHK(dalloc(pb, &pb->Jold, jslice<2, double, false>(F.geom())));
    CHK(dalloc(pb, &pb->lam, nd));
    CHK(dalloc(pb, &pb->lamn, nd));
    CHK(dalloc(pb, &pb->arhs, nd));
    CHK(dalloc(pb, &pb->ay, nd));
    CHK(dalloc(pb, &pb->agrad, 3));
    CHK(dalloc(pb, &pb->abnd, (size_t)(pb->Bmax + 1) * nd));
    CHK(dalloc(pb, &pb->aout, (size_t)pb->Bmax * nd));
    std::vector<DragFace> f = drag_faces(F);
    pb->nfaces = (int)f.size();
    CHK(dalloc(pb, &pb->faces, f.size()));
    HIPCHK(hipMemcpy(pb->faces, f.data(), f.size() * sizeof(DragFace), hipMemcpyHostToDevice));
  }
  if (nstates > pb->traj_cap) {
    CHK(dalloc(pb, &pb->traj, nstates * nd));
    CHK(dalloc(pb, &pb->dvals, nstates));
    pb->traj_cap = nstates;
  }
  (void)N;
  return FSI_OK;
}

// Sequential fine solve with slice-boundary checkpoints, a batched recompute of
// every step from the checkpoints, the functional J = k sum D(U^n), and the
// backward sweep of transposed Newton-Jacobian solves (FP64).
fsi_status adjoint_run(fsi_problem* pb, double T, int N, int m, const double* U0, double* J_out, double* grad_out,
                       fsi_stats* stats, hipStream_t caller) {
  FSI_DIM(2);
  Level& F = pb->lev[pb->nlev - 1];
  const Geom g = F.geom();
  const size_t nd = (size_t)F.nn * NC;
  const double dl = T / N, k = dl / m;
  const StepPar sp = step_par(pb, k);
  const double rn = pb->p.rho_f * pb->p.nu_f;
  const size_t S = (size_t)N * m;
  CHK(adjoint_alloc(pb, S, N));
  auto t_start = std::chrono::steady_clock::now();
  fsi_stats tmp;
  int ntot = 0, ktot = 0;
  // forward: sequential slices, checkpoints abnd[0..N]
  HIPCHK(hipMemcpyAsync(pb->abnd, U0, nd * sizeof(double), hipMemcpyDeviceToDevice, caller));
  for (int l = 0; l < N; ++l) {
    const double t0 = l * dl;
    CHK(run_propagate(pb, 1, &t0, dl, m, pb->abnd + l * nd, pb->abnd + (l + 1) * nd, &tmp, caller));
    ntot += tmp.newton_total;
    ktot += tmp.krylov_total;
  }
  // recompute all slices at once from the checkpoints, keeping every step: traj[n-1][l]
  std::vector<double> t0s(N);
  for (int l = 0; l < N; ++l) t0s[l] = l * dl;
  pb->traj_out = pb->traj;
  fsi_status rs = run_propagate(pb, N, t0s.data(), dl, m, pb->abnd, pb->aout, &tmp, caller);
  pb->traj_out = nullptr;
  CHK(rs);
  ntot += tmp.newton_total;
  ktot += tmp.krylov_total;
  hipStream_t st = pb->ist;
  HIPCHK(hipEventRecord(pb->iev, caller));
  HIPCHK(hipStreamWaitEvent(st, pb->iev, 0));
  // U^s (s = 1..S) and the old state its step started from
  auto cur = [&](size_t s) -> const double* {
    const size_t l = (s - 1) / m, n = (s - 1) % m + 1;
    return pb->traj + ((n - 1) * (size_t)N + l) * nd;
  };
  auto prev = [&](size_t s) -> const double* {
    const size_t l = (s - 1) / m, n = (s - 1) % m + 1;
    return n == 1 ? pb->abnd + l * nd : pb->traj + ((n - 2) * (size_t)N + l) * nd;
  };
  // functional
  k_drag_values<<<(unsigned)((S + 63) / 64), 64, 0, st>>>(g, rn, pb->faces, pb->nfaces, pb->traj, nd, (int)S,
                                                          pb->dvals);
  std::vector<double> dv(S);
  HIPCHK(hipMemcpyAsync(dv.data(), pb->dvals, S * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemsetAsync(pb->agrad, 0, 3 * sizeof(double), st));
  HIPCHK(hipStreamSynchronize(st));
  double J = 0.0;
  for (size_t s = 0; s < S; ++s) J += k * dv[s];
  // backward sweep: (dR_s/dU^s)^T lam_s = -k dD/dU(U^s) - (dR_{s+1}/dU^s)^T lam_{s+1}
  pb->ltol_h[0] = pb->adj_rtol;
  const int one = 1;
  HIPCHK(hipMemcpyAsync(pb->nact, &one, sizeof(int), hipMemcpyHostToDevice, st));
  fsi_status ret = FSI_OK;
  std::vector<int> kits(1, 0);
  for (size_t s = S; s >= 1; --s) {
    const size_t l = (s - 1) / m, n = (s - 1) % m + 1;
    const double ts = l * dl + n * k;
    HIPCHK(hipMemsetAsync(pb->arhs, 0, nd * sizeof(double), st));
    k_drag_gradient<<<1, 1, 0, st>>>(g, rn, pb->faces, pb->nfaces, cur(s), -k, pb->arhs);
    if (s < S) {
      k_elem_jacobian<2, true><<<dim3((g.ncell + jac_cells<2>() - 1) / jac_cells<2>(), 1),
                                 jac_cells<2>() * jac_waves<2>(), 0, st>>>(
          g, sp, cur(s + 1), prev(s + 1), pb->Ke, nullptr);
      k_gather_jacobian<2, double, false><<<grid1(g.nn, 1), TPB, 0, st>>>(g, k, pb->Ke, pb->Jold, nullptr, nullptr, 0);
      k_spmv_T<double><<<grid1(g.nn, 1), TPB, 0, st>>>(g, k, pb->Jold, pb->lamn, pb->ay, 0);
      k_daxpy<<<64, TPB, 0, st>>>(nd, -1.0, pb->ay, pb->arhs);
    }
    // transposed multigrid hierarchy at (U^s, U^{s-1})
    HIPCHK(hipMemcpyAsync(pb->U, cur(s), nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(pb->Uold, prev(s), nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    CHK(assemble_levels<2, double, false>(pb, 1, sp, pb->nact, st, true, true, pb->Jcopy));
    // free unknowns: Krylov solve with the Dirichlet entries of the right-hand side removed
    k_adjoint_rhs<<<grid1(g.nn, 1), TPB, 0, st>>>(g, pb->arhs, pb->Res);
    HIPCHK(hipGetLastError());
    fsi_status ls = fgmres<2, double, false>(pb, 1, k, kits, st);
    if (ls != FSI_OK) { ret = ls; break; }
    HIPCHK(hipMemcpyAsync(pb->lam, pb->xs, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    // Dirichlet unknowns: lam_D = rhs_D - (J^T lam)_D
    k_spmv_T<double><<<grid1(g.nn, 1), TPB, 0, st>>>(g, k, pb->Jcopy, pb->lam, pb->ay, 1);
    k_fix_dirichlet<<<grid1(g.nn, 1), TPB, 0, st>>>(g, pb->lam, pb->arhs, pb->ay);
    k_param_sens<<<1, TPB, 0, st>>>(g, sp, cur(s), prev(s), pb->lam, ts, pb->agrad);
    HIPCHK(hipGetLastError());
    std::swap(pb->lam, pb->lamn);
  }
  double gh[3] = {0, 0, 0};
  HIPCHK(hipMemcpyAsync(gh, pb->agrad, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (J_out) *J_out = J;
  if (grad_out)
    for (int q = 0; q < 3; ++q) grad_out[q] = gh[q];
  if (stats) {
    std::memset(stats, 0, sizeof(fsi_stats));
    stats->newton_total = ntot;
    stats->krylov_total = ktot + kits[0];
    stats->krylov_its[0] = kits[0];
    stats->stage_ms[4] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return ret;
}

}  // namespace

// ------------------------------------------------------------ static scratch
// Scratch of fsi_residual_noalloc: the element residuals of the batch and the
// per-slice times, in a file-scope device array that exists on every GPU the
// library runs on (each GPU holds its own copy until the process ends).  Host
// code never passes the array's name to a kernel or copy: that is a host-side
// stand-in, not a device address.  Its device address on a device comes from
// hipGetSymbolAddress, called once per device with that device current (at
// fsi_setup) and kept per device.
constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Device address of the scratch array on the current device (looked up once).
static fsi_status scratch_address(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return FSI_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return FSI_ERR_HIP;
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return FSI_OK;
}

// =================================================================== C ABI
extern "C" {

const char* fsi_status_string(fsi_status s) {
  switch (s) {
    case FSI_OK: return "ok";
    case FSI_ERR_ARG: return "invalid argument";
    case FSI_ERR_HIP: return "HIP runtime error";
    case FSI_ERR_OOM: return "out of device memory";
    case FSI_ERR_NEWTON: return "Newton did not converge";
    case FSI_ERR_LINEAR: return "linear solver did not converge";
    case FSI_ERR_NONFINITE: return "non-finite value";
    case FSI_ERR_PARAREAL: return "Parareal did not converge";
  }
  return "unknown status";
}

void fsi_destroy(fsi_problem* pb) {
  if (!pb) return;
  if (pb->pipe) fsi_destroy(pb->pipe);
  for (fsi_problem* q : pb->sub) fsi_destroy(q);
  if (pb->vc_exec) (void)hipGraphExecDestroy(pb->vc_exec);
  if (pb->ist) (void)hipStreamSynchronize(pb->ist);
  for (auto& e : pb->sg)
    for (hipGraphExec_t x : e.ex)
      if (x) (void)hipGraphExecDestroy(x);
  if (pb->hst_pin) (void)hipHostFree(pb->hst_pin);
  for (hipEvent_t e : pb->step_ev)
    if (e) (void)hipEventDestroy(e);
  if (pb->ist) (void)hipStreamSynchronize(pb->ist);
  if (pb->ist) (void)hipStreamDestroy(pb->ist);
  if (pb->iev) (void)hipEventDestroy(pb->iev);
  for (void* q : pb->allocs) (void)hipFree(q);
  for (hipEvent_t e : pb->prof.pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : pb->spool) (void)hipEventDestroy(e);
  delete pb;
}

static fsi_status setup_impl(const fsi_params* prm, fsi_problem** out);

fsi_status fsi_setup(const fsi_params* prm, fsi_problem** out) {
  return guarded([&] { return setup_impl(prm, out); });
}

static fsi_status setup_impl(const fsi_params* prm, fsi_problem** out) {
  if (!prm || !out) return FSI_ERR_ARG;
  *out = nullptr;
  const fsi_params& p = *prm;
  if ((p.dim != 2 && p.dim != 3) || p.level < (p.degree == 2 ? 0 : 1) || p.level > MAXLEV - 2 || p.max_batch < 1 ||
      p.max_batch > FSI_MAX_SLICES ||
      p.gmres_restart < 1 || p.gmres_restart > 63 || p.newton_maxit < 1 || p.vanka_sweeps < 1 ||
      p.vanka_sweeps_coarse < 1 ||
      p.gmres_maxit < 1 || (p.precision != FSI_FP64 && p.precision != FSI_MIXED) ||
      (p.precond_lag != 0 && p.precond_lag != 1) || !(p.lin_rtol_first > 0.0 && p.lin_rtol_first < 1.0) ||
      p.parareal_theta < 0 || p.parareal_theta > 2 || !(p.theta_ref_k >= 0.0) || p.parareal_pipeline < 0 ||
      p.parareal_pipeline > p.max_batch || p.batch_split < 0 || p.batch_split > 8 || p.newton_guess < 0 || p.newton_guess > 3 ||
      !(p.precond_lps_scale >= 0 && p.precond_lps_scale < 1e6) || p.batch_split > p.max_batch)
    return FSI_ERR_ARG;
  for (int a = 0; a < p.dim; ++a) {
    if (p.nseg[a] < 1 || p.nseg[a] > 4) return FSI_ERR_ARG;
    for (int s = 0; s < p.nseg[a]; ++s)
      if (p.seg_cells[a][s] < 1 || !(p.seg_pts[a][s + 1] > p.seg_pts[a][s])) return FSI_ERR_ARG;
  }
  if (!(p.rho_f > 0 && p.nu_f > 0 && p.rho_s > 0 && p.ramp_time > 0)) return FSI_ERR_ARG;
  // the remaining physical and solver constants: finite, and in the range where
  // the scheme and the solver are defined
  for (double v : {p.rho_f, p.nu_f, p.rho_s, p.mu_s, p.lambda_s, p.inflow_peak, p.ramp_time, p.theta0, p.lps_alpha0,
                   p.cip_gamma, p.vanka_omega, p.newton_rtol, p.lin_rtol, p.newton_res_rtol})
    if (!std::isfinite(v)) return FSI_ERR_ARG;
  if (!(p.mu_s > 0) || p.lambda_s < 0 || p.theta0 < 0 || p.lps_alpha0 < 0 || p.cip_gamma < 0 ||
      !(p.vanka_omega > 0 && p.vanka_omega < 2) || !(p.newton_rtol > 0) || !(p.lin_rtol > 0 && p.lin_rtol < 1) ||
      !(p.newton_res_rtol > 0 && p.newton_res_rtol < 1) || !(p.newton_res_accept >= 0 && p.newton_res_accept < 1) || p.spmv_slice_fast < -1 || p.spmv_slice_fast > 1 ||
      p.vanka_slice_fast < -1 || p.vanka_slice_fast > 1 || p.vanka_wide_cells < 0 ||
      (p.degree != 1 && p.degree != 2) ||
      (p.degree == 2 && (p.dim != 2 || p.level + 2 > MAXLEV - 1)))
    return FSI_ERR_ARG;
  fsi_problem* pb = new (std::nothrow) fsi_problem();
  if (!pb) return FSI_ERR_OOM;
  pb->p = p;
  pb->Bmax = p.max_batch;
  pb->mixed = p.precision == FSI_MIXED;
  pb->ssz = pb->mixed ? sizeof(float) : sizeof(double);
  pb->R = p.gmres_restart;
  pb->deg = p.degree;
  pb->nlev = p.level + 1 + (p.degree - 1);   // Q2: the Q1 hierarchy reaches the Q2 node grid
  {
    // FSI_GRAPHS=0 replays nothing from graphs (every kernel launched directly)
    const char* e = std::getenv("FSI_GRAPHS");
    pb->use_graphs = !(e && e[0] == '0');
    const char* v = std::getenv("FSI_VERBOSE");
    pb->verbose = v && v[0] == '1';
  }
  fsi_status s = FSI_OK;
  for (int l = 0; l < pb->nlev && s == FSI_OK; ++l) s = p.dim == 3 ? build_level<3>(pb, l) : build_level<2>(pb, l);
  if (s != FSI_OK) { fsi_destroy(pb); return s; }
  Level& F = pb->lev[pb->nlev - 1];
  Level& C = pb->lev[0];
  const int B = pb->Bmax;
  const int NC = p.dim == 3 ? Dm<3>::NC : Dm<2>::NC;
  const int NE = p.dim == 3 ? Dm<3>::NE : Dm<2>::NE;
  const size_t ndof = (size_t)F.nn * NC;
  const size_t ss = pb->ssz;
  const int R = pb->R;
  pb->chunk_n = 2048;
  pb->nchunk_n = (F.nn + pb->chunk_n - 1) / pb->chunk_n;
  // 2d coarsest level: block-tridiagonal direct solve over super-columns of two node columns
  const bool direct = p.dim == 2;
  pb->cbs = direct ? 2 * (C.ny + 1) * NC : 1;
  pb->cnsb = direct ? (C.nx + 1 + 1) / 2 : 1;
  if (direct && (pb->cbs > 64 || C.nn * NC > 2048)) { fsi_destroy(pb); return FSI_ERR_ARG; }
  const size_t cb2 = (size_t)pb->cbs * pb->cbs * pb->cnsb * B;
#define A_(x) do { s = (x); if (s != FSI_OK) { fsi_destroy(pb); return s; } } while (0)
  A_(dalloc(pb, &pb->U, B * ndof));
  A_(dalloc(pb, &pb->Uold, B * ndof));
  A_(dalloc(pb, &pb->Uprev, B * ndof));
  if (p.newton_guess >= 2) A_(dalloc(pb, &pb->Uprev2, B * ndof));
  if (p.newton_guess >= 3) A_(dalloc(pb, &pb->Uprev3, B * ndof));
  A_(dalloc(pb, &pb->Res, B * ndof));
  A_(dalloc(pb, &pb->Re, (size_t)B * NE * F.ncell));
  A_(dalloc(pb, &pb->Ke, (size_t)B * NE * NE * F.ncell));
  A_(dalloc(pb, &pb->tdev, B));
  A_(dalloc(pb, &pb->nact, B));
  A_(dalloc(pb, &pb->gact, B));
  A_(dalloc(pb, &pb->gord, B));
  A_(dalloc(pb, &pb->flag, B));
  A_(dalloc_bytes(pb, &pb->V, (size_t)B * (R + 1) * ndof * ss));
  A_(dalloc_bytes(pb, &pb->Z, (size_t)B * R * ndof * ss));
  A_(dalloc_bytes(pb, &pb->w, (size_t)B * ndof * ss));
  A_(dalloc_bytes(pb, &pb->xs, (size_t)B * ndof * ss));
  A_(dalloc_bytes(pb, &pb->tmp, (size_t)B * ndof * ss));
  A_(dalloc(pb, &pb->H, (size_t)B * (R + 1) * R));
  A_(dalloc(pb, &pb->hcol, (size_t)B * 64));
  A_(dalloc(pb, &pb->hcol2, (size_t)B * 64));
  A_(dalloc(pb, &pb->cs, (size_t)B * R));
  A_(dalloc(pb, &pb->sn, (size_t)B * R));
  A_(dalloc(pb, &pb->gv, (size_t)B * (R + 1)));
  A_(dalloc(pb, &pb->res, B));
  A_(dalloc(pb, &pb->beta0, B));
  A_(dalloc(pb, &pb->beta, B));
  A_(dalloc(pb, &pb->ycoef, (size_t)B * 64));
  A_(dalloc(pb, &pb->partial, (size_t)B * 64 * ((ndof + KDOT_CHUNK - 1) / KDOT_CHUNK + 1)));
  A_(dalloc(pb, &pb->gstate, B));
  A_(dalloc(pb, &pb->ncol, B));
  A_(dalloc(pb, &pb->ltol, B));
  pb->ltol_h.assign(B, p.lin_rtol);
  A_(dalloc(pb, &pb->cDinv, cb2));
  A_(dalloc(pb, &pb->cW, cb2));
  A_(dalloc(pb, &pb->cL, cb2));
  A_(dalloc(pb, &pb->cY, (size_t)B * pb->cnsb * pb->cnsb * pb->cbs * pb->cbs));
  A_(dalloc_bytes(pb, &pb->cAinv, direct ? (size_t)B * C.nn * NC * C.nn * NC * ss : 1));
  A_(dalloc(pb, &pb->npart, (size_t)B * 6 * pb->nchunk_n));
  A_(dalloc(pb, &pb->nmax, (size_t)B * 6));
  if (pb->deg == 2) {
    const Level& Cq = pb->lev[pb->nlev - 2];   // the Q2 cells
    A_(upload(pb, &pb->pst2, q2_lps_stencil(Cq, F, p)));
    A_(dalloc_bytes(pb, &pb->J2, (size_t)B * 625 * F.nn * ss));
    A_(dalloc(pb, &pb->Ke2, (size_t)B * 45 * 45 * Cq.ncell));
    A_(dalloc(pb, &pb->Re2, (size_t)B * 45 * Cq.ncell));
  }
#undef A_
  if (hipFuncSetAttribute((const void*)k_coarse_factor<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          5 * pb->cbs * pb->cbs * sizeof(double)) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_coarse_factor<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          5 * pb->cbs * pb->cbs * sizeof(double)) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_coarse_factor<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          5 * pb->cbs * pb->cbs * sizeof(double)) != hipSuccess) {
    fsi_destroy(pb);
    return FSI_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&pb->ist, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&pb->iev, hipEventDisableTiming) != hipSuccess) {
    fsi_destroy(pb);
    return FSI_ERR_HIP;
  }
  if (hipHostMalloc((void**)&pb->hst_pin, 2 * (size_t)B * sizeof(int), hipHostMallocCoherent) != hipSuccess) {
    pb->hst_pin = nullptr;
    fsi_destroy(pb);
    return FSI_ERR_OOM;
  }
  std::memset(pb->hst_pin, 0, 2 * (size_t)B * sizeof(int));
  if (hipEventCreateWithFlags(&pb->step_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pb->step_ev[1], hipEventDisableTiming) != hipSuccess) {
    fsi_destroy(pb);
    return FSI_ERR_HIP;
  }
  if ((s = scratch_address(&pb->scratch)) != FSI_OK) {
    fsi_destroy(pb);
    return s;
  }
  *out = pb;
  return FSI_OK;
}

fsi_status fsi_sizes(const fsi_problem* pb, int64_t* n_nodes, int64_t* n_dofs) {
  if (!pb) return FSI_ERR_ARG;
  const Level& F = pb->lev[pb->nlev - 1];
  if (n_nodes) *n_nodes = F.nn;
  if (n_dofs) *n_dofs = (int64_t)F.nn * (2 * pb->p.dim + 1);
  return FSI_OK;
}

fsi_status fsi_initial_state(fsi_problem* pb, double* U0, hipStream_t st) {
  if (!pb || !U0) return FSI_ERR_ARG;
  Level& F = pb->lev[pb->nlev - 1];
  const size_t ndof = (size_t)F.nn * (2 * pb->p.dim + 1);
  HIPCHK(hipMemsetAsync(U0, 0, ndof * sizeof(double), st));
  double t0 = 0.0;
  HIPCHK(hipMemcpyAsync(pb->tdev, &t0, sizeof(double), hipMemcpyHostToDevice, st));
  if (pb->p.dim == 3)
    k_apply_dirichlet<3><<<grid1(F.nn, 1), TPB, 0, st>>>(F.geom(), step_par(pb, 1.0), U0, pb->tdev, nullptr);
  else
    k_apply_dirichlet<2><<<grid1(F.nn, 1), TPB, 0, st>>>(F.geom(), step_par(pb, 1.0), U0, pb->tdev, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return FSI_OK;
}

fsi_status fine_propagate(fsi_problem* pb, int32_t B, const double* t0, double slice_len, int32_t m,
                          const double* U_in, double* U_out, fsi_stats* stats, hipStream_t st) {
  return guarded([&] { return run_propagate(pb, B, t0, slice_len, m, U_in, U_out, stats, st); });
}

fsi_status coarse_propagate(fsi_problem* pb, int32_t B, const double* t0, double slice_len, int32_t M,
                            const double* U_in, double* U_out, fsi_stats* stats, hipStream_t st) {
  return guarded([&] { return run_propagate(pb, B, t0, slice_len, M, U_in, U_out, stats, st); });
}

}  // extern "C"

namespace {

// Device scratch of a Parareal run and the host copies of its partial sums.
struct PararealBufs {
  double *Cold = nullptr, *Fv = nullptr, *Up = nullptr, *Cn = nullptr, *part = nullptr, *tpart = nullptr;
  int chunk = 4096, nchunk = 1;
  std::vector<double> htp, hp;
  ~PararealBufs() {
    (void)hipDeviceSynchronize();
    (void)hipFree(Cold); (void)hipFree(Fv); (void)hipFree(Up); (void)hipFree(Cn); (void)hipFree(part);
    (void)hipFree(tpart);
  }
  // nfv: number of fine-result buffers of N slices each
  fsi_status alloc(int nn, size_t nd, int N, int nfv) {
    nchunk = (nn + chunk - 1) / chunk;
    htp.resize((size_t)18 * nchunk);
    hp.resize((size_t)(N + 1) * 4 * nchunk);
    if (hipMalloc(&Cold, N * nd * sizeof(double)) != hipSuccess ||
        hipMalloc(&Fv, (size_t)nfv * N * nd * sizeof(double)) != hipSuccess ||
        hipMalloc(&Up, (N + 1) * nd * sizeof(double)) != hipSuccess || hipMalloc(&Cn, nd * sizeof(double)) != hipSuccess ||
        hipMalloc(&part, (size_t)(N + 1) * 4 * nchunk * sizeof(double)) != hipSuccess ||
        hipMalloc(&tpart, (size_t)18 * nchunk * sizeof(double)) != hipSuccess)
      return FSI_ERR_OOM;
    return FSI_OK;
  }
};

// theta-Parareal weight from F = F(U^i_l) and C = C(U^{i+1}_l), per velocity /
// displacement component, averaged (host-synchronous on st).
fsi_status theta_weight(fsi_problem* pb, PararealBufs& w, const double* Fl, const double* Cl, double& th,
                        hipStream_t st) {
  const int dim = pb->p.dim, nq = 3 * 2 * dim;
  const int nn = pb->lev[pb->nlev - 1].nn;
  th = 1.0;
  if (pb->p.parareal_theta == 0) return FSI_OK;
  if (dim == 3)
    k_theta_dots<3><<<w.nchunk, RED_T, 0, st>>>(nn, Fl, Cl, w.chunk, w.tpart, w.nchunk);
  else
    k_theta_dots<2><<<w.nchunk, RED_T, 0, st>>>(nn, Fl, Cl, w.chunk, w.tpart, w.nchunk);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(w.htp.data(), w.tpart, (size_t)nq * w.nchunk * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double sum = 0.0;
  int cnt = 0;
  for (int c = 0; c < 2 * dim; ++c) {
    double ff = 0.0, fg = 0.0, gg = 0.0;
    for (int q = 0; q < w.nchunk; ++q) {
      ff += w.htp[(size_t)(3 * c) * w.nchunk + q];
      fg += w.htp[(size_t)(3 * c + 1) * w.nchunk + q];
      gg += w.htp[(size_t)(3 * c + 2) * w.nchunk + q];
    }
    if (pb->p.parareal_theta == 1 && gg > 0.0 && ff > 0.0) { sum += fg / std::sqrt(gg * ff); ++cnt; }
    if (pb->p.parareal_theta == 2 && gg > 0.0) { sum += fg / gg; ++cnt; }
  }
  th = cnt ? sum / cnt : 1.0;
  return FSI_OK;
}

// Largest relative change of v and of u over the N + 1 slice boundaries.
fsi_status boundary_change(fsi_problem* pb, PararealBufs& w, int N, const double* Ub, double& change,
                           hipStream_t st) {
  const int nn = pb->lev[pb->nlev - 1].nn;
  if (pb->p.dim == 3)
    k_change_norms<3><<<dim3(w.nchunk, N + 1), RED_T, 0, st>>>(nn, Ub, w.Up, w.chunk, w.part, w.nchunk);
  else
    k_change_norms<2><<<dim3(w.nchunk, N + 1), RED_T, 0, st>>>(nn, Ub, w.Up, w.chunk, w.part, w.nchunk);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(w.hp.data(), w.part, w.hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  change = 0.0;
  for (int l = 0; l <= N; ++l)
    for (int f = 0; f < 2; ++f) {
      double dd = 0.0, nn2 = 0.0;
      for (int c = 0; c < w.nchunk; ++c) {
        dd += w.hp[((size_t)l * 4 + 2 * f) * w.nchunk + c];
        nn2 += w.hp[((size_t)l * 4 + 2 * f + 1) * w.nchunk + c];
      }
      const double r = nn2 > 0.0 ? std::sqrt(dd / nn2) : std::sqrt(dd);
      change = std::max(change, r);
    }
  return FSI_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Plain schedule: each iteration is one batched fine sweep over the slices that
// are not yet exact, then the sequential coarse / correction sweep.
fsi_status parareal_plain(fsi_problem* pb, double T, int N, int m, int M, double tol, int max_iter,
                          const double* U0, double* Ub, fsi_stats* sp, double& coarse_ms, double& fine_ms,
                          hipStream_t st) {
  const size_t nd = (size_t)pb->lev[pb->nlev - 1].nn * (2 * pb->p.dim + 1);
  const double dl = T / N;
  PararealBufs w;
  CHK(w.alloc(pb->lev[pb->nlev - 1].nn, nd, N, 1));
  fsi_stats tmp;
  HIPCHK(hipMemcpyAsync(Ub, U0, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  // initial coarse sweep U^0_{l+1} = C(U^0_l)
  for (int l = 0; l < N; ++l) {
    const double t0 = l * dl;
    auto c0 = std::chrono::steady_clock::now();
    CHK(run_propagate(pb, 1, &t0, dl, M, Ub + l * nd, Ub + (l + 1) * nd, &tmp, st));
    coarse_ms += ms_since(c0);
    HIPCHK(hipMemcpyAsync(w.Cold + l * nd, Ub + (l + 1) * nd, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  int it = 0;
  double change = 1e300;
  std::vector<double> t0s(N);
  for (int i = 0; i < max_iter; ++i) {
    // fine sweep over the slices that are not yet exact, batched in one call
    const int Bf = N - i;
    for (int l = i; l < N; ++l) t0s[l - i] = l * dl;
    auto f0 = std::chrono::steady_clock::now();
    CHK(run_propagate(pb, Bf, t0s.data(), dl, m, Ub + i * nd, w.Fv + i * nd, &tmp, st));
    fine_ms += ms_since(f0);
    sp->newton_total += tmp.newton_total;
    sp->krylov_total += tmp.krylov_total;
    HIPCHK(hipMemcpyAsync(w.Up, Ub, (N + 1) * nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    // sequential correction sweep
    for (int l = 0; l < N; ++l) {
      const double* cn = w.Cold + l * nd;
      double th = 1.0;
      if (l >= i) {
        const double t0 = l * dl;
        auto c0 = std::chrono::steady_clock::now();
        CHK(run_propagate(pb, 1, &t0, dl, M, Ub + l * nd, w.Cn, &tmp, st));
        coarse_ms += ms_since(c0);
        cn = w.Cn;
        CHK(theta_weight(pb, w, w.Fv + l * nd, w.Cn, th, st));
      }
      k_parareal_update<<<256, TPB, 0, st>>>(nd, cn, w.Fv + l * nd, w.Cold + l * nd, Ub + (l + 1) * nd, th);
      if (cn != w.Cold + l * nd)
        HIPCHK(hipMemcpyAsync(w.Cold + l * nd, w.Cn, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    CHK(boundary_change(pb, w, N, Ub, change, st));
    it = i + 1;
    sp->parareal_iters = it;   // completed iterations, also when a later one fails
    if (change < tol) break;
  }
  return (!(change < tol) && it < N) ? FSI_ERR_PARAREAL : FSI_OK;
}

// Pipelined schedule (the task view of the iteration): the fine propagation of
// a chunk of G consecutive slices in iteration i + 1 depends only on the
// corrected states of those slices, which the correction sweep of iteration i
// produces one after another.  A worker host thread with its own workspace and
// stream runs the fine chunks in order as soon as their inputs are written,
// while this thread runs the sequential coarse / correction sweep; a sweep step
// waits only for the chunks it reads.  Chunks of an iteration that turns out
// not to be needed are discarded.  The iterates are those of the plain
// schedule: every slice sees the same inputs and the same arithmetic.
struct FineTask {
  int iter, l0, cnt;
  hipEvent_t ready;
};

fsi_status parareal_pipelined(fsi_problem* pb, double T, int N, int m, int M, double tol, int max_iter,
                              const double* U0, double* Ub, fsi_stats* sp, double& coarse_ms, double& fine_ms,
                              hipStream_t st) {
  const int G = pb->p.parareal_pipeline;
  const size_t nd = (size_t)pb->lev[pb->nlev - 1].nn * (2 * pb->p.dim + 1);
  const double dl = T / N;
  if (!pb->pipe) {
    fsi_params q = pb->p;
    q.max_batch = G;
    q.parareal_pipeline = 0;
    q.batch_split = 0;
    CHK(fsi_setup(&q, &pb->pipe));
  }
  fsi_problem* wp = pb->pipe;
  if (wp->Bmax < G) return FSI_ERR_ARG;
  PararealBufs w;
  CHK(w.alloc(pb->lev[pb->nlev - 1].nn, nd, N, 2));   // fine results double-buffered by iteration parity
  auto fbuf = [&](int iter) { return w.Fv + (size_t)(iter & 1) * N * nd; };
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipStream_t ws = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));

  const int ng = (N + G - 1) / G;
  std::vector<FineTask> tasks;
  std::vector<int> tid((size_t)max_iter * ng, -1);
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int> queue;
  int done = 0;
  bool stop = false;
  fsi_status werr = FSI_OK;
  double wfine_ms = 0.0;
  int wnewton = 0, wkrylov = 0;
  tasks.reserve((size_t)max_iter * ng);

  std::thread worker([&]() {
    (void)hipSetDevice(dev);
    std::vector<double> t0s(G);
    for (;;) {
      FineTask t;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !queue.empty(); });
        if (stop) return;
        t = tasks[queue.front()];
        queue.pop_front();
      }
      fsi_status s = hipStreamWaitEvent(ws, t.ready, 0) == hipSuccess ? FSI_OK : FSI_ERR_HIP;
      for (int k = 0; k < t.cnt; ++k) t0s[k] = (t.l0 + k) * dl;
      fsi_stats tmp{};
      auto f0 = std::chrono::steady_clock::now();
      if (s == FSI_OK)
        s = run_propagate(wp, t.cnt, t0s.data(), dl, m, Ub + t.l0 * nd, fbuf(t.iter) + t.l0 * nd, &tmp, ws);
      {
        std::lock_guard<std::mutex> lk(mu);
        wfine_ms += ms_since(f0);
        wnewton += tmp.newton_total;
        wkrylov += tmp.krylov_total;
        if (s != FSI_OK && werr == FSI_OK) werr = s;
        ++done;
      }
      cv.notify_all();
      if (s != FSI_OK) return;
    }
  });

  // chunk g of iteration it: slices [max(gG, it), min((g+1)G, N))
  auto enqueue = [&](int it, int g) -> fsi_status {
    const int l0 = std::max(g * G, it), l1 = std::min((g + 1) * G, N);
    if (l1 <= l0) return FSI_OK;
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (hipEventRecord(ev, st) != hipSuccess) {
      (void)hipEventDestroy(ev);
      return FSI_ERR_HIP;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      tasks.push_back({it, l0, l1 - l0, ev});
      tid[(size_t)it * ng + g] = (int)tasks.size() - 1;
      queue.push_back((int)tasks.size() - 1);
    }
    cv.notify_all();
    return FSI_OK;
  };
  // the input state of slice j for iteration it has just been written on st
  auto input_ready = [&](int it, int j) -> fsi_status {
    if (it >= max_iter || j >= N || j < it) return FSI_OK;
    const int g = j / G;
    return j == std::min((g + 1) * G, N) - 1 ? enqueue(it, g) : FSI_OK;
  };
  // wait until the chunk of iteration it holding slice j has finished (no-op if it has no work)
  auto wait_chunk = [&](int it, int j) -> fsi_status {
    const int t = tid[(size_t)it * ng + j / G];
    if (t < 0) return FSI_OK;
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return done > t || werr != FSI_OK; });
    return done > t ? FSI_OK : werr;
  };

  fsi_status ret = FSI_OK;
  int it = 0;
  double change = 1e300;
  fsi_stats tmp;
#define PP_(x) do { fsi_status s_ = (x); if (s_ != FSI_OK) { ret = s_; goto finish; } } while (0)
  if (hipMemcpyAsync(Ub, U0, nd * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) {
    ret = FSI_ERR_HIP;
    goto finish;
  }
  PP_(input_ready(0, 0));
  for (int l = 0; l < N; ++l) {
    const double t0 = l * dl;
    auto c0 = std::chrono::steady_clock::now();
    PP_(run_propagate(pb, 1, &t0, dl, M, Ub + l * nd, Ub + (l + 1) * nd, &tmp, st));
    coarse_ms += ms_since(c0);
    if (hipMemcpyAsync(w.Cold + l * nd, Ub + (l + 1) * nd, nd * sizeof(double), hipMemcpyDeviceToDevice, st) !=
        hipSuccess) {
      ret = FSI_ERR_HIP;
      goto finish;
    }
    PP_(input_ready(0, l + 1));
  }
  for (int i = 0; i < max_iter; ++i) {
    if (hipMemcpyAsync(w.Up, Ub, (N + 1) * nd * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) {
      ret = FSI_ERR_HIP;
      goto finish;
    }
    for (int l = 0; l < N; ++l) {
      // Ub[l + 1] may still be an input of a running chunk of this iteration, and
      // F(U^i_l) must be there: chunks finish in order, so wait for the later one
      if (l + 1 < N && l + 1 >= i) PP_(wait_chunk(i, l + 1));
      if (l >= i) PP_(wait_chunk(i, l));
      // a slice l < i is exact; its fine result was last computed in iteration l
      const double* fl = (l >= i ? fbuf(i) : fbuf(l)) + l * nd;
      const double* cn = w.Cold + l * nd;
      double th = 1.0;
      if (l >= i) {
        const double t0 = l * dl;
        auto c0 = std::chrono::steady_clock::now();
        PP_(run_propagate(pb, 1, &t0, dl, M, Ub + l * nd, w.Cn, &tmp, st));
        coarse_ms += ms_since(c0);
        cn = w.Cn;
        PP_(theta_weight(pb, w, fl, w.Cn, th, st));
      }
      k_parareal_update<<<256, TPB, 0, st>>>(nd, cn, fl, w.Cold + l * nd, Ub + (l + 1) * nd, th);
      if (cn != w.Cold + l * nd &&
          hipMemcpyAsync(w.Cold + l * nd, w.Cn, nd * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) {
        ret = FSI_ERR_HIP;
        goto finish;
      }
      if (l >= i) PP_(input_ready(i + 1, l + 1));
    }
    PP_(boundary_change(pb, w, N, Ub, change, st));
    it = i + 1;
    sp->parareal_iters = it;
    if (change < tol) break;
  }
  if (!(change < tol) && it < N) ret = FSI_ERR_PARAREAL;
finish:
#undef PP_
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;   // queued chunks that are not needed any more are dropped
  }
  cv.notify_all();
  worker.join();   // a chunk already running finishes first
  (void)hipStreamSynchronize(ws);
  (void)hipStreamDestroy(ws);
  for (FineTask& t : tasks) (void)hipEventDestroy(t.ready);
  fine_ms += wfine_ms;
  sp->newton_total += wnewton;
  sp->krylov_total += wkrylov;
  return ret;
}

}  // namespace

extern "C" {

fsi_status parareal_run(fsi_problem* pb, double T, int32_t N, int32_t m, int32_t M, double tol, int32_t max_iter,
                        const double* U0, double* Ub, fsi_stats* stats, hipStream_t st) {
  if (!pb || !U0 || !Ub || N < 1 || N > pb->Bmax || m < 1 || M < 1 || !(T > 0.0) || max_iter < 1) return FSI_ERR_ARG;
  if (max_iter > N) max_iter = N;
  fsi_stats local;
  fsi_stats* sp = stats ? stats : &local;
  std::memset(sp, 0, sizeof(fsi_stats));
  auto t_start = std::chrono::steady_clock::now();
  double coarse_ms = 0.0, fine_ms = 0.0;
  const fsi_status ret = guarded([&] {
    return pb->p.parareal_pipeline > 0
               ? parareal_pipelined(pb, T, N, m, M, tol, max_iter, U0, Ub, sp, coarse_ms, fine_ms, st)
               : parareal_plain(pb, T, N, m, M, tol, max_iter, U0, Ub, sp, coarse_ms, fine_ms, st);
  });
  (void)hipStreamSynchronize(st);
  sp->stage_ms[5] = coarse_ms;
  sp->stage_ms[6] = fine_ms;
  sp->stage_ms[4] = ms_since(t_start);
  return ret;
}

fsi_status adjoint_gradient(fsi_problem* pb, double T, int32_t N, int32_t m, const double* U0, double* J_out,
                            double* grad_out, fsi_stats* stats, hipStream_t st) {
  if (!pb || !U0 || !J_out || !grad_out || N < 1 || N > pb->Bmax || m < 1 || !(T > 0.0)) return FSI_ERR_ARG;
  if (pb->mixed || pb->p.dim != 2 || pb->deg != 1) return FSI_ERR_ARG;   // the adjoint runs in the 2d Q1 FP64 path
  return guarded([&] { return adjoint_run(pb, T, N, m, U0, J_out, grad_out, stats, st); });
}

fsi_status fsi_debug_residual(fsi_problem* pb, int32_t B, const double* U, const double* Uo, const double* t,
                              double k, double* R, hipStream_t st) {
  if (!pb || !U || !Uo || !t || !R || B <= 0 || B > pb->Bmax || !(k > 0)) return FSI_ERR_ARG;
  HIPCHK(hipMemcpyAsync(pb->tdev, t, B * sizeof(double), hipMemcpyHostToDevice, st));
  if (pb->p.dim == 3)
    CHK(residual<3>(pb, B, step_par(pb, k), U, Uo, R, nullptr, st));
  else
    CHK(residual<2>(pb, B, step_par(pb, k), U, Uo, R, nullptr, st));
  HIPCHK(hipStreamSynchronize(st));
  return FSI_OK;
}

fsi_status fsi_residual_noalloc(fsi_problem* pb, int32_t B, const double* U, const double* Uo, const double* t,
                                double k, double* R, hipStream_t st) {
  if (!pb || !U || !Uo || !t || !R || B <= 0 || B > pb->Bmax || !(k > 0) || !pb->scratch) return FSI_ERR_ARG;
  const Level& F = pb->lev[pb->nlev - 1];
  const Level& Cq = pb->lev[pb->nlev - (pb->deg == 2 ? 2 : 1)];   // the cells of the element kernels
  const int NE = pb->deg == 2 ? 45 : (pb->p.dim == 3 ? Dm<3>::NE : Dm<2>::NE);
  // element residuals [B][NE][ncell], then the B slice times at a 256-byte boundary
  const size_t re_vals = (size_t)B * NE * Cq.ncell;
  const size_t t_off = (re_vals + 31) / 32 * 32;
  if ((t_off + (size_t)B) * sizeof(double) > SCRATCH_BYTES) {
    std::fprintf(stderr, "fsi_residual_noalloc: %d slices need %zu bytes of scratch, more than its %zu\n", B,
                 (t_off + (size_t)B) * sizeof(double), SCRATCH_BYTES);
    return FSI_ERR_ARG;
  }
  double* re = pb->scratch;
  double* td = pb->scratch + t_off;
  HIPCHK(hipMemcpyAsync(td, t, B * sizeof(double), hipMemcpyHostToDevice, st));
  const StepPar sp = step_par(pb, k);
  const Geom g = F.geom();
  if (pb->deg == 2) {
    const Geom gc = Cq.geom();
    k_elem_residual_q2<<<grid1(gc.ncell, B), TPB, 0, st>>>(gc, g, sp, U, Uo, re, nullptr);
    k_gather_residual_q2<<<grid1(g.nn, B), TPB, 0, st>>>(gc, g, sp, pb->pst2, re, U, td, R, nullptr);
  } else if (pb->p.dim == 3) {
    k_elem_residual<3><<<grid1(g.ncell, B), TPB, 0, st>>>(g, sp, U, Uo, re, nullptr);
    k_gather_residual<3><<<grid1(g.nn, B), TPB, 0, st>>>(g, sp, re, U, td, R, nullptr);
  } else {
    k_elem_residual<2><<<grid1(g.ncell, B), TPB, 0, st>>>(g, sp, U, Uo, re, nullptr);
    k_gather_residual<2><<<grid1(g.nn, B), TPB, 0, st>>>(g, sp, re, U, td, R, nullptr);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return FSI_OK;
}

}  // extern "C"

namespace {

// Debug entries: assemble the hierarchy at (U, Uo, t, k), then Y = J X (what = 0)
// or Y = one V-cycle applied to X (what = 1); FP64 in and out.
template <int D, class S>
fsi_status debug_apply(fsi_problem* pb, int B, const double* U, const double* Uo, const double* t, double k,
                       const double* X, double* Y, int what, hipStream_t st) {
  FSI_DIM(D);
  Level& F = pb->lev[pb->nlev - 1];
  const size_t ndof = (size_t)F.nn * NC;
  const StepPar sp = step_par(pb, k);
  pb->prof.pact = B;   // every slice works (profiled bytes)
  HIPCHK(hipMemcpyAsync(pb->tdev, t, B * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pb->U, U, B * ndof * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(pb->Uold, Uo, B * ndof * sizeof(double), hipMemcpyDeviceToDevice, st));
  CHK(assemble_levels<D, S, true>(pb, B, sp, nullptr, st));
  k_convert<double, S><<<1024, TPB, 0, st>>>(B * ndof, X, (S*)pb->tmp);
  if (what == 0)
    krylov_spmv<D, S, true>(pb, B, k, (const S*)pb->tmp, nullptr, nullptr, (S*)pb->w, nullptr, st);
  else
    vcycle<D, S, true>(pb, B, k, (const S*)pb->tmp, (S*)pb->w, nullptr, st);
  k_convert<S, double><<<1024, TPB, 0, st>>>(B * ndof, (const S*)pb->w, Y);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return FSI_OK;
}

fsi_status debug_dispatch(fsi_problem* pb, int B, const double* U, const double* Uo, const double* t, double k,
                          const double* X, double* Y, int what, hipStream_t st) {
  if (!pb || !U || !Uo || !t || !X || !Y || B <= 0 || B > pb->Bmax || !(k > 0)) return FSI_ERR_ARG;
  if (pb->p.dim == 3)
    return pb->mixed ? debug_apply<3, float>(pb, B, U, Uo, t, k, X, Y, what, st)
                     : debug_apply<3, double>(pb, B, U, Uo, t, k, X, Y, what, st);
  return pb->mixed ? debug_apply<2, float>(pb, B, U, Uo, t, k, X, Y, what, st)
                   : debug_apply<2, double>(pb, B, U, Uo, t, k, X, Y, what, st);
}

}  // namespace

extern "C" {

fsi_status fsi_debug_jacobian_apply(fsi_problem* pb, int32_t B, const double* U, const double* Uo, const double* t,
                                    double k, const double* X, double* Y, hipStream_t st) {
  return guarded([&] { return debug_dispatch(pb, B, U, Uo, t, k, X, Y, 0, st); });
}

fsi_status fsi_debug_vcycle(fsi_problem* pb, int32_t B, const double* U, const double* Uo, const double* t, double k,
                            const double* X, double* Y, hipStream_t st) {
  return guarded([&] { return debug_dispatch(pb, B, U, Uo, t, k, X, Y, 1, st); });
}

fsi_status fsi_profile_enable(fsi_problem* pb, int32_t on) {
  if (!pb) return FSI_ERR_ARG;
  pb->prof.on = on != 0;
  if (on) {
    pb->prof.used = 0;
    for (int f = 0; f < F_NFAM; ++f) {
      pb->prof.ev[f].clear();
      pb->prof.bytes[f] = 0;
      pb->prof.launches[f] = 0;
    }
  }
  return FSI_OK;
}

fsi_status fsi_profile_query(const fsi_problem* pb, int32_t which, int64_t* launches, double* ms, double* bytes) {
  if (!pb || which < 0 || which >= F_NFAM) return FSI_ERR_ARG;
  double tot = 0.0;
  for (auto& e : pb->prof.ev[which]) {
    float m = 0.f;
    if (hipEventSynchronize(e.second) != hipSuccess) return FSI_ERR_HIP;
    if (hipEventElapsedTime(&m, e.first, e.second) != hipSuccess) return FSI_ERR_HIP;
    tot += m;
  }
  if (launches) *launches = pb->prof.launches[which];
  if (ms) *ms = tot;
  if (bytes) *bytes = pb->prof.bytes[which];
  return FSI_OK;
}

}  // extern "C"
