// Host side of the C ABI declared in include/ift.h: argument validation,
// mesh preprocessing (face pairing and gather maps), reference-element
// tables, workspace management and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/ift.h"
#include "kernels.hpp"
#include "batch.hpp"
#include "mixed.hpp"
#include "mlp.hpp"

namespace ift {
__constant__ RefTab c_tab[2];
}

using namespace ift;

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return IFT_EDEVICE;           \
  } while (0)

struct ift_problem {
  int pde = 0, p = 1, n_elem = 0, n_gnode = 0;
  int nn = 3, nc = 1, nue = 3, nun = 6, nxe = 6;
  long long N_u = 0, N_x = 0;
  double gamma = 1.4, kappa = 0.0, eps_g = 1e-8, bc_mu_scale = 0.5;
  int all_farfield = 0;
  double src_amp = 0.0;   // Burgers source amplitude (0: none)
  int bc_spacetime = 0;
  std::vector<int> h_gn, h_face;
  std::vector<long long> h_Pn;
  std::vector<double> h_X;
  int* d_gn = nullptr;
  int* d_face = nullptr;
  int* d_Pn = nullptr;
  double* d_X = nullptr;
  int* d_flags = nullptr;
  double* d_eta_ref = nullptr;   // distortion of each reference element [n_elem]
  void* d_pts = nullptr;   // point-data workspace of the Jacobian path [n_elem]
  double* d_hn_part = nullptr;   // residual-norm block sums [points][blocks] (grown on demand)
  int* d_hn_bad = nullptr;
  long long hn_cap = 0;
};

struct ift_rom {
  ift_problem* prob = nullptr;
  int n = 0, m = 0, D = 0, n_s = 0;
  ift_precision precision = IFT_FP64;
  int* d_eq = nullptr;
  double* d_rho = nullptr;
  double* d_srho = nullptr;
  double* d_Phi_s = nullptr;
  double* d_phisum = nullptr;   // [n_c][n]: sum over the nodes of Phi's component-c rows
  double* d_Phin_s = nullptr;
  double* d_Psi_s = nullptr;
  double* d_X_s = nullptr;
  int* d_face_s = nullptr;    // [n_s][3]: face codes of the sampled elements
  double* d_eta_ref_s = nullptr;   // [n_s]: distortion of each sampled reference element
  double* d_LiftU = nullptr;  // [n_s][n][nue + nun]: the gathered Phi rows, column-major per element
  double* d_LiftX = nullptr;  // [n_s][m][nxe]: the gathered Psi rows, column-major per element
  double* d_Bw = nullptr;   // reduced state basis at the quadrature points [n_s][KWP][n]
  double* d_Bx = nullptr;   // mapping-basis geometry derivatives [n_s][KXP][m]
  short* d_Bw16 = nullptr;  // BF16 copies, column-major per element (mixed precision)
  short* d_Bx16 = nullptr;
  // workspaces
  long long nrows = 0;
  int n_gram_blk = 0;
  int gram_rows_per = 0;
  int max_pts = 0;        // evaluation points the per-point workspaces hold
  double* d_Jt = nullptr;
  double* d_Ft = nullptr;
  double* d_Jpart = nullptr;
  int* d_flags = nullptr;
  double* d_PTR = nullptr;
  double* d_gram_part = nullptr;
  void* d_pts = nullptr;
  PhysConst* d_pcs = nullptr;   // physical constants of the points of a multi-point call [max_pts]
  int fused_nt = 0;             // column tiles of the fused assembly + Gram (0: two-kernel path)
  double* d_fpart = nullptr;    // fused block partials
  int* d_fbad = nullptr;
  // Gauss-Newton state
  double* d_H = nullptr;
  double* d_g = nullptr;
  double* d_J = nullptr;
  double* d_Jtrial = nullptr;
  double* d_dz = nullptr;
  double* d_solve_out = nullptr;
  double* d_qr[2] = {nullptr, nullptr};   // QR step: stacked triangles (allocated by the first QR step)
  double* d_wt = nullptr;
  double* d_tt = nullptr;
  int* d_nbad = nullptr;
  int* d_flag_or = nullptr;
};

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRec {
  int kind;
  hipEvent_t a, b;
  bool own_a;   // false: a is the end event of the preceding record
};
bool g_prof_on = false;
hipEvent_t g_prof_tail = nullptr;     // end event of the last record
hipStream_t g_prof_tail_st = nullptr;
std::vector<ProfRec> g_prof_live;     // recorded, not yet read
std::vector<hipEvent_t> g_prof_pool;  // idle events
int g_prof_count[IFT_PROF_NKIND] = {};
double g_prof_ms[IFT_PROF_NKIND] = {};

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch: events recorded before and after enqueueing it.  A
// chained scope directly follows the previous scope on the same stream and
// starts at that scope's end event (fewer events between back-to-back
// kernels).
struct ProfScope {
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  bool own_a = true;
  bool on;
  ProfScope(int k, hipStream_t s, bool chain = false, bool enable = true) : kind(k), st(s), on(enable && g_prof_on) {
    if (!on) return;
    if (chain && g_prof_tail && g_prof_tail_st == s) {
      a = g_prof_tail;
      own_a = false;
    } else {
      a = prof_event();
      if (a) (void)hipEventRecord(a, st);
    }
    b = prof_event();
  }
  ~ProfScope() {
    if (!on || !a || !b) return;
    (void)hipEventRecord(b, st);
    g_prof_live.push_back({kind, a, b, own_a});
    g_prof_tail = b;
    g_prof_tail_st = st;
  }
};

void prof_drain() {
  for (auto& r : g_prof_live) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_prof_count[r.kind] += 1;
      g_prof_ms[r.kind] += ms;
    }
  }
  for (auto& r : g_prof_live) {
    if (r.own_a) g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_live.clear();
  g_prof_tail = nullptr;
}
}  // namespace

extern "C" ift_status ift_profile_enable(int on) {
  g_prof_on = on != 0;
  g_prof_tail = nullptr;
  return IFT_OK;
}

extern "C" ift_status ift_profile_reset(void) {
  prof_drain();
  for (int k = 0; k < IFT_PROF_NKIND; ++k) {
    g_prof_count[k] = 0;
    g_prof_ms[k] = 0.0;
  }
  return IFT_OK;
}

extern "C" ift_status ift_profile_read(int which, int* count, double* total_ms) {
  if (which < 0 || which >= IFT_PROF_NKIND) return IFT_EINVAL;
  prof_drain();
  if (count) *count = g_prof_count[which];
  if (total_ms) *total_ms = g_prof_ms[which];
  return IFT_OK;
}

// --------------------------------------------------------- reference tables
// Closed forms: barycentric Lagrange bases of degree 1 and 2; the 3-point
// degree-2 rule; the 6-point degree-4 rule of Dunavant (1985) in its
// closed form; Gauss-Legendre with p+1 points on [0, 1].
static void build_tables(int p, RefTab& t) {
  std::memset(&t, 0, sizeof(t));
  const int nn = (p + 1) * (p + 2) / 2;
  std::vector<double> qx, qy, qw;
  if (p == 1) {
    const double a = 1.0 / 6.0, b = 2.0 / 3.0;
    qx = {a, b, a};
    qy = {a, a, b};
    qw = {1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
  } else {
    const double s10 = std::sqrt(10.0);
    const double r = std::sqrt(38.0 - 44.0 * std::sqrt(0.4));
    const double a1 = (8.0 - s10 + r) / 18.0, a2 = (8.0 - s10 - r) / 18.0;
    const double rw = std::sqrt(213125.0 - 53320.0 * s10);
    const double w1 = 0.5 * (620.0 + rw) / 3720.0, w2 = 0.5 * (620.0 - rw) / 3720.0;
    for (double a : {a1, a2}) {
      const double w = (a == a1) ? w1 : w2;
      const double c = 1.0 - 2.0 * a;
      qx.insert(qx.end(), {a, c, a});
      qy.insert(qy.end(), {a, a, c});
      qw.insert(qw.end(), {w, w, w});
    }
  }
  const int nq = (int)qw.size();
  for (int q = 0; q < nq; ++q) {
    const double xi = qx[q], eta = qy[q];
    const double l[3] = {1.0 - xi - eta, xi, eta};
    const double dl[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
    t.wv[q] = qw[q];
    for (int i = 0; i < 3; ++i) {
      if (p == 1) {
        t.phiv[q][i] = l[i];
        t.dphiv[q][i][0] = dl[i][0];
        t.dphiv[q][i][1] = dl[i][1];
      } else {
        t.phiv[q][i] = l[i] * (2.0 * l[i] - 1.0);
        t.dphiv[q][i][0] = (4.0 * l[i] - 1.0) * dl[i][0];
        t.dphiv[q][i][1] = (4.0 * l[i] - 1.0) * dl[i][1];
      }
    }
    if (p == 2) {
      for (int f = 0; f < 3; ++f) {
        const int a = f, b = (f + 1) % 3;
        t.phiv[q][3 + f] = 4.0 * l[a] * l[b];
        t.dphiv[q][3 + f][0] = 4.0 * (l[b] * dl[a][0] + l[a] * dl[b][0]);
        t.dphiv[q][3 + f][1] = 4.0 * (l[b] * dl[a][1] + l[a] * dl[b][1]);
      }
    }
  }
  std::vector<double> s, ws;
  if (p == 1) {
    const double h = 0.5 / std::sqrt(3.0);
    s = {0.5 - h, 0.5 + h};
    ws = {0.5, 0.5};
  } else {
    const double h = 0.5 * std::sqrt(0.6);
    s = {0.5 - h, 0.5, 0.5 + h};
    ws = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  }
  for (int q = 0; q <= p; ++q) {
    const double x = s[q];
    t.wf[q] = ws[q];
    if (p == 1) {
      t.L[q][0] = 1.0 - x;
      t.L[q][1] = x;
      t.dL[q][0] = -1.0;
      t.dL[q][1] = 1.0;
    } else {
      t.L[q][0] = 2.0 * (x - 0.5) * (x - 1.0);
      t.L[q][1] = -4.0 * x * (x - 1.0);
      t.L[q][2] = 2.0 * x * (x - 0.5);
      t.dL[q][0] = 4.0 * x - 3.0;
      t.dL[q][1] = -8.0 * x + 4.0;
      t.dL[q][2] = 4.0 * x - 1.0;
    }
  }
  for (int f = 0; f < 3; ++f) {
    t.en[f][0] = f;
    if (p == 1) {
      t.en[f][1] = (f + 1) % 3;
    } else {
      t.en[f][1] = 3 + f;
      t.en[f][2] = (f + 1) % 3;
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int f = 0; f < 3; ++f) {
      t.nfk[i][f] = -1;
      if (i < nn)
        for (int k = 0; k <= p; ++k)
          if (t.en[f][k] == i) t.nfk[i][f] = k;
      for (int q = 0; q <= p; ++q) t.wl[i][f][q] = t.nfk[i][f] >= 0 ? t.wf[q] * t.L[q][t.nfk[i][f]] : 0.0;
    }
}

static bool g_tables_ready = false;

static ift_status ensure_tables() {
  if (g_tables_ready) return IFT_OK;
  RefTab t[2];
  build_tables(1, t[0]);
  build_tables(2, t[1]);
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_tab), t, sizeof(t)));
  g_tables_ready = true;
  return IFT_OK;
}

template <class T>
static ift_status dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) return IFT_ENOMEM;
  return IFT_OK;
}

template <class T>
static void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static PhysConst phys_const(const ift_problem* pr, const double* mu) {
  PhysConst pc;
  std::memset(&pc, 0, sizeof(pc));
  pc.gamma = pr->gamma;
  pc.all_farfield = pr->all_farfield;
  if (pr->pde == IFT_BURGERS2D) {
    pc.src_amp = pr->src_amp;
    pc.bc_st = pr->bc_spacetime;
    if (mu) {
      pc.uinf[0] = pr->bc_spacetime ? mu[0] : 1.0 + pr->bc_mu_scale * mu[0];
      pc.uinf[1] = pr->bc_spacetime ? 1.0 : pc.uinf[0];
      pc.src_b = pr->src_amp != 0.0 ? mu[1] : 0.0;
    }
  } else {
    const double M = mu[0];
    const double a = mu[1] * (M_PI / 180.0);
    const double c = std::sqrt(pr->gamma);
    pc.uinf[0] = 1.0;
    pc.uinf[1] = M * c * std::cos(a);
    pc.uinf[2] = M * c * std::sin(a);
    pc.uinf[3] = 1.0 / (pr->gamma - 1.0) + 0.5 * pr->gamma * M * M;
  }
  return pc;
}

static bool finite_mu(const ift_problem* pr, const double* mu) {
  if (!mu) return false;
  const int nmu = pr->pde == IFT_BURGERS2D && pr->src_amp == 0.0 ? 1 : 2;
  for (int i = 0; i < nmu; ++i)
    if (!std::isfinite(mu[i])) return false;
  if (pr->pde == IFT_EULER2D && !(mu[0] > 0.0)) return false;
  return true;
}

static size_t gram_shm_bytes(int D, int rows_per) {
  const int Dp = (D + 3) & ~3, TD = Dp / 4;
  const int G = TD * TD <= 64 ? 4 : (TD * TD <= 128 ? 2 : 1);
  const size_t rows = (size_t)rows_per * (Dp + 1);
  const size_t red = (size_t)(G - 1) * TD * TD * 20;
  return sizeof(double) * std::max(rows, red);
}

// Bytes of one element's point data (the double layout is the larger one).
static size_t pts_bytes(const ift_problem* pr) {
  if (pr->pde == IFT_BURGERS2D)
    return pr->p == 1 ? sizeof(Pts<Disc<PDE_BURGERS, 1>, double>) : sizeof(Pts<Disc<PDE_BURGERS, 2>, double>);
  return pr->p == 1 ? sizeof(Pts<Disc<PDE_EULER, 1>, double>) : sizeof(Pts<Disc<PDE_EULER, 2>, double>);
}

// Calls f.template run<Disc<...>>() for the problem's discretisation.
template <class F>
static void with_disc(const ift_problem* pr, F&& f) {
  if (pr->pde == IFT_BURGERS2D) {
    if (pr->p == 1) f.template run<Disc<PDE_BURGERS, 1>>();
    else f.template run<Disc<PDE_BURGERS, 2>>();
  } else {
    if (pr->p == 1) f.template run<Disc<PDE_EULER, 1>>();
    else f.template run<Disc<PDE_EULER, 2>>();
  }
}

// Distortion of every reference element (the reference term of N_e).
struct EtaRef {
  ift_problem* pr;
  template <class D>
  void run() {
    hipLaunchKernelGGL((k_eta_ref<D>), dim3((pr->n_elem + 255) / 256), dim3(256), 0, 0, (const double*)pr->d_X,
                       (const int*)pr->d_gn, pr->n_elem, pr->d_eta_ref);
  }
};

// ------------------------------------------------------------------- problem
extern "C" ift_status ift_problem_create(const ift_problem_desc* d, ift_problem** out) {
  if (!d || !out) return IFT_EINVAL;
  *out = nullptr;
  if (d->pde != IFT_BURGERS2D && d->pde != IFT_EULER2D) return IFT_EINVAL;
  if (d->p != 1 && d->p != 2) return IFT_EINVAL;
  if (d->n_elem <= 0 || d->n_gnode <= 0 || !d->X || !d->elem_gnodes || !d->elem_nbr) return IFT_EINVAL;
  if (!(d->eps_g > 0.0) || !(d->kappa >= 0.0) || !std::isfinite(d->kappa)) return IFT_EINVAL;
  if (d->pde == IFT_EULER2D && !(d->gamma > 1.0)) return IFT_EINVAL;
  if (!std::isfinite(d->src_amp) || (d->bc_spacetime != 0 && d->bc_spacetime != 1)) return IFT_EINVAL;
  if (d->pde == IFT_EULER2D && (d->src_amp != 0.0 || d->bc_spacetime != 0)) return IFT_EINVAL;
  ift_status st;
  ift_problem* pr = new ift_problem();
  pr->pde = d->pde;
  pr->p = d->p;
  pr->n_elem = d->n_elem;
  pr->n_gnode = d->n_gnode;
  pr->nn = (d->p + 1) * (d->p + 2) / 2;
  pr->nc = d->pde == IFT_BURGERS2D ? 1 : 4;
  pr->nue = pr->nn * pr->nc;
  pr->nun = 3 * (d->p + 1) * pr->nc;
  pr->nxe = 2 * pr->nn;
  pr->N_u = (long long)d->n_elem * pr->nue;
  pr->N_x = 2LL * d->n_gnode;
  pr->gamma = d->gamma;
  pr->kappa = d->kappa;
  pr->eps_g = d->eps_g;
  pr->bc_mu_scale = d->bc_mu_scale;
  pr->all_farfield = d->all_farfield;
  pr->src_amp = d->src_amp;
  pr->bc_spacetime = d->bc_spacetime;
  const int Ne = d->n_elem, nn = pr->nn;
  pr->h_gn.assign(d->elem_gnodes, d->elem_gnodes + (size_t)Ne * nn);
  pr->h_face.assign(d->elem_nbr, d->elem_nbr + (size_t)Ne * 3);
  pr->h_X.assign(d->X, d->X + (size_t)2 * d->n_gnode);
  for (double v : pr->h_X)
    if (!std::isfinite(v)) { delete pr; return IFT_EINVAL; }
  for (int g : pr->h_gn)
    if (g < 0 || g >= d->n_gnode) { delete pr; return IFT_EINVAL; }
  // face pairing: the neighbour E across face f of e must list e exactly once;
  // the shared edge is traversed in opposite directions.
  const int P = d->p, NC = pr->nc, NE = P + 1;
  pr->h_Pn.assign((size_t)Ne * pr->nun, -1);
  for (int e = 0; e < Ne; ++e) {
    for (int f = 0; f < 3; ++f) {
      const int E = pr->h_face[e * 3 + f];
      if (E < 0) {
        if (E < -4) { delete pr; return IFT_EINVAL; }
        continue;
      }
      if (E >= Ne || E == e) { delete pr; return IFT_EINVAL; }
      int g = -1, cnt = 0;
      for (int h = 0; h < 3; ++h)
        if (pr->h_face[E * 3 + h] == e) { g = h; ++cnt; }
      if (cnt != 1) { delete pr; return IFT_EINVAL; }
      if (pr->h_gn[e * nn + f] != pr->h_gn[E * nn + (g + 1) % 3] ||
          pr->h_gn[e * nn + (f + 1) % 3] != pr->h_gn[E * nn + g]) {
        delete pr;
        return IFT_EINVAL;
      }
      for (int k = 0; k < NE; ++k) {
        // neighbour's edge node p-k of face g sits at e's edge node k
        const int kk = P - k;
        int node;
        if (kk == 0) node = g;
        else if (kk == P) node = (g + 1) % 3;
        else node = 3 + g;
        for (int c = 0; c < NC; ++c)
          pr->h_Pn[((size_t)e * 3 + f) * NE * NC + k * NC + c] = ((long long)E * nn + node) * NC + c;
      }
    }
  }
  std::vector<int> pn32(pr->h_Pn.size());
  if (pr->N_u > 0x7fffffffLL) { delete pr; return IFT_EINVAL; }
  // all host-side checks passed: from here on the device is touched
  if ((st = ensure_tables()) != IFT_OK) { delete pr; return st; }
  for (size_t i = 0; i < pn32.size(); ++i) pn32[i] = (int)pr->h_Pn[i];
  if ((st = dalloc(&pr->d_gn, pr->h_gn.size())) != IFT_OK ||
      (st = dalloc(&pr->d_face, pr->h_face.size())) != IFT_OK ||
      (st = dalloc(&pr->d_Pn, pn32.size())) != IFT_OK ||
      (st = dalloc(&pr->d_X, pr->h_X.size())) != IFT_OK ||
      (st = dalloc(&pr->d_flags, (size_t)Ne)) != IFT_OK ||
      (st = dalloc(&pr->d_eta_ref, (size_t)Ne)) != IFT_OK) {
    ift_problem_destroy(pr);
    return st;
  }
  if (hipMalloc(&pr->d_pts, (size_t)Ne * pts_bytes(pr)) != hipSuccess) {
    ift_problem_destroy(pr);
    return IFT_ENOMEM;
  }
  if (hipMemcpy(pr->d_gn, pr->h_gn.data(), pr->h_gn.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pr->d_face, pr->h_face.data(), pr->h_face.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pr->d_Pn, pn32.data(), pn32.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pr->d_X, pr->h_X.data(), pr->h_X.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    ift_problem_destroy(pr);
    return IFT_EDEVICE;
  }
  with_disc(pr, EtaRef{pr});
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    ift_problem_destroy(pr);
    return IFT_EDEVICE;
  }
  *out = pr;
  return IFT_OK;
}

extern "C" void ift_problem_destroy(ift_problem* pr) {
  if (!pr) return;
  dfree(pr->d_gn);
  dfree(pr->d_face);
  dfree(pr->d_Pn);
  dfree(pr->d_X);
  dfree(pr->d_flags);
  dfree(pr->d_eta_ref);
  dfree(pr->d_hn_part);
  dfree(pr->d_hn_bad);
  if (pr->d_pts) (void)hipFree(pr->d_pts);
  delete pr;
}

extern "C" ift_status ift_problem_sizes(const ift_problem* pr, int* nue, int* nun, int* nxe, long long* N_u,
                                        long long* N_x) {
  if (!pr) return IFT_EINVAL;
  if (nue) *nue = pr->nue;
  if (nun) *nun = pr->nun;
  if (nxe) *nxe = pr->nxe;
  if (N_u) *N_u = pr->N_u;
  if (N_x) *N_x = pr->N_x;
  return IFT_OK;
}

extern "C" ift_status ift_problem_neighbour_map(const ift_problem* pr, long long* Pn) {
  if (!pr || !Pn) return IFT_EINVAL;
  std::copy(pr->h_Pn.begin(), pr->h_Pn.end(), Pn);
  return IFT_OK;
}

// --------------------------------------------------------------- dispatch
struct HdmLaunch {
  const HdmArgs& a;
  bool jac;
  hipStream_t st;
  template <class D>
  void run() {
    if (jac && D::NC == 4) {
      // one pass: point physics and the blocks written from the same LDS
      ProfScope ps(IFT_PROF_HDM, st);
      if constexpr (pair_layout<D>())
        hipLaunchKernelGGL((k_hdm_fused2<D, double>), dim3((a.n_elem + 1) / 2), dim3(2 * NTHR_PTS), 0, st, a);
      else
        hipLaunchKernelGGL((k_hdm_fused<D, double>), dim3(a.n_elem), dim3(NTHR_PTS), 0, st, a);
    } else if (jac) {
      {
        ProfScope ps(IFT_PROF_POINTS, st);
        hipLaunchKernelGGL((k_points_hdm<D, double>), dim3(a.n_elem), dim3(NTHR_PTS), 0, st, a);
      }
      ProfScope ps(IFT_PROF_HDM, st);
      hipLaunchKernelGGL((k_hdm_asm<D, double>), dim3(a.n_elem), dim3(NTHR), 0, st, a);
    } else {
      ProfScope ps(IFT_PROF_HDM, st);
      hipLaunchKernelGGL((k_hdm_val<D, double>), dim3(a.n_elem), dim3(NTHR), 0, st, a);
    }
  }
};

extern "C" ift_status hdm_assemble(ift_problem* pr, const double* mu, const double* U, const double* x, double* R,
                                   double* N, double* dRdU, double* dRdUn, double* dRdx, double* dNdx, int* n_bad,
                                   hipStream_t stream) {
  if (!pr || !U || !x || !finite_mu(pr, mu)) return IFT_EINVAL;
  HdmArgs a;
  a.U = U;
  a.x = x;
  a.gn = pr->d_gn;
  a.face = pr->d_face;
  a.Pn = pr->d_Pn;
  a.X = pr->d_X;
  a.R = R;
  a.N = N;
  a.dRdU = dRdU;
  a.dRdUn = dRdUn;
  a.dRdx = dRdx;
  a.dNdx = dNdx;
  a.flags = pr->d_flags;
  a.eta_ref = pr->d_eta_ref;
  a.pts = pr->d_pts;
  a.pc = phys_const(pr, mu);
  a.kappa = pr->kappa;
  a.eps = pr->eps_g;
  a.n_elem = pr->n_elem;
  const bool jac = dRdU || dRdUn || dRdx || dNdx;
  ift_status s;
  with_disc(pr, HdmLaunch{a, jac, stream});
  s = hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
  if (s != IFT_OK) return s;
  if (n_bad) {
    hipLaunchKernelGGL(k_obj_final, dim3(1), dim3(256), 0, stream, (const double*)nullptr, (const int*)pr->d_flags,
                       pr->n_elem, (double*)nullptr, n_bad, (int*)nullptr);
    if (hipGetLastError() != hipSuccess) return IFT_EDEVICE;
  }
  return IFT_OK;
}

// Full-order residual norms at reduced solutions (greedy indicator).
struct HdmRomLaunch {
  const HdmRomArgs& a;
  int n_pts;
  hipStream_t st;
  template <class D>
  void run() {
    ProfScope ps(IFT_PROF_HDM, st);
    hipLaunchKernelGGL((k_hdm_res_rom<D, double>), dim3(a.nblk, n_pts), dim3(RV_THR), 0, st, a);
  }
};

extern "C" ift_status hdm_residual_norm_batched(ift_problem* pr, int n_pts, const double* mu, const double* Phi, int n,
                                                const double* w, const double* Psi, int m, const double* tau,
                                                double* norms, int* n_bad, hipStream_t stream) {
  if (!pr || n_pts < 1 || !mu || !Phi || n < 1 || !w || m < 0 || (m > 0 && (!Psi || !tau)) || !norms)
    return IFT_EINVAL;
  const int nblk = (pr->n_elem + RV_SLOTS - 1) / RV_SLOTS;
  const long long need = (long long)n_pts * nblk;
  if (need > pr->hn_cap) {
    dfree(pr->d_hn_part);
    dfree(pr->d_hn_bad);
    pr->hn_cap = 0;
    ift_status e;
    if ((e = dalloc(&pr->d_hn_part, need)) != IFT_OK || (e = dalloc(&pr->d_hn_bad, need)) != IFT_OK) return e;
    pr->hn_cap = need;
  }
  const double mu0[2] = {1.0, 0.0};
  HdmRomArgs a;
  a.Phi = Phi;
  a.Psi = Psi;
  a.w = w;
  a.tau = tau;
  a.mu = mu;
  a.gn = pr->d_gn;
  a.face = pr->d_face;
  a.Pn = pr->d_Pn;
  a.X = pr->d_X;
  a.pc = phys_const(pr, mu0);
  a.eps = pr->eps_g;
  a.bc_mu_scale = pr->bc_mu_scale;
  a.n = n;
  a.m = m;
  a.n_elem = pr->n_elem;
  a.nblk = nblk;
  a.part = pr->d_hn_part;
  a.nbad = pr->d_hn_bad;
  with_disc(pr, HdmRomLaunch{a, n_pts, stream});
  hipLaunchKernelGGL(k_hdm_norm_final, dim3(n_pts), dim3(256), 0, stream, (const double*)pr->d_hn_part,
                     (const int*)pr->d_hn_bad, nblk, norms, n_bad);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

// -------------------------------------------------------------------- ROM
extern "C" void ift_rom_destroy(ift_rom* r) {
  if (!r) return;
  dfree(r->d_eq);
  dfree(r->d_rho);
  dfree(r->d_srho);
  dfree(r->d_Phi_s);
  dfree(r->d_phisum);
  dfree(r->d_Phin_s);
  dfree(r->d_Psi_s);
  dfree(r->d_X_s);
  dfree(r->d_face_s);
  dfree(r->d_eta_ref_s);
  dfree(r->d_LiftU);
  dfree(r->d_LiftX);
  dfree(r->d_Jt);
  dfree(r->d_Ft);
  dfree(r->d_Jpart);
  dfree(r->d_flags);
  dfree(r->d_PTR);
  dfree(r->d_gram_part);
  dfree(r->d_fpart);
  dfree(r->d_fbad);
  dfree(r->d_H);
  dfree(r->d_g);
  dfree(r->d_J);
  dfree(r->d_Jtrial);
  dfree(r->d_dz);
  dfree(r->d_solve_out);
  dfree(r->d_qr[0]);
  dfree(r->d_qr[1]);
  dfree(r->d_wt);
  dfree(r->d_tt);
  dfree(r->d_nbad);
  dfree(r->d_flag_or);
  if (r->d_pts) (void)hipFree(r->d_pts);
  dfree(r->d_pcs);
  dfree(r->d_Bw);
  dfree(r->d_Bx);
  dfree(r->d_Bw16);
  dfree(r->d_Bx16);
  delete r;
}

// Reduced bases at the quadrature points of every sampled element (they
// depend only on the ROM): allocated and computed once at creation.
struct PointBases {
  ift_rom* r;
  bool ok;
  template <class D>
  void run() {
    using O = EqOp<D>;
    if (dalloc(&r->d_Bw, (size_t)r->n_s * O::KWP * (r->n + 1)) != IFT_OK ||
        dalloc(&r->d_Bx, (size_t)r->n_s * O::KXP * (r->m + 1)) != IFT_OK) {
      ok = false;
      return;
    }
    hipLaunchKernelGGL((k_point_bases<D>), dim3(r->n_s), dim3(256), 0, 0, (const double*)r->d_Phi_s,
                       (const double*)r->d_Phin_s, (const double*)r->d_Psi_s, r->n, r->m, r->d_Bw, r->d_Bx);
    ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (ok && r->precision == IFT_MIXED_BF16) {
      using Q = EqOp16<D>;
      if (dalloc(&r->d_Bw16, (size_t)r->n_s * (r->n + 1) * Q::KW16) != IFT_OK ||
          dalloc(&r->d_Bx16, (size_t)r->n_s * (r->m + 1) * Q::KX16) != IFT_OK) {
        ok = false;
        return;
      }
      hipLaunchKernelGGL((k_point_bases16<D>), dim3(r->n_s), dim3(256), 0, 0, (const double*)r->d_Bw,
                         (const double*)r->d_Bx, r->n, r->m, r->d_Bw16, r->d_Bx16);
      ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
  }
};

static bool build_point_bases(ift_rom* r) {
  PointBases pb{r, true};
  with_disc(r->prob, pb);
  return pb.ok;
}

// Work split of the fused assembly for n_pts points: E sampled elements per
// wave, nblk blocks of four waves per point.  About four waves per SIMD in
// total; nblk is a multiple of 8 so that the blocks of every point that
// cover the same elements run on the same XCD and share its L2.
struct FusedLayout {
  int E, nblk;
};
static constexpr long long FUSED_TARGET_WAVES = 2048;   // waves resident at two per SIMD
static FusedLayout fused_layout_units(long long ns, long long groups) {
  int E = (int)std::max<long long>(1, (ns * groups + FUSED_TARGET_WAVES - 1) / FUSED_TARGET_WAVES);
  int nblk = (int)((ns + 4LL * E - 1) / (4LL * E));
  if (nblk > 8) nblk = (nblk + 7) / 8 * 8;
  E = (int)((ns + 4LL * nblk - 1) / (4LL * nblk));
  return {E, nblk};
}
static FusedLayout fused_layout(const ift_rom* r, int n_pts) { return fused_layout_units(r->n_s, n_pts); }

// Multi-point FP64 calls of the four-component P2 discretisation take two
// points of an element per wave (k_eq_fused_pts2): the work items are
// (element, point pair), and the blocks of a pair write one partial per
// point.  Its iterations pair w and x steps (m > 0), and its B ring holds
// both stripes of an iteration in one 1 KB slot (n + m <= 30).
static bool fused_pts2_used(const ift_rom* r, int n_pts, bool rows) {
  const ift_problem* pr = r->prob;
  return !rows && n_pts >= 2 && r->precision == IFT_FP64 && pr->nc == 4 && pr->p == 2 && r->fused_nt >= 1 &&
         r->fused_nt <= 2 && r->m > 0 && r->n + r->m <= 30;
}
// Its blocks: two per CU in all (the kernel's occupancy), a multiple of 8 per
// point pair, each block's elements split over its four waves (E is the most
// any wave takes).
static FusedLayout fused_layout_pts2(const ift_rom* r, int n_pts) {
  const long long ns = r->n_s, groups = (n_pts + 1) / 2;
  long long nblk = (FUSED_TARGET_WAVES / 4 + groups - 1) / groups;
  nblk = std::min(nblk, (ns + 3) / 4);
  nblk = std::max(8LL, (nblk + 7) / 8 * 8);
  const long long bmax = (ns + nblk - 1) / nblk;
  return {(int)std::max(1LL, (bmax + 3) / 4), (int)nblk};
}

// (Re)allocates every workspace that scales with the number of evaluation
// points of one call.
static ift_status reserve_points(ift_rom* r, int max_pts) {
  if (max_pts <= r->max_pts) return IFT_OK;
  const ift_problem* pr = r->prob;
  const size_t P = (size_t)max_pts, ns = (size_t)r->n_s, D = (size_t)r->D;
  dfree(r->d_Jt);
  dfree(r->d_Ft);
  dfree(r->d_Jpart);
  dfree(r->d_flags);
  dfree(r->d_PTR);
  dfree(r->d_gram_part);
  dfree(r->d_fpart);
  dfree(r->d_fbad);
  if (r->d_pts) (void)hipFree(r->d_pts);
  r->d_pts = nullptr;
  dfree(r->d_H);
  dfree(r->d_g);
  dfree(r->d_J);
  dfree(r->d_Jtrial);
  dfree(r->d_dz);
  dfree(r->d_solve_out);
  dfree(r->d_qr[0]);
  dfree(r->d_qr[1]);
  dfree(r->d_wt);
  dfree(r->d_tt);
  dfree(r->d_nbad);
  dfree(r->d_flag_or);
  dfree(r->d_pcs);
  r->max_pts = 0;
  ift_status st;
  if ((st = dalloc(&r->d_Jt, P * r->nrows * D)) != IFT_OK || (st = dalloc(&r->d_Ft, P * r->nrows)) != IFT_OK ||
      (st = dalloc(&r->d_Jpart, P * ns)) != IFT_OK || (st = dalloc(&r->d_flags, P * ns)) != IFT_OK ||
      (st = dalloc(&r->d_PTR, P * ns * r->n)) != IFT_OK ||
      (st = dalloc(&r->d_gram_part, P * r->n_gram_blk * (D * D + D))) != IFT_OK ||
      (st = dalloc(&r->d_H, P * D * D)) != IFT_OK || (st = dalloc(&r->d_g, P * D)) != IFT_OK ||
      (st = dalloc(&r->d_J, P)) != IFT_OK || (st = dalloc(&r->d_Jtrial, P)) != IFT_OK ||
      (st = dalloc(&r->d_dz, P * D)) != IFT_OK || (st = dalloc(&r->d_solve_out, P * 8)) != IFT_OK ||
      (st = dalloc(&r->d_wt, P * r->n)) != IFT_OK || (st = dalloc(&r->d_tt, P * std::max(r->m, 1))) != IFT_OK ||
      (st = dalloc(&r->d_nbad, P)) != IFT_OK || (st = dalloc(&r->d_flag_or, P)) != IFT_OK ||
      (st = dalloc(&r->d_pcs, P)) != IFT_OK)
    return st;
  if (hipMalloc(&r->d_pts, P * ns * pts_bytes(pr)) != hipSuccess) return IFT_ENOMEM;
  if (r->fused_nt > 0) {
    size_t nb = 0;
    for (int q = 1; q <= max_pts; ++q) {
      nb = std::max(nb, (size_t)q * fused_layout(r, q).nblk);
      if (fused_pts2_used(r, q, false)) nb = std::max(nb, (size_t)q * fused_layout_pts2(r, q).nblk);
    }
    const size_t nh = (size_t)r->fused_nt * (r->fused_nt + 1) / 2;
    if ((st = dalloc(&r->d_fpart, nb * nh * 256)) != IFT_OK || (st = dalloc(&r->d_fbad, nb * 2)) != IFT_OK) return st;
  }
  r->max_pts = max_pts;
  return IFT_OK;
}

// Per-point workspaces are allocated on first use, so that handles used
// only through a batch never hold them.
static bool lazy_points(ift_rom* r) { return r->max_pts >= 1 || reserve_points(r, 1) == IFT_OK; }

extern "C" ift_status ift_rom_reserve(ift_rom* r, int max_pts) {
  if (!r || max_pts < 1) return IFT_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return IFT_EDEVICE;
  return reserve_points(r, max_pts);
}

extern "C" ift_status ift_rom_create(ift_problem* pr, int n, int m, const double* Phi, const double* Psi, int n_s,
                                     const int* eq_elem, const double* eq_rho, ift_precision precision,
                                     ift_rom** out) {
  if (!pr || !out || !Phi || (m > 0 && !Psi) || !eq_elem || !eq_rho) return IFT_EINVAL;
  *out = nullptr;
  if (n < 1 || m < 0 || n + m > 64 || n_s < 1) return IFT_EINVAL;
  if (precision != IFT_FP64 && precision != IFT_FP32_ELEM && precision != IFT_MIXED_BF16) return IFT_EINVAL;
  for (int k = 0; k < n_s; ++k) {
    if (eq_elem[k] < 0 || eq_elem[k] >= pr->n_elem) return IFT_EINVAL;
    if (!(eq_rho[k] >= 0.0) || !std::isfinite(eq_rho[k])) return IFT_EINVAL;
  }
  ift_rom* r = new ift_rom();
  r->prob = pr;
  r->n = n;
  r->m = m;
  r->D = n + m;
  r->n_s = n_s;
  r->precision = precision;
  const int nue = pr->nue, nun = pr->nun, nxe = pr->nxe, nn = pr->nn;
  r->nrows = (long long)n_s * nue + n_s;
  // Gram row blocks: about one per compute unit, at most GRAM_MAXROWS rows each
  const int Dp = (r->D + 3) & ~3;
  const long long cap = std::min<long long>(GRAM_MAXROWS, 6144 / (Dp + 1));   // row buffer <= 48 KB
  r->gram_rows_per = (int)std::min<long long>(cap, std::max<long long>(4, (r->nrows + 255) / 256));
  r->n_gram_blk = (int)((r->nrows + r->gram_rows_per - 1) / r->gram_rows_per);
  r->fused_nt = (r->D + 1 + 15) / 16 <= FUSED_MAXNT ? (r->D + 1 + 15) / 16 : 0;
  std::vector<long long> rows_u((size_t)n_s * nue), rows_n((size_t)n_s * nun), rows_x((size_t)n_s * nxe), rows_e(n_s);
  std::vector<double> hXs((size_t)n_s * nxe), hsr(n_s);
  std::vector<int> hfs((size_t)n_s * 3);
  for (int k = 0; k < n_s; ++k) {
    const int e = eq_elem[k];
    for (int f = 0; f < 3; ++f) hfs[(size_t)k * 3 + f] = pr->h_face[(size_t)e * 3 + f];
    for (int i = 0; i < nue; ++i) rows_u[(size_t)k * nue + i] = (long long)e * nue + i;
    for (int i = 0; i < nun; ++i) rows_n[(size_t)k * nun + i] = pr->h_Pn[(size_t)e * nun + i];
    for (int i = 0; i < nxe; ++i) {
      const long long gi = 2LL * pr->h_gn[(size_t)e * nn + i / 2] + (i & 1);
      rows_x[(size_t)k * nxe + i] = gi;
      hXs[(size_t)k * nxe + i] = pr->h_X[gi];
    }
    hsr[k] = std::sqrt(eq_rho[k]);
    rows_e[k] = e;
  }
  ift_status st;
  long long* d_rows = nullptr;
  const size_t maxrows = std::max({rows_u.size(), rows_n.size(), rows_x.size()});
#define ALLOC(ptr, cnt)                                       \
  if ((st = dalloc(&(ptr), (size_t)(cnt))) != IFT_OK) {       \
    dfree(d_rows);                                            \
    ift_rom_destroy(r);                                       \
    return st;                                                \
  }
  ALLOC(d_rows, maxrows);
  ALLOC(r->d_eq, n_s);
  ALLOC(r->d_rho, n_s);
  ALLOC(r->d_srho, n_s);
  ALLOC(r->d_Phi_s, (size_t)n_s * nue * n);
  ALLOC(r->d_Phin_s, (size_t)n_s * nun * n);
  ALLOC(r->d_Psi_s, (size_t)n_s * nxe * std::max(m, 1));
  ALLOC(r->d_X_s, (size_t)n_s * nxe);
  ALLOC(r->d_face_s, (size_t)n_s * 3);
  ALLOC(r->d_eta_ref_s, (size_t)n_s);
  ALLOC(r->d_LiftU, (size_t)n_s * n * (nue + nun));
  ALLOC(r->d_LiftX, (size_t)n_s * std::max(m, 1) * nxe);
#undef ALLOC
  bool ok = hipMemcpy(r->d_eq, eq_elem, n_s * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(r->d_rho, eq_rho, n_s * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(r->d_srho, hsr.data(), n_s * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(r->d_X_s, hXs.data(), hXs.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(r->d_face_s, hfs.data(), hfs.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
  auto gather = [&](const double* src, int ncol, const std::vector<long long>& rows, double* dst) {
    if (!ok || ncol == 0) return;
    ok = hipMemcpy(d_rows, rows.data(), rows.size() * sizeof(long long), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return;
    const long long tot = (long long)rows.size() * ncol;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, 0, src, ncol,
                       (const long long*)d_rows, (long long)rows.size(), dst);
    ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  };
  gather(Phi, n, rows_u, r->d_Phi_s);
  gather(Phi, n, rows_n, r->d_Phin_s);
  if (ok) {
    ok = dalloc(&r->d_phisum, (size_t)pr->nc * n) == IFT_OK;
    if (ok) {
      hipLaunchKernelGGL(k_phi_colsum, dim3(pr->nc * n), dim3(256), 0, 0, Phi, (long long)(pr->N_u / pr->nc), pr->nc,
                         n, r->d_phisum);
      ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
  }
  gather(Psi, m, rows_x, r->d_Psi_s);
  gather(pr->d_eta_ref, 1, rows_e, r->d_eta_ref_s);
  dfree(d_rows);
  if (ok) {
    const long long tot = (long long)n_s * (n * (nue + nun) + m * nxe);
    hipLaunchKernelGGL(k_lift_bases, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, 0, (const double*)r->d_Phi_s,
                       (const double*)r->d_Phin_s, (const double*)r->d_Psi_s, nue, nun, nxe, n, m, (long long)n_s,
                       r->d_LiftU, r->d_LiftX);
    ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  }
  if (ok) ok = build_point_bases(r);
  if (!ok) {
    ift_rom_destroy(r);
    return IFT_EDEVICE;
  }
  *out = r;
  return IFT_OK;
}

extern "C" ift_status ift_rom_get_gathers(ift_rom* r, double* Phi_s, double* Phin_s, double* Psi_s, double* X_s,
                                          hipStream_t stream) {
  if (!r) return IFT_EINVAL;
  const ift_problem* pr = r->prob;
  const size_t ns = r->n_s;
  if (Phi_s) HIP_TRY(hipMemcpyAsync(Phi_s, r->d_Phi_s, ns * pr->nue * r->n * sizeof(double), hipMemcpyDeviceToDevice, stream));
  if (Phin_s) HIP_TRY(hipMemcpyAsync(Phin_s, r->d_Phin_s, ns * pr->nun * r->n * sizeof(double), hipMemcpyDeviceToDevice, stream));
  if (Psi_s && r->m > 0) HIP_TRY(hipMemcpyAsync(Psi_s, r->d_Psi_s, ns * pr->nxe * r->m * sizeof(double), hipMemcpyDeviceToDevice, stream));
  if (X_s) HIP_TRY(hipMemcpyAsync(X_s, r->d_X_s, ns * pr->nxe * sizeof(double), hipMemcpyDeviceToDevice, stream));
  return IFT_OK;
}

static EqArgs eq_args(ift_rom* r, const double* mu, const double* w, const double* tau) {
  const ift_problem* pr = r->prob;
  EqArgs a;
  a.n_s = r->n_s;
  a.n = r->n;
  a.m = r->m;
  a.D = r->D;
  a.nrows = r->nrows;
  a.mu = nullptr;
  a.pcs = nullptr;
  a.face_s = r->d_face_s;
  a.eta_ref_s = r->d_eta_ref_s;
  a.rho = r->d_rho;
  a.srho = r->d_srho;
  a.Phi_s = r->d_Phi_s;
  a.Phin_s = r->d_Phin_s;
  a.Psi_s = r->d_Psi_s;
  a.X_s = r->d_X_s;
  a.LiftU = r->d_LiftU;
  a.LiftX = r->d_LiftX;
  a.w = w;
  a.tau = tau;
  a.Jt = r->d_Jt;
  a.Ft = r->d_Ft;
  a.Jpart = r->d_Jpart;
  a.flags = r->d_flags;
  a.PTR = nullptr;
  a.pts = r->d_pts;
  a.pc = phys_const(pr, mu);
  a.kappa = pr->kappa;
  a.eps = pr->eps_g;
  a.bc_mu_scale = pr->bc_mu_scale;
  return a;
}

// Workgroups are dealt to the 8 XCDs round-robin in linear order; padding
// the element axis of an (element, point) grid to a multiple of 8 keeps
// every point of one element on the same XCD, so its gathered operands are
// read from that XCD's L2 after the first point.
static inline int xcd_pad(int n) { return n > 8 ? (n + 7) / 8 * 8 : n; }

template <class R>
struct EqLaunch {
  const EqArgs& a;
  bool jac;
  int n_pts;
  hipStream_t st;
  const double* Bw;
  const double* Bx;
  const FusedArgs* fa;   // fused assembly + Gram, or null
  int nt;
  const short* Bw16;     // non-null: projection on BF16 matrix cores (R = float)
  const short* Bx16;
  template <class D, int NT>
  void fused() {
    if constexpr (std::is_same<R, double>::value && fused_pts2_ok<D, NT>()) {
      if (fa->pts2) {
        if constexpr (NT == 2) {
          if (pts2_tiles<NT>(a.n, a.m) == PTS2_TILES_N17) {
            hipLaunchKernelGGL((k_eq_fused_pts2<D, NT, PTS2_TILES_N17>), dim3(fa->nblk, (n_pts + 1) / 2), dim3(NTHR),
                               0, st, a, Bw, Bx, *fa, n_pts);
            return;
          }
        }
        hipLaunchKernelGGL((k_eq_fused_pts2<D, NT, pts2_tiles_all<NT>()>), dim3(fa->nblk, (n_pts + 1) / 2), dim3(NTHR),
                           0, st, a, Bw, Bx, *fa, n_pts);
        return;
      }
    }
    if constexpr (std::is_same<R, float>::value) {
      if (Bw16) {
        hipLaunchKernelGGL((k_eq_fused_mixed<D, NT>), dim3(fa->nblk, n_pts), dim3(NTHR), 0, st, a, Bw16, Bx16, *fa);
        return;
      }
    }
    hipLaunchKernelGGL((k_eq_fused<D, R, NT>), dim3(fa->nblk, n_pts), dim3(NTHR), 0, st, a, Bw, Bx, *fa);
  }
  template <class D>
  void run() {
    if (jac) {
      {
        ProfScope ps(IFT_PROF_POINTS, st);
        if (a.mu)   // the points' physical constants, which the point kernels read (dispatch_eq checks a.pcs)
          hipLaunchKernelGGL(k_phys_points, dim3((n_pts + 63) / 64), dim3(64), 0, st, a.pc, D::PDE, a.bc_mu_scale,
                             a.mu, n_pts, const_cast<PhysConst*>(a.pcs));
        if constexpr (pair_layout<D>())
          hipLaunchKernelGGL((k_points_eq2<D, R>), dim3(xcd_pad((a.n_s + 1) / 2), n_pts), dim3(2 * NTHR_PTS), 0, st, a);
        else
          hipLaunchKernelGGL((k_points_eq<D, R>), dim3(xcd_pad(a.n_s), n_pts), dim3(NTHR_PTS), 0, st, a);
      }
      ProfScope ps(IFT_PROF_EQ_JAC, st, true);
      if (!fa) hipLaunchKernelGGL((k_eq_asm<D, R>), dim3(a.n_s, n_pts), dim3(NTHR), 0, st, a, Bw, Bx);
      else if (nt == 1) fused<D, 1>();
      else if (nt == 2) fused<D, 2>();
      else fused<D, 3>();
    } else {
      ProfScope ps(IFT_PROF_EQ_RES, st);
      const long long items = (long long)n_pts * a.n_s;
      hipLaunchKernelGGL((k_eq_res16<D, R>), dim3((unsigned)((items + RV_SLOTS - 1) / RV_SLOTS)), dim3(RV_THR), 0, st,
                         a, n_pts);
    }
  }
};

static ift_status dispatch_eq(const ift_rom* r, const EqArgs& a, bool jac, int n_pts, hipStream_t st,
                              const FusedArgs* fa = nullptr) {
  // the point kernels of the Jacobian path take a call's per-point constants
  // from a.pcs, which their launch fills from a.mu
  if (jac && a.mu && !a.pcs) return IFT_EINVAL;
  if (r->precision != IFT_FP64)
    with_disc(r->prob, EqLaunch<float>{a, jac, n_pts, st, r->d_Bw, r->d_Bx, fa, r->fused_nt, r->d_Bw16, r->d_Bx16});
  else
    with_disc(r->prob, EqLaunch<double>{a, jac, n_pts, st, r->d_Bw, r->d_Bx, fa, r->fused_nt, nullptr, nullptr});
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

// Device workspace of one fused Jacobian assembly: the block partials, their
// flag counts and the OR of the invalid flags (the point data go in EqArgs).
struct FusedWork {
  double* part;
  int* part_bad;
  int* flag_or;
  double* Jobj;   // objective when the caller passes none
};

static FusedWork rom_fused_work(ift_rom* r) { return {r->d_fpart, r->d_fbad, r->d_flag_or, r->d_J}; }

// Jacobian path through the fused assembly + Gram; rows: also leave the
// rows of J~ and F~ in the workspace (d_Jt, d_Ft).
static ift_status eq_jacobian_fused(ift_rom* r, const EqArgs& a, int n_pts, double* H, double* g, double* Jobj,
                                    int* n_bad, bool rows, hipStream_t stream, const FusedWork& w) {
  const bool pts2 = fused_pts2_used(r, n_pts, rows);
  const FusedLayout L = pts2 ? fused_layout_pts2(r, n_pts) : fused_layout(r, n_pts);
  FusedArgs fa;
  fa.E = L.E;
  fa.nblk = L.nblk;
  fa.part = w.part;
  fa.part_bad = w.part_bad;
  fa.rows = rows ? 1 : 0;
  fa.pts2 = pts2 ? 1 : 0;
  ift_status s = dispatch_eq(r, a, true, n_pts, stream, &fa);
  if (s != IFT_OK) return s;
  const int D1 = r->D + 1;
  const int nbe = (D1 * (D1 + 1) / 2 + GF_ENT - 1) / GF_ENT;
  ProfScope ps(IFT_PROF_GRAM, stream, true);
  hipLaunchKernelGGL(k_fused_final, dim3(nbe + 1, n_pts), dim3(256), 0, stream, (const double*)w.part,
                     (const int*)w.part_bad, L.nblk, r->fused_nt, r->D, H, g, Jobj ? Jobj : w.Jobj, n_bad, w.flag_or);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

static ift_status eq_jacobian_fused(ift_rom* r, const EqArgs& a, int n_pts, double* H, double* g, double* Jobj,
                                    int* n_bad, bool rows, hipStream_t stream) {
  return eq_jacobian_fused(r, a, n_pts, H, g, Jobj, n_bad, rows, stream, rom_fused_work(r));
}

extern "C" ift_status eq_assemble_residual(ift_rom* r, const double* mu, const double* w, const double* tau,
                                           double* Jobj, double* Ft, double* PhiT_r, int* n_bad,
                                           hipStream_t stream) {
  if (!r || !w || (r->m > 0 && !tau) || !finite_mu(r->prob, mu)) return IFT_EINVAL;
  if (!lazy_points(r)) return IFT_ENOMEM;
  EqArgs a = eq_args(r, mu, w, tau);
  a.Ft = Ft;
  a.PTR = PhiT_r ? r->d_PTR : nullptr;
  ift_status s = dispatch_eq(r, a, false, 1, stream);
  if (s != IFT_OK) return s;
  hipLaunchKernelGGL(k_obj_final, dim3(1), dim3(256), 0, stream, (const double*)r->d_Jpart, (const int*)r->d_flags,
                     r->n_s, Jobj, n_bad, r->d_flag_or);
  if (PhiT_r)
    hipLaunchKernelGGL(k_sum_rows, dim3((r->n + 63) / 64), dim3(64), 0, stream, (const double*)r->d_PTR, r->n_s,
                       r->n, PhiT_r);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

static ift_status gram(ift_rom* r, int n_pts, double* H, double* g, double* Jobj, int* n_bad, hipStream_t stream) {
  const int D = r->D;
  GramArgs ga;
  ga.Jt = r->d_Jt;
  ga.Ft = r->d_Ft;
  ga.Jpart = r->d_Jpart;
  ga.flags = r->d_flags;
  ga.nrows = r->nrows;
  ga.n_s = r->n_s;
  ga.D = D;
  ga.nblk = r->n_gram_blk;
  ga.rows_per = r->gram_rows_per;
  ga.part = r->d_gram_part;
  ga.H = H;
  ga.g = g;
  ga.Jobj = Jobj ? Jobj : r->d_J;
  ga.n_bad = n_bad;
  ga.flag_or = r->d_flag_or;
  ProfScope ps(IFT_PROF_GRAM, stream);
  hipLaunchKernelGGL(k_gram_part, dim3(ga.nblk, n_pts), dim3(256), gram_shm_bytes(D, ga.rows_per), stream, ga);
  const int nbe = (D * D + D + GF_ENT - 1) / GF_ENT;
  hipLaunchKernelGGL(k_gram_final, dim3(nbe + 1, n_pts), dim3(256), 0, stream, ga);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

extern "C" ift_status eq_assemble_jacobian(ift_rom* r, const double* mu, const double* w, const double* tau,
                                           double* Jobj, double* g, double* H, double* Jt, int* n_bad,
                                           hipStream_t stream) {
  if (!r || !w || (r->m > 0 && !tau) || !finite_mu(r->prob, mu)) return IFT_EINVAL;
  if (!lazy_points(r)) return IFT_ENOMEM;
  EqArgs a = eq_args(r, mu, w, tau);
  ift_status s;
  if (r->fused_nt > 0) {
    s = eq_jacobian_fused(r, a, 1, H ? H : r->d_H, g ? g : r->d_g, Jobj, n_bad, Jt != nullptr, stream);
  } else {
    s = dispatch_eq(r, a, true, 1, stream);
    if (s == IFT_OK) s = gram(r, 1, H ? H : r->d_H, g ? g : r->d_g, Jobj, n_bad, stream);
  }
  if (s != IFT_OK) return s;
  if (Jt) HIP_TRY(hipMemcpyAsync(Jt, r->d_Jt, (size_t)r->nrows * r->D * sizeof(double), hipMemcpyDeviceToDevice, stream));
  return IFT_OK;
}

// ------------------------------------------- assembly without allocation
// eq_assemble_jacobian_noalloc keeps its workspace (point data, block
// partials, flag counts) in one static device array of fixed size instead of
// the ROM's lazily allocated buffers.  Each device holds its own copy of the
// array; its address on a device is taken once, with that device current, on
// the first call there, and only that address is ever handed to kernels.
// Every call on a device shares that device's array: calls that overlap on
// one device race.  Nothing in it needs clearing: every byte a call reads was
// written earlier in the same call.
static __device__ __align__(256) unsigned char scratch[IFT_NOALLOC_SCRATCH_BYTES];

static constexpr int SCRATCH_MAX_DEV = 64;
static void* g_scratch_ptr[SCRATCH_MAX_DEV] = {};
static std::mutex g_scratch_mu;

static ift_status scratch_on_device(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEV) return IFT_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IFT_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IFT_OK;
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

extern "C" size_t eq_noalloc_scratch_bytes(const ift_rom* r) {
  if (!r || r->fused_nt < 1) return 0;
  const FusedLayout L = fused_layout(r, 1);
  const size_t nh = (size_t)r->fused_nt * (r->fused_nt + 1) / 2;
  return align256((size_t)r->n_s * pts_bytes(r->prob)) + align256((size_t)L.nblk * nh * 256 * sizeof(double)) +
         align256((size_t)L.nblk * 2 * sizeof(int)) + align256(sizeof(int)) + align256(sizeof(double));
}

extern "C" ift_status eq_assemble_jacobian_noalloc(ift_rom* r, const double* mu, const double* w, const double* tau,
                                                   double* Jobj, double* g, double* H, int* n_bad,
                                                   hipStream_t stream) {
  if (!r || !w || (r->m > 0 && !tau) || !Jobj || !g || !H || !finite_mu(r->prob, mu) || r->fused_nt < 1)
    return IFT_EINVAL;
  if (eq_noalloc_scratch_bytes(r) > (size_t)IFT_NOALLOC_SCRATCH_BYTES) return IFT_ESCRATCH;
  void* base = nullptr;
  ift_status s = scratch_on_device(&base);
  if (s != IFT_OK) return s;
  const FusedLayout L = fused_layout(r, 1);
  const size_t nh = (size_t)r->fused_nt * (r->fused_nt + 1) / 2;
  unsigned char* p = static_cast<unsigned char*>(base);
  EqArgs a = eq_args(r, mu, w, tau);
  a.pts = p;
  p += align256((size_t)r->n_s * pts_bytes(r->prob));
  FusedWork fw;
  fw.part = reinterpret_cast<double*>(p);
  p += align256((size_t)L.nblk * nh * 256 * sizeof(double));
  fw.part_bad = reinterpret_cast<int*>(p);
  p += align256((size_t)L.nblk * 2 * sizeof(int));
  fw.flag_or = reinterpret_cast<int*>(p);
  p += align256(sizeof(int));
  fw.Jobj = reinterpret_cast<double*>(p);
  // the Jacobian-path kernels read only the point data, the gathered
  // operands and the point bases; the row outputs stay off
  a.Jt = nullptr;
  a.Ft = nullptr;
  a.Jpart = nullptr;
  a.flags = nullptr;
  return eq_jacobian_fused(r, a, 1, H, g, Jobj, n_bad, false, stream, fw);
}

extern "C" ift_status eq_element_contributions(ift_rom* r, const double* mu, const double* w, const double* tau,
                                               double* C, hipStream_t stream) {
  if (!r || !w || (r->m > 0 && !tau) || !C || !finite_mu(r->prob, mu)) return IFT_EINVAL;
  if (!lazy_points(r)) return IFT_ENOMEM;
  EqArgs a = eq_args(r, mu, w, tau);
  ift_status s;
  if (r->fused_nt > 0) {
    s = eq_jacobian_fused(r, a, 1, r->d_H, r->d_g, r->d_J, r->d_nbad, true, stream);
  } else {
    s = dispatch_eq(r, a, true, 1, stream);
    if (s == IFT_OK) s = gram(r, 1, r->d_H, r->d_g, r->d_J, r->d_nbad, stream);
  }
  if (s != IFT_OK) return s;
  const long long cnt = (long long)r->n_s * r->D;
  hipLaunchKernelGGL(k_elem_contrib, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, (const double*)r->d_Jt,
                     (const double*)r->d_Ft, (const double*)r->d_rho, r->n_s, r->prob->nue, r->D, C);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

extern "C" ift_status eq_assemble_residual_batch(ift_rom* r, int n_pts, const double* mu, const double* w,
                                                 const double* tau, double* Jobj, int* n_bad, hipStream_t stream) {
  if (r && !lazy_points(r)) return IFT_ENOMEM;
  if (!r || n_pts < 1 || n_pts > r->max_pts || !mu || !w || (r->m > 0 && !tau) || !Jobj) return IFT_EINVAL;
  double mu0[2] = {1.0, 0.0};
  EqArgs a = eq_args(r, mu0, w, tau);
  a.mu = mu;
  a.Ft = nullptr;
  ift_status s = dispatch_eq(r, a, false, n_pts, stream);
  if (s != IFT_OK) return s;
  hipLaunchKernelGGL(k_obj_final, dim3(n_pts), dim3(256), 0, stream, (const double*)r->d_Jpart, (const int*)r->d_flags,
                     r->n_s, Jobj, n_bad, r->d_flag_or);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

extern "C" ift_status eq_assemble_jacobian_batch(ift_rom* r, int n_pts, const double* mu, const double* w,
                                                 const double* tau, double* Jobj, double* g, double* H, int* n_bad,
                                                 hipStream_t stream) {
  if (r && !lazy_points(r)) return IFT_ENOMEM;
  if (!r || n_pts < 1 || n_pts > r->max_pts || !mu || !w || (r->m > 0 && !tau) || !Jobj || !g || !H)
    return IFT_EINVAL;
  double mu0[2] = {1.0, 0.0};
  EqArgs a = eq_args(r, mu0, w, tau);
  a.mu = mu;
  a.pcs = r->d_pcs;   // filled by the point kernels' launch
  if (r->fused_nt > 0) return eq_jacobian_fused(r, a, n_pts, H, g, Jobj, n_bad, false, stream);
  ift_status s = dispatch_eq(r, a, true, n_pts, stream);
  if (s != IFT_OK) return s;
  return gram(r, n_pts, H, g, Jobj, n_bad, stream);
}

// LM step of eq. (levmarq-step) by TSQR of the point-0 rows in d_Jt / d_Ft:
// dz into d_dz and {failed, |S~|, |T~|, g . dz} into d_solve_out.  The
// triangle buffers are allocated by the first call.
static ift_status qr_step(ift_rom* r, double lambda, bool w_only, hipStream_t st) {
  const int ns = w_only ? r->n : r->D;
  const int C = ns + 1;
  const long long rows1 = r->nrows + (lambda > 0.0 && !w_only ? r->m : 0);
  const long long nb1 = (rows1 + QR_RB - 1) / QR_RB;
  if (!r->d_qr[0]) {
    // sized for the full step with mapping rows, the largest case
    const long long nbmax = (r->nrows + r->m + QR_RB - 1) / QR_RB;
    const size_t sz = (size_t)nbmax * (r->D + 1) * (r->D + 1);
    ift_status e;
    if ((e = dalloc(&r->d_qr[0], sz)) != IFT_OK || (e = dalloc(&r->d_qr[1], sz)) != IFT_OK) return e;
  }
  QrArgs q;
  q.Jt = r->d_Jt;
  q.Ft = r->d_Ft;
  q.src = nullptr;
  q.rows = (int)rows1;
  q.nrows = (int)r->nrows;
  q.D = r->D;
  q.n = r->n;
  q.ns = ns;
  q.C = C;
  q.sqlam = std::sqrt(lambda);
  q.g = r->d_g;
  q.dz = r->d_dz;
  q.out = r->d_solve_out;
  long long nb = nb1;
  for (int cur = 0;; cur ^= 1) {
    q.dst = r->d_qr[cur];
    hipLaunchKernelGGL(k_qr_rows, dim3((unsigned)nb), dim3(QR_RB), 0, st, q, nb == 1 ? 1 : 0);
    HIP_TRY(hipGetLastError());
    if (nb == 1) break;
    q.src = r->d_qr[cur];
    q.rows = (int)(nb * C);
    nb = (q.rows + QR_RB - 1) / QR_RB;
  }
  return IFT_OK;
}

extern "C" ift_status rom_gauss_newton_step(ift_rom* r, const double* mu, double* w, double* tau,
                                            const ift_gn_params* prm, ift_gn_info* info, hipStream_t stream) {
  if (!r || !w || (r->m > 0 && !tau) || !prm || !info || !finite_mu(r->prob, mu)) return IFT_EINVAL;
  if (!(prm->lambda >= 0.0) || !(prm->c1 > 0.0 && prm->c1 < 1.0) || prm->max_backtrack < 0 || !(prm->tol >= 0.0))
    return IFT_EINVAL;
  if (prm->use_qr && r->D + 1 > QR_MAXC) return IFT_EINVAL;
  std::memset(info, 0, sizeof(*info));
  if (!lazy_points(r)) return IFT_ENOMEM;
  const int n = r->n, m = r->m, D = r->D;
  ift_status s;
  if (prm->use_qr) {
    // the stacked rows of the point in the ROM's row workspace, then TSQR
    EqArgs a = eq_args(r, mu, w, tau);
    if (r->fused_nt > 0) {
      s = eq_jacobian_fused(r, a, 1, r->d_H, r->d_g, r->d_J, r->d_nbad, true, stream);
    } else {
      s = dispatch_eq(r, a, true, 1, stream);
      if (s == IFT_OK) s = gram(r, 1, r->d_H, r->d_g, r->d_J, r->d_nbad, stream);
    }
    if (s != IFT_OK) return s;
    if ((s = qr_step(r, prm->lambda, prm->w_only != 0, stream)) != IFT_OK) return s;
  } else {
    s = eq_assemble_jacobian(r, mu, w, tau, r->d_J, r->d_g, r->d_H, nullptr, r->d_nbad, stream);
    if (s != IFT_OK) return s;
    hipLaunchKernelGGL(k_lm_solve, dim3(1), dim3(64), 0, stream, (const double*)r->d_H, (const double*)r->d_g, D, n,
                       prm->w_only ? n : D, prm->lambda, r->d_dz, r->d_solve_out);
    HIP_TRY(hipGetLastError());
  }
  double so[4], J0;
  int fo;
  HIP_TRY(hipMemcpyAsync(so, r->d_solve_out, 4 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&J0, r->d_J, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&fo, r->d_flag_or, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  info->J_old = J0;
  info->J_new = J0;
  info->norm_S = so[1];
  info->norm_T = so[2];
  if (!std::isfinite(J0)) {
    info->status = (fo & BAD_GEOM) ? IFT_EBADMESH : IFT_ENONPHYS;
    return (ift_status)info->status;
  }
  if (so[1] <= prm->tol && (prm->w_only || so[2] <= prm->tol)) {
    info->converged = 1;
    info->status = IFT_OK;
    return IFT_OK;
  }
  if (so[0] != 0.0) {
    info->status = IFT_ESINGULAR;
    return IFT_ESINGULAR;
  }
  // the Armijo reference J~(z_n) from the kernels that evaluate the trials
  // (the Gram corner sums the same squares in another order, and near a
  // minimum that rounding difference is as large as the decrease tested)
  s = eq_assemble_residual(r, mu, w, tau, r->d_Jtrial, nullptr, nullptr, nullptr, stream);
  if (s != IFT_OK) return s;
  HIP_TRY(hipMemcpyAsync(&J0, r->d_Jtrial, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const double slope = so[3];
  double alpha = 1.0;
  for (int bt = 0; bt <= prm->max_backtrack; ++bt) {
    hipLaunchKernelGGL(k_axpy2, dim3((D + 63) / 64), dim3(64), 0, stream, (const double*)w, (const double*)tau,
                       (const double*)r->d_dz, alpha, n, m, r->d_wt, r->d_tt);
    HIP_TRY(hipGetLastError());
    s = eq_assemble_residual(r, mu, r->d_wt, r->d_tt, r->d_Jtrial, nullptr, nullptr, nullptr, stream);
    if (s != IFT_OK) return s;
    double Jt;
    HIP_TRY(hipMemcpyAsync(&Jt, r->d_Jtrial, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (Jt <= J0 + prm->c1 * alpha * slope) {
      HIP_TRY(hipMemcpyAsync(w, r->d_wt, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
      if (m > 0) HIP_TRY(hipMemcpyAsync(tau, r->d_tt, m * sizeof(double), hipMemcpyDeviceToDevice, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      info->J_new = Jt;
      info->alpha = alpha;
      info->n_backtrack = bt;
      info->status = IFT_OK;
      return IFT_OK;
    }
    alpha *= 0.5;
  }
  info->n_backtrack = prm->max_backtrack + 1;
  info->status = IFT_ELINESEARCH;
  return IFT_ELINESEARCH;
}

// ============================================================ batched solves
struct ift_batch {
  ift_problem* prob = nullptr;
  ift_precision precision = IFT_FP64;
  int n_inst = 0;
  std::vector<ift_rom*> roms;
  std::vector<int> zoff, hoff, nsoff;   // packed offsets [n_inst + 1]
  std::vector<BatchInst> h_inst;
  long long sum_ns = 0;
  int E = 8;                 // sampled elements per wave of the fused assembly
  int nbe_max = 0;           // final-reduction workgroups of the widest instance
  bool has_nt[FUSED_MAXNT + 1] = {};
  BatchInst* d_inst = nullptr;
  BatchState* d_state = nullptr;
  BatchParams* d_params = nullptr;
  int* d_off = nullptr;
  int* d_cnt = nullptr;
  double* d_z = nullptr;
  double* d_zt = nullptr;
  double* d_zp = nullptr;
  double* d_dz = nullptr;
  double* d_H = nullptr;
  double* d_g = nullptr;
  double* d_mu = nullptr;
  void* d_pts = nullptr;
  double* d_Jpart = nullptr;
  int* d_flags = nullptr;
  double* d_part = nullptr;
  int* d_pbad = nullptr;
  size_t part_cap = 0, pbad_cap = 0;   // capacities (doubles, ints) for the smallest E
  int* d_remaining = nullptr;
  int* h_remaining = nullptr;          // pinned
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;       // BATCH_ROUNDS rounds
};

static constexpr int BATCH_E_CAND[] = {4, 8, 16, 32};
static constexpr int BATCH_T = 2;           // line-search trials per round
static constexpr float BATCH_TUNE_TAIL = 4.f;    // weight of the one-in-eight timing in the autotuner
static constexpr float BATCH_TUNE_MARGIN = 0.97f; // a larger work split must be 3 % faster
static constexpr int BATCH_ROUNDS = 4;      // rounds per graph replay (one completion check each)
static constexpr double BATCH_TOL_MIX = 1e-5;   // gradient norms that end the mixed-precision rounds
static constexpr int BATCH_BT_MIX = 3;          // mixed-precision halvings before the switch to FP64
static constexpr int BATCH_GRID_PTS = 2048, BATCH_GRID_RES = 1024, BATCH_GRID_FUSED = 1024;
// the two-item points kernel: one 4-wave block per resident slot (two per CU
// at two waves per SIMD; 512 blocks ran 1 % faster than 1024 or 2048)
static constexpr int BATCH_GRID_PTS2 = 512;

static int batch_nblk(int n_s, int E) { return (n_s + 4 * E - 1) / (4 * E); }

// Per-instance descriptors for the current E (fused partial slices depend on it).
static ift_status batch_upload(ift_batch* b) {
  const ift_problem* pr = b->prob;
  const size_t pb = pts_bytes(pr);
  size_t po = 0, bo = 0;
  for (int i = 0; i < b->n_inst; ++i) {
    ift_rom* r = b->roms[i];
    const double mu0[2] = {1.0, 0.0};
    BatchInst& bi = b->h_inst[i];
    EqArgs a = eq_args(r, mu0, nullptr, nullptr);
    a.w = b->d_z + b->zoff[i];
    a.tau = b->d_z + b->zoff[i] + r->n;
    a.mu = b->d_mu + 2 * i;
    a.Jt = nullptr;
    a.Ft = nullptr;
    a.PTR = nullptr;
    a.Jpart = b->d_Jpart + b->nsoff[i];
    a.flags = b->d_flags + b->nsoff[i];
    a.pts = static_cast<char*>(b->d_pts) + (size_t)b->nsoff[i] * pb;
    bi.a = a;
    bi.Bw = r->d_Bw;
    bi.Bx = r->d_Bx;
    bi.Bw16 = r->d_Bw16;
    bi.Bx16 = r->d_Bx16;
    bi.phisum = r->d_phisum;
    bi.z = b->d_z + b->zoff[i];
    bi.zt = b->d_zt + b->zoff[i];
    bi.dz = b->d_dz + b->zoff[i];
    bi.zp = b->d_zp + b->zoff[i];
    bi.H = b->d_H + b->hoff[i];
    bi.g = b->d_g + b->zoff[i];
    bi.nt = r->fused_nt;
    bi.nblk = batch_nblk(r->n_s, b->E);
    bi.part = b->d_part + po;
    bi.part_bad = b->d_pbad + bo;
    po += (size_t)bi.nblk * (bi.nt * (bi.nt + 1) / 2) * 256;
    bo += (size_t)bi.nblk * 2;
  }
  if (po > b->part_cap || bo > b->pbad_cap) return IFT_EINVAL;
  HIP_TRY(hipMemcpy(b->d_inst, b->h_inst.data(), b->n_inst * sizeof(BatchInst), hipMemcpyHostToDevice));
  return IFT_OK;
}

extern "C" void ift_batch_destroy(ift_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  dfree(b->d_remaining);
  if (b->h_remaining) (void)hipHostFree(b->h_remaining);
  dfree(b->d_inst);
  dfree(b->d_state);
  dfree(b->d_params);
  dfree(b->d_off);
  dfree(b->d_cnt);
  dfree(b->d_z);
  dfree(b->d_zt);
  dfree(b->d_dz);
  dfree(b->d_zp);
  dfree(b->d_H);
  dfree(b->d_g);
  dfree(b->d_mu);
  if (b->d_pts) (void)hipFree(b->d_pts);
  dfree(b->d_Jpart);
  dfree(b->d_flags);
  dfree(b->d_part);
  dfree(b->d_pbad);
  delete b;
}

extern "C" ift_status ift_batch_create(int n_inst, ift_rom* const* roms, ift_batch** out) {
  if (!out || !roms || n_inst < 1) return IFT_EINVAL;
  *out = nullptr;
  for (int i = 0; i < n_inst; ++i) {
    if (!roms[i] || roms[i]->prob != roms[0]->prob || roms[i]->precision != roms[0]->precision) return IFT_EINVAL;
    if (roms[i]->fused_nt < 1) return IFT_EINVAL;
  }
  ift_batch* b = new ift_batch;
  b->prob = roms[0]->prob;
  b->precision = roms[0]->precision;
  b->n_inst = n_inst;
  b->roms.assign(roms, roms + n_inst);
  b->zoff.assign(n_inst + 1, 0);
  b->hoff.assign(n_inst + 1, 0);
  b->nsoff.assign(n_inst + 1, 0);
  size_t part_max = 0, pbad_max = 0;
  for (int i = 0; i < n_inst; ++i) {
    const ift_rom* r = roms[i];
    b->zoff[i + 1] = b->zoff[i] + r->D;
    b->hoff[i + 1] = b->hoff[i] + r->D * r->D;
    b->nsoff[i + 1] = b->nsoff[i] + r->n_s;
    const int D1 = r->D + 1;
    b->nbe_max = std::max(b->nbe_max, (D1 * (D1 + 1) / 2 + GF_ENT - 1) / GF_ENT);
    b->has_nt[r->fused_nt] = true;
    const int nb = batch_nblk(r->n_s, BATCH_E_CAND[0]);
    part_max += (size_t)nb * (r->fused_nt * (r->fused_nt + 1) / 2) * 256;
    pbad_max += (size_t)nb * 2;
  }
  b->sum_ns = b->nsoff[n_inst];
  b->h_inst.resize(n_inst);
  const size_t Z = b->zoff[n_inst], HH = b->hoff[n_inst], NS = b->sum_ns;
  ift_status st;
  if ((st = dalloc(&b->d_inst, n_inst)) != IFT_OK || (st = dalloc(&b->d_state, n_inst)) != IFT_OK ||
      (st = dalloc(&b->d_params, 1)) != IFT_OK || (st = dalloc(&b->d_off, 4 * (size_t)(n_inst + 1))) != IFT_OK ||
      (st = dalloc(&b->d_cnt, 4)) != IFT_OK || (st = dalloc(&b->d_z, Z)) != IFT_OK ||
      (st = dalloc(&b->d_zt, Z)) != IFT_OK || (st = dalloc(&b->d_dz, Z)) != IFT_OK ||
      (st = dalloc(&b->d_zp, Z)) != IFT_OK ||
      (st = dalloc(&b->d_H, HH)) != IFT_OK || (st = dalloc(&b->d_g, Z)) != IFT_OK ||
      (st = dalloc(&b->d_mu, 2 * (size_t)n_inst)) != IFT_OK || (st = dalloc(&b->d_Jpart, NS)) != IFT_OK ||
      (st = dalloc(&b->d_flags, NS)) != IFT_OK || (st = dalloc(&b->d_part, part_max)) != IFT_OK ||
      (st = dalloc(&b->d_pbad, pbad_max)) != IFT_OK) {
    ift_batch_destroy(b);
    return st;
  }
  b->part_cap = part_max;
  b->pbad_cap = pbad_max;
  if (hipMalloc(&b->d_pts, NS * pts_bytes(b->prob)) != hipSuccess) {
    ift_batch_destroy(b);
    return IFT_ENOMEM;
  }
  if (dalloc(&b->d_remaining, 1) != IFT_OK ||
      hipHostMalloc((void**)&b->h_remaining, sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      (st = batch_upload(b)) != IFT_OK) {
    ift_batch_destroy(b);
    return st == IFT_OK ? IFT_EDEVICE : st;
  }
  *out = b;
  return IFT_OK;
}

extern "C" ift_status ift_batch_layout(const ift_batch* b, int* zoff, int* hoff) {
  if (!b) return IFT_EINVAL;
  if (zoff) std::memcpy(zoff, b->zoff.data(), (b->n_inst + 1) * sizeof(int));
  if (hoff) std::memcpy(hoff, b->hoff.data(), (b->n_inst + 1) * sizeof(int));
  return IFT_OK;
}

// Kernels of one phase for the batch's discretisation.  A mixed-precision
// batch runs each phase twice: for its instances still in mixed rounds
// (FP32 points, BF16 projection, FP32 element residuals) and for those in
// FP64 rounds.
struct BatchLaunch {
  ift_batch* b;
  hipStream_t st;
  int phase;   // 0: Jacobian assembly of the JAC instances, 1: trial residuals of the SEARCH instances
  bool prof = false;   // time the points, projection and final kernels separately (never under capture)
  template <class D, class R, int NT>
  void fused(const BatchLists& L, bool mixed) {
    if (!b->has_nt[NT]) return;
    if constexpr (std::is_same<R, float>::value) {
      if (mixed) {
        hipLaunchKernelGGL((k_fused_batch_mixed<D, NT>), dim3(BATCH_GRID_FUSED), dim3(NTHR), 0, st,
                           (const BatchInst*)b->d_inst, L, b->n_inst, b->E);
        return;
      }
    }
    hipLaunchKernelGGL((k_fused_batch<D, R, NT>), dim3(BATCH_GRID_FUSED), dim3(NTHR), 0, st,
                       (const BatchInst*)b->d_inst, L, b->n_inst, b->E);
  }
  // the instances of one precision phase (want_prec: 1 mixed, 0 FP64, -1 all)
  template <class D, class R>
  void group(int want_prec, bool mixed) {
    BatchLists L{b->d_off, b->d_cnt};
    const int ni = b->n_inst;
    if (phase == 0) {
      hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(BC_THR), 0, st, (const BatchInst*)b->d_inst,
                         (const BatchState*)b->d_state, L, ni, (int)BS_JAC, want_prec, 1);
      {
        ProfScope ps(IFT_PROF_POINTS, st, false, prof);
        if constexpr (pair_layout<D>())
          hipLaunchKernelGGL((k_points_batch2<D, R>), dim3(BATCH_GRID_PTS2), dim3(2 * NTHR_PTS), 0, st,
                             (const BatchInst*)b->d_inst, L, ni);
        else
          hipLaunchKernelGGL((k_points_batch<D, R>), dim3(BATCH_GRID_PTS), dim3(NTHR_PTS), 0, st,
                             (const BatchInst*)b->d_inst, L, ni);
      }
      ProfScope ps(IFT_PROF_EQ_JAC, st, true, prof);
      fused<D, R, 1>(L, mixed);
      fused<D, R, 2>(L, mixed);
      fused<D, R, 3>(L, mixed);
    } else {
      hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(BC_THR), 0, st, (const BatchInst*)b->d_inst,
                         (const BatchState*)b->d_state, L, ni, (int)BS_SEARCH, want_prec, 0);
      hipLaunchKernelGGL((k_res_batch<D, R>), dim3(BATCH_GRID_RES), dim3(RV_THR), 0, st, (const BatchInst*)b->d_inst,
                         L, ni);
    }
  }
  template <class D>
  void run() {
    const int ni = b->n_inst;
    if (phase == 1)
      hipLaunchKernelGGL(k_trial_batch, dim3(ni), dim3(64), 0, st, (const BatchInst*)b->d_inst,
                         (const BatchState*)b->d_state);
    if (b->precision == IFT_MIXED_BF16) {
      group<D, float>(1, true);
      group<D, double>(0, false);
    } else if (b->precision == IFT_FP32_ELEM) {
      group<D, float>(-1, false);
    } else {
      group<D, double>(-1, false);
    }
    if (phase == 0) {
      ProfScope ps(IFT_PROF_GRAM, st, true, prof);
      hipLaunchKernelGGL(k_final_batch, dim3(b->nbe_max + 1, ni), dim3(256), 0, st, (const BatchInst*)b->d_inst,
                         b->d_state);
    } else
      hipLaunchKernelGGL(k_ls_batch, dim3(ni), dim3(256), 0, st, (const BatchInst*)b->d_inst, b->d_state,
                         (const BatchParams*)b->d_params);
  }
};

static void batch_phase(ift_batch* b, int phase, hipStream_t st, bool prof = false) {
  with_disc(b->prob, BatchLaunch{b, st, phase, prof});
}

// `rounds` rounds of the solve: the Jacobian phase of the JAC instances,
// their LM step (or stop), then BATCH_T line-search trials of the SEARCH
// instances.  An instance still backtracking continues in the next round.
static void batch_rounds(ift_batch* b, int rounds, hipStream_t st) {
  for (int r = 0; r < rounds; ++r) {
    batch_phase(b, 0, st);
    hipLaunchKernelGGL(k_lm_batch, dim3(b->n_inst), dim3(64), 0, st, (const BatchInst*)b->d_inst, b->d_state,
                       (const BatchParams*)b->d_params);
    for (int t = 0; t < BATCH_T; ++t) batch_phase(b, 1, st);
  }
}

__global__ void k_batch_info(const BatchState* S, int n_inst, ift_gn_info* info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  const BatchState st = S[i];
  ift_gn_info o;
  o.J_old = st.J0;
  o.J_new = st.J;
  o.alpha = st.alpha_acc;
  o.norm_S = st.nS;
  o.norm_T = st.nT;
  o.n_backtrack = st.n_bt_total;
  o.converged = st.converged;
  o.status = st.state == BS_DONE ? st.status : IFT_ENOTCONV;   // (round cap reached; not expected)
  o.iterations = st.it;
  o.fallback = st.fallback;
  o.mixed_iterations = st.it_mixed;
  o.presolve_iterations = st.it_w;
  info[i] = o;
}

static ift_status batch_inputs(ift_batch* b, const double* mu, const double* z, hipStream_t stream) {
  HIP_TRY(hipMemcpyAsync(b->d_mu, mu, 2 * (size_t)b->n_inst * sizeof(double), hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpyAsync(b->d_z, z, (size_t)b->zoff[b->n_inst] * sizeof(double), hipMemcpyDeviceToDevice, stream));
  return IFT_OK;
}

extern "C" ift_status eq_assemble_jacobian_batched(ift_batch* b, const double* mu, const double* z, double* Jobj,
                                                   double* g, double* H, int* n_bad, hipStream_t stream) {
  if (!b || !mu || !z || !Jobj || !g || !H) return IFT_EINVAL;
  ift_status s = batch_inputs(b, mu, z, stream);
  if (s != IFT_OK) return s;
  hipLaunchKernelGGL(k_batch_init, dim3((b->n_inst + 255) / 256), dim3(256), 0, stream, b->d_state, b->n_inst,
                     b->precision == IFT_MIXED_BF16 ? 1 : 0, 0, 0.0);
  batch_phase(b, 0, stream, true);
  HIP_TRY(hipGetLastError());
  const size_t Z = b->zoff[b->n_inst], HH = b->hoff[b->n_inst];
  HIP_TRY(hipMemcpyAsync(g, b->d_g, Z * sizeof(double), hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpyAsync(H, b->d_H, HH * sizeof(double), hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpy2DAsync(Jobj, sizeof(double), &b->d_state->J, sizeof(BatchState), sizeof(double), b->n_inst,
                           hipMemcpyDeviceToDevice, stream));
  if (n_bad)
    HIP_TRY(hipMemcpy2DAsync(n_bad, sizeof(int), &b->d_state->n_bad, sizeof(BatchState), sizeof(int), b->n_inst,
                             hipMemcpyDeviceToDevice, stream));
  return IFT_OK;
}

extern "C" ift_status ift_batch_autotune(ift_batch* b, const double* mu, const double* z, int* chosen,
                                         hipStream_t stream) {
  if (!b || !mu || !z) return IFT_EINVAL;
  ift_status s = batch_inputs(b, mu, z, stream);
  if (s != IFT_OK) return s;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 0.f;
  int bestE = b->E;
  for (int E : BATCH_E_CAND) {
    b->E = E;
    if ((s = batch_upload(b)) != IFT_OK) break;
    // the Jacobian phase with every instance active and with one in eight
    // (the late rounds of a solve, where few instances remain), weighted
    // by the share of a solve's rounds each stands for; the fastest of four
    // timed runs of each
    float tot = 0.f;
    for (int sub = 0; sub < 2; ++sub) {
      float fastest = 0.f;
      for (int rep = 0; rep < 5; ++rep) {
        hipLaunchKernelGGL(k_batch_init, dim3((b->n_inst + 255) / 256), dim3(256), 0, stream, b->d_state, b->n_inst,
                           b->precision == IFT_MIXED_BF16 ? 1 : 0, 0, 0.0);
        if (sub)
          hipLaunchKernelGGL(k_batch_keep_every, dim3((b->n_inst + 255) / 256), dim3(256), 0, stream, b->d_state,
                             b->n_inst, 8);
        HIP_TRY(hipEventRecord(e0, stream));
        batch_phase(b, 0, stream);
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0 && (fastest == 0.f || ms < fastest)) fastest = ms;   // the first run warms up
      }
      tot += (sub ? BATCH_TUNE_TAIL : 1.f) * fastest;
    }
    // candidates ascend in E: a larger split must be clearly faster (the
    // late rounds with very few instances, not timed here, favour small E)
    if (best == 0.f || tot < BATCH_TUNE_MARGIN * best) {
      best = tot;
      bestE = E;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->E = bestE;
  if (s == IFT_OK) s = batch_upload(b);
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (chosen) *chosen = b->E;
  return s;
}

// FP64 residual phase over the SEARCH instances (objective parts at zt).
struct BatchResidual64 {
  ift_batch* b;
  hipStream_t st;
  template <class D>
  void run() {
    BatchLists L{b->d_off, b->d_cnt};
    hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(BC_THR), 0, st, (const BatchInst*)b->d_inst,
                       (const BatchState*)b->d_state, L, b->n_inst, (int)BS_SEARCH, -1, 0);
    hipLaunchKernelGGL((k_res_batch<D, double>), dim3(BATCH_GRID_RES), dim3(RV_THR), 0, st,
                       (const BatchInst*)b->d_inst, L, b->n_inst);
  }
};

// Warm start or plain start per instance: J~ (FP64) at both, keep the smaller.
static void batch_select_start(ift_batch* b, hipStream_t st) {
  const ift_problem* pr = b->prob;
  const int ni = b->n_inst;
  hipLaunchKernelGGL(k_plain_batch, dim3(ni), dim3(64), 0, st, (const BatchInst*)b->d_inst,
                     pr->pde == IFT_BURGERS2D ? (int)PDE_BURGERS : (int)PDE_EULER, pr->nc, (double* const*)nullptr, 2);
  for (int which = 0; which < 2; ++which) {
    hipLaunchKernelGGL(k_start_stage, dim3(ni), dim3(64), 0, st, (const BatchInst*)b->d_inst, b->d_state, which);
    with_disc(pr, BatchResidual64{b, st});
    hipLaunchKernelGGL(k_start_obj, dim3(ni), dim3(256), 0, st, (const BatchInst*)b->d_inst, b->d_state, which);
  }
  hipLaunchKernelGGL(k_start_select, dim3(ni), dim3(64), 0, st, (const BatchInst*)b->d_inst, b->d_state);
}

extern "C" ift_status rom_gauss_newton_solve_batched(ift_batch* b, const double* mu, double* z,
                                                     const ift_gn_params* prm, int max_it, ift_gn_info* info,
                                                     int flags, hipStream_t stream) {
  if (!b || !mu || !z || !prm || !info || max_it < 0 || prm->use_qr || prm->w_only) return IFT_EINVAL;
  if (!(prm->lambda >= 0.0) || !(prm->c1 > 0.0 && prm->c1 < 1.0) || prm->max_backtrack < 0 || !(prm->tol >= 0.0))
    return IFT_EINVAL;
  BatchParams bp{prm->lambda, prm->c1, prm->tol, prm->tol_mix > 0.0 ? std::max(prm->tol, prm->tol_mix)
                                                                     : std::max(prm->tol, BATCH_TOL_MIX),
                 prm->max_backtrack, max_it,
                 std::min(prm->max_backtrack, prm->max_backtrack_mixed > 0 ? prm->max_backtrack_mixed : BATCH_BT_MIX),
                 (flags & 8) ? 1 : 0};
  HIP_TRY(hipMemcpyAsync(b->d_params, &bp, sizeof(bp), hipMemcpyHostToDevice, stream));
  ift_status s = batch_inputs(b, mu, z, stream);
  if (s != IFT_OK) return s;
  const bool graph = !(flags & 1);
  if (graph && !b->exec) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    batch_rounds(b, BATCH_ROUNDS, b->cap_stream);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
    if (le != hipSuccess || ce != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return IFT_EDEVICE;
    }
    const hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      b->exec = nullptr;
      return IFT_EDEVICE;
    }
  }
  hipLaunchKernelGGL(k_batch_init, dim3((b->n_inst + 255) / 256), dim3(256), 0, stream, b->d_state, b->n_inst,
                     b->precision == IFT_MIXED_BF16 ? 1 : 0, (flags & 4) ? 1 : 0, prm->lambda);
  if (flags & 2) batch_select_start(b, stream);
  // every instance finishes within (max_it + 1) Jacobian rounds, each
  // followed by at most ceil((max_backtrack + 2) / T) rounds of trials (the
  // halvings and the re-evaluation of J~ at the iterate; a few more for the
  // rounds that take no step: the end of the w-only initialisation, the
  // switch to FP64, a restart)
  const long long cap = (long long)(max_it + 4) * (2 + (prm->max_backtrack + 2 + BATCH_T - 1) / BATCH_T);
  for (long long done = 0; done < cap; done += BATCH_ROUNDS) {
    if (graph) HIP_TRY(hipGraphLaunch(b->exec, stream));
    else batch_rounds(b, BATCH_ROUNDS, stream);
    hipLaunchKernelGGL(k_batch_remaining, dim3(1), dim3(256), 0, stream, (const BatchState*)b->d_state, b->n_inst,
                       b->d_remaining);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(b->h_remaining, b->d_remaining, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (*b->h_remaining == 0) break;
  }
  HIP_TRY(hipMemcpyAsync(z, b->d_z, (size_t)b->zoff[b->n_inst] * sizeof(double), hipMemcpyDeviceToDevice, stream));
  hipLaunchKernelGGL(k_batch_info, dim3((b->n_inst + 255) / 256), dim3(256), 0, stream, (const BatchState*)b->d_state,
                     b->n_inst, info);
  HIP_TRY(hipGetLastError());
  return IFT_OK;
}

// ------------------------------------------------------------ plain start
// w0 = Phi^T U_fs(mu) with U_fs the uniform free stream (Euler) or inflow
// value (Burgers) on every node, tau0 = 0.
__global__ void k_plain_start(const double* phisum, int nc, int n, int m, PhysConst pc, int pde, double bc_scale,
                              const double* mu, double* w, double* tau) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const PhysConst q = mu ? phys_from_mu(pc, pde, bc_scale, mu) : pc;
  if (j < n) {
    double a = 0.0;
    for (int c = 0; c < nc; ++c) a += q.uinf[c] * phisum[c * n + j];
    w[j] = a;
  } else if (j < n + m) {
    tau[j - n] = 0.0;
  }
}

extern "C" ift_status rom_plain_start(ift_rom* r, const double* mu, double* w, double* tau, hipStream_t stream) {
  if (!r || !w || (r->m > 0 && !tau) || !finite_mu(r->prob, mu)) return IFT_EINVAL;
  const ift_problem* pr = r->prob;
  hipLaunchKernelGGL(k_plain_start, dim3((r->D + 63) / 64), dim3(64), 0, stream, (const double*)r->d_phisum, pr->nc,
                     r->n, r->m, phys_const(pr, mu), pr->pde == IFT_BURGERS2D ? (int)PDE_BURGERS : (int)PDE_EULER,
                     pr->bc_mu_scale, (const double*)nullptr, w, tau);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}

extern "C" ift_status rom_plain_start_batched(ift_batch* b, const double* mu, double* z, hipStream_t stream) {
  if (!b || !mu || !z) return IFT_EINVAL;
  ift_status s = batch_inputs(b, mu, z, stream);   // mu into the batch; z is overwritten below
  if (s != IFT_OK) return s;
  const ift_problem* pr = b->prob;
  hipLaunchKernelGGL(k_plain_batch, dim3(b->n_inst), dim3(64), 0, stream, (const BatchInst*)b->d_inst,
                     pr->pde == IFT_BURGERS2D ? (int)PDE_BURGERS : (int)PDE_EULER, pr->nc, (double* const*)nullptr, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(z, b->d_z, (size_t)b->zoff[b->n_inst] * sizeof(double), hipMemcpyDeviceToDevice, stream));
  return IFT_OK;
}

// ============================================================ warm-start network
struct ift_mlp {
  int n_in = 0, hidden = 0, n_out = 0;
  int n_par = 0;
  float* d_par = nullptr;     // flat parameters
  float* d_grad = nullptr;
  float* d_m = nullptr;       // Adam moments
  float* d_v = nullptr;
  long long adam_t = 0;
  double* d_norm = nullptr;   // x_mean[n_in], x_scale[n_in], y_mean[n_out], y_scale[n_out]
  // activations for up to cap samples
  int cap = 0;
  float *d_X = nullptr, *d_T = nullptr, *d_A1 = nullptr, *d_H1 = nullptr, *d_A2 = nullptr, *d_H2 = nullptr,
        *d_Y = nullptr, *d_dY = nullptr, *d_d1 = nullptr, *d_d2 = nullptr;
  double* d_lpart = nullptr;
  double* d_loss = nullptr;
  float* d_wpart = nullptr;   // [MLP_WCHUNKS][out][in + 1] weight-gradient partials
};

static constexpr int MLP_LOSS_BLOCKS = 64;

static int mlp_offsets(const ift_mlp* p, int layer, int* in, int* out) {
  const int dims[3][2] = {{p->hidden, p->n_in}, {p->hidden, p->hidden}, {p->n_out, p->hidden}};
  int o = 0;
  for (int l = 0; l < layer; ++l) o += dims[l][0] * dims[l][1] + dims[l][0];
  *out = dims[layer][0];
  *in = dims[layer][1];
  return o;
}

static ift_status mlp_reserve(ift_mlp* p, int N) {
  if (N <= p->cap) return IFT_OK;
  dfree(p->d_X);
  dfree(p->d_T);
  dfree(p->d_A1);
  dfree(p->d_H1);
  dfree(p->d_A2);
  dfree(p->d_H2);
  dfree(p->d_Y);
  dfree(p->d_dY);
  dfree(p->d_d1);
  dfree(p->d_d2);
  p->cap = 0;
  const size_t n = N, h = p->hidden;
  ift_status st;
  if ((st = dalloc(&p->d_X, n * p->n_in)) != IFT_OK || (st = dalloc(&p->d_T, n * p->n_out)) != IFT_OK ||
      (st = dalloc(&p->d_A1, n * h)) != IFT_OK || (st = dalloc(&p->d_H1, n * h)) != IFT_OK ||
      (st = dalloc(&p->d_A2, n * h)) != IFT_OK || (st = dalloc(&p->d_H2, n * h)) != IFT_OK ||
      (st = dalloc(&p->d_Y, n * p->n_out)) != IFT_OK || (st = dalloc(&p->d_dY, n * p->n_out)) != IFT_OK ||
      (st = dalloc(&p->d_d1, n * h)) != IFT_OK || (st = dalloc(&p->d_d2, n * h)) != IFT_OK)
    return st;
  p->cap = N;
  return IFT_OK;
}

extern "C" void ift_mlp_destroy(ift_mlp* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  dfree(p->d_par);
  dfree(p->d_grad);
  dfree(p->d_m);
  dfree(p->d_v);
  dfree(p->d_norm);
  dfree(p->d_X);
  dfree(p->d_T);
  dfree(p->d_A1);
  dfree(p->d_H1);
  dfree(p->d_A2);
  dfree(p->d_H2);
  dfree(p->d_Y);
  dfree(p->d_dY);
  dfree(p->d_d1);
  dfree(p->d_d2);
  dfree(p->d_lpart);
  dfree(p->d_loss);
  dfree(p->d_wpart);
  delete p;
}

// splitmix64 (Steele, Lea and Flood 2014): the initialisation stream.
static unsigned long long splitmix64(unsigned long long& s) {
  unsigned long long z = (s += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

extern "C" ift_status ift_mlp_create(int n_in, int hidden, int n_out, unsigned long long seed, ift_mlp** out) {
  if (!out || n_in < 1 || n_in > 8 || hidden < 1 || hidden > 256 || n_out < 1 || n_out > 64) return IFT_EINVAL;
  *out = nullptr;
  ift_mlp* p = new ift_mlp;
  p->n_in = n_in;
  p->hidden = hidden;
  p->n_out = n_out;
  p->n_par = hidden * n_in + hidden + hidden * hidden + hidden + n_out * hidden + n_out;
  // W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0; unit normalisation
  std::vector<float> h(p->n_par, 0.f);
  unsigned long long st = seed;
  for (int l = 0; l < 3; ++l) {
    int in, o;
    const int off = mlp_offsets(p, l, &in, &o);
    const double lim = 1.0 / std::sqrt((double)in);
    for (int i = 0; i < o * in; ++i)
      h[off + i] = float(lim * (2.0 * (double)(splitmix64(st) >> 11) * 0x1.0p-53 - 1.0));
  }
  std::vector<double> nrm(2 * n_in + 2 * n_out, 0.0);
  for (int i = 0; i < n_in; ++i) nrm[n_in + i] = 1.0;
  for (int o = 0; o < n_out; ++o) nrm[2 * n_in + n_out + o] = 1.0;
  if (dalloc(&p->d_par, p->n_par) != IFT_OK || dalloc(&p->d_grad, p->n_par) != IFT_OK ||
      dalloc(&p->d_m, p->n_par) != IFT_OK || dalloc(&p->d_v, p->n_par) != IFT_OK ||
      dalloc(&p->d_norm, nrm.size()) != IFT_OK || dalloc(&p->d_lpart, MLP_LOSS_BLOCKS) != IFT_OK ||
      dalloc(&p->d_loss, 1) != IFT_OK ||
      dalloc(&p->d_wpart, (size_t)MLP_WCHUNKS * std::max(hidden, n_out) * (std::max(hidden, n_in) + 1)) != IFT_OK ||
      hipMemcpy(p->d_par, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_norm, nrm.data(), nrm.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(p->d_m, 0, p->n_par * sizeof(float)) != hipSuccess ||
      hipMemset(p->d_v, 0, p->n_par * sizeof(float)) != hipSuccess) {
    ift_mlp_destroy(p);
    return IFT_ENOMEM;
  }
  *out = p;
  return IFT_OK;
}

extern "C" ift_status ift_mlp_num_params(const ift_mlp* p, int* n) {
  if (!p || !n) return IFT_EINVAL;
  *n = p->n_par;
  return IFT_OK;
}

extern "C" ift_status ift_mlp_set_params(ift_mlp* p, const float* params, hipStream_t stream) {
  if (!p || !params) return IFT_EINVAL;
  HIP_TRY(hipMemcpyAsync(p->d_par, params, p->n_par * sizeof(float), hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemsetAsync(p->d_m, 0, p->n_par * sizeof(float), stream));
  HIP_TRY(hipMemsetAsync(p->d_v, 0, p->n_par * sizeof(float), stream));
  p->adam_t = 0;
  return IFT_OK;
}

extern "C" ift_status ift_mlp_get_params(const ift_mlp* p, float* params, hipStream_t stream) {
  if (!p || !params) return IFT_EINVAL;
  HIP_TRY(hipMemcpyAsync(params, p->d_par, p->n_par * sizeof(float), hipMemcpyDeviceToDevice, stream));
  return IFT_OK;
}

extern "C" ift_status ift_mlp_set_normalization(ift_mlp* p, const double* x_mean, const double* x_scale,
                                                const double* y_mean, const double* y_scale) {
  if (!p || !x_mean || !x_scale || !y_mean || !y_scale) return IFT_EINVAL;
  std::vector<double> nrm;
  nrm.insert(nrm.end(), x_mean, x_mean + p->n_in);
  nrm.insert(nrm.end(), x_scale, x_scale + p->n_in);
  nrm.insert(nrm.end(), y_mean, y_mean + p->n_out);
  nrm.insert(nrm.end(), y_scale, y_scale + p->n_out);
  for (int i = 0; i < p->n_in; ++i)
    if (!(x_scale[i] > 0.0) || !std::isfinite(x_mean[i])) return IFT_EINVAL;
  for (int o = 0; o < p->n_out; ++o)
    if (!(y_scale[o] > 0.0) || !std::isfinite(y_mean[o])) return IFT_EINVAL;
  HIP_TRY(hipMemcpy(p->d_norm, nrm.data(), nrm.size() * sizeof(double), hipMemcpyHostToDevice));
  return IFT_OK;
}

static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Forward pass on d_X (FP32) for N samples into d_Y; keeps pre-activations.
static void mlp_forward(ift_mlp* p, int N, hipStream_t st) {
  int in, o;
  const float* par = p->d_par;
  int off = mlp_offsets(p, 0, &in, &o);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk((long long)N * o, 256)), dim3(256), 0, st, (const float*)p->d_X, in,
                     par + off, par + off + o * in, o, N, p->d_A1, p->d_H1, 1);
  off = mlp_offsets(p, 1, &in, &o);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk((long long)N * o, 256)), dim3(256), 0, st, (const float*)p->d_H1, in,
                     par + off, par + off + o * in, o, N, p->d_A2, p->d_H2, 1);
  off = mlp_offsets(p, 2, &in, &o);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk((long long)N * o, 256)), dim3(256), 0, st, (const float*)p->d_H2, in,
                     par + off, par + off + o * in, o, N, (float*)nullptr, p->d_Y, 0);
}

// Loss of d_Y against d_T and the gradient into d_grad.
static void mlp_backward(ift_mlp* p, int N, hipStream_t st) {
  const long long cnt = (long long)N * p->n_out;
  hipLaunchKernelGGL(k_mlp_loss, dim3(MLP_LOSS_BLOCKS), dim3(256), 0, st, (const float*)p->d_Y, (const float*)p->d_T,
                     cnt, float(1.0 / (double)cnt), p->d_dY, p->d_lpart);
  hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(64), 0, st, (const double*)p->d_lpart, MLP_LOSS_BLOCKS,
                     1.0 / (double)cnt, p->d_loss);
  const float* par = p->d_par;
  float* gr = p->d_grad;
  int in, o;
  // layer 3: dY -> dW3, db3, dH2
  int off = mlp_offsets(p, 2, &in, &o);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((long long)o * (in + 1), 256), MLP_WCHUNKS), dim3(256), 0, st,
                     (const float*)p->d_dY, (const float*)p->d_H2, in, o, N, p->d_wpart);
  hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3(nblk((long long)o * (in + 1), 256)), dim3(256), 0, st,
                     (const float*)p->d_wpart, in, o, gr + off, gr + off + o * in);
  hipLaunchKernelGGL(k_mlp_xgrad, dim3(nblk((long long)N * in, 256)), dim3(256), 0, st, (const float*)p->d_dY,
                     par + off, in, o, N, p->d_d2);
  hipLaunchKernelGGL(k_mlp_act_bwd, dim3(nblk((long long)N * in, 256)), dim3(256), 0, st, (const float*)p->d_A2,
                     p->d_d2, (long long)N * in);
  // layer 2
  off = mlp_offsets(p, 1, &in, &o);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((long long)o * (in + 1), 256), MLP_WCHUNKS), dim3(256), 0, st,
                     (const float*)p->d_d2, (const float*)p->d_H1, in, o, N, p->d_wpart);
  hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3(nblk((long long)o * (in + 1), 256)), dim3(256), 0, st,
                     (const float*)p->d_wpart, in, o, gr + off, gr + off + o * in);
  hipLaunchKernelGGL(k_mlp_xgrad, dim3(nblk((long long)N * in, 256)), dim3(256), 0, st, (const float*)p->d_d2,
                     par + off, in, o, N, p->d_d1);
  hipLaunchKernelGGL(k_mlp_act_bwd, dim3(nblk((long long)N * in, 256)), dim3(256), 0, st, (const float*)p->d_A1,
                     p->d_d1, (long long)N * in);
  // layer 1
  off = mlp_offsets(p, 0, &in, &o);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(nblk((long long)o * (in + 1), 256), MLP_WCHUNKS), dim3(256), 0, st,
                     (const float*)p->d_d1, (const float*)p->d_X, in, o, N, p->d_wpart);
  hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3(nblk((long long)o * (in + 1), 256)), dim3(256), 0, st,
                     (const float*)p->d_wpart, in, o, gr + off, gr + off + o * in);
}

extern "C" ift_status ift_mlp_loss_grad(ift_mlp* p, const float* X, const float* T, int N, float* grad, double* loss,
                                        hipStream_t stream) {
  if (!p || !X || !T || N < 1) return IFT_EINVAL;
  ift_status s = mlp_reserve(p, N);
  if (s != IFT_OK) return s;
  HIP_TRY(hipMemcpyAsync(p->d_X, X, (size_t)N * p->n_in * sizeof(float), hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->d_T, T, (size_t)N * p->n_out * sizeof(float), hipMemcpyDeviceToDevice, stream));
  mlp_forward(p, N, stream);
  mlp_backward(p, N, stream);
  HIP_TRY(hipGetLastError());
  if (grad) HIP_TRY(hipMemcpyAsync(grad, p->d_grad, p->n_par * sizeof(float), hipMemcpyDeviceToDevice, stream));
  if (loss) {
    HIP_TRY(hipMemcpyAsync(loss, p->d_loss, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  return IFT_OK;
}

extern "C" ift_status ift_mlp_train(ift_mlp* p, const double* mu, const double* z, int N, int steps, double lr,
                                    double* loss_hist, hipStream_t stream) {
  if (!p || !mu || !z || N < 1 || steps < 0 || !(lr > 0.0)) return IFT_EINVAL;
  ift_status s = mlp_reserve(p, N);
  if (s != IFT_OK) return s;
  const double* nm = p->d_norm;
  const int ni = p->n_in, no = p->n_out;
  hipLaunchKernelGGL(k_mlp_normalize, dim3(nblk((long long)N * std::max(ni, no), 256)), dim3(256), 0, stream, mu, z, N,
                     ni, no, nm, nm + ni, nm + 2 * ni, nm + 2 * ni + no, p->d_X, p->d_T);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int it = 0; it < steps; ++it) {
    mlp_forward(p, N, stream);
    mlp_backward(p, N, stream);
    p->adam_t += 1;
    const float c1 = float(1.0 - std::pow(0.9, (double)p->adam_t));
    const float c2 = float(1.0 - std::pow(0.999, (double)p->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(p->n_par, 256)), dim3(256), 0, stream, p->d_par, (const float*)p->d_grad,
                       p->d_m, p->d_v, p->n_par, float(lr), b1, b2, eps, c1, c2);
    if (loss_hist) HIP_TRY(hipMemcpyAsync(loss_hist + it, p->d_loss, sizeof(double), hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(stream));
  return IFT_OK;
}

extern "C" ift_status ift_mlp_predict(ift_mlp* p, const double* mu, int N, double* z, int bf16, hipStream_t stream) {
  if (!p || !mu || !z || N < 1) return IFT_EINVAL;
  ift_status s = mlp_reserve(p, N);
  if (s != IFT_OK) return s;
  const double* nm = p->d_norm;
  const int ni = p->n_in, no = p->n_out;
  hipLaunchKernelGGL(k_mlp_normalize, dim3(nblk((long long)N * ni, 256)), dim3(256), 0, stream, mu,
                     (const double*)nullptr, N, ni, no, nm, nm + ni, nm + 2 * ni, nm + 2 * ni + no, p->d_X, p->d_T);
  if (bf16) {
    const float* par = p->d_par;
    const float* H[4] = {p->d_X, p->d_H1, p->d_H2, nullptr};
    float* Ho[3] = {p->d_H1, p->d_H2, p->d_Y};
    for (int l = 0; l < 3; ++l) {
      int in, o;
      const int off = mlp_offsets(p, l, &in, &o);
      hipLaunchKernelGGL(k_mlp_fwd_bf16, dim3(nblk(N, 16), nblk(o, 16)), dim3(64), 0, stream, H[l], in, par + off,
                         par + off + o * in, o, N, Ho[l], l < 2 ? 1 : 0);
    }
  } else {
    mlp_forward(p, N, stream);
  }
  hipLaunchKernelGGL(k_mlp_denormalize, dim3(nblk((long long)N * no, 256)), dim3(256), 0, stream, (const float*)p->d_Y,
                     N, no, nm + 2 * ni, nm + 2 * ni + no, z);
  return hipGetLastError() == hipSuccess ? IFT_OK : IFT_EDEVICE;
}
