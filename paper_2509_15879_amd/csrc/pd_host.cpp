// Host runtime of the polar-disk θ-scheme solver: C ABI (include/polardisk.h),
// mesh construction, coefficient preparation, device memory, the batched
// level driver, and the continuous-batching request loop.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/polardisk.h"
#include "pd_device.h"
#include "pd_launch.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PD_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                  __FILE__, __LINE__);                                                \
  } while (0)

constexpr int kMaxM = 2048;
constexpr int kMaxN = 2048;
constexpr double kPi = 3.14159265358979323846;

using Clock = std::chrono::steady_clock;

// ------------------------------------------------------------------ mesh

// §2.1 / §3.1: h = 1/(m+1), r_i = υ(i h) with υ from (2.4) or (2.13); the
// end points are exact.
int radial_nodes(const pd_mesh_desc &d, std::vector<double> &r) {
  const int m = d.nr;
  r.assign(m + 2, 0.0);
  const double h = 1.0 / (m + 1);
  for (int i = 0; i <= m + 1; ++i) {
    const double s = i * h;
    switch (d.r_kind) {
      case PD_MESH_UNIFORM: r[i] = s; break;
      case PD_MESH_SINE: r[i] = std::sin(std::pow(s, d.p) * kPi / 2.0); break;
      case PD_MESH_POLY: r[i] = 1.0 - std::pow(1.0 - s, d.p + 1.0); break;
      case PD_MESH_EXPLICIT:
        if (!d.r_explicit) return fail(PD_EINVAL, "r_explicit is NULL");
        r[i] = d.r_explicit[i];
        break;
      default: return fail(PD_EINVAL, "unknown r_kind %d", d.r_kind);
    }
  }
  if ((d.r_kind == PD_MESH_SINE || d.r_kind == PD_MESH_POLY) && !(d.p > 0.0))
    return fail(PD_EINVAL, "stretch exponent p must be > 0 (got %g)", d.p);
  r[0] = 0.0;
  r[m + 1] = 1.0;
  for (int i = 1; i <= m + 1; ++i)
    if (!(r[i] > r[i - 1])) return fail(PD_EINVAL, "radial nodes not strictly increasing at %d", i);
  return PD_OK;
}

// §3.1 angular stretch: θ_j = v(j μ̃), v(ι) = 2π sin((ι/2π)^q π/2).
int angular_nodes(const pd_mesh_desc &d, std::vector<double> &th) {
  const int n = d.ntheta;
  th.assign(n + 1, 0.0);
  for (int j = 0; j <= n; ++j) {
    const double s = (double)j / n;
    switch (d.th_kind) {
      case PD_MESH_UNIFORM: th[j] = 2.0 * kPi * s; break;
      case PD_MESH_SINE: th[j] = 2.0 * kPi * std::sin(std::pow(s, d.q) * kPi / 2.0); break;
      case PD_MESH_EXPLICIT:
        if (!d.th_explicit) return fail(PD_EINVAL, "th_explicit is NULL");
        th[j] = d.th_explicit[j];
        break;
      default: return fail(PD_EINVAL, "unknown th_kind %d", d.th_kind);
    }
  }
  if (d.th_kind == PD_MESH_SINE && !(d.q > 0.0))
    return fail(PD_EINVAL, "angular stretch exponent q must be > 0 (got %g)", d.q);
  th[0] = 0.0;
  th[n] = 2.0 * kPi;
  for (int j = 1; j <= n; ++j)
    if (!(th[j] > th[j - 1])) return fail(PD_EINVAL, "angular nodes not strictly increasing at %d", j);
  return PD_OK;
}

int check_mesh(const pd_mesh_desc *d) {
  if (!d) return fail(PD_EINVAL, "mesh descriptor is NULL");
  if (d->nr < 2 || d->nr > kMaxM) return fail(PD_EINVAL, "nr must be in [2, %d] (got %d)", kMaxM, d->nr);
  if (d->ntheta < 4 || d->ntheta > kMaxN)
    return fail(PD_EINVAL, "ntheta must be in [4, %d] (got %d)", kMaxN, d->ntheta);
  return PD_OK;
}

struct MeshH {
  int m = 0, n = 0;
  std::vector<double> r, th;     // nodes
  std::vector<double> h, rh;     // h_i (i = 1..m+1), r_{i+1/2} (i = 0..m)
  std::vector<double> mu, dth;   // μ_j (j = 0..n, μ_0 = μ_n), Δθ_j = (μ_j + μ_{j+1})/2
  std::vector<double> w;         // (h_i + h_{i+1})/2, i = 1..m
};

int build_mesh(const pd_mesh_desc *d, MeshH &M) {
  int rc = check_mesh(d);
  if (rc) return rc;
  M.m = d->nr;
  M.n = d->ntheta;
  if ((rc = radial_nodes(*d, M.r))) return rc;
  if ((rc = angular_nodes(*d, M.th))) return rc;
  const int m = M.m, n = M.n;
  M.h.assign(m + 2, 0.0);
  for (int i = 1; i <= m + 1; ++i) M.h[i] = M.r[i] - M.r[i - 1];
  M.rh.assign(m + 1, 0.0);
  for (int i = 0; i <= m; ++i) M.rh[i] = 0.5 * (M.r[i] + M.r[i + 1]);
  M.mu.assign(n + 1, 0.0);
  for (int j = 1; j <= n; ++j) M.mu[j] = M.th[j] - M.th[j - 1];
  M.mu[0] = M.mu[n];
  M.dth.assign(n, 0.0);
  for (int j = 0; j < n; ++j) M.dth[j] = 0.5 * (M.mu[j] + M.mu[j + 1]);
  M.w.assign(m + 2, 0.0);
  for (int i = 1; i <= m; ++i) M.w[i] = 0.5 * (M.h[i] + M.h[i + 1]);
  return PD_OK;
}

// ------------------------------------------------------------------ tiling

struct Tiling {
  int rb, ncg, nrg, nb_sten, nb_elem, cw, nseg, brad, nb_rad, bang, aw, nb_ang, nb_frad, nb_fang, npad;
};

// Stencil blocks of an instance whose waves take `rb` rings each.
int sten_blocks(int m, int n, int rb) {
  const int nrg = (m + rb - 1) / rb;
  return ((n + 63) / 64) * ((nrg + PD_STEN_WAVES - 1) / PD_STEN_WAVES);
}

// Launch geometry of an instance (the stencil's for PD_RB rings per wave,
// the most blocks a schedule can ask for; see make_plan).
Tiling make_tiling(int m, int n) {
  Tiling t;
  t.rb = PD_RB;
  t.ncg = (n + 63) / 64;
  t.nrg = (m + t.rb - 1) / t.rb;
  t.nb_sten = sten_blocks(m, n, t.rb);
  const int N = m * n + 1;
  t.nb_elem = (N + PD_ELEM_PER_BLOCK - 1) / PD_ELEM_PER_BLOCK;
  // radial sweep and factorisation: 16 columns (one 128-byte line of FP64)
  // per block, 64 segments per column
  t.cw = 16;
  t.nseg = PD_RAD_THREADS / t.cw;
  t.brad = (m + t.nseg - 1) / t.nseg;
  t.nb_rad = (n + t.cw - 1) / t.cw;
  // ring sweeps: one wave per ring up to 1024 nodes; beyond, 4 waves of 8
  // nodes per lane (the lane span rounded up to 32).  Two waves for 513-1024
  // nodes cost a small batch more in barriers than they gained.
  const int b0 = (n + 63) / 64;
  t.aw = b0 <= 16 ? 1 : 4;
  t.bang = t.aw == 1 ? b0 : 8 * t.aw;
  t.nb_ang = (m + 3) / 4;
  t.nb_frad = t.nb_rad;
  t.nb_fang = t.nb_ang;
  t.npad = ((N + 63) / 64) * 64;
  return t;
}

}  // namespace

// ------------------------------------------------------------------ instance

namespace {
struct MgHier;   // multigrid levels of an instance (below)
}

struct pd_instance {
  MeshH M;
  Tiling T;
  int precision = PD_FP64;
  int pde = 0, flux = 0, bc = 0, nsrc = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  void *dmem = nullptr;
  size_t dbytes = 0;
  PdInst H{};            // host image of the device descriptor
  PdScalars *sc = nullptr;   // device scalars
  double *t_table = nullptr; // device time table (capacity kcap+1)
  double *stats = nullptr;   // device level stats (PD_LSTAT * kcap)
  int kcap = 0;
  bool arena = false;         // dmem, t_table and stats are one chunk of a serving arena
  int rot = 0;               // host mirror of the buffer rotation
  double t = 0.0;            // current time
  bool have_prev = false;
  std::atomic<int> busy{0};
  // carrier of a coupled system (pd_set_mobility): created without drift,
  // its faces then take the drift of a potential
  bool zero_drift = false;    // no drift at creation: gp = gm = G on every face
  std::vector<double> lam_h;  // host copies of the source exponents and powers
  std::vector<int> tp_h;
  double b0 = 0.0;            // reaction at the origin (the origin diagonal l0)
  double *drift = nullptr;    // device: G_r, c_r ((m+1) n each), G_t, c_t (m n each)
  int precond = PD_PRECOND_LINE;   // pd_set_preconditioner
  MgHier *mg = nullptr;            // its multigrid levels, built at the first solve that needs them
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
  char *base;
  size_t off = 0;
  bool dry;
  template <typename T>
  T *take(size_t count) {
    size_t o = off;
    off = align_up(off + count * sizeof(T));
    return dry ? nullptr : reinterpret_cast<T *>(base + o);
  }
};

// Lays out every device array of an instance; a dry run only measures.
void carve(pd_instance *I, Carver &c) {
  const int m = I->M.m, n = I->M.n, mn = m * n;
  const int ma = m * 64 * I->T.bang;   // angular factors, ring stride 64*bang
  const int np = I->T.npad;
  const int ns = std::max(1, I->nsrc);
  PdInst &H = I->H;
  const bool mixed = I->precision == PD_MIXED;
  H.inv_rw = c.take<double>(m + 2);
  H.inv_dth = c.take<double>(n);
  H.r_nodes = c.take<double>(m + 2);
  H.th_nodes = c.take<double>(n + 1);
  H.b_node = c.take<double>(np);
  H.g = c.take<double>((size_t)ns * np);
  H.nb = c.take<double>((size_t)ns * n);
  H.lam = c.take<double>(PD_MAXSRC);
  H.tpow = c.take<int>(PD_MAXSRC);
  for (int k = 0; k < PD_NSOL; ++k) H.sol[k] = c.take<double>(np);
  for (int k = 0; k < PD_NSOL; ++k) H.lsol[k] = c.take<double>(np);
  H.ldiag = c.take<double>(np);
  for (int k = 0; k < 3; ++k) H.fdot[k] = c.take<double>(np);
  H.bvec = c.take<double>(np);
  H.diag = c.take<double>(np);
  H.inv_diag = c.take<double>(np);
  H.k64.inv_d = H.inv_diag;
  H.inv_diag32 = mixed ? c.take<float>(np) : nullptr;
  H.k32.inv_d = H.inv_diag32;
  H.rf_uinv = c.take<float>(mn);
  H.rf_f = c.take<float>(mn);
  H.rf_g = c.take<float>(mn);
  H.af_uinv = c.take<float>(ma);
  H.af_f = c.take<float>(ma);
  H.af_g = c.take<float>(ma);
  H.af_z = c.take<float>(ma);
  H.af_kappa = c.take<double>(m);
  H.af_alpha0 = c.take<double>(m);
  H.af_q = c.take<float>(64 * I->T.bang);
  H.af_c = c.take<float>(64 * I->T.bang);
  H.af_sigma = c.take<double>(1);
  H.k64.gp_r = c.take<double>((size_t)(m + 1) * n);
  H.k64.gm_r = c.take<double>((size_t)(m + 1) * n);
  H.k64.gp_t = c.take<double>(mn);
  H.k64.gm_t = c.take<double>(mn);
  if (!mixed) {
    H.k64.r = c.take<double>(np);
    H.k64.rh = c.take<double>(np);
    H.k64.p = c.take<double>(np);
    H.k64.v = c.take<double>(np);
    H.k64.ph = c.take<double>(np);
    H.k64.s = c.take<double>(np);
    H.k64.sh = c.take<double>(np);
    H.k64.t = c.take<double>(np);
    H.k64.w = c.take<double>(np);
    H.rout = nullptr;
  } else {
    H.rout = c.take<double>(np);
    H.k32.r = c.take<float>(np);
    H.k32.rh = c.take<float>(np);
    H.k32.p = c.take<float>(np);
    H.k32.v = c.take<float>(np);
    H.k32.ph = c.take<float>(np);
    H.k32.s = c.take<float>(np);
    H.k32.sh = c.take<float>(np);
    H.k32.t = c.take<float>(np);
    H.k32.w = c.take<float>(np);
    H.k32.d = c.take<float>(np);
    H.k32.gp_r = c.take<float>((size_t)(m + 1) * n);
    H.k32.gm_r = c.take<float>((size_t)(m + 1) * n);
    H.k32.gp_t = c.take<float>(mn);
    H.k32.gm_t = c.take<float>(mn);
  }
  const int nbs = I->T.nb_sten;
  H.part_b = c.take<double>(PD_NBEGIN * (size_t)nbs);
  H.part_g = c.take<double>(PD_NGRAM * (size_t)nbs);
  H.gram_tot = c.take<double>(PD_NGRAM);
  H.part_v = c.take<double>(2 * (size_t)nbs);
  H.part_t = c.take<double>(3 * (size_t)nbs);
  H.part_ur = c.take<double>(2 * (size_t)nbs);
  H.part_a = c.take<double>(1 * (size_t)nbs);
  H.part_e = c.take<double>(3 * (size_t)nbs);
  H.part_x = c.take<double>(2 * (size_t)I->T.nb_elem);
  H.crs = c.take<double>(6 * (size_t)(m + 1));
  H.cr_c = c.take<double>(m + 1);
  H.part_c = c.take<double>((size_t)m * I->T.ncg);
  H.cr_f = c.take<double>((size_t)m + 1);
  H.part_c0 = c.take<double>(nbs);
  I->sc = c.take<PdScalars>(1);
  H.sc = I->sc;
}

// Input node vector (N values, `layout`) -> internal ring-major layout with
// the origin at m*n (npad entries, zero padded).
void to_internal(const double *src, int layout, int m, int n, int npad, double *dst) {
  std::fill(dst, dst + npad, 0.0);
  dst[m * n] = src[0];
  for (int i = 1; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t s = (layout == PD_LAYOUT_PAPER) ? 1 + (size_t)j * m + (i - 1)
                                                    : 1 + (size_t)(i - 1) * n + j;
      dst[(size_t)(i - 1) * n + j] = src[s];
    }
}

void from_internal(const double *src, int layout, int m, int n, double *dst) {
  dst[0] = src[m * n];
  for (int i = 1; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t d = (layout == PD_LAYOUT_PAPER) ? 1 + (size_t)j * m + (i - 1)
                                                    : 1 + (size_t)(i - 1) * n + j;
      dst[d] = src[(size_t)(i - 1) * n + j];
    }
}

// Fetches a caller array (host or device) into a host vector.
int fetch(const double *p, size_t count, int device_ptrs, std::vector<double> &out) {
  out.resize(count);
  if (!p) return fail(PD_EINVAL, "required array is NULL");
  if (device_ptrs) {
    HIPCHK(hipMemcpy(out.data(), p, count * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(out.data(), p, count * sizeof(double));
  }
  return PD_OK;
}

// Face coefficients of the numerical flux P -> Q, F = gp x_P - gm x_Q, from
// the conductance G and the drift coefficient K of the face.
inline void face_pair(double G, double K, int flux, double &gp, double &gm) {
  if (flux == 0) {
    gp = G + 0.5 * K;
    gm = G - 0.5 * K;
  } else {
    gp = G + std::max(K, 0.0);
    gm = G - std::min(K, 0.0);
  }
}

int ensure_time_capacity(pd_instance *I, int K) {
  if (K <= I->kcap) return PD_OK;
  if (I->arena) return fail(PD_EINVAL, "a served request's level capacity is fixed at admission");
  if (I->t_table) (void)hipFree(I->t_table);
  if (I->stats) (void)hipFree(I->stats);
  I->t_table = nullptr;
  I->stats = nullptr;
  const int cap = std::max(K, 16);
  HIPCHK(hipMalloc(&I->t_table, (cap + 1) * sizeof(double)));
  HIPCHK(hipMalloc(&I->stats, PD_LSTAT * (size_t)cap * sizeof(double)));
  I->kcap = cap;
  I->H.t_table = I->t_table;
  I->H.level_stats = I->stats;
  return PD_OK;
}

// Adaptive stepping: the first step from t_start (clamped to [dt_min,
// dt_max], landing on T as every later step does); the device writes the
// later levels as it decides them.
double first_adaptive_level(const pd_time_desc *td, double t_start) {
  double dt = std::min(std::max(td->dt0, td->dt_min), td->dt_max);
  const double rem = td->T;
  if (dt >= rem) return t_start + td->T;
  if (dt > 0.5 * rem) dt = 0.5 * rem;
  return t_start + dt;
}

int build_time_table(const pd_time_desc *td, double t_start, std::vector<double> &t) {
  if (!td) return fail(PD_EINVAL, "time descriptor is NULL");
  if (td->K < 1) return fail(PD_EINVAL, "K must be >= 1");
  const int K = td->K;
  if (td->t_kind == PD_TIME_ADAPTIVE) {
    if (!(td->T > 0.0)) return fail(PD_EINVAL, "T must be > 0");
    if (!(td->dt0 > 0.0) || !(td->dt_min > 0.0) || !(td->dt_max >= td->dt_min))
      return fail(PD_EINVAL, "adaptive stepping needs dt0 > 0 and 0 < dt_min <= dt_max");
    if (!(td->tol_time > 0.0)) return fail(PD_EINVAL, "adaptive stepping needs tol_time > 0");
    if (K < 2) return fail(PD_EINVAL, "K (the cap on adaptive steps) must be >= 2");
    t = {t_start, first_adaptive_level(td, t_start)};
    return PD_OK;
  }
  t.assign(K + 1, 0.0);
  if (td->t_kind == PD_TIME_TABLE) {
    if (!td->t_table) return fail(PD_EINVAL, "t_table is NULL");
    for (int k = 0; k <= K; ++k) t[k] = td->t_table[k];
  } else {
    if (!(td->T > 0.0)) return fail(PD_EINVAL, "T must be > 0");
    for (int k = 0; k <= K; ++k) {
      const double s = (double)k / K;
      if (td->t_kind == PD_TIME_UNIFORM)
        t[k] = td->T * s;
      else if (td->t_kind == PD_TIME_SINE) {
        if (!(td->l > 0.0)) return fail(PD_EINVAL, "time stretch exponent l must be > 0");
        t[k] = td->T * std::sin(std::pow(s, td->l) * kPi / 2.0);
      } else
        return fail(PD_EINVAL, "unknown t_kind %d", td->t_kind);
    }
    t[0] = 0.0;
    t[K] = td->T;
    for (int k = 0; k <= K; ++k) t[k] += t_start;
  }
  for (int k = 1; k <= K; ++k)
    if (!(t[k] > t[k - 1])) return fail(PD_EINVAL, "time levels must increase (level %d)", k);
  if (std::fabs(t[0] - t_start) > 1e-12 * std::max(1.0, std::fabs(t_start)))
    return fail(PD_EINVAL, "time table starts at %g but the state is at t = %g", t[0], t_start);
  t[0] = t_start;
  return PD_OK;
}

// ------------------------------------------------------------------ timing

struct EventTimer : pd::KTimer {
  std::vector<hipEvent_t> pool;
  struct Rec { int f; hipEvent_t a, b; };
  std::vector<Rec> pending;
  double total_ms[PD_KF_N] = {};
  int64_t launches[PD_KF_N] = {};
  hipEvent_t take() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  bool pair(int f, hipEvent_t *a, hipEvent_t *b) override {
    hipEvent_t e0 = take();
    if (!e0) return false;
    hipEvent_t e1 = take();
    if (!e1) {
      pool.push_back(e0);
      return false;
    }
    pending.push_back({f, e0, e1});
    *a = e0;
    *b = e1;
    return true;
  }
  // Reads every finished pair (the caller has synchronised the stream).
  void harvest() {
    for (auto &r : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        total_ms[r.f] += ms;
        launches[r.f] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    for (int k = 0; k < PD_KF_N; ++k) {
      total_ms[k] = 0;
      launches[k] = 0;
    }
  }
  ~EventTimer() override {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

EventTimer *g_event_timer = nullptr;

// ------------------------------------------------------------------ engine

// Launch plan of a set of instances.  Its device data (active counter,
// level words, instance descriptors, block maps) lives in one buffer staged
// through one pinned host buffer; both grow only and are kept when the plan
// is rebuilt for another set, so that a serving loop re-plans without
// allocating or freeing device memory (hipFree waits for the whole device).
struct Plan {
  pd::LaunchSet L;
  std::vector<const pd::MgSet *> mg;   // L.mg: the multigrid sets of its instances
  char *dbuf = nullptr, *hbuf = nullptr;   // device data and its pinned staging
  size_t cap = 0;
  int *n_active = nullptr;
  int *h_active = nullptr;   // pinned, 2 slots
  int *lvl = nullptr;        // device: (levels done, status) per instance
  hipEvent_t ev[2] = {nullptr, nullptr};
  int reserve(size_t bytes, hipStream_t s) {
    if (bytes <= cap) return PD_OK;
    if (dbuf) {
      HIPCHK(hipStreamSynchronize(s));
      (void)hipFree(dbuf);
      (void)hipHostFree(hbuf);
      dbuf = hbuf = nullptr;
    }
    const size_t c = std::max(bytes, cap + cap / 2);
    HIPCHK(hipMalloc(&dbuf, c));
    HIPCHK(hipHostMalloc((void **)&hbuf, c));
    cap = c;
    return PD_OK;
  }
  ~Plan() {
    if (dbuf) (void)hipFree(dbuf);
    if (hbuf) (void)hipHostFree(hbuf);
    if (h_active) (void)hipHostFree(h_active);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

template <typename F>
int build_map(std::vector<pd_instance *> const &insts, F per_inst, std::vector<int2> &map) {
  map.clear();
  for (size_t q = 0; q < insts.size(); ++q) {
    const int nb = per_inst(insts[q]);
    for (int b = 0; b < nb; ++b) map.push_back(make_int2((int)q, b));
  }
  return (int)map.size();
}

// Workgroups of a launch are dealt to the 8 XCDs (each with its own L2) in
// turn: workgroup b runs on XCD b % 8.  This reorders a block map so that
// XCD x receives a contiguous run of logical blocks (its b = x, x+8, x+16,
// ... take the next logical blocks in order), so that neighbouring tiles,
// which read each other's edge rings and columns, share an L2.
constexpr int kXcds = 8;
void xcd_contiguous(std::vector<int2> &map) {
  const size_t nb = map.size();
  std::vector<int2> out(nb);
  size_t next = 0;
  for (int x = 0; x < kXcds; ++x)
    for (size_t b = x; b < nb; b += kXcds) out[b] = map[next++];
  map.swap(out);
}

// stencil_rings: stencil rings per wave of the plan's instances (PD_RB or
// 2 PD_RB, either precision).
int make_plan(std::vector<pd_instance *> const &insts, hipStream_t s, Plan &P, int stencil_rings = PD_RB) {
  const int ninst = (int)insts.size();
  auto rings = [&](const pd_instance *) { return stencil_rings; };
  P.L = pd::LaunchSet{};
  // host side first: the block maps, then one layout for everything
  constexpr int NMAP = 9;
  std::vector<int2> maps[NMAP];
  int *counts[NMAP] = {&P.L.nb_sten, &P.L.nb_elem, &P.L.nb_rad, &P.L.nb_rs[0], &P.L.nb_rs[1], &P.L.nb_rs[2],
                       &P.L.nb_ang, &P.L.nb_angs[0], &P.L.nb_angs[1]};
  int2 **dsts[NMAP] = {&P.L.map_sten, &P.L.map_elem, &P.L.map_rad, &P.L.map_rs[0], &P.L.map_rs[1], &P.L.map_rs[2],
                       &P.L.map_ang, &P.L.map_angs[0], &P.L.map_angs[1]};
  *counts[0] = build_map(insts, [&](pd_instance *I) { return sten_blocks(I->M.m, I->M.n, rings(I)); }, maps[0]);
  *counts[1] = build_map(insts, [](pd_instance *I) { return I->T.nb_elem; }, maps[1]);
  // radial sweep blocks: neighbouring column blocks share the 128-byte
  // lines of FP32 rows (16 columns x 4 bytes), so they go to the same XCD
  // (L2).  The factorisation keeps the plain order: only the instances
  // starting a level take part in it, and a contiguous run per XCD would
  // crowd them onto a few XCDs.
  *counts[2] = build_map(insts, [](pd_instance *I) { return I->T.nb_rad; }, maps[2]);
  for (int c = 0; c < 3; ++c)
    *counts[3 + c] =
        build_map(insts, [c](pd_instance *I) { return pd::rad_class(I->M.m) == c ? pd::rad_blocks(I->M.m, I->M.n) : 0; },
                  maps[3 + c]);
  // factorisation of the rings: 4 rings (waves) per block for every
  // instance; sweeps: the same for one-wave rings, 4/aw rings per block for
  // the wider ones
  *counts[6] = build_map(insts, [](pd_instance *I) { return I->T.nb_ang; }, maps[6]);
  *counts[7] = build_map(insts, [](pd_instance *I) { return I->T.aw == 1 ? I->T.nb_ang : 0; }, maps[7]);
  *counts[8] = build_map(insts, [](pd_instance *I) {
    return I->T.aw == 1 ? 0 : (I->M.m * I->T.aw + 3) / 4;
  }, maps[8]);
  xcd_contiguous(maps[0]);
  xcd_contiguous(maps[3]);
  xcd_contiguous(maps[4]);
  xcd_contiguous(maps[5]);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t off = 0;
  const size_t o_act = off;
  off += al(sizeof(int));
  const size_t o_lvl = off;
  off += al(2 * (size_t)ninst * sizeof(int));
  const size_t o_inst = off;
  off += al((size_t)ninst * sizeof(PdInst));
  size_t o_map[NMAP];
  for (int k = 0; k < NMAP; ++k) {
    o_map[k] = off;
    off += al(maps[k].size() * sizeof(int2));
  }
  int rc;
  if ((rc = P.reserve(off, s))) return rc;
  P.n_active = (int *)(P.dbuf + o_act);
  P.lvl = (int *)(P.dbuf + o_lvl);
  P.L.insts = (PdInst *)(P.dbuf + o_inst);
  std::memset(P.hbuf, 0, off);
  PdInst *hv = (PdInst *)(P.hbuf + o_inst);
  for (int q = 0; q < ninst; ++q) {
    hv[q] = insts[q]->H;
    hv[q].rb = rings(insts[q]);
    hv[q].nrg = (insts[q]->M.m + hv[q].rb - 1) / hv[q].rb;
    hv[q].nb_sten = sten_blocks(insts[q]->M.m, insts[q]->M.n, hv[q].rb);
    hv[q].n_active = P.n_active;
    hv[q].lvl_out = P.lvl + 2 * q;
    P.L.mixed_any |= insts[q]->precision == PD_MIXED;
    P.L.fp64_any |= insts[q]->precision != PD_MIXED;
    P.L.max_bang = std::max(P.L.max_bang, insts[q]->T.bang);
    if (insts[q]->T.aw == 1) P.L.max_bang1 = std::max(P.L.max_bang1, insts[q]->T.bang);
    P.L.max_bfrad = std::max(P.L.max_bfrad, insts[q]->T.brad);
  }
  for (auto *I : insts) {
    const int c = pd::rad_class(I->M.m);
    P.L.max_brs[c] = std::max(P.L.max_brs[c], pd::rad_rows(I->M.m));
  }
  for (int k = 0; k < NMAP; ++k) {
    *dsts[k] = maps[k].empty() ? nullptr : (int2 *)(P.dbuf + o_map[k]);
    if (!maps[k].empty()) std::memcpy(P.hbuf + o_map[k], maps[k].data(), maps[k].size() * sizeof(int2));
  }
  P.L.ninst = ninst;
  // one copy (the pinned staging is rewritten only after the next plan's
  // copy has been ordered behind this one on the same stream, and the
  // stream is synchronised before the host writes it again)
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpyAsync(P.dbuf, P.hbuf, off, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!P.h_active) {
    HIPCHK(hipHostMalloc((void **)&P.h_active, 2 * sizeof(int)));
    for (auto &e : P.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  P.h_active[0] = P.h_active[1] = 1;
  return PD_OK;
}

// ------------------------------------------------------------------ multigrid
//
// The θ-semi-coarsening levels of an instance (PdMgLevel): level l+1 merges
// the θ-lines of level l in pairs while n_l >= kMgMin, and the ring means
// lie below the last level.  Each coarse level is laid out like an instance
// of its own (faces, widths, reaction, factors, vectors) so that the
// instance's factorisation and line-sweep kernels serve it unchanged; a
// "shadow" descriptor of level 0 gives the instance's own factors the
// V-cycle's vectors.  All of them point at the instance's scalars, so that
// they run exactly when the instance's own kernels do.

constexpr int kMgMin = 16;   // lines are merged while a level has at least this many

struct MgHier {
  int m = 0, n0 = 0, nlev = 0;
  std::vector<int> ns;                                // θ-lines per level
  void *dmem = nullptr;
  std::vector<std::unique_ptr<pd_instance>> shadow;   // [0..nlev]
  std::vector<std::unique_ptr<Plan>> plans;           // [0..nlev]
  std::vector<PdMgLevel> hl;                          // host copies of the level descriptors
  PdMgLevel *dlev = nullptr;
  pd::MgSet set;
  ~MgHier() {
    plans.clear();
    if (dmem) (void)hipFree(dmem);
  }
};

void mg_free(pd_instance *I) {
  delete I->mg;
  I->mg = nullptr;
}

// Lays out the levels' arrays (a dry run only measures).
void mg_carve(MgHier &H, const pd_instance *I, Carver &c) {
  const int m = H.m;
  const bool hb = I->H.has_b != 0;
  H.hl.assign(H.nlev + 1, PdMgLevel{});
  for (int l = 0; l <= H.nlev; ++l) {
    const int n = H.ns[l];
    const Tiling T = make_tiling(m, n);
    const int np = T.npad, mn = m * n, ma = m * 64 * T.bang;
    PdMgLevel &L = H.hl[l];
    pd_instance &S = *H.shadow[l];
    PdInst &D = S.H;
    L.m = m;
    L.n = n;
    L.npad = np;
    L.has_b = hb ? 1 : 0;
    L.inv_rw = I->H.inv_rw;
    L.inv_V0 = I->H.inv_V0;
    L.r = c.take<double>(np);
    L.w = c.take<double>(np);
    L.sh = c.take<double>(np);
    if (l == 0) {
      L.gp_r = I->H.k64.gp_r;
      L.gm_r = I->H.k64.gm_r;
      L.gp_t = I->H.k64.gp_t;
      L.gm_t = I->H.k64.gm_t;
      L.inv_dth = I->H.inv_dth;
      L.b_node = I->H.b_node;
      L.diag = I->H.diag;
      L.inv_diag = I->H.inv_diag;
      continue;
    }
    L.gp_r = c.take<double>((size_t)(m + 1) * n);
    L.gm_r = c.take<double>((size_t)(m + 1) * n);
    L.gp_t = c.take<double>(mn);
    L.gm_t = c.take<double>(mn);
    L.inv_dth = c.take<double>(n);
    L.b_node = hb ? c.take<double>(np) : nullptr;
    double *dg = c.take<double>(np), *idg = c.take<double>(np);
    L.diag = dg;
    L.inv_diag = idg;
    L.g = c.take<double>(np);
    L.x = c.take<double>(np);
    D.diag = dg;
    D.inv_diag = idg;
    D.rf_uinv = c.take<float>(mn);
    D.rf_f = c.take<float>(mn);
    D.rf_g = c.take<float>(mn);
    D.af_uinv = c.take<float>(ma);
    D.af_f = c.take<float>(ma);
    D.af_g = c.take<float>(ma);
    D.af_z = c.take<float>(ma);
    D.af_kappa = c.take<double>(m);
    D.af_alpha0 = c.take<double>(m);
    D.af_q = c.take<float>(64 * T.bang);
    D.af_c = c.take<float>(64 * T.bang);
    D.af_sigma = c.take<double>(1);
  }
  H.dlev = c.take<PdMgLevel>(H.nlev + 1);
  H.set.btot = c.take<double>(m + 1);
  H.set.cring = c.take<double>(m + 1);
}

// The shadow descriptor of level l: the instance's descriptor with the
// level's geometry, faces, factors and vectors (fields no sweep or
// factorisation reads are cleared, so that a stray use fails loudly).
void mg_shadow(MgHier &H, const pd_instance *I, int l) {
  pd_instance &S = *H.shadow[l];
  const PdMgLevel &L = H.hl[l];
  const int m = H.m, n = H.ns[l];
  S.M.m = m;
  S.M.n = n;
  S.T = l == 0 ? I->T : make_tiling(m, n);
  S.precision = PD_FP64;
  S.stream = I->stream;
  PdInst D = I->H;
  if (l > 0) {
    const PdInst &K = S.H;   // factor arrays set by mg_carve
    D.diag = K.diag;
    D.inv_diag = K.inv_diag;
    D.rf_uinv = K.rf_uinv;
    D.rf_f = K.rf_f;
    D.rf_g = K.rf_g;
    D.af_uinv = K.af_uinv;
    D.af_f = K.af_f;
    D.af_g = K.af_g;
    D.af_z = K.af_z;
    D.af_kappa = K.af_kappa;
    D.af_alpha0 = K.af_alpha0;
    D.af_q = K.af_q;
    D.af_c = K.af_c;
    D.af_sigma = K.af_sigma;
    D.inv_dth = L.inv_dth;
    D.b_node = L.b_node;
  }
  D.m = m;
  D.n = n;
  D.npad = S.T.npad;
  D.mixed = 0;
  D.rb = S.T.rb;
  D.ncg = S.T.ncg;
  D.nrg = S.T.nrg;
  D.nb_sten = S.T.nb_sten;
  D.nb_elem = S.T.nb_elem;
  D.cw = S.T.cw;
  D.nseg = S.T.nseg;
  D.brad = S.T.brad;
  D.nb_rad = S.T.nb_rad;
  D.bang = S.T.bang;
  D.aw = S.T.aw;
  D.nb_ang = S.T.nb_ang;
  D.nb_frad = S.T.nb_frad;
  D.nb_fang = S.T.nb_fang;
  D.k64 = KSet<double>{};
  D.k64.r = D.k64.rh = D.k64.p = D.k64.v = D.k64.ph = D.k64.s = D.k64.t = D.k64.d = L.r;
  D.k64.w = L.w;
  D.k64.sh = L.sh;
  D.k64.gp_r = L.gp_r;
  D.k64.gm_r = L.gm_r;
  D.k64.gp_t = L.gp_t;
  D.k64.gm_t = L.gm_t;
  D.k64.inv_d = D.inv_diag;
  D.k32 = KSet<float>{};
  D.inv_diag32 = nullptr;
  for (int k = 0; k < PD_NSOL; ++k) D.sol[k] = D.lsol[k] = nullptr;
  for (int k = 0; k < 3; ++k) D.fdot[k] = nullptr;
  D.ldiag = D.bvec = D.rout = nullptr;
  D.part_b = D.part_v = D.part_t = D.part_ur = D.part_a = D.part_x = D.part_g = D.gram_tot = nullptr;
  D.part_e = D.cr_c = D.part_c = D.cr_f = D.part_c0 = nullptr;
  D.level_stats = nullptr;
  D.sc = I->H.sc;
  S.H = D;
}

// Builds (or reuses) the instance's levels for a solve on stream s: the
// coarse faces from the instance's current faces, the level descriptors,
// and one launch set per level.
int mg_prepare(pd_instance *I, hipStream_t s, const pd::MgSet **out) {
  if (I->precision != PD_FP64) return fail(PD_EINVAL, "the multigrid preconditioner takes FP64 instances");
  const int m = I->M.m, n = I->M.n;
  MgHier *H = I->mg;
  if (!H || H->m != m || H->n0 != n) {
    mg_free(I);
    std::unique_ptr<MgHier> N(new MgHier);
    N->m = m;
    N->n0 = n;
    N->ns = {n};
    while (N->ns.back() >= kMgMin) N->ns.push_back(N->ns.back() / 2);
    N->nlev = (int)N->ns.size() - 1;
    if (N->nlev > PD_MG_MAXLEV) return fail(PD_EINVAL, "too many multigrid levels for %d lines", n);
    for (int l = 0; l <= N->nlev; ++l) {
      N->shadow.emplace_back(new pd_instance);
      N->plans.emplace_back(new Plan);
    }
    Carver dry{nullptr, 0, true};
    mg_carve(*N, I, dry);
    const size_t bytes = dry.off;
    hipError_t e = hipMalloc(&N->dmem, bytes);
    if (e != hipSuccess) {
      N->dmem = nullptr;
      return fail(e == hipErrorOutOfMemory ? PD_ENOMEM : PD_EHIP, "multigrid allocation of %zu bytes failed: %s",
                  bytes, hipGetErrorString(e));
    }
    HIPCHK(hipMemsetAsync(N->dmem, 0, bytes, s));
    Carver cv{(char *)N->dmem, 0, false};
    mg_carve(*N, I, cv);
    I->mg = H = N.release();
  }
  // level 0 follows the instance (its faces may have changed since the last
  // call: a carrier's drift); the coarse faces are formed again from them
  {
    Carver cv{(char *)H->dmem, 0, false};
    mg_carve(*H, I, cv);   // the same layout again, with level 0's pointers into the instance
  }
  HIPCHK(hipMemcpyAsync(H->dlev, H->hl.data(), H->hl.size() * sizeof(PdMgLevel), hipMemcpyHostToDevice, s));
  for (int l = 1; l <= H->nlev; ++l) {
    PdMgLevel &L = H->hl[l];
    pd::launch_mg_faces(H->dlev, l - 1, m, H->ns[l], const_cast<double *>(L.gp_r), const_cast<double *>(L.gm_r),
                        const_cast<double *>(L.gp_t), const_cast<double *>(L.gm_t),
                        const_cast<double *>(L.inv_dth), const_cast<double *>(L.b_node), s);
    HIPCHK(hipGetLastError());
  }
  pd::MgSet &M = H->set;
  M.nlev = H->nlev;
  M.m = m;
  for (int l = 0; l <= H->nlev; ++l) {
    M.n[l] = H->ns[l];
    mg_shadow(*H, I, l);
    int rc = make_plan({H->shadow[l].get()}, s, *H->plans[l]);
    if (rc) return rc;
    M.lev[l] = H->plans[l]->L;
  }
  M.dlev = H->dlev;
  M.sc = I->sc;
  M.crs = I->H.crs;
  M.p = I->H.k64.p;
  M.s = I->H.k64.s;
  M.r = I->H.k64.r;
  M.ph = I->H.k64.ph;
  M.sh = I->H.k64.sh;
  *out = &M;
  return PD_OK;
}

// The V-cycles of a plan's multigrid instances (built or refreshed for
// this solve).  They batch with FP64 instances only.
int attach_mg(std::vector<pd_instance *> const &part, hipStream_t s, Plan &P) {
  P.mg.clear();
  bool mixed = false;
  for (auto *I : part) mixed |= I->precision == PD_MIXED;
  for (auto *I : part) {
    if (I->precond != PD_PRECOND_MG) continue;
    if (mixed) return fail(PD_EINVAL, "a multigrid instance batches with FP64 instances only");
    const pd::MgSet *ms = nullptr;
    int rc = mg_prepare(I, s, &ms);
    if (rc) return rc;
    P.mg.push_back(ms);
  }
  P.L.mg = P.mg.empty() ? nullptr : P.mg.data();
  P.L.nmg = (int)P.mg.size();
  return PD_OK;
}

struct SolveParams {
  double theta, tol, tol_inner;
  int maxit, maxit_inner, max_outer;
  int adaptive = 0;
  double T = 0.0, dt_min = 0.0, dt_max = 0.0, tol_time = 0.0;
  double max_seconds = 0.0;   // host wall-clock limit of the call (0: kDefaultMaxSeconds)
};

constexpr double kDefaultMaxSeconds = 600.0;

int init_scalars(pd_instance *I, const SolveParams &sp, int K, hipStream_t s) {
  PdScalars h{};
  h.theta = sp.theta;
  h.theta_run = sp.theta;
  h.tol = sp.tol;
  h.tol_inner = sp.tol_inner;
  h.maxit = sp.maxit;
  h.maxit_inner = sp.maxit_inner;
  h.max_outer = sp.max_outer;
  h.K = K;
  h.level = 0;
  h.status = ST_DONE;          // ready to start a level
  h.rot = I->rot;
  h.have_prev = 0;             // extrapolation restarts with each solve call
  h.fact_dt = -1.0;
  h.fact_theta = -1.0;
  h.t_now = I->t;
  h.adaptive = sp.adaptive;
  h.need_f0 = sp.adaptive;
  h.t_end = I->t + sp.T;
  h.dt_min = sp.dt_min;
  h.dt_max = sp.dt_max;
  h.tol_time = sp.tol_time;
  HIPCHK(hipMemcpyAsync(I->sc, &h, sizeof h, hipMemcpyHostToDevice, s));
  // levels never taken read as not done
  if (I->stats) HIPCHK(hipMemsetAsync(I->stats, 0, PD_LSTAT * (size_t)K * sizeof(double), s));
  return PD_OK;
}

// Library-owned helper streams (default priority), one pool per device,
// created on first use and kept for the life of the process.
hipStream_t helper_stream(int device, int k) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, hipStream_t> pool;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(device, k);
  auto it = pool.find(key);
  if (it != pool.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
  pool.emplace(key, st);
  return st;
}

// Launch schedule of an engine: how many stream groups a batch is split
// into and how many Krylov cycles one captured graph holds.
struct Schedule {
  int groups = 1;
  int cycles_per_graph = 2;
  int stencil_rings = PD_RB;  // stencil rings per wave
};

std::atomic<int> g_sched_groups{1}, g_sched_cpg{2}, g_sched_rings{PD_RB};

Schedule default_schedule() {
  Schedule sc;
  sc.groups = g_sched_groups.load();
  sc.cycles_per_graph = g_sched_cpg.load();
  sc.stencil_rings = g_sched_rings.load();
  return sc;
}

// A set of instances advancing through their time levels in shared
// launches, each at its own pace (asynchronous levels: an instance whose
// level has ended starts its next one at the next round, whatever the
// others are doing).  A round is the level-control head (control kernel,
// factorisations and right-hand sides of the instances starting a level)
// and cycles_per_graph Krylov cycles; it is captured, with the read-back of
// the active-instance counter, in one HIP graph and replayed until every
// instance has taken all its levels (one graph of look-ahead; launches for
// finished instances are no-ops).  The batch is split into `groups` parts
// (by cells, largest first, to the part with the fewest), each with its own
// launch plan and graph on its own stream, so that one part's launch ramps
// and tails overlap the other parts' work; group 0 runs on the caller's
// stream, which every run forks from and joins.  Per-kernel event timing
// needs plain launches.
struct Engine {
  struct Group {
    hipStream_t s = nullptr;
    std::unique_ptr<Plan> P;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> members;   // engine instance indices, in plan order
  };
  hipStream_t s = nullptr;
  std::vector<Group> G;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  bool use_graph = false;
  int max_cycles = 0;
  int ninst = 0;
  int cpg = 2;
  int rings = PD_RB;

  std::vector<std::unique_ptr<Plan>> spare;   // plans kept for the next build

  void release() {
    for (auto &g : G) {
      if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
      // a kept plan may next serve another stream: nothing may still read it
      if (g.s) (void)hipStreamSynchronize(g.s);
      if (g.P) spare.push_back(std::move(g.P));
    }
    G.clear();
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (auto e : join_ev) (void)hipEventDestroy(e);
    fork_ev = nullptr;
    join_ev.clear();
  }
  ~Engine() { release(); }

  int build(std::vector<pd_instance *> const &insts, int cycles_cap, hipStream_t st, Schedule sch = {},
            bool adaptive = false) {
    release();
    s = st;
    ninst = (int)insts.size();
    max_cycles = cycles_cap;
    cpg = std::max(1, sch.cycles_per_graph);
    rings = sch.stencil_rings;
    const int ng = std::max(1, std::min(sch.groups, ninst));
    int device = 0;
    HIPCHK(hipGetDevice(&device));
    // partition by cells, largest first, each to the part with the fewest
    std::vector<int> order(ninst);
    for (int q = 0; q < ninst; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return (int64_t)insts[x]->M.m * insts[x]->M.n > (int64_t)insts[y]->M.m * insts[y]->M.n;
    });
    G.resize(ng);
    std::vector<int64_t> load(ng, 0);
    for (int q : order) {
      int g = 0;
      for (int k = 1; k < ng; ++k)
        if (load[k] < load[g]) g = k;
      G[g].members.push_back(q);
      load[g] += (int64_t)insts[q]->M.m * insts[q]->M.n;
    }
    for (auto &g : G) std::sort(g.members.begin(), g.members.end());
    HIPCHK(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
    join_ev.assign(ng, nullptr);
    for (auto &e : join_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    use_graph = !pd::g_timer && !getenv("PD_NO_GRAPH");
    for (int k = 0; k < ng; ++k) {
      Group &g = G[k];
      g.s = (k == 0) ? s : helper_stream(device, k);
      if (!g.s) return fail(PD_EHIP, "could not create a helper stream");
      std::vector<pd_instance *> part;
      for (int q : g.members) part.push_back(insts[q]);
      if (!spare.empty()) {
        g.P = std::move(spare.back());
        spare.pop_back();
      } else {
        g.P.reset(new Plan);
      }
      int rc = make_plan(part, g.s, *g.P, rings);
      if (rc) return rc;
      if ((rc = attach_mg(part, g.s, *g.P))) return rc;
      g.P->L.adaptive_any = adaptive ? 1 : 0;
      // every member still has levels to take
      HIPCHK(hipMemsetD32Async((hipDeviceptr_t)g.P->n_active, (int)part.size(), 1, g.s));
      if (use_graph) {
        HIPCHK(hipStreamBeginCapture(g.s, hipStreamCaptureModeThreadLocal));
        pd::launch_round(g.P->L, cpg, g.s);
        hipError_t ce = hipMemcpyAsync(&g.P->h_active[0], g.P->n_active, sizeof(int), hipMemcpyDeviceToHost, g.s);
        hipError_t ee = hipStreamEndCapture(g.s, &g.graph);
        if (ce != hipSuccess || ee != hipSuccess)
          return fail(PD_EHIP, "graph capture failed: %s / %s", hipGetErrorString(ce), hipGetErrorString(ee));
        HIPCHK(hipGraphInstantiate(&g.gexec, g.graph, nullptr, nullptr, 0));
      }
    }
    return PD_OK;
  }

  // Replays cycles until every part's active-instance count reaches 0 (all
  // instances have taken all their levels) or max_cycles cycles have been
  // launched; returns whether everything finished.  Work stays queued on
  // the parts' streams; the caller's stream is joined to them.
  // Replays stop early, with *timed_out set, once the host clock passes
  // `deadline` (the work already queued still completes).
  int run(long max_cycles_run, bool *finished, Clock::time_point deadline = Clock::time_point::max(),
          bool *timed_out = nullptr) {
    const int ng = (int)G.size();
    if (timed_out) *timed_out = false;
    HIPCHK(hipEventRecord(fork_ev, s));
    for (int k = 1; k < ng; ++k) HIPCHK(hipStreamWaitEvent(G[k].s, fork_ev, 0));
    std::vector<char> live(ng, 1);
    int left = ng;
    const long max_launch = (max_cycles_run + cpg - 1) / cpg;   // rounds of cpg cycles
    for (long c = 0; c < max_launch && left > 0; ++c) {
      if (Clock::now() > deadline) {
        if (timed_out) *timed_out = true;
        break;
      }
      for (int k = 0; k < ng; ++k) {
        if (!live[k]) continue;
        Plan &Q = *G[k].P;
        if (use_graph) {
          HIPCHK(hipGraphLaunch(G[k].gexec, G[k].s));
        } else {
          pd::launch_round(Q.L, cpg, G[k].s);
          HIPCHK(hipMemcpyAsync(&Q.h_active[c & 1], Q.n_active, sizeof(int), hipMemcpyDeviceToHost, G[k].s));
        }
        HIPCHK(hipEventRecord(Q.ev[c & 1], G[k].s));
      }
      if (c < 1) continue;
      for (int k = 0; k < ng; ++k) {
        if (!live[k]) continue;
        Plan &Q = *G[k].P;
        // the slot holds the part's count after launch c-1 or a later one;
        // the count never grows, so 0 means the part is done
        HIPCHK(hipEventSynchronize(Q.ev[(c - 1) & 1]));
        const int na = use_graph ? __atomic_load_n(&Q.h_active[0], __ATOMIC_ACQUIRE) : Q.h_active[(c - 1) & 1];
        if (na == 0) {
          live[k] = 0;
          --left;
        }
      }
      if (g_event_timer && pd::g_timer) {
        for (auto &g : G) HIPCHK(hipStreamSynchronize(g.s));
        g_event_timer->harvest();
      }
    }
    HIPCHK(hipGetLastError());
    for (int k = 1; k < ng; ++k) {
      HIPCHK(hipEventRecord(join_ev[k], G[k].s));
      HIPCHK(hipStreamWaitEvent(s, join_ev[k], 0));
    }
    if (finished) *finished = left == 0;
    return PD_OK;
  }

  // (levels done, left-the-batch flag) of every instance (synchronises).
  int levels_done(std::vector<int> &out) {
    out.assign(2 * (size_t)ninst, 0);
    for (auto &g : G) {
      std::vector<int> part(2 * g.members.size());
      HIPCHK(hipMemcpyAsync(part.data(), g.P->lvl, part.size() * sizeof(int), hipMemcpyDeviceToHost, g.s));
      HIPCHK(hipStreamSynchronize(g.s));
      for (size_t k = 0; k < g.members.size(); ++k) {
        out[2 * (size_t)g.members[k]] = part[2 * k];
        out[2 * (size_t)g.members[k] + 1] = part[2 * k + 1];
      }
    }
    return PD_OK;
  }
};

int cycles_cap(SolveParams const &sp) { return sp.maxit + sp.max_outer + 8; }

// Krylov cycles a solve of K levels can need: levels x attempts per level x
// cycles per attempt.  An adaptive solve takes at most ceil(T/dt_min) + 2
// accepted steps (every step but the last two is at least dt_min long) and,
// per step, at most ceil(ln(dt_max/dt_min)/ln 1.4) + 1 rejected attempts: a
// rejection has e > 2 tol_time, so it shrinks Δt by 0.9 (1/2)^{1/(q+1)} <=
// 1/1.4 or more, and stops once Δt reaches dt_min.
long solve_cycle_bound(SolveParams const &sp, int K) {
  long levels = K, attempts = 1;
  if (sp.adaptive && sp.dt_min > 0.0) {
    levels = std::min<long>(K, (long)std::ceil(sp.T / sp.dt_min) + 2);
    attempts = 2 + (long)std::ceil(std::log(std::max(1.0, sp.dt_max / sp.dt_min)) / std::log(1.4));
  }
  return levels * attempts * (long)cycles_cap(sp) + 2 * levels;
}

// After a solve that stopped early: the host mirror of the instance follows
// its last completed level (the level under way, if any, is dropped).
int sync_host_state(pd_instance *I) {
  PdScalars h{};
  HIPCHK(hipMemcpy(&h, I->sc, sizeof h, hipMemcpyDeviceToHost));
  I->rot = h.rot;
  I->t = h.t_now;
  I->have_prev = false;
  return PD_OK;
}

// Per-level statistics of an instance after a solve: PD_LSTAT doubles per
// level; an adaptive solve takes fewer levels than its cap K (the rest stay
// zero), and fails when the cap came before T.
int read_level_stats(pd_instance *I, int K, std::vector<double> &st, int &worst) {
  PdScalars h{};
  HIPCHK(hipMemcpy(&h, I->sc, sizeof h, hipMemcpyDeviceToHost));
  I->rot = h.rot;
  I->t = h.t_now;
  I->have_prev = true;
  st.assign(PD_LSTAT * (size_t)K, 0.0);
  HIPCHK(hipMemcpy(st.data(), I->stats, st.size() * sizeof(double), hipMemcpyDeviceToHost));
  const int taken = h.adaptive ? std::min(h.level, K) : K;
  if (h.adaptive && h.t_now < h.t_end && worst == PD_OK) worst = PD_ENOCONV;
  for (int k = 0; k < taken; ++k) {
    const int status = (int)st[PD_LSTAT * k + 2];
    if (status == ST_BREAKDOWN) worst = PD_EBREAKDOWN;
    else if (status != ST_DONE && worst == PD_OK) worst = PD_ENOCONV;
  }
  return PD_OK;
}

// Runs all levels of every instance (instance q has Ks[q] levels).
int run_levels(std::vector<pd_instance *> const &insts, std::vector<int> const &Ks,
               std::vector<SolveParams> const &sps, hipStream_t s, std::vector<std::vector<double>> *stats_out) {
  const Clock::time_point t_start = Clock::now();
  int rc, cap = 0;
  long bound = 0;
  double max_s = 0.0;
  for (size_t q = 0; q < insts.size(); ++q) {
    if ((rc = init_scalars(insts[q], sps[q], Ks[q], s))) return rc;
    cap = std::max(cap, cycles_cap(sps[q]));
    bound = std::max(bound, solve_cycle_bound(sps[q], Ks[q]));
    const double lim = sps[q].max_seconds > 0.0 ? sps[q].max_seconds : kDefaultMaxSeconds;
    max_s = q == 0 ? lim : std::min(max_s, lim);
  }
  Engine E;
  bool adaptive = false;
  for (auto const &sp : sps) adaptive |= sp.adaptive != 0;
  if ((rc = E.build(insts, cap, s, default_schedule(), adaptive))) return rc;
  bool finished = false, timed_out = false;
  const auto deadline = t_start + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(max_s));
  if ((rc = E.run(bound, &finished, deadline, &timed_out))) return rc;
  HIPCHK(hipGetLastError());
  for (auto &g : E.G) HIPCHK(hipStreamSynchronize(g.s));
  HIPCHK(hipStreamSynchronize(s));
  if (!finished) {
    for (auto *I : insts) (void)sync_host_state(I);
    if (timed_out) return fail(PD_ENOCONV, "the solve passed its wall-clock limit of %g s", max_s);
    return fail(PD_ENOCONV, "the batch did not finish within its cycle bound (%ld cycles)", bound);
  }
  int worst = PD_OK;
  for (size_t q = 0; q < insts.size(); ++q) {
    std::vector<double> st;
    if ((rc = read_level_stats(insts[q], Ks[q], st, worst))) return rc;
    if (stats_out) (*stats_out)[q] = std::move(st);
  }
  if (worst == PD_EBREAKDOWN) return fail(worst, "Krylov breakdown in at least one step");
  if (worst == PD_ENOCONV)
    return fail(worst, adaptive ? "an adaptive solve stopped before T (a step hit its iteration cap, the level cap "
                                  "came first, or the local error stayed above 2 tol_time at dt_min)"
                                : "a step did not reach the tolerance within the iteration cap");
  return PD_OK;
}

void fill_stats(const std::vector<double> &st, int k, pd_step_stats *o) {
  const double *e = st.data() + PD_LSTAT * (size_t)k;
  o->iters = (int)e[0];
  o->refinements = (int)e[1];
  o->err_time = e[7];
  o->rejected = (int)e[8];
  o->pad = 0;
  if (e[4] == 0.0) {                      // a level an adaptive solve did not need
    o->status = PD_OK;
    o->reserved = 0;
    o->rel_resid = 0.0;
    o->dt = 0.0;
    o->t = 0.0;
    return;
  }
  const int status = (int)e[2];
  o->status = status == ST_DONE ? PD_OK : (status == ST_BREAKDOWN ? PD_EBREAKDOWN : PD_ENOCONV);
  o->reserved = (int)e[6];
  o->rel_resid = e[3];
  o->dt = e[4];
  o->t = e[5];
}

SolveParams params_from(const pd_time_desc *td, int precision) {
  SolveParams sp;
  sp.theta = td->theta;
  sp.tol = td->tol > 0 ? td->tol : 1e-12;
  sp.maxit = td->max_iters > 0 ? td->max_iters : 5000;
  sp.tol_inner = 1e-3;
  sp.maxit_inner = 400;
  sp.max_outer = precision == PD_MIXED ? 40 : 0;
  sp.max_seconds = td->max_seconds;
  if (td->t_kind == PD_TIME_ADAPTIVE) {
    sp.adaptive = 1;
    sp.T = td->T;
    sp.dt_min = td->dt_min;
    sp.dt_max = td->dt_max;
    sp.tol_time = td->tol_time;
  }
  return sp;
}

int validate_theta(double th) {
  if (!(th > 0.0 && th <= 1.0)) return fail(PD_EINVAL, "theta (implicit weight 1-a) must be in (0, 1], got %g", th);
  return PD_OK;
}

struct BusyGuard {
  std::vector<pd_instance *> v;
  bool ok = true;
  explicit BusyGuard(std::vector<pd_instance *> const &insts) {
    for (auto *I : insts) {
      int z = 0;
      if (!I->busy.compare_exchange_strong(z, 1)) {
        ok = false;
        break;
      }
      v.push_back(I);
    }
  }
  ~BusyGuard() { release(); }
  void release() {
    for (auto *I : v) I->busy = 0;
    v.clear();
  }
};

int solve_many(std::vector<pd_instance *> const &insts, std::vector<const pd_time_desc *> const &tds,
               std::vector<std::vector<double>> *stats) {
  if (insts.empty()) return fail(PD_EINVAL, "no instances");
  BusyGuard g(insts);
  if (!g.ok) return fail(PD_EBUSY, "instance is in use by another call");
  hipStream_t s = insts[0]->stream;
  for (auto *I : insts)
    if (I->stream != s) return fail(PD_EINVAL, "all instances of a batch must share one stream");
  std::vector<int> Ks;
  std::vector<SolveParams> sps;
  for (size_t q = 0; q < insts.size(); ++q) {
    pd_instance *I = insts[q];
    const pd_time_desc *td = tds[q];
    int rc;
    if ((rc = validate_theta(td ? td->theta : -1))) return rc;
    std::vector<double> t;
    if ((rc = build_time_table(td, I->t, t))) return rc;
    if ((rc = ensure_time_capacity(I, td->K))) return rc;
    HIPCHK(hipMemcpyAsync(I->t_table, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, s));
    Ks.push_back(td->K);
    sps.push_back(params_from(td, I->precision));
  }
  // the descriptor array may have been rebuilt (time capacity): it is
  // copied per call in make_plan
  return run_levels(insts, Ks, sps, s, stats);
}

}  // namespace

// ------------------------------------------------------------------ instance set-up
//
// Creating an instance has a host part (mesh, face coefficients, layout
// changes: no device call) and a device part (allocation and uploads), so
// that a serving loop can prepare requests on the submitting thread and
// only upload them when it admits them.

// Host staging of every array an instance uploads.
struct HostImage {
  std::vector<double> inv_rw, inv_dth, r, th;
  std::vector<double> gpr, gmr, gpt, gmt;
  std::vector<float> f_gpr, f_gmr, f_gpt, f_gmt;
  std::vector<double> b_int, g_int, nb, u0_int;
  std::vector<double> crs;   // ring sums of the ring-mean correction (PdInst::crs)
  double lam[PD_MAXSRC] = {0, 0, 0, 0};
  int tp[PD_MAXSRC] = {0, 0, 0, 0};
  bool has_b = false;
};

// The operator ϖ_h of §3.2.1 and the origin row of §3.2.2 as printed (scalar
// E at the nodes, one-sided drift differences), written into the face-pair
// form the kernels apply.  Row (i, j) of the printed stencil, with
// s = h_i + h_{i+1} and the face diffusivities D_{i±1/2,j}, D_{i,j±1/2}:
//   diagonal  2/(r_i s) (r_{i+1/2} D_{i+1/2,j}/h_{i+1} + r_{i-1/2} D_{i-1/2,j}/h_i)
//             + 2/(r_i² (μ_j+μ_{j+1})) (D_{i,j+1/2}/μ_{j+1} + D_{i,j-1/2}/μ_j)
//             + E_ij (1/(r_i μ_{j+1}) + 1/h_{i+1})
//   (i-1, j)  -2 r_{i-1/2} D_{i-1/2,j} / (r_i h_i s)            (the origin for i = 1)
//   (i+1, j)  -(2 r_{i+1/2} D_{i+1/2,j} / (r_i h_{i+1} s) + E_ij/h_{i+1})   (N_j for i = m)
//   (i, j-1)  -2 D_{i,j-1/2} / (r_i² μ_j (μ_j+μ_{j+1}))
//   (i, j+1)  -(2 D_{i,j+1/2} / (r_i² μ_{j+1} (μ_j+μ_{j+1})) + E_ij/(r_i μ_{j+1}))
// and the origin row  (4 D_00/h_1² + E_00/h_1) n_0 - (4 D_00/(n h_1²) - E_00/(n h_1)) Σ_j n_{1,j}.
// A kernel row is ivV_P (Σ_faces gp x_P - gm x_Q) + b_P x_P: every
// off-diagonal coefficient of a row fixes one face coefficient (the one that
// multiplies the neighbour in that row), and what the faces leave of the
// printed diagonal goes into b_P (added to the reaction already in b).
int literal_stencil(const MeshH &M, const std::vector<double> &Dr, const std::vector<double> &Dt,
                    const std::vector<double> &E, double D00, double inv_V0, const std::vector<double> &inv_rw,
                    const std::vector<double> &inv_dth, HostImage &X, std::vector<double> &b) {
  const int m = M.m, n = M.n;
  const std::vector<double> &r = M.r, &h = M.h, &rh = M.rh, &mu = M.mu;
  auto ivV = [&](int i, int j) { return inv_rw[i] * inv_dth[j]; };
  std::fill(X.gpr.begin(), X.gpr.end(), 0.0);
  std::fill(X.gmr.begin(), X.gmr.end(), 0.0);
  std::fill(X.gpt.begin(), X.gpt.end(), 0.0);
  std::fill(X.gmt.begin(), X.gmt.end(), 0.0);
  std::vector<double> diag((size_t)m * n);
  for (int i = 1; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const int jm = (j + n - 1) % n;
      const double Dp = Dr[(size_t)i * n + j], Dm = Dr[(size_t)(i - 1) * n + j];
      const double Dtp = Dt[(size_t)(i - 1) * n + j], Dtm = Dt[(size_t)(i - 1) * n + jm];
      const double mj = mu[j], mj1 = mu[j + 1], e = E[(size_t)(i - 1) * n + j];
      const double s = h[i] + h[i + 1], w = ivV(i, j);
      diag[(size_t)(i - 1) * n + j] = 2.0 / (r[i] * s) * (rh[i] * Dp / h[i + 1] + rh[i - 1] * Dm / h[i]) +
                                      2.0 / (r[i] * r[i] * (mj + mj1)) * (Dtp / mj1 + Dtm / mj) +
                                      e * (1.0 / (r[i] * mj1) + 1.0 / h[i + 1]);
      const double c_in = -2.0 * rh[i - 1] * Dm / (r[i] * h[i] * s);
      const double c_out = -(2.0 * rh[i] * Dp / (r[i] * h[i + 1] * s) + e / h[i + 1]);
      const double c_lo = -2.0 * Dtm / (r[i] * r[i] * mj * (mj + mj1));
      const double c_hi = -(2.0 * Dtp / (r[i] * r[i] * mj1 * (mj + mj1)) + e / (r[i] * mj1));
      X.gpr[(size_t)(i - 1) * n + j] = -c_in / w;    // face i-1/2 times the inner neighbour
      X.gmr[(size_t)i * n + j] = -c_out / w;         // face i+1/2 times the outer neighbour (or N_j)
      X.gmt[(size_t)(i - 1) * n + j] = -c_hi / w;    // face j+1/2 times (i, j+1)
      X.gpt[(size_t)(i - 1) * n + jm] = -c_lo / w;   // face j-1/2 times (i, j-1)
    }
  const double E00 = E[(size_t)m * n], h1 = h[1];
  const double d0 = 4.0 * D00 / (h1 * h1) + E00 / h1;
  const double off = -(4.0 * D00 / (n * h1 * h1) - E00 / (n * h1));
  for (int j = 0; j < n; ++j) X.gmr[j] = -off / inv_V0;   // the origin row times ring 1
  for (int i = 1; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const int jm = (j + n - 1) % n;
      const size_t k = (size_t)(i - 1) * n + j;
      const double faces = X.gpr[(size_t)i * n + j] + X.gmr[(size_t)(i - 1) * n + j] + X.gpt[k] +
                           X.gmt[(size_t)(i - 1) * n + jm];
      b[k] += diag[k] - ivV(i, j) * faces;
    }
  double s0 = 0.0;
  for (int j = 0; j < n; ++j) s0 += X.gpr[j];
  b[(size_t)m * n] += d0 - inv_V0 * s0;
  for (double v : b)
    if (!std::isfinite(v)) return fail(PD_EINVAL, "the printed stencil gave a non-finite coefficient");
  return PD_OK;
}

int prepare_instance(const pd_mesh_desc *mesh, const pd_problem_desc *pb, int32_t precision,
                     std::unique_ptr<pd_instance> &out, std::unique_ptr<HostImage> &img_out) {
  if (!pb) return fail(PD_EINVAL, "problem descriptor is NULL");
  if (precision != PD_FP64 && precision != PD_MIXED) return fail(PD_EINVAL, "unknown precision %d", precision);
  if (pb->nsrc < 0 || pb->nsrc > PD_MAXSRC) return fail(PD_EINVAL, "nsrc must be in [0, %d]", PD_MAXSRC);
  if (pb->flux < 0 || pb->flux > 2) return fail(PD_EINVAL, "flux must be 0, 1 or 2");
  if (pb->flux == 2 && pb->bc != 0) return fail(PD_EINVAL, "the printed stencil (flux 2) takes Dirichlet data only");
  if (pb->flux == 2 && !pb->E_node) return fail(PD_EINVAL, "the printed stencil (flux 2) needs E_node");
  if (pb->bc != 0 && pb->bc != 1) return fail(PD_EINVAL, "bc must be 0 or 1");
  if (pb->layout != PD_LAYOUT_RING && pb->layout != PD_LAYOUT_PAPER) return fail(PD_EINVAL, "bad layout");
  std::unique_ptr<pd_instance> I(new pd_instance);
  std::unique_ptr<HostImage> img(new HostImage);
  HostImage &X = *img;
  int rc = build_mesh(mesh, I->M);
  if (rc) return rc;
  const int m = I->M.m, n = I->M.n, N = m * n + 1;
  I->T = make_tiling(m, n);
  I->precision = precision;
  I->pde = pb->pde;
  I->flux = pb->flux;
  I->bc = pb->bc;
  I->nsrc = pb->nsrc;
  const MeshH &M = I->M;
  const int np = I->T.npad;
  std::vector<double> Dr, Er, Dt, Et, bn, g, u0;
  const int dp = pb->device_ptrs;
  if (pb->D_rface) { if ((rc = fetch(pb->D_rface, (size_t)(m + 1) * n, dp, Dr))) return rc; }
  else Dr.assign((size_t)(m + 1) * n, 1.0);
  if (pb->Er_rface) { if ((rc = fetch(pb->Er_rface, (size_t)(m + 1) * n, dp, Er))) return rc; }
  else Er.assign((size_t)(m + 1) * n, 0.0);
  if (pb->D_tface) { if ((rc = fetch(pb->D_tface, (size_t)m * n, dp, Dt))) return rc; }
  else Dt.assign((size_t)m * n, 1.0);
  if (pb->Et_tface) { if ((rc = fetch(pb->Et_tface, (size_t)m * n, dp, Et))) return rc; }
  else Et.assign((size_t)m * n, 0.0);
  I->zero_drift = std::all_of(Er.begin(), Er.end(), [](double v) { return v == 0.0; }) &&
                  std::all_of(Et.begin(), Et.end(), [](double v) { return v == 0.0; });
  if ((rc = fetch(pb->u0, N, dp, u0))) return rc;
  if (pb->nsrc > 0) {
    if (!pb->lambda) return fail(PD_EINVAL, "lambda is NULL");
    if ((rc = fetch(pb->g, (size_t)pb->nsrc * N, dp, g))) return rc;
    if (pb->nb) { if ((rc = fetch(pb->nb, (size_t)pb->nsrc * n, dp, X.nb))) return rc; }
    else X.nb.assign((size_t)pb->nsrc * n, 0.0);
    std::vector<double> lam;
    if ((rc = fetch(pb->lambda, (size_t)pb->nsrc, dp, lam))) return rc;
    int32_t tp[PD_MAXSRC] = {0, 0, 0, 0};
    if (pb->tpow) {
      if (dp) {
        HIPCHK(hipMemcpy(tp, pb->tpow, pb->nsrc * sizeof(int32_t), hipMemcpyDeviceToHost));
      } else {
        std::memcpy(tp, pb->tpow, pb->nsrc * sizeof(int32_t));
      }
    }
    for (int q = 0; q < pb->nsrc; ++q) {
      X.lam[q] = lam[q];
      X.tp[q] = tp[q];
      if (X.tp[q] < 0 || X.tp[q] > 8) return fail(PD_EINVAL, "tpow must be in [0, 8]");
    }
    I->lam_h.assign(X.lam, X.lam + pb->nsrc);
    I->tp_h.assign(X.tp, X.tp + pb->nsrc);
  }
  X.has_b = pb->b_node != nullptr;
  if (X.has_b && (rc = fetch(pb->b_node, N, dp, bn))) return rc;
  for (double v : Dr) if (!std::isfinite(v) || v < 0) return fail(PD_EINVAL, "D_rface must be finite and >= 0");
  for (double v : Dt) if (!std::isfinite(v) || v < 0) return fail(PD_EINVAL, "D_tface must be finite and >= 0");
  for (double v : u0) if (!std::isfinite(v)) return fail(PD_EINVAL, "u0 has a non-finite value");
  // faces
  X.gpr.resize((size_t)(m + 1) * n);
  X.gmr.resize((size_t)(m + 1) * n);
  X.gpt.resize((size_t)m * n);
  X.gmt.resize((size_t)m * n);
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t k = (size_t)i * n + j;
      const double area = M.rh[i] * M.dth[j];
      double G = Dr[k] * area / M.h[i + 1], K = Er[k] * area;
      if (i == m && I->bc == 1) G = K = 0.0;
      face_pair(G, K, I->flux, X.gpr[k], X.gmr[k]);
    }
  for (int i = 1; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t k = (size_t)(i - 1) * n + j;
      const double G = Dt[k] * M.w[i] / (M.r[i] * M.mu[j + 1]);
      const double K = Et[k] * M.w[i];
      face_pair(G, K, I->flux, X.gpt[k], X.gmt[k]);
    }
  X.inv_rw.assign(m + 2, 0.0);
  X.inv_dth.resize(n);
  for (int i = 1; i <= m; ++i) X.inv_rw[i] = 1.0 / (M.r[i] * M.w[i]);
  for (int j = 0; j < n; ++j) X.inv_dth[j] = 1.0 / M.dth[j];
  I->H.inv_V0 = 1.0 / (kPi * 0.25 * M.h[1] * M.h[1]);
  if (pb->flux == 2) {
    std::vector<double> En;
    if ((rc = fetch(pb->E_node, N, dp, En))) return rc;
    std::vector<double> E_int(np, 0.0), b_lit;
    to_internal(En.data(), pb->layout, m, n, np, E_int.data());
    if (X.has_b) {
      b_lit.resize(np);
      to_internal(bn.data(), pb->layout, m, n, np, b_lit.data());
    } else {
      b_lit.assign(np, 0.0);
    }
    if ((rc = literal_stencil(M, Dr, Dt, E_int, pb->D_origin, I->H.inv_V0, X.inv_rw, X.inv_dth, X, b_lit)))
      return rc;
    // the literal rows' diagonals live in the node reaction term
    X.has_b = true;
    bn.assign(N, 0.0);
    from_internal(b_lit.data(), pb->layout, m, n, bn.data());
  }
  X.r = M.r;
  X.th = M.th;
  if (precision == PD_MIXED) {
    X.f_gpr.assign(X.gpr.begin(), X.gpr.end());
    X.f_gmr.assign(X.gmr.begin(), X.gmr.end());
    X.f_gpt.assign(X.gpt.begin(), X.gpt.end());
    X.f_gmt.assign(X.gmt.begin(), X.gmt.end());
  }
  if (X.has_b) {
    X.b_int.resize(np);
    to_internal(bn.data(), pb->layout, m, n, np, X.b_int.data());
  }
  X.g_int.resize((size_t)pb->nsrc * np);
  for (int q = 0; q < pb->nsrc; ++q)
    to_internal(g.data() + (size_t)q * N, pb->layout, m, n, np, X.g_int.data() + (size_t)q * np);
  X.u0_int.resize(np);
  to_internal(u0.data(), pb->layout, m, n, np, X.u0_int.data());
  {
    // diagonal of L at the origin, with the ring-1 faces summed in order
    double s0 = 0.0;
    for (int j = 0; j < n; ++j) s0 += X.gpr[j];
    const double b0 = X.has_b ? X.b_int[m * n] : 0.0;
    I->H.l0 = std::fma(I->H.inv_V0, s0, b0);
    I->b0 = b0;
  }
  {
    // ring sums of the ring-mean (Galerkin) correction: with P the
    // prolongation of ring values to their nodes and V the cell volumes
    // (those the stencil divides by), P^T V (I/dt + θ L) P is tridiagonal:
    //   row i: (Σ V)/dt + θ (Σ V b + Σ gp_r(i+1/2) + Σ gm_r(i-1/2)) on the
    //   diagonal, -θ Σ gm_r(i+1/2) above and -θ Σ gp_r(i-1/2) below (the
    //   angular fluxes of a ring-constant vector cancel around the ring)
    const int M1 = m + 1;
    X.crs.assign(6 * (size_t)M1, 0.0);
    double *cV = &X.crs[0], *cB = &X.crs[M1], *cO = &X.crs[2 * M1], *cI = &X.crs[3 * M1];
    double *cU = &X.crs[4 * M1], *cL = &X.crs[5 * M1];
    const double V0 = 1.0 / I->H.inv_V0;
    cV[0] = V0;
    cB[0] = V0 * (X.has_b ? X.b_int[m * n] : 0.0);
    for (int i = 1; i <= m; ++i)
      for (int j = 0; j < n; ++j) {
        const double V = 1.0 / (X.inv_rw[i] * X.inv_dth[j]);
        cV[i] += V;
        if (X.has_b) cB[i] += V * X.b_int[(size_t)(i - 1) * n + j];
      }
    for (int i = 0; i <= m; ++i)
      for (int j = 0; j < n; ++j) {
        cO[i] += X.gpr[(size_t)i * n + j];
        if (i < m) cU[i] += X.gmr[(size_t)i * n + j];
        if (i >= 1) {
          cI[i] += X.gmr[(size_t)(i - 1) * n + j];
          cL[i] += X.gpr[(size_t)(i - 1) * n + j];
        }
      }
  }
  out = std::move(I);
  img_out = std::move(img);
  return PD_OK;
}

// Device allocation and uploads of a prepared instance on I->stream
// (returns once the uploads are done; the image may then be dropped).
// mem: device memory of at least instance_bytes(I) to carve into, or NULL
// to allocate it.
int upload_instance(pd_instance *I, const HostImage &X, void *mem = nullptr) {
  const int m = I->M.m, n = I->M.n;
  const int np = I->T.npad;
  Carver dry{nullptr, 0, true};
  carve(I, dry);
  I->dbytes = dry.off;
  if (mem) {
    I->dmem = mem;
  } else {
    hipError_t e = hipMalloc(&I->dmem, I->dbytes);
    if (e != hipSuccess) {
      I->dmem = nullptr;
      return fail(e == hipErrorOutOfMemory ? PD_ENOMEM : PD_EHIP, "device allocation of %zu bytes failed: %s",
                  I->dbytes, hipGetErrorString(e));
    }
  }
  hipStream_t s = I->stream;
  HIPCHK(hipMemsetAsync(I->dmem, 0, I->dbytes, s));
  Carver cv{(char *)I->dmem, 0, false};
  carve(I, cv);
  PdInst &H = I->H;
  H.m = m;
  H.n = n;
  H.npad = np;
  H.nsrc = I->nsrc;
  H.mixed = I->precision == PD_MIXED;
  H.has_b = X.has_b;
  H.zero_flux = I->bc;
  H.rb = I->T.rb;
  H.ncg = I->T.ncg;
  H.nrg = I->T.nrg;
  H.nb_sten = I->T.nb_sten;
  H.nb_elem = I->T.nb_elem;
  H.cw = I->T.cw;
  H.nseg = I->T.nseg;
  H.brad = I->T.brad;
  H.nb_rad = I->T.nb_rad;
  H.bang = I->T.bang;
  H.aw = I->T.aw;
  H.nb_ang = I->T.nb_ang;
  H.nb_frad = I->T.nb_frad;
  H.nb_fang = I->T.nb_fang;
  if (!X.has_b) H.b_node = nullptr;
  auto up = [&](const void *dst, const void *src, size_t bytes) -> int {
    if (bytes == 0) return PD_OK;
    HIPCHK(hipMemcpyAsync(const_cast<void *>(dst), src, bytes, hipMemcpyHostToDevice, s));
    return PD_OK;
  };
  int rc;
  if ((rc = up(H.inv_rw, X.inv_rw.data(), X.inv_rw.size() * 8))) return rc;
  if ((rc = up(H.inv_dth, X.inv_dth.data(), X.inv_dth.size() * 8))) return rc;
  if ((rc = up(H.r_nodes, X.r.data(), X.r.size() * 8))) return rc;
  if ((rc = up(H.th_nodes, X.th.data(), X.th.size() * 8))) return rc;
  if ((rc = up(H.k64.gp_r, X.gpr.data(), X.gpr.size() * 8))) return rc;
  if ((rc = up(H.k64.gm_r, X.gmr.data(), X.gmr.size() * 8))) return rc;
  if ((rc = up(H.k64.gp_t, X.gpt.data(), X.gpt.size() * 8))) return rc;
  if ((rc = up(H.k64.gm_t, X.gmt.data(), X.gmt.size() * 8))) return rc;
  if ((rc = up(H.crs, X.crs.data(), X.crs.size() * 8))) return rc;
  if (H.mixed) {
    if ((rc = up(H.k32.gp_r, X.f_gpr.data(), X.f_gpr.size() * 4))) return rc;
    if ((rc = up(H.k32.gm_r, X.f_gmr.data(), X.f_gmr.size() * 4))) return rc;
    if ((rc = up(H.k32.gp_t, X.f_gpt.data(), X.f_gpt.size() * 4))) return rc;
    if ((rc = up(H.k32.gm_t, X.f_gmt.data(), X.f_gmt.size() * 4))) return rc;
  }
  if (X.has_b && (rc = up(H.b_node, X.b_int.data(), (size_t)np * 8))) return rc;
  if ((rc = up(H.g, X.g_int.data(), X.g_int.size() * 8))) return rc;
  if (I->nsrc > 0) {
    if ((rc = up(H.nb, X.nb.data(), X.nb.size() * 8))) return rc;
    if ((rc = up(H.lam, X.lam, sizeof X.lam))) return rc;
    if ((rc = up(H.tpow, X.tp, sizeof X.tp))) return rc;
  }
  I->rot = 0;
  if ((rc = up(H.sol[sol_slot(0, 0)], X.u0_int.data(), (size_t)np * 8))) return rc;
  if ((rc = ensure_time_capacity(I, 16))) return rc;
  HIPCHK(hipStreamSynchronize(s));
  I->t = 0.0;
  return PD_OK;
}

// ================================================================== C ABI

extern "C" {

const char *pd_last_error(void) { return g_err.c_str(); }

int pd_set_schedule(const pd_schedule *sc) {
  if (!sc) {
    g_sched_groups = 1;
    g_sched_cpg = 2;
    g_sched_rings = PD_RB;
    return PD_OK;
  }
  if (sc->groups < 1 || sc->groups > 8) return fail(PD_EINVAL, "groups must be in [1, 8]");
  if (sc->cycles_per_graph < 1 || sc->cycles_per_graph > 16)
    return fail(PD_EINVAL, "cycles_per_graph must be in [1, 16]");
  if (sc->stencil_rings != 0 && sc->stencil_rings != PD_RB && sc->stencil_rings != 2 * PD_RB)
    return fail(PD_EINVAL, "stencil_rings must be 0, %d or %d", PD_RB, 2 * PD_RB);
  g_sched_groups = sc->groups;
  g_sched_cpg = sc->cycles_per_graph;
  g_sched_rings = sc->stencil_rings ? sc->stencil_rings : PD_RB;
  return PD_OK;
}

int pd_set_preconditioner(pd_instance *I, int32_t kind) {
  if (!I) return fail(PD_EINVAL, "instance is NULL");
  if (kind != PD_PRECOND_LINE && kind != PD_PRECOND_MG) return fail(PD_EINVAL, "unknown preconditioner %d", kind);
  if (kind == PD_PRECOND_MG && I->precision != PD_FP64)
    return fail(PD_EINVAL, "the multigrid preconditioner takes FP64 instances");
  BusyGuard g({I});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  I->precond = kind;
  if (kind == PD_PRECOND_LINE) {
    if (I->stream) HIPCHK(hipStreamSynchronize(I->stream));
    mg_free(I);
  }
  return PD_OK;
}

int pd_get_schedule(pd_schedule *sc) {
  if (!sc) return fail(PD_EINVAL, "NULL argument");
  sc->groups = g_sched_groups.load();
  sc->cycles_per_graph = g_sched_cpg.load();
  sc->stencil_rings = g_sched_rings.load();
  return PD_OK;
}

int pd_time_levels(const pd_time_desc *td, double t_start, double *out) {
  try {
    if (!out) return fail(PD_EINVAL, "output buffer is NULL");
    std::vector<double> t;
    int rc = build_time_table(td, t_start, t);
    if (rc) return rc;
    std::copy(t.begin(), t.end(), out);
    return PD_OK;
  } catch (...) {
    return fail(PD_EINVAL, "unexpected host exception");
  }
}

int pd_mesh_coords(const pd_mesh_desc *mesh, double *r_nodes, double *r_faces, double *th_nodes,
                   double *th_faces) {
  MeshH M;
  int rc = build_mesh(mesh, M);
  if (rc) return rc;
  if (r_nodes) std::copy(M.r.begin(), M.r.end(), r_nodes);
  if (r_faces) std::copy(M.rh.begin(), M.rh.end(), r_faces);
  if (th_nodes) std::copy(M.th.begin(), M.th.end(), th_nodes);
  if (th_faces)
    for (int j = 0; j < M.n; ++j) th_faces[j] = 0.5 * (M.th[j] + M.th[j + 1]);
  return PD_OK;
}

int pd_footprint(const pd_mesh_desc *mesh, int32_t nsrc, int32_t precision, size_t *bytes) {
  if (!bytes) return fail(PD_EINVAL, "bytes is NULL");
  int rc = check_mesh(mesh);
  if (rc) return rc;
  pd_instance tmp;
  tmp.M.m = mesh->nr;
  tmp.M.n = mesh->ntheta;
  tmp.T = make_tiling(mesh->nr, mesh->ntheta);
  tmp.nsrc = nsrc;
  tmp.precision = precision;
  Carver c{nullptr, 0, true};
  carve(&tmp, c);
  *bytes = c.off + 8 * 1024;   // + time table / stats for short runs
  return PD_OK;
}

int pd_mesh_create(const pd_mesh_desc *mesh, const pd_problem_desc *pb, int32_t precision,
                   void *hip_stream, pd_instance **out) {
  if (!out) return fail(PD_EINVAL, "out is NULL");
  *out = nullptr;
  std::unique_ptr<pd_instance> I;
  std::unique_ptr<HostImage> img;
  int rc = prepare_instance(mesh, pb, precision, I, img);
  if (rc) return rc;
  HIPCHK(hipGetDevice(&I->device));
  if (hip_stream) {
    I->stream = (hipStream_t)hip_stream;
  } else {
    // one library-owned stream per device for every instance created
    // without a stream, so that such instances can be batched together
    static std::mutex mu;
    static std::map<int, hipStream_t> shared;
    std::lock_guard<std::mutex> lk(mu);
    auto it = shared.find(I->device);
    if (it == shared.end()) {
      hipStream_t st;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      it = shared.emplace(I->device, st).first;
    }
    I->stream = it->second;
    I->own_stream = false;
  }
  if ((rc = upload_instance(I.get(), *img))) {
    if (I->dmem) (void)hipFree(I->dmem);
    if (I->t_table) (void)hipFree(I->t_table);
    if (I->stats) (void)hipFree(I->stats);
    return rc;
  }
  *out = I.release();
  return PD_OK;
}

int pd_destroy(pd_instance *I) {
  if (!I) return PD_OK;
  if (I->busy) return fail(PD_EBUSY, "instance is in use");
  if (I->stream) (void)hipStreamSynchronize(I->stream);
  if (I->drift) (void)hipFree(I->drift);
  mg_free(I);
  if (!I->arena) {          // a serving arena takes its chunk back itself
    if (I->dmem) (void)hipFree(I->dmem);
    if (I->t_table) (void)hipFree(I->t_table);
    if (I->stats) (void)hipFree(I->stats);
  }
  if (I->own_stream) (void)hipStreamDestroy(I->stream);
  delete I;
  return PD_OK;
}

int pd_solve_to_T(pd_instance *I, const pd_time_desc *td, pd_step_stats *per_step) {
  if (!I) return fail(PD_EINVAL, "instance is NULL");
  std::vector<std::vector<double>> st(1);
  int rc = solve_many({I}, {td}, &st);
  if (per_step && !st[0].empty())
    for (int k = 0; k < td->K; ++k) fill_stats(st[0], k, per_step + k);
  return rc;
}

int pd_scheme_step(pd_instance *I, double t_k, double dt, double theta, double tol, pd_step_stats *stats) {
  if (!I) return fail(PD_EINVAL, "instance is NULL");
  if (!(dt > 0.0)) return fail(PD_EINVAL, "dt must be > 0");
  double tab[2] = {t_k, t_k + dt};
  pd_time_desc td{};
  td.t_kind = PD_TIME_TABLE;
  td.K = 1;
  td.t_table = tab;
  td.theta = theta;
  td.tol = tol;
  return pd_solve_to_T(I, &td, stats);
}

int pd_solve_batch(pd_instance *const *insts, int32_t count, const pd_time_desc *times,
                   pd_step_stats *const *per_step) {
  if (!insts || count <= 0 || !times) return fail(PD_EINVAL, "empty batch");
  std::vector<pd_instance *> v(insts, insts + count);
  std::vector<const pd_time_desc *> tds;
  for (int q = 0; q < count; ++q) {
    if (!v[q]) return fail(PD_EINVAL, "instance %d is NULL", q);
    tds.push_back(times + q);
  }
  std::vector<std::vector<double>> st(count);
  int rc = solve_many(v, tds, &st);
  if (per_step)
    for (int q = 0; q < count; ++q)
      if (per_step[q] && !st[q].empty())
        for (int k = 0; k < times[q].K; ++k) fill_stats(st[q], k, per_step[q] + k);
  return rc;
}

int pd_kernel_timing(int32_t enable, int32_t reset, double *total_ms, int64_t *launches) {
  if (enable && !g_event_timer) g_event_timer = new EventTimer;
  if (g_event_timer) {
    if (total_ms)
      for (int k = 0; k < PD_KF_N; ++k) total_ms[k] = g_event_timer->total_ms[k];
    if (launches)
      for (int k = 0; k < PD_KF_N; ++k) launches[k] = g_event_timer->launches[k];
    if (reset) g_event_timer->reset();
  } else {
    if (total_ms)
      for (int k = 0; k < PD_KF_N; ++k) total_ms[k] = 0;
    if (launches)
      for (int k = 0; k < PD_KF_N; ++k) launches[k] = 0;
  }
  pd::g_timer = enable ? g_event_timer : nullptr;
  return PD_OK;
}

int pd_get_solution(const pd_instance *I, double *out, int32_t layout, int32_t device_ptr) {
  if (!I || !out) return fail(PD_EINVAL, "NULL argument");
  if (layout != PD_LAYOUT_RING && layout != PD_LAYOUT_PAPER) return fail(PD_EINVAL, "bad layout");
  const int m = I->M.m, n = I->M.n, N = m * n + 1;
  std::vector<double> h(I->T.npad), o(N);
  HIPCHK(hipStreamSynchronize(I->stream));
  HIPCHK(hipMemcpy(h.data(), I->H.sol[sol_slot(I->rot, 0)], I->T.npad * sizeof(double), hipMemcpyDeviceToHost));
  from_internal(h.data(), layout, m, n, o.data());
  if (device_ptr) {
    HIPCHK(hipMemcpy(out, o.data(), N * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::memcpy(out, o.data(), N * sizeof(double));
  }
  return PD_OK;
}

int pd_get_time(const pd_instance *I, double *t) {
  if (!I || !t) return fail(PD_EINVAL, "NULL argument");
  *t = I->t;
  return PD_OK;
}

int pd_set_solution(pd_instance *I, const double *in, int32_t layout, int32_t device_ptr, double t) {
  if (!I || !in) return fail(PD_EINVAL, "NULL argument");
  if (layout != PD_LAYOUT_RING && layout != PD_LAYOUT_PAPER) return fail(PD_EINVAL, "bad layout");
  if (I->busy) return fail(PD_EBUSY, "instance is in use");
  const int m = I->M.m, n = I->M.n, N = m * n + 1;
  std::vector<double> src;
  int rc = fetch(in, N, device_ptr, src);
  if (rc) return rc;
  std::vector<double> h(I->T.npad);
  to_internal(src.data(), layout, m, n, I->T.npad, h.data());
  HIPCHK(hipMemcpy(I->H.sol[sol_slot(I->rot, 0)], h.data(), I->T.npad * sizeof(double), hipMemcpyHostToDevice));
  I->t = t;
  I->have_prev = false;
  return PD_OK;
}

int pd_apply_operator(pd_instance *I, double dt, double theta, const double *x, double *y, int32_t layout,
                      int32_t device_ptrs, int32_t precision) {
  if (!I || !x || !y) return fail(PD_EINVAL, "NULL argument");
  if (!(dt > 0.0)) return fail(PD_EINVAL, "dt must be > 0");
  int rc = validate_theta(theta);
  if (rc) return rc;
  if (precision == 1 && I->precision != PD_MIXED)
    return fail(PD_EINVAL, "the FP32 stencil needs a mixed-precision instance");
  const int m = I->M.m, n = I->M.n, N = m * n + 1, np = I->T.npad;
  std::vector<double> src;
  if ((rc = fetch(x, N, device_ptrs, src))) return rc;
  std::vector<double> hin(np), hout(np), o(N);
  to_internal(src.data(), layout, m, n, np, hin.data());
  hipStream_t s = I->stream;
  void *dx = nullptr, *dy = nullptr;
  const size_t es = precision == 1 ? 4 : 8;
  HIPCHK(hipMalloc(&dx, np * es));
  HIPCHK(hipMalloc(&dy, np * es));
  std::vector<float> fin, fout;
  if (precision == 1) {
    fin.assign(hin.begin(), hin.end());
    HIPCHK(hipMemcpy(dx, fin.data(), np * 4, hipMemcpyHostToDevice));
  } else {
    HIPCHK(hipMemcpy(dx, hin.data(), np * 8, hipMemcpyHostToDevice));
  }
  Plan P;
  if ((rc = make_plan({I}, s, P))) return rc;
  pd::launch_apply(P.L, dt, theta, dx, dy, precision == 1, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (precision == 1) {
    fout.resize(np);
    HIPCHK(hipMemcpy(fout.data(), dy, np * 4, hipMemcpyDeviceToHost));
    for (int k = 0; k < np; ++k) hout[k] = fout[k];
  } else {
    HIPCHK(hipMemcpy(hout.data(), dy, np * 8, hipMemcpyDeviceToHost));
  }
  (void)hipFree(dx);
  (void)hipFree(dy);
  from_internal(hout.data(), layout, m, n, o.data());
  if (device_ptrs) {
    HIPCHK(hipMemcpy(y, o.data(), N * 8, hipMemcpyHostToDevice));
  } else {
    std::memcpy(y, o.data(), N * 8);
  }
  return PD_OK;
}

int pd_assemble_rhs(pd_instance *I, double t_k, double dt, double theta, double *rhs, int32_t layout,
                    int32_t device_ptr) {
  if (!I || !rhs) return fail(PD_EINVAL, "NULL argument");
  if (!(dt > 0.0)) return fail(PD_EINVAL, "dt must be > 0");
  int rc = validate_theta(theta);
  if (rc) return rc;
  BusyGuard g({I});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  hipStream_t s = I->stream;
  // one level whose Krylov phase is skipped: the begin kernel leaves the
  // right-hand side in bvec; the state is not advanced
  double tab[2] = {t_k, t_k + dt};
  if ((rc = ensure_time_capacity(I, 1))) return rc;
  HIPCHK(hipMemcpyAsync(I->t_table, tab, sizeof tab, hipMemcpyHostToDevice, s));
  Plan P;
  if ((rc = make_plan({I}, s, P))) return rc;
  SolveParams sp{theta, 1e-300, 1e-3, 1, 1, 1};
  if ((rc = init_scalars(I, sp, 1, s))) return rc;
  pd::launch_level_begin(P.L, s);
  pd::launch_factor(P.L, s);
  pd::launch_begin(P.L, s);
  pd::launch_begin_origin(P.L, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  const int m = I->M.m, n = I->M.n, N = m * n + 1;
  std::vector<double> h(I->T.npad), o(N);
  HIPCHK(hipMemcpy(h.data(), I->H.bvec, I->T.npad * 8, hipMemcpyDeviceToHost));
  from_internal(h.data(), layout, m, n, o.data());
  if (device_ptr) {
    HIPCHK(hipMemcpy(rhs, o.data(), N * 8, hipMemcpyHostToDevice));
  } else {
    std::memcpy(rhs, o.data(), N * 8);
  }
  return PD_OK;
}

// ------------------------------------------------------------ two carriers

int pd_set_mobility(pd_instance *I, const double *mu_rface, const double *mu_tface, double sign,
                    int32_t device_ptrs) {
  if (!I || !mu_rface || !mu_tface) return fail(PD_EINVAL, "NULL argument");
  if (I->precision != PD_FP64) return fail(PD_EINVAL, "a carrier of the coupled system must be an FP64 instance");
  if (I->flux != 0 && I->flux != 1) return fail(PD_EINVAL, "a carrier takes the central or upwind flux (0 or 1)");
  if (!I->zero_drift) return fail(PD_EINVAL, "a carrier must be created without drift (Er_rface = Et_tface = 0)");
  if (sign != 1.0 && sign != -1.0) return fail(PD_EINVAL, "sign must be +1 (holes) or -1 (electrons)");
  BusyGuard g({I});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  const MeshH &M = I->M;
  const int m = M.m, n = M.n;
  const size_t nr = (size_t)(m + 1) * n, nt = (size_t)m * n;
  std::vector<double> mr, mt;
  int rc = fetch(mu_rface, nr, device_ptrs, mr);
  if (rc || (rc = fetch(mu_tface, nt, device_ptrs, mt))) return rc;
  for (double v : mr) if (!std::isfinite(v) || v < 0) return fail(PD_EINVAL, "mu_rface must be finite and >= 0");
  for (double v : mt) if (!std::isfinite(v) || v < 0) return fail(PD_EINVAL, "mu_tface must be finite and >= 0");
  // c = s μ (face length) / (node distance), so that the face's drift
  // coefficient is K = c (ψ_P - ψ_Q); the outer faces of a zero-flux
  // carrier carry nothing
  std::vector<double> c(nr + nt);
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t k = (size_t)i * n + j;
      c[k] = (i == m && I->bc == 1) ? 0.0 : sign * mr[k] * (M.rh[i] * M.dth[j]) / M.h[i + 1];
    }
  for (int i = 1; i <= m; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t k = (size_t)(i - 1) * n + j;
      c[nr + k] = sign * mt[k] * M.w[i] / (M.r[i] * M.mu[j + 1]);
    }
  if (!I->drift) HIPCHK(hipMalloc(&I->drift, 2 * (nr + nt) * sizeof(double)));
  double *G_r = I->drift, *c_r = G_r + nr, *G_t = c_r + nr, *c_t = G_t + nt;
  // created without drift, the faces hold the conductances: gp = gm = G
  HIPCHK(hipMemcpy(G_r, I->H.k64.gp_r, nr * sizeof(double), hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(G_t, I->H.k64.gp_t, nt * sizeof(double), hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(c_r, c.data(), nr * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c_t, c.data() + nr, nt * sizeof(double), hipMemcpyHostToDevice));
  return PD_OK;
}

namespace {
constexpr double kSteadyDt = 1e30;   // a level this long is the steady problem (θ = 1)

bool same_mesh(const pd_instance *a, const pd_instance *b) {
  return a->M.m == b->M.m && a->M.n == b->M.n && a->M.r == b->M.r && a->M.th == b->M.th;
}

// The carrier's faces from the potential's state, then its ring sums and
// origin diagonal (read back into the descriptor the next plans copy).
int drift_from(pd_instance *C, pd_instance *P, double *l0_dev) {
  const int m = C->M.m, n = C->M.n;
  const size_t nr = (size_t)(m + 1) * n, nt = (size_t)m * n;
  const double *G_r = C->drift, *c_r = G_r + nr, *G_t = c_r + nr, *c_t = G_t + nt;
  PdInst &H = C->H;
  pd::launch_drift(m, n, C->flux, G_r, c_r, G_t, c_t, P->H.sol[sol_slot(P->rot, 0)], P->H.nb, P->H.lam, P->H.tpow,
                   P->nsrc, const_cast<double *>(H.k64.gp_r), const_cast<double *>(H.k64.gm_r),
                   const_cast<double *>(H.k64.gp_t), const_cast<double *>(H.k64.gm_t), const_cast<double *>(H.crs),
                   H.inv_V0, C->b0, l0_dev, C->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(&H.l0, l0_dev, sizeof(double), hipMemcpyDeviceToHost, C->stream));
  HIPCHK(hipStreamSynchronize(C->stream));
  return PD_OK;
}
}  // namespace

int pd_gummel_step(pd_instance *psi, pd_instance *ne, pd_instance *pe, double t_k, double dt, double theta,
                   double tol, double gummel_tol, int32_t max_gummel, pd_gummel_stats *stats) {
  if (!psi || !ne || !pe) return fail(PD_EINVAL, "instance is NULL");
  if (psi == ne || psi == pe || ne == pe) return fail(PD_EINVAL, "the potential and the carriers must be three instances");
  if (!(dt > 0.0)) return fail(PD_EINVAL, "dt must be > 0");
  int rc = validate_theta(theta);
  if (rc) return rc;
  if (max_gummel < 1 || !(gummel_tol >= 0.0)) return fail(PD_EINVAL, "max_gummel must be >= 1 and gummel_tol >= 0");
  if (psi->precision != PD_FP64) return fail(PD_EINVAL, "the potential must be an FP64 instance");
  if (!ne->drift || !pe->drift) return fail(PD_EINVAL, "pd_set_mobility has not been called for both carriers");
  if (!same_mesh(psi, ne) || !same_mesh(psi, pe)) return fail(PD_EINVAL, "the three instances must share one mesh");
  if (psi->bc != 0) return fail(PD_EINVAL, "the potential takes Dirichlet data");
  if (psi->nsrc < 1) return fail(PD_EINVAL, "the potential needs its charge slot (source mode 0)");
  for (int q = 0; q < psi->nsrc; ++q)
    if (psi->lam_h[q] != 0.0 || psi->tp_h[q] != 0)
      return fail(PD_EINVAL, "the potential's sources and boundary data must be steady (lambda = 0, tpow = 0)");
  if (ne->stream != pe->stream) return fail(PD_EINVAL, "the two carriers must share one stream");
  for (const pd_instance *C : {ne, pe})
    if (std::fabs(C->t - t_k) > 1e-12 * std::max(1.0, std::fabs(t_k)))
      return fail(PD_EINVAL, "the step starts at %g but a carrier is at t = %g", t_k, C->t);
  BusyGuard g({psi, ne, pe});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  const int np = psi->T.npad;
  const int nblk = std::max(1, std::min(1024, (np + 2047) / 2048));
  double *tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, (3 * (size_t)np + 2 * nblk + 4) * sizeof(double)));
  struct Free { double *p; ~Free() { if (p) (void)hipFree(p); } } fr{tmp};
  double *n0 = tmp, *p0 = n0 + np, *prev = p0 + np, *part = prev + np, *out = part + 2 * nblk, *l0 = out + 2;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(n0, ne->H.sol[sol_slot(ne->rot, 0)], np * sizeof(double), hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(p0, pe->H.sol[sol_slot(pe->rot, 0)], np * sizeof(double), hipMemcpyDeviceToDevice));
  double tab_c[2] = {t_k, t_k + dt}, tab_p[2] = {0.0, kSteadyDt};
  pd_time_desc tdc{}, tdp{};
  tdc.t_kind = tdp.t_kind = PD_TIME_TABLE;
  tdc.K = tdp.K = 1;
  tdc.t_table = tab_c;
  tdp.t_table = tab_p;
  tdc.theta = theta;
  tdp.theta = 1.0;
  tdc.tol = tdp.tol = tol;
  int it = 0, krylov = 0;
  double change = 0.0;
  g.release();   // each solve below takes the instances itself
  for (; it < max_gummel; ++it) {
    // ψ from the charge p - n (the potential's source mode 0)
    double *charge = const_cast<double *>(psi->H.g);
    pd::launch_sub(pe->H.sol[sol_slot(pe->rot, 0)], ne->H.sol[sol_slot(ne->rot, 0)], charge, np, psi->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(prev, psi->H.sol[sol_slot(psi->rot, 0)], np * sizeof(double), hipMemcpyDeviceToDevice,
                          psi->stream));
    HIPCHK(hipStreamSynchronize(psi->stream));
    psi->t = 0.0;     // every steady solve is the level [0, kSteadyDt] from the last potential
    std::vector<std::vector<double>> st(1);
    if ((rc = solve_many({psi}, {&tdp}, &st))) return rc;
    krylov += (int)st[0][0];
    pd::launch_maxdiff(psi->H.sol[sol_slot(psi->rot, 0)], prev, np, part, nblk, out, psi->stream);
    HIPCHK(hipGetLastError());
    double hd[2];
    HIPCHK(hipMemcpyAsync(hd, out, sizeof hd, hipMemcpyDeviceToHost, psi->stream));
    HIPCHK(hipStreamSynchronize(psi->stream));
    change = hd[1] > 0.0 ? hd[0] / hd[1] : hd[0];
    // the carriers' drift from ψ, then their level from the level's start
    for (pd_instance *C : {ne, pe}) {
      if ((rc = drift_from(C, psi, l0))) return rc;
      HIPCHK(hipMemcpy(C->H.sol[sol_slot(C->rot, 0)], C == ne ? n0 : p0, np * sizeof(double),
                       hipMemcpyDeviceToDevice));
      C->t = t_k;
      C->have_prev = false;
    }
    std::vector<std::vector<double>> sc(2);
    if ((rc = solve_many({ne, pe}, {&tdc, &tdc}, &sc))) return rc;
    krylov += (int)sc[0][0] + (int)sc[1][0];
    if (it >= 1 && change <= gummel_tol) {
      ++it;
      break;
    }
  }
  psi->t = 0.0;
  if (stats) {
    stats->gummel_iters = it;
    stats->krylov_iters = krylov;
    stats->change = change;
  }
  return PD_OK;
}

int pd_apply_preconditioner(pd_instance *I, double dt, double theta, const double *y, double *z, int32_t layout,
                            int32_t device_ptrs) {
  if (!I || !y || !z) return fail(PD_EINVAL, "NULL argument");
  if (!(dt > 0.0)) return fail(PD_EINVAL, "dt must be > 0");
  int rc = validate_theta(theta);
  if (rc) return rc;
  if (layout != PD_LAYOUT_RING && layout != PD_LAYOUT_PAPER) return fail(PD_EINVAL, "bad layout");
  BusyGuard g({I});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  const int m = I->M.m, n = I->M.n, N = m * n + 1, np = I->T.npad;
  std::vector<double> src;
  if ((rc = fetch(y, N, device_ptrs, src))) return rc;
  std::vector<double> hin(np), hout(np), o(N);
  to_internal(src.data(), layout, m, n, np, hin.data());
  hipStream_t s = I->stream;
  // one level t -> t + dt set up and factored (its Krylov phase is not run);
  // the state of the instance is not touched
  double tab[2] = {I->t, I->t + dt};
  if ((rc = ensure_time_capacity(I, 1))) return rc;
  HIPCHK(hipMemcpyAsync(I->t_table, tab, sizeof tab, hipMemcpyHostToDevice, s));
  Plan P;
  if ((rc = make_plan({I}, s, P))) return rc;
  if ((rc = attach_mg({I}, s, P))) return rc;
  SolveParams sp{theta, 1e-300, 1e-3, 1, 1, 1};
  if ((rc = init_scalars(I, sp, 1, s))) return rc;
  pd::launch_level_begin(P.L, s);
  pd::launch_factor(P.L, s);
  const bool fp32 = I->precision == PD_MIXED;
  if (fp32) {
    std::vector<float> f(hin.begin(), hin.end());
    HIPCHK(hipMemcpyAsync(I->H.k32.r, f.data(), np * 4, hipMemcpyHostToDevice, s));
    pd::launch_precond_apply(P.L, 1, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(f.data(), I->H.k32.ph, np * 4, hipMemcpyDeviceToHost));
    for (int k = 0; k < np; ++k) hout[k] = f[k];
  } else {
    HIPCHK(hipMemcpyAsync(I->H.k64.r, hin.data(), np * 8, hipMemcpyHostToDevice, s));
    pd::launch_precond_apply(P.L, 0, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(hout.data(), I->H.k64.ph, np * 8, hipMemcpyDeviceToHost));
  }
  from_internal(hout.data(), layout, m, n, o.data());
  if (device_ptrs) {
    HIPCHK(hipMemcpy(z, o.data(), N * 8, hipMemcpyHostToDevice));
  } else {
    std::memcpy(z, o.data(), N * 8);
  }
  return PD_OK;
}

}  // extern "C"

// ================================================================== adaptivity

// Scratch of the allocation-free indicator: the per-ring values of
// k_indicator (4 doubles per ring), up to kMaxM rings.  Each device holds
// its own copy for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns for that device.
constexpr size_t kIndScratch = 4 * (size_t)kMaxM;
static __device__ __align__(256) double scratch[kIndScratch];

namespace {

// Node k of the radial stretch (2.4) with exponent p: r_k = sin((k h)^p π/2),
// the end points exact.
double sine_node(int m, double p, int k) {
  if (k <= 0) return 0.0;
  if (k >= m + 1) return 1.0;
  return std::sin(std::pow(k * (1.0 / (m + 1)), p) * kPi / 2.0);
}

// κ at v by linear interpolation between (xs[k], ys[k]), k = 0..cnt-1 (xs
// increasing), constant beyond the ends.
double interp_linear(const double *xs, const double *ys, int cnt, double v) {
  if (v <= xs[0]) return ys[0];
  if (v >= xs[cnt - 1]) return ys[cnt - 1];
  const int k = (int)(std::upper_bound(xs, xs + cnt, v) - xs);   // xs[k-1] <= v < xs[k]
  const double w = (v - xs[k - 1]) / (xs[k] - xs[k - 1]);
  return ys[k - 1] + w * (ys[k] - ys[k - 1]);
}

// Predicted largest radial indicator max_k ĥ'_k² κ(r'_k) of the stretch with
// exponent p; r_old holds r_0..r_{m+1} of the current mesh, kappa κ_1..κ_m.
// Allocates nothing.
double predicted_max(const double *r_old, const double *kappa, int m, double p) {
  double best = 0.0;
  double rl = sine_node(m, p, 0), rc = sine_node(m, p, 1);
  for (int k = 1; k <= m; ++k) {
    const double rr = sine_node(m, p, k + 1);
    const double hl = 0.5 * ((rc - rl) + (rr - rc));
    best = std::max(best, hl * hl * interp_linear(r_old + 1, kappa, m, rc));
    rl = rc;
    rc = rr;
  }
  return best;
}

// The indicator summary from the per-ring values of k_indicator (4 per
// ring: κ_i, max_j η, its first j, Σ_j η) and the candidate exponents.
// Allocates nothing; kappa (m values) may be NULL.
void indicator_summary(const pd_instance *I, const double *ring, double p_current, const double *p_candidates,
                       int n_candidates, double *kappa, double *kap_work, pd_indicator *out) {
  const int m = I->M.m;
  pd_indicator R{};
  R.eta_max = -1.0;
  for (int i = 1; i <= m; ++i) {
    const double *q = ring + 4 * (size_t)(i - 1);
    kap_work[i - 1] = q[0];
    if (q[1] > R.eta_max) {
      R.eta_max = q[1];
      R.i_max = i;
      R.j_max = (int)q[2];
    }
    R.eta_sum += q[3];
  }
  if (kappa) std::copy(kap_work, kap_work + m, kappa);
  R.p_best = p_current;
  R.pred_current = predicted_max(I->M.r.data(), kap_work, m, p_current);
  R.pred_best = R.pred_current;
  bool found = false;
  for (int c = 0; c < n_candidates; ++c) {
    const double v = predicted_max(I->M.r.data(), kap_work, m, p_candidates[c]);
    if (!found || v < R.pred_best) {
      R.pred_best = v;
      R.p_best = p_candidates[c];
      found = true;
    }
  }
  R.recommend = (found && R.pred_best <= 0.8 * R.pred_current) ? 1 : 0;
  *out = R;
}

int check_indicator_args(pd_instance *I, double p_current, const double *p_candidates, int32_t n_candidates,
                         pd_indicator *out) {
  if (!I || !out) return fail(PD_EINVAL, "NULL argument");
  if (n_candidates < 0 || (n_candidates > 0 && !p_candidates)) return fail(PD_EINVAL, "bad candidate list");
  for (int c = 0; c < n_candidates; ++c)
    if (!(p_candidates[c] > 0.0)) return fail(PD_EINVAL, "stretch exponents must be > 0");
  if (!(p_current > 0.0)) return fail(PD_EINVAL, "p_current must be > 0");
  return PD_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device
// with that device current (the caller's current device is restored).
int scratch_on(int device, double **ptr) {
  if (device < 0 || device >= kMaxDevices) return fail(PD_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return fail(PD_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = (double *)p;
  }
  *ptr = g_scratch_ptr[device];
  return PD_OK;
}

}  // namespace

extern "C" {

int pd_error_indicator(pd_instance *I, double p_current, const double *p_candidates, int32_t n_candidates,
                       double *kappa, double *eta, pd_indicator *out) {
  int rc = check_indicator_args(I, p_current, p_candidates, n_candidates, out);
  if (rc) return rc;
  BusyGuard g({I});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  const int m = I->M.m, n = I->M.n;
  hipStream_t s = I->stream;
  double *dbuf = nullptr;
  const size_t ring_vals = 4 * (size_t)m, eta_vals = eta ? (size_t)m * n : 0;
  HIPCHK(hipMalloc(&dbuf, (ring_vals + eta_vals) * sizeof(double)));
  struct Free {
    double *p;
    ~Free() { (void)hipFree(p); }
  } fr{dbuf};
  const PdInst &H = I->H;
  pd::launch_indicator(H.sol[sol_slot(I->rot, 0)], m, n, H.r_nodes, H.th_nodes, H.nb, H.lam, H.tpow, H.nsrc,
                       I->t, I->bc == 0 ? 1 : 0, dbuf, eta ? dbuf + ring_vals : nullptr, s);
  HIPCHK(hipGetLastError());
  std::vector<double> ring(ring_vals), kap(m);
  HIPCHK(hipMemcpyAsync(ring.data(), dbuf, ring_vals * sizeof(double), hipMemcpyDeviceToHost, s));
  if (eta) HIPCHK(hipMemcpyAsync(eta, dbuf + ring_vals, eta_vals * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  indicator_summary(I, ring.data(), p_current, p_candidates, n_candidates, kappa, kap.data(), out);
  return PD_OK;
}

int pd_error_indicator_noalloc(pd_instance *I, double p_current, const double *p_candidates,
                               int32_t n_candidates, double *kappa, double *eta_device, pd_indicator *out) {
  int rc = check_indicator_args(I, p_current, p_candidates, n_candidates, out);
  if (rc) return rc;
  const int m = I->M.m, n = I->M.n;
  if (4 * (size_t)m > kIndScratch)
    return fail(PD_EINVAL, "m = %d exceeds the scratch of the allocation-free indicator (%d rings)", m, kMaxM);
  double *ring_dev = nullptr;
  if ((rc = scratch_on(I->device, &ring_dev))) return rc;
  BusyGuard g({I});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  hipStream_t s = I->stream;
  const PdInst &H = I->H;
  // k_indicator writes every ring's four values: nothing needs clearing
  pd::launch_indicator(H.sol[sol_slot(I->rot, 0)], m, n, H.r_nodes, H.th_nodes, H.nb, H.lam, H.tpow, H.nsrc,
                       I->t, I->bc == 0 ? 1 : 0, ring_dev, eta_device, s);
  HIPCHK(hipGetLastError());
  double ring[kIndScratch];
  double kap[kMaxM];
  HIPCHK(hipMemcpyAsync(ring, ring_dev, 4 * (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  indicator_summary(I, ring, p_current, p_candidates, n_candidates, kappa, kap, out);
  return PD_OK;
}

int pd_remesh_transfer(pd_instance *from, pd_instance *to) {
  if (!from || !to) return fail(PD_EINVAL, "NULL argument");
  if (from == to) return fail(PD_EINVAL, "source and target must differ");
  if (from->device != to->device) return fail(PD_EINVAL, "instances live on different devices");
  if (from->bc != to->bc) return fail(PD_EINVAL, "boundary conditions differ");
  if (from->bc == 1 && from->M.m < 3) return fail(PD_EINVAL, "zero-flux transfer needs m >= 3");
  BusyGuard g({from, to});
  if (!g.ok) return fail(PD_EBUSY, "instance is in use");
  HIPCHK(hipStreamSynchronize(from->stream));
  const PdInst &A = from->H;
  const PdInst &B = to->H;
  pd::launch_transfer(A.sol[sol_slot(from->rot, 0)], from->M.m, from->M.n, A.r_nodes, A.th_nodes, A.nb, A.lam,
                      A.tpow, A.nsrc, from->t, from->bc == 0 ? 1 : 0, B.r_nodes, B.th_nodes, to->M.m, to->M.n,
                      B.sol[sol_slot(to->rot, 0)], to->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(to->stream));
  to->t = from->t;
  to->have_prev = false;
  return PD_OK;
}

}  // extern "C"

// ================================================================== serving
//
// Continuous batching: a worker thread steps every admitted request one
// time level at a time in shared launches (Engine); between levels it
// retires finished requests and admits queued ones (arrival order, while
// the slot count and the memory pool allow), rebuilding the launch plan
// whenever the set changed.

namespace {


struct Request {
  uint64_t ticket = 0;
  std::unique_ptr<pd_instance> prepared;   // host part, until admission
  std::unique_ptr<HostImage> image;        // uploads, until admission
  int layout = PD_LAYOUT_RING;
  std::vector<double> ttab;                // the K+1 levels from t = 0
  int K = 0, N = 0;
  size_t footprint = 0;
  SolveParams sp{};
  pd_instance *inst = nullptr;
  void *chunk = nullptr;                   // its device memory, from the loop's arena
  size_t chunk_bytes = 0;
  int status = PD_PENDING;
  std::string err;
  std::vector<double> result;
  pd_request_summary sum{};
  Clock::time_point t_submit, t_admit;
};

double seconds(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

}  // namespace

// Device memory of a serving loop: segments allocated on demand (at least
// seg_bytes) and kept until the loop ends, carved first-fit with free
// lists that coalesce, so that requests are admitted and retired without
// hipMalloc or hipFree (hipFree waits for the whole device).  Used by the
// loop's worker thread only.
struct Arena {
  struct Seg {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;   // offset -> bytes
  };
  std::vector<Seg> segs;
  size_t seg_bytes = size_t(1) << 30;
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  void *alloc(size_t bytes) {
    bytes = round(bytes);
    for (auto &g : segs)
      for (auto it = g.free.begin(); it != g.free.end(); ++it)
        if (it->second >= bytes) {
          const size_t off = it->first, rest = it->second - bytes;
          g.free.erase(it);
          if (rest) g.free.emplace(off + bytes, rest);
          return g.base + off;
        }
    Seg g;
    g.size = std::max(seg_bytes, bytes);
    if (hipMalloc((void **)&g.base, g.size) != hipSuccess) return nullptr;
    if (g.size > bytes) g.free.emplace(bytes, g.size - bytes);
    segs.push_back(std::move(g));
    return segs.back().base;
  }
  void release(void *p, size_t bytes) {
    bytes = round(bytes);
    for (auto &g : segs) {
      if ((char *)p < g.base || (char *)p >= g.base + g.size) continue;
      size_t off = (char *)p - g.base;
      auto nx = g.free.lower_bound(off);
      if (nx != g.free.end() && nx->first == off + bytes) {   // merge with the next free run
        bytes += nx->second;
        nx = g.free.erase(nx);
      }
      if (nx != g.free.begin()) {                              // and with the previous one
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
          off = pv->first;
          bytes += pv->second;
          g.free.erase(pv);
        }
      }
      g.free.emplace(off, bytes);
      return;
    }
  }
  void destroy() {
    for (auto &g : segs) (void)hipFree(g.base);
    segs.clear();
  }
};

struct pd_batch {
  size_t pool = 0;
  Arena arena;
  int max_slots = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> pending;                         // arrival order
  std::map<uint64_t, std::unique_ptr<Request>> reqs;     // every unreported ticket
  uint64_t next = 1;
  bool stop = false;
  pd_batch_info info{};
  std::thread worker;
};

namespace {

// Uploads the request's prepared instance on the loop's stream and readies its solve.
int admit_request(pd_batch *B, Request *R) {
  pd_instance *I = R->prepared.get();
  I->device = B->device;
  I->stream = B->stream;
  I->own_stream = false;
  // one arena chunk: the instance's arrays, then its time table and statistics
  Carver dry{nullptr, 0, true};
  carve(I, dry);
  const size_t kcap = (size_t)std::max(R->K, 16);
  const size_t db = Arena::round(dry.off), tb = Arena::round((kcap + 1) * sizeof(double));
  R->chunk_bytes = db + tb + PD_LSTAT * kcap * sizeof(double);
  R->chunk = B->arena.alloc(R->chunk_bytes);
  if (!R->chunk) {
    R->prepared.reset();
    return fail(PD_ENOMEM, "device allocation of %zu bytes for a request failed", R->chunk_bytes);
  }
  // the time table and statistics live in the chunk too (set before the
  // upload, which would otherwise allocate them)
  I->arena = true;
  I->t_table = (double *)((char *)R->chunk + db);
  I->stats = (double *)((char *)R->chunk + db + tb);
  I->kcap = (int)kcap;
  int rc = upload_instance(I, *R->image, R->chunk);
  R->image.reset();
  I->H.t_table = I->t_table;
  I->H.level_stats = I->stats;
  if (rc) {
    R->prepared.reset();
    B->arena.release(R->chunk, R->chunk_bytes);
    R->chunk = nullptr;
    return rc;
  }
  R->inst = R->prepared.release();
  HIPCHK(hipMemcpyAsync(R->inst->t_table, R->ttab.data(), R->ttab.size() * sizeof(double), hipMemcpyHostToDevice,
                        B->stream));
  return init_scalars(R->inst, R->sp, R->K, B->stream);
}

// Collects a finished request's result and statistics (its first `levels`
// levels were taken) and frees its instance.
void retire_request(pd_batch *B, Request *R, int rc, int levels) {
  int worst = PD_OK;
  std::string err;
  if (rc) err = g_err;
  if (!rc && R->inst && levels > 0) {
    std::vector<double> st;
    rc = read_level_stats(R->inst, levels, st, worst);
    if (!rc) {
      pd_request_summary &S = R->sum;
      for (int k = 0; k < levels; ++k) {
        S.levels = k + 1;
        S.iters += (int)st[PD_LSTAT * k + 0];
        S.refinements += (int)st[PD_LSTAT * k + 1];
        S.max_rel_resid = std::max(S.max_rel_resid, st[PD_LSTAT * k + 3]);
        S.t = st[PD_LSTAT * k + 5];
      }
      R->result.resize(R->N);
      rc = pd_get_solution(R->inst, R->result.data(), R->layout, 0);
    }
    if (rc) err = g_err;
    if (!rc && worst != PD_OK) {
      rc = worst;
      err = worst == PD_EBREAKDOWN ? "Krylov breakdown in a step"
                                   : "a step did not reach the tolerance within the iteration cap";
    }
  }
  if (R->inst) (void)pd_destroy(R->inst);
  R->inst = nullptr;
  if (R->chunk) B->arena.release(R->chunk, R->chunk_bytes);
  R->chunk = nullptr;
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(B->mu);
  R->sum.status = rc;
  R->sum.queue_s = seconds(R->t_submit, R->t_admit);
  R->sum.latency_s = seconds(R->t_submit, now);
  R->err = err;
  R->status = rc;
  B->info.used_bytes -= R->footprint;
  B->info.active -= 1;
  B->info.completed += 1;
}

// Cycles the loop runs between looks at its queue and its finished requests.
constexpr long kServeSlice = 8;
constexpr int kServeRound = 4;   // most Krylov cycles per round in the serving loop

void serve(pd_batch *B) {
  (void)hipSetDevice(B->device);
  Engine E;
  std::vector<Request *> active;
  std::vector<int> lv;
  bool dirty = false;
  for (;;) {
    std::vector<Request *> admit;
    {
      std::unique_lock<std::mutex> lk(B->mu);
      B->cv.wait(lk, [&] { return B->stop || !active.empty() || !B->pending.empty(); });
      if (B->stop) break;
      while (!B->pending.empty() && (int)(active.size() + admit.size()) < B->max_slots &&
             B->info.used_bytes + B->pending.front()->footprint <= B->pool) {
        Request *R = B->pending.front();
        B->pending.pop_front();
        B->info.used_bytes += R->footprint;
        B->info.peak_bytes = std::max(B->info.peak_bytes, B->info.used_bytes);
        B->info.pending -= 1;
        B->info.active += 1;
        admit.push_back(R);
      }
      B->info.peak_active = std::max(B->info.peak_active, B->info.active);
    }
    const auto t_a = Clock::now();
    for (Request *R : admit) {
      R->t_admit = Clock::now();
      const int rc = admit_request(B, R);
      if (rc) {
        retire_request(B, R, rc, 0);
      } else {
        active.push_back(R);
        dirty = true;
      }
    }
    const auto t_b = Clock::now();
    if (!admit.empty()) {
      std::lock_guard<std::mutex> lk(B->mu);
      B->info.admit_s += std::chrono::duration<double>(t_b - t_a).count();
    }
    if (active.empty()) continue;
    int rc = PD_OK;
    if (dirty) {
      std::vector<pd_instance *> insts;
      int cap = 0;
      for (Request *R : active) {
        insts.push_back(R->inst);
        cap = std::max(cap, cycles_cap(R->sp));
      }
      // short rounds: a request's level can only start at a round head, and
      // a slice of the loop is at least one round
      Schedule sch = default_schedule();
      sch.cycles_per_graph = std::min(sch.cycles_per_graph, kServeRound);
      rc = E.build(insts, cap, B->stream, sch);
      dirty = false;
      std::lock_guard<std::mutex> lk(B->mu);
      B->info.plans_built += 1;
      B->info.build_s += std::chrono::duration<double>(Clock::now() - t_b).count();
    }
    // a slice of asynchronous cycles, then retire whoever left the batch
    const auto t_r = Clock::now();
    bool fin = false;
    if (!rc) rc = E.run(kServeSlice, &fin);
    if (!rc) rc = E.levels_done(lv);
    const auto t_d = Clock::now();
    if (rc) {
      // a failure of the loop itself ends every active request
      E.release();
      for (Request *R : active) retire_request(B, R, rc, 0);
      active.clear();
      continue;
    }
    std::vector<Request *> keep;
    for (size_t q = 0; q < active.size(); ++q) {
      Request *R = active[q];
      if (lv[2 * q + 1]) {
        retire_request(B, R, PD_OK, lv[2 * q]);
        dirty = true;
      } else {
        keep.push_back(R);
      }
    }
    active.swap(keep);
    if (active.empty()) E.release();
    std::lock_guard<std::mutex> lk(B->mu);
    B->info.slices_run += 1;       // slices of cycles run
    B->info.run_s += std::chrono::duration<double>(t_d - t_r).count();
    B->info.retire_s += std::chrono::duration<double>(Clock::now() - t_d).count();
  }
  E.release();
  for (Request *R : active)
    if (R->inst) (void)pd_destroy(R->inst);
}

}  // namespace

extern "C" {

int pd_batch_create(size_t hbm_pool_bytes, int32_t max_slots, void *hip_stream, pd_batch **out) {
  if (!out) return fail(PD_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_pool_bytes == 0) return fail(PD_EINVAL, "hbm_pool_bytes must be > 0");
  if (max_slots < 1) return fail(PD_EINVAL, "max_slots must be >= 1");
  std::unique_ptr<pd_batch> B(new pd_batch);
  B->pool = hbm_pool_bytes;
  B->max_slots = max_slots;
  HIPCHK(hipGetDevice(&B->device));
  if (hip_stream) {
    B->stream = (hipStream_t)hip_stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
    B->own_stream = true;
  }
  pd_batch *raw = B.get();
  try {
    B->worker = std::thread(serve, raw);
  } catch (...) {
    if (B->own_stream) (void)hipStreamDestroy(B->stream);
    return fail(PD_EINVAL, "could not start the serving thread");
  }
  *out = B.release();
  return PD_OK;
}

int pd_batch_submit(pd_batch *B, const pd_mesh_desc *mesh, const pd_problem_desc *pb, const pd_time_desc *td,
                    int32_t precision, uint64_t *ticket) {
  try {
    if (!B || !mesh || !pb || !td || !ticket) return fail(PD_EINVAL, "NULL argument");
    if (precision != PD_FP64 && precision != PD_MIXED) return fail(PD_EINVAL, "unknown precision %d", precision);
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if ((rc = validate_theta(td->theta))) return rc;
    if (pb->nsrc < 0 || pb->nsrc > PD_MAXSRC) return fail(PD_EINVAL, "nsrc must be in [0, %d]", PD_MAXSRC);
    if (pb->flux < 0 || pb->flux > 2) return fail(PD_EINVAL, "flux must be 0, 1 or 2");
  if (pb->flux == 2 && pb->bc != 0) return fail(PD_EINVAL, "the printed stencil (flux 2) takes Dirichlet data only");
  if (pb->flux == 2 && !pb->E_node) return fail(PD_EINVAL, "the printed stencil (flux 2) needs E_node");
    if (pb->bc != 0 && pb->bc != 1) return fail(PD_EINVAL, "bc must be 0 or 1");
    if (pb->layout != PD_LAYOUT_RING && pb->layout != PD_LAYOUT_PAPER) return fail(PD_EINVAL, "bad layout");
    if (!pb->u0) return fail(PD_EINVAL, "u0 is NULL");
    if (pb->nsrc > 0 && (!pb->lambda || !pb->g)) return fail(PD_EINVAL, "lambda and g are required when nsrc > 0");
    const auto t_submit = Clock::now();
    std::unique_ptr<Request> R(new Request);
    const int m = mesh->nr, n = mesh->ntheta, N = m * n + 1;
    R->N = N;
    R->layout = pb->layout;
    if (td->t_kind == PD_TIME_ADAPTIVE)
      return fail(PD_EINVAL, "adaptive time stepping is not served; use pd_solve_to_T or pd_solve_batch");
    if ((rc = build_time_table(td, 0.0, R->ttab))) return rc;
    R->K = td->K;
    R->sp = params_from(td, precision);
    size_t fp = 0;
    if ((rc = pd_footprint(mesh, pb->nsrc, precision, &fp))) return rc;
    R->footprint = fp + ((PD_LSTAT + 1) * (size_t)std::max(R->K, 16) + 1) * sizeof(double);
    if (R->footprint > B->pool)
      return fail(PD_ENOMEM, "request needs %zu bytes, the pool holds %zu", R->footprint, B->pool);
    // the host part of the instance is built here, on the caller's thread
    if ((rc = prepare_instance(mesh, pb, precision, R->prepared, R->image))) return rc;
    {
      std::lock_guard<std::mutex> lk(B->mu);
      if (B->stop) return fail(PD_EINVAL, "batch is shutting down");
      R->ticket = B->next++;
      R->t_submit = t_submit;
      *ticket = R->ticket;
      B->pending.push_back(R.get());
      B->reqs.emplace(R->ticket, std::move(R));
      B->info.pending += 1;
      B->info.submitted += 1;
    }
    B->cv.notify_all();
    return PD_OK;
  } catch (const std::bad_alloc &) {
    return fail(PD_ENOMEM, "host allocation failed");
  }
}

int pd_batch_poll(pd_batch *B, uint64_t ticket, double *out, pd_request_summary *summary) {
  if (!B) return fail(PD_EINVAL, "batch is NULL");
  std::unique_ptr<Request> R;
  {
    std::lock_guard<std::mutex> lk(B->mu);
    auto it = B->reqs.find(ticket);
    if (it == B->reqs.end()) return fail(PD_EINVAL, "unknown or already reported ticket %llu", (unsigned long long)ticket);
    if (it->second->status == PD_PENDING) return PD_PENDING;
    R = std::move(it->second);
    B->reqs.erase(it);
  }
  if (summary) *summary = R->sum;
  if (R->status == PD_OK && out) std::memcpy(out, R->result.data(), R->result.size() * sizeof(double));
  if (R->status < 0) return fail(R->status, "%s", R->err.c_str());
  return R->status;
}

int pd_batch_stats(pd_batch *B, pd_batch_info *info) {
  if (!B || !info) return fail(PD_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(B->mu);
  *info = B->info;
  return PD_OK;
}

int pd_batch_destroy(pd_batch *B) {
  if (!B) return PD_OK;
  {
    std::lock_guard<std::mutex> lk(B->mu);
    B->stop = true;
  }
  B->cv.notify_all();
  if (B->worker.joinable()) B->worker.join();
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  B->arena.destroy();
  if (B->own_stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return PD_OK;
}

}  // extern "C"
