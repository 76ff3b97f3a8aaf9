// C ABI of the PQMC field-update sweep: context, workspace layout, setup
// (K = e^{-dtau H0}, initial stack) and the sweep driver (Sec. II B).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pqmc.h"
#include "engine.hpp"
#include "soc.hpp"

namespace {
thread_local std::string g_last_error;

pqmc_status set_error(pqmc_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}
}  // namespace

namespace pq {
int api_error(int st, const char *msg) {
  g_last_error = msg;
  return st;
}

int fail_device(hipError_t e, const char *expr, const char *file, int line) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e),
                expr, file, line);
  g_last_error = buf;
  return PQMC_EDEVICE;
}
}  // namespace pq

using namespace pq;

struct pqmc_ctx {
  // U < 0: the paper's one-sector complex model, run by the complex engine;
  // every call below forwards to it
  pqmc_soc_ctx *cx = nullptr;
  int N = 0, Ns[2] = {0, 0}, M = 0, kt = 0, nst = 0;
  double U = 0, dtau = 0, alpha = 0;
  uint64_t seed = 0, walker = 0;
  pqmc_update_opts opts{};
  int kmax = 1, bmax = 1, gmax = 1;
  bool log_alloc = false;
  hipStream_t st = nullptr;

  double *K = nullptr, *Kinv = nullptr, *Tay0 = nullptr, *Tay1 = nullptr;
  // H0 as ELL rows (sparse propagation): ell_w entries per row, Taylor degree
  // taylor_J; sparse_prop when H0 qualifies (see setup_sparse)
  int *ell_idx = nullptr;
  double *ell_val = nullptr;
  int ell_w = 0, taylor_J = 0;
  bool sparse_prop = false;
  int8_t *fields = nullptr;
  int8_t *replay = nullptr;   // 2 M x N forced outcomes of pqmc_replay
  bool replaying = false;
  double *P[2] = {nullptr, nullptr};
  double *URw[2][2] = {}, *ULw[2][2] = {};
  double *Lstack[2] = {}, *Rstack[2] = {};
  double *T[2] = {};
  float *T32[2] = {};
  double *E[2] = {}, *F[2] = {}, *BR[2] = {}, *Z[2] = {};
  int *prow[2] = {}, *slot[2] = {};
  LocalBufs lb{};
  GroupBufs gb{};
  unsigned long long *stats = nullptr;
  int32_t *log_meta = nullptr, *hb_meta = nullptr;
  double *log_margin = nullptr, *hb_margin = nullptr;
  long long log_cap = 0;
  double *gtmp = nullptr, *xtmp = nullptr;
  // stabilisation drift: sampled columns of U_R T U_L before / after
  double *drift_y[2] = {}, *drift_z[2][2] = {};
  // persistent local kernels: partial buffers and the grid barrier
  double *lp_y[2] = {}, *lp_x[2] = {}, *lp_s[2] = {};
  unsigned *lp_sync = nullptr;
  // G-form local update (sized when created with PQMC_LOCAL_G): G_s, a
  // work copy for the propagation and the stabilisation, published rows
  bool gsized = false;
  bool g_valid = false;   // G holds the current G-form state
  // graph-captured sweeps (PQMC_FLAG_GRAPH): the sweep counter on the device,
  // and, in a batch's first context, the captured sweep of that batch
  uint64_t *sweep_dev = nullptr;
  bool capturing = false;
  uint64_t generation = 0;   // bumped by every change that a captured sweep bakes in
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<pqmc_ctx *> gkey;
  std::vector<uint64_t> ggen;
  long long glog = 0, ghb = 0;   // log entries one captured sweep writes
  double *G[2] = {}, *Gw[2] = {}, *grow_buf[2] = {};

  double *UR[2] = {};
  double *ULt[2] = {};
  int position = 0;
  bool failed = false, windowed = false;
  bool t32_ahead = false;   // precision form: T32 holds flushes that T does not
  uint64_t sweep_index = 0;
  long long log_count = 0, hb_count = 0, hb_total = 0;
  std::vector<hipEvent_t> evs;
  // per-launch kernel timing (PQMC_FLAG_KTIME)
  std::vector<hipEvent_t> kevs;
  std::vector<int> kclass;
  size_t kused = 0;
  double kt_total[PQMC_K_COUNT] = {};
  uint64_t kt_count[PQMC_K_COUNT] = {};
};

namespace {

constexpr size_t kAlign = 256;
// columns of G sampled for the stabilisation drift statistic
constexpr int kDriftCols = 16;

struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Assign every device buffer inside the workspace (or only size it).
void layout(pqmc_ctx &c, char *base, size_t *bytes) {
  Carver cv{base};
  const size_t N = c.N;
  const size_t NN = N * N;
  c.K = cv.take<double>(NN);
  c.Kinv = cv.take<double>(NN);
  c.Tay0 = cv.take<double>(NN);
  c.Tay1 = cv.take<double>(NN);
  c.gtmp = c.Tay0;   // Green's function output reuses the Taylor scratch
  c.ell_idx = cv.take<int>(N * kExpMaxW);
  c.ell_val = cv.take<double>(N * kExpMaxW);
  c.fields = cv.take<int8_t>((size_t)c.M * N);
  c.replay = cv.take<int8_t>((size_t)2 * c.M * N);
  c.sweep_dev = cv.take<uint64_t>(1);
  c.stats = cv.take<unsigned long long>(16);
  const int kmax = c.gmax;
  for (int s = 0; s < 2; ++s) {
    const size_t ns = c.Ns[s];
    const size_t nt = ceil_div(c.Ns[s], 64);
    c.P[s] = cv.take<double>(N * ns);
    c.URw[s][0] = cv.take<double>(N * ns);
    c.URw[s][1] = cv.take<double>(N * ns);
    c.ULw[s][0] = cv.take<double>(N * ns);
    c.ULw[s][1] = cv.take<double>(N * ns);
    c.Lstack[s] = cv.take<double>((size_t)(c.nst + 1) * N * ns);
    c.Rstack[s] = cv.take<double>((size_t)(c.nst + 1) * N * ns);
    c.T[s] = cv.take<double>(ns * ns);
    c.T32[s] = cv.take<float>(ns * ns);
    c.E[s] = cv.take<double>(ns * 2 * ns);
    c.F[s] = cv.take<double>(ns * ns);
    c.BR[s] = cv.take<double>((size_t)2 * kNB * 2 * ns);
    c.Z[s] = cv.take<double>(kNB * kNB);
    c.prow[s] = cv.take<int>(ns);
    c.slot[s] = cv.take<int>(ns);
    for (int p = 0; p < 2; ++p) {
      c.lb.ypart[s][p] = cv.take<double>(nt * ns);
      c.lb.tpart[s][p] = cv.take<double>(nt * ns);
      c.lb.spart[s][p] = cv.take<double>(nt * nt);
    }
    c.gb.P2part[s] = cv.take<double>(nt * kmax * ns);
    c.gb.P1part[s] = cv.take<double>(nt * ns * kmax);
    c.gb.P2[s] = cv.take<double>(kmax * ns);
    c.gb.P1[s] = cv.take<double>(ns * kmax);
    c.gb.W0part[s] = cv.take<double>(nt * nt * kmax * kmax);
    c.gb.W0[s] = cv.take<double>(kmax * kmax);
    c.gb.Mc[s] = cv.take<double>(kmax * kmax);
    c.gb.sc[s] = cv.take<double>(kmax);
    c.gb.Q[s] = cv.take<double>(ns * kmax);
  }
  c.lb.delta[0] = cv.take<double>(2);
  c.lb.delta[1] = cv.take<double>(2);
  c.gb.nA = cv.take<int>(2);
  c.gb.alist = cv.take<int>(kmax);
  c.gb.uni = cv.take<double>(kmax + 1);
  c.gb.kmax = kmax;
  c.gb.chunks = c.opts.tile_chunks > 0 ? c.opts.tile_chunks : 2;
  c.gb.Ns[0] = c.Ns[0];
  c.gb.Ns[1] = c.Ns[1];
  c.xtmp = cv.take<double>(N * (size_t)std::max(c.Ns[0], c.Ns[1]));
  for (int s = 0; s < 2; ++s) {
    int pr = 1, pc = 1;
    local_persist_grid(c.Ns[s], &pr, &pc);
    c.lp_y[s] = cv.take<double>((size_t)2 * pr * c.Ns[s]);
    c.lp_x[s] = cv.take<double>((size_t)2 * pc * c.Ns[s]);
    c.lp_s[s] = cv.take<double>((size_t)2 * pr * pc);
    if (c.gsized) {
      c.G[s] = cv.take<double>(NN);
      c.Gw[s] = cv.take<double>(NN);
      c.grow_buf[s] = cv.take<double>(2 * N);
    }
  }
  c.lp_sync = cv.take<unsigned>(kLocalMaxGroups + 1);
  for (int s = 0; s < 2; ++s) {
    c.drift_y[s] = cv.take<double>((size_t)kDriftCols * c.Ns[s]);
    c.drift_z[s][0] = cv.take<double>((size_t)kDriftCols * N);
    c.drift_z[s][1] = cv.take<double>((size_t)kDriftCols * N);
  }
  if (c.log_alloc) {
    c.log_cap = 2LL * c.M * c.N;
    c.log_meta = cv.take<int32_t>(3 * (size_t)c.log_cap);
    c.log_margin = cv.take<double>((size_t)c.log_cap);
    c.hb_meta = cv.take<int32_t>(3 * (size_t)c.log_cap);
    c.hb_margin = cv.take<double>((size_t)c.log_cap);
  }
  *bytes = cv.off + kAlign;
}

pqmc_status validate(const pqmc_problem *p, const pqmc_update_opts *o) {
  if (!p || !o) return set_error(PQMC_EINVAL, "null problem or options");
  if (p->n_sites < 1) return set_error(PQMC_EINVAL, "n_sites must be >= 1");
  if (p->n_up < 1 || p->n_dn < 1 || p->n_up > p->n_sites || p->n_dn > p->n_sites)
    return set_error(PQMC_EINVAL, "need 1 <= n_up, n_dn <= n_sites");
  if (p->n_up > 1024 || p->n_dn > 1024)
    return set_error(PQMC_EINVAL, "particle numbers above 1024 are not supported");
  if (!p->hopping || !p->trial_up || !p->trial_dn) return set_error(PQMC_EINVAL, "null input");
  if (!(p->dtau > 0) || !std::isfinite(p->dtau)) return set_error(PQMC_EINVAL, "dtau must be > 0");
  if (!std::isfinite(p->U)) return set_error(PQMC_EINVAL, "U must be finite");
  if (p->n_slices < 1 || p->stab_every < 1 || p->n_slices % p->stab_every)
    return set_error(PQMC_EINVAL, "stab_every must divide n_slices");
  if (o->scheme < PQMC_LOCAL || o->scheme > PQMC_LOCAL_G) return set_error(PQMC_EINVAL, "scheme");
  if (o->scheme == PQMC_LOCAL_G && !local_persist_fits(p->n_up, p->n_dn, p->n_sites, true))
    return set_error(PQMC_EINVAL, "the G-form local update holds N <= 2048 sites");
  if (o->delay_k < 1 || o->delay_k > 128) return set_error(PQMC_EINVAL, "delay_k in [1, 128]");
  if (o->block_b < 1 || o->block_b > 64) return set_error(PQMC_EINVAL, "block_b in [1, 64]");
  if (o->tile_chunks < 0) return set_error(PQMC_EINVAL, "tile_chunks must be >= 0");
  if ((o->flags & PQMC_FLAG_FP32) &&
      (o->scheme == PQMC_LOCAL || o->scheme == PQMC_LOCAL_G ||
       (o->scheme == PQMC_DELAYED ? o->delay_k : o->block_b) > 64))
    return set_error(PQMC_EINVAL, "the float32 form needs the delayed or block scheme, k, b <= 64");
  const size_t NN = (size_t)p->n_sites * p->n_sites;
  for (size_t e = 0; e < NN; ++e)
    if (!std::isfinite(p->hopping[e])) return set_error(PQMC_EINVAL, "non-finite hopping matrix");
  return PQMC_OK;
}

void fill_problem(pqmc_ctx &c, const pqmc_problem *p, const pqmc_update_opts *o) {
  c.N = p->n_sites;
  c.Ns[0] = p->n_up;
  c.Ns[1] = p->n_dn;
  c.M = p->n_slices;
  c.kt = p->stab_every;
  c.nst = c.M / c.kt;
  c.U = p->U;
  c.dtau = p->dtau;
  c.alpha = p->U > 0 ? std::acosh(std::exp(p->dtau * p->U / 2.0)) : 0.0;
  c.seed = p->seed;
  c.walker = p->walker_id;
  c.opts = *o;
  c.kmax = std::min(o->delay_k, c.N);
  c.bmax = std::min(o->block_b, c.N);
  c.gmax = std::max(c.kmax, c.bmax);
  c.log_alloc = (o->flags & PQMC_FLAG_LOG) != 0;
  c.gsized = o->scheme == PQMC_LOCAL_G;
}

const double kSpin[2] = {1.0, -1.0};

// PQMC_FLAG_KTIME: an event pair around one launch, resolved after the call
struct KTimer {
  pqmc_ctx &c;
  int cls;
  size_t i0 = 0;
  bool on;
  KTimer(pqmc_ctx &cc, int k)
      : c(cc), cls(k), on((cc.opts.flags & PQMC_FLAG_KTIME) != 0 && !cc.capturing) {
    if (!on) return;
    while (c.kevs.size() < c.kused + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      c.kevs.push_back(e);
    }
    i0 = c.kused;
    c.kused += 2;
    c.kclass.push_back(cls);
    (void)hipEventRecord(c.kevs[i0], c.st);
  }
  ~KTimer() {
    if (on) (void)hipEventRecord(c.kevs[i0 + 1], c.st);
  }
};

// ------------------------------------------------------------------ helpers
double *other(double *cur, double *const w[2]) { return cur == w[0] ? w[1] : w[0]; }

int sync_check(pqmc_ctx &c) {
  PQ_HIP_CHECK(hipStreamSynchronize(c.st));
  unsigned long long h[16];
  PQ_HIP_CHECK(d2h(h, c.stats, sizeof h, c.st));
  if (h[kStError] & kErrSingular) {
    c.failed = true;
    return set_error(PQMC_ESINGULAR, "stabilisation factorisation broke down (zero pivot)");
  }
  if (h[kStError] & kErrNonFinite) {
    c.failed = true;
    return set_error(PQMC_ENONFINITE, "non-finite determinant ratio");
  }
  if (h[kStError] & kErrBarrier) {
    c.failed = true;
    return set_error(PQMC_EDEVICE, "persistent local update: a grid barrier timed out");
  }
  return PQMC_OK;
}

// A set of walkers of one shape (N, N_sigma, M, k_tau, scheme, k, b) run in
// lockstep on the lead walker's stream: every launch covers all of them.
struct Walkers {
  pqmc_ctx *const *w;
  int n;
  pqmc_ctx &lead() const { return *w[0]; }
  pqmc_ctx &operator[](int i) const { return *w[i]; }
};

// GEMM descriptors queued and launched kGemmMaxBatch at a time.
struct GemmQueue {
  hipStream_t st;
  bool ta, tb;
  GemmBatch cur{};
  int add(const GemmDesc &d) {
    cur.d[cur.count++] = d;
    return cur.count == kGemmMaxBatch ? flush() : PQMC_OK;
  }
  int flush() {
    if (cur.count == 0) return PQMC_OK;
    hipError_t e = gemm(cur, ta, tb, st);
    cur.count = 0;
    if (e != hipSuccess) return fail_device(e, "gemm", __FILE__, __LINE__);
    return PQMC_OK;
  }
};

struct ExpvQueue {
  hipStream_t st;
  ExpvBatch cur{};
  int add(const ExpvDesc &d) {
    cur.d[cur.count++] = d;
    return cur.count == kExpvMaxBatch ? flush() : PQMC_OK;
  }
  int flush() {
    if (cur.count == 0) return PQMC_OK;
    hipError_t e = expv(cur, st);
    cur.count = 0;
    if (e != hipSuccess) return fail_device(e, "sparse propagation", __FILE__, __LINE__);
    return PQMC_OK;
  }
};

// the walker propagates with the sparse H0 (and not the dense K, K^{-1})
bool sparse(const pqmc_ctx &c) {
  return c.sparse_prop && !(c.opts.flags & PQMC_FLAG_DENSE_PROP);
}

// Y = rs * e^{sign dtau H0} (ks * X) for the N x n matrix X (field row
// scaling after the product, or before it when pre)
ExpvDesc expv_desc(const pqmc_ctx &c, const double *X, double *Y, int n, double sign,
                   const int8_t *row, double pos, double neg, bool pre) {
  ExpvDesc d{};
  d.X = X;
  d.ldx = n;
  d.Y = Y;
  d.ldy = n;
  d.N = c.N;
  d.n = n;
  d.idx = c.ell_idx;
  d.val = c.ell_val;
  d.w = c.ell_w;
  d.J = c.taylor_J;
  d.a = sign * c.dtau;
  d.field = row;
  d.pos = pos;
  d.neg = neg;
  d.pre = pre ? 1 : 0;
  return d;
}

bool fp32_form(const pqmc_ctx &c) { return (c.opts.flags & PQMC_FLAG_FP32) != 0; }
// the G-form local update: G (not T) is the updated state between stabilisations
bool gform(const pqmc_ctx &c) { return c.opts.scheme == PQMC_LOCAL_G; }

// G_s = 1 - U_R T U_L (Eq. (15)) into dst[s], both spins (xtmp as scratch)
int assemble_G(pqmc_ctx &c, double *const *dst) {
  const int N = c.N;
  for (int s = 0; s < 2; ++s) {
    const int n = c.Ns[s];
    GemmBatch a{};
    a.d[a.count++] = gemm_desc(c.UR[s], n, c.T[s], n, c.xtmp, n, N, n, n);
    PQ_HIP_CHECK(gemm(a, false, false, c.st));
    GemmBatch b{};
    GemmDesc d = gemm_desc(c.xtmp, n, c.ULt[s], n, dst[s], N, N, N, n, -1.0);
    d.addI = 1;
    b.d[b.count++] = d;
    PQ_HIP_CHECK(gemm(b, false, true, c.st));
  }
  return PQMC_OK;
}

// G-form propagation of G with the slice-l propagator B_l = diag(e^{alpha f x_l}) K:
// forward G <- B_l G B_l^{-1}, backward G <- B_l^{-1} G B_l (the same moves as
// U_R and U_L, Eq. (9)); the field scalings ride on the GEMM epilogue / depth.
int wrap_G(pqmc_ctx &c, int l, bool forward) {
  const int N = c.N;
  const int8_t *row = c.fields + (size_t)(l - 1) * N;
  GemmBatch g1{}, g2{};
  for (int s = 0; s < 2; ++s) {
    const double ep = std::exp(c.alpha * (s ? -1.0 : 1.0)), em = 1.0 / ep;
    if (forward) {
      GemmDesc d1 = gemm_desc(c.K, N, c.G[s], N, c.Gw[s], N, N, N, N);
      d1.rs_field = row; d1.rs_pos = ep; d1.rs_neg = em;
      GemmDesc d2 = gemm_desc(c.Gw[s], N, c.Kinv, N, c.G[s], N, N, N, N);
      d2.cs_field = row; d2.cs_pos = em; d2.cs_neg = ep;
      g1.d[g1.count++] = d1;
      g2.d[g2.count++] = d2;
    } else {
      GemmDesc d1 = gemm_desc(c.Kinv, N, c.G[s], N, c.Gw[s], N, N, N, N);
      d1.ks_field = row; d1.ks_pos = em; d1.ks_neg = ep;
      GemmDesc d2 = gemm_desc(c.Gw[s], N, c.K, N, c.G[s], N, N, N, N);
      d2.ks_field = row; d2.ks_pos = ep; d2.ks_neg = em;
      g1.d[g1.count++] = d1;
      g2.d[g2.count++] = d2;
    }
  }
  PQ_HIP_CHECK(gemm(g1, false, false, c.st));
  PQ_HIP_CHECK(gemm(g2, false, false, c.st));
  return PQMC_OK;
}

// The float32 copy of T from the float64 one (precision form), all walkers
// of the batch that use the form.
int round_T(const Walkers &b) {
  const double *src[kMaxMats];
  float *dst[kMaxMats];
  long n[kMaxMats];
  int m = 0;
  for (int i = 0; i < b.n; ++i) {
    b[i].t32_ahead = false;
    if (!fp32_form(b[i])) continue;
    for (int s = 0; s < 2; ++s) {
      src[m] = b[i].T[s];
      dst[m] = b[i].T32[s];
      n[m] = (long)b[i].Ns[s] * b[i].Ns[s];
      ++m;
    }
  }
  if (m) PQ_HIP_CHECK(round_to_f32(src, dst, m, n, b.lead().st));
  return PQMC_OK;
}

ElimSpin elim_spin(pqmc_ctx &c, int s) {
  const int n = c.Ns[s];
  return ElimSpin{c.E[s], 2L * n, n, 2 * n, c.Z[s], c.prow[s], c.slot[s], c.BR[s], c.F[s], c.stats};
}

// The (walker, spin) matrices of a batch grouped by their size N_sigma, in
// order of first appearance: one elimination launch per size.
struct SizeClass {
  int n, m;
  int w[kMaxMats], s[kMaxMats];
};
std::vector<SizeClass> size_classes(const Walkers &b) {
  std::vector<SizeClass> out;
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      const int n = b[i].Ns[s];
      SizeClass *sc = nullptr;
      for (SizeClass &x : out)
        if (x.n == n) sc = &x;
      if (!sc) {
        out.push_back(SizeClass{n, 0, {}, {}});
        sc = &out.back();
      }
      sc->w[sc->m] = i;
      sc->s[sc->m] = s;
      ++sc->m;
    }
  return out;
}

// One pass of Cholesky QR on the columns of A (N x Ns per walker and spin,
// index 2 w + s) into dst: S = A^T A = R^T R, dst = A R^{-1}.
int cholqr_pass(const Walkers &b, double *const *A, double *const *dst) {
  pqmc_ctx &L = b.lead();
  GemmQueue gram{L.st, true, false};
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      const int n = b[i].Ns[s];
      int rc = gram.add(gemm_desc(A[2 * i + s], n, A[2 * i + s], n, b[i].E[s], 2 * n, n, n, b[i].N));
      if (rc) return rc;
    }
  int rc = gram.flush();
  if (rc) return rc;
  // matrices of equal size go in one elimination call
  for (const SizeClass &sc : size_classes(b)) {
    ElimSpin es[kMaxMats];
    double *E[kMaxMats];
    for (int j = 0; j < sc.m; ++j) {
      es[j] = elim_spin(b[sc.w[j]], sc.s[j]);
      E[j] = es[j].E;
    }
    PQ_HIP_CHECK(set_identity_block(E, sc.m, 2 * sc.n, sc.n, sc.n, L.st));
    PQ_HIP_CHECK(chol_eliminate(es, sc.m, L.st));
  }
  GemmQueue q{L.st, false, true};
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      const int n = b[i].Ns[s];
      rc = q.add(gemm_desc(A[2 * i + s], n, b[i].F[s], n, dst[2 * i + s], n, b[i].N, n, n));
      if (rc) return rc;
    }
  return q.flush();
}

// QR stabilisation of Sec. II B: the columns of A orthonormalised into dst by
// Cholesky QR applied twice (A -> tmp -> dst).  One pass leaves Q^T Q - 1 of
// order kappa(A)^2 eps; the second pass starts from a basis with condition
// number close to one and leaves it at the rounding level.  A Cholesky
// breakdown (kappa(A)^2 eps near one) sets the singular-factorisation error.
// The Green's function depends on U_R (U_L) only through its column (row)
// space; tmp is a free work buffer of the same shape.
int orthonormalize(const Walkers &b, double *const *A, double *const *tmp, double *const *dst) {
  int rc = cholqr_pass(b, A, tmp);
  if (rc) return rc;
  return cholqr_pass(b, tmp, dst);
}

// T = (U_L U_R)^{-1} by blocked Gauss-Jordan with partial pivoting.
int refresh_T(const Walkers &b) {
  pqmc_ctx &L = b.lead();
  GemmQueue q{L.st, true, false};
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      const int n = b[i].Ns[s];
      int rc = q.add(gemm_desc(b[i].ULt[s], n, b[i].UR[s], n, b[i].E[s], 2 * n, n, n, b[i].N));
      if (rc) return rc;
    }
  int rc = q.flush();
  if (rc) return rc;
  for (const SizeClass &sc : size_classes(b)) {
    ElimSpin es[kMaxMats];
    double *E[kMaxMats], *out[kMaxMats];
    for (int j = 0; j < sc.m; ++j) {
      es[j] = elim_spin(b[sc.w[j]], sc.s[j]);
      E[j] = es[j].E;
      out[j] = b[sc.w[j]].T[sc.s[j]];
    }
    PQ_HIP_CHECK(set_identity_block(E, sc.m, 2 * sc.n, sc.n, sc.n, L.st));
    PQ_HIP_CHECK(gj_invert(es, sc.m, out, sc.n, L.st));
  }
  return round_T(b);
}

double *slot(double *stack, int j, const pqmc_ctx &c, int s) {
  return stack + (size_t)j * c.N * c.Ns[s];
}

// position l-1 -> l: U_R <- B_l U_R, U_L <- U_L B_l^{-1}   (Eq. (9))
int prop_forward(const Walkers &b, int l) {
  pqmc_ctx &L = b.lead();
  GemmQueue q{L.st, false, false};
  ExpvQueue xq{L.st};
  KTimer kt(L, PQMC_K_PROPAGATE);
  for (int i = 0; i < b.n; ++i) {
    pqmc_ctx &c = b[i];
    const int8_t *row = c.fields + (size_t)(l - 1) * c.N;
    for (int s = 0; s < 2; ++s) {
      const int n = c.Ns[s];
      const double ep = std::exp(c.alpha * kSpin[s]), em = std::exp(-c.alpha * kSpin[s]);
      double *nur = other(c.UR[s], c.URw[s]);
      double *nul = other(c.ULt[s], c.ULw[s]);
      int rc;
      if (sparse(c)) {
        rc = xq.add(expv_desc(c, c.UR[s], nur, n, -1.0, row, ep, em, false));
        if (!rc) rc = xq.add(expv_desc(c, c.ULt[s], nul, n, +1.0, row, em, ep, false));
      } else {
        GemmDesc d = gemm_desc(c.K, c.N, c.UR[s], n, nur, n, c.N, n, c.N);
        d.rs_field = row; d.rs_pos = ep; d.rs_neg = em;
        rc = q.add(d);
        GemmDesc e = gemm_desc(c.Kinv, c.N, c.ULt[s], n, nul, n, c.N, n, c.N);
        e.rs_field = row; e.rs_pos = em; e.rs_neg = ep;
        if (!rc) rc = q.add(e);
      }
      if (rc) return rc;
      c.UR[s] = nur;
      c.ULt[s] = nul;
    }
  }
  int rc = q.flush();
  if (!rc) rc = xq.flush();
  for (int i = 0; i < b.n && !rc; ++i)
    if (gform(b[i])) rc = wrap_G(b[i], l, true);
  return rc;
}

// position l -> l-1: U_L <- U_L B_l, U_R <- B_l^{-1} U_R
int prop_backward(const Walkers &b, int l, bool with_R) {
  pqmc_ctx &L = b.lead();
  GemmQueue q{L.st, false, false};
  ExpvQueue xq{L.st};
  KTimer kt(L, with_R ? PQMC_K_PROPAGATE : -1);
  for (int i = 0; i < b.n; ++i) {
    pqmc_ctx &c = b[i];
    const int8_t *row = c.fields + (size_t)(l - 1) * c.N;
    for (int s = 0; s < 2; ++s) {
      const int n = c.Ns[s];
      const double ep = std::exp(c.alpha * kSpin[s]), em = std::exp(-c.alpha * kSpin[s]);
      double *nul = other(c.ULt[s], c.ULw[s]);
      int rc;
      if (sparse(c)) {
        rc = xq.add(expv_desc(c, c.ULt[s], nul, n, -1.0, row, ep, em, true));
      } else {
        GemmDesc d = gemm_desc(c.K, c.N, c.ULt[s], n, nul, n, c.N, n, c.N);
        d.ks_field = row; d.ks_pos = ep; d.ks_neg = em;
        rc = q.add(d);
      }
      if (rc) return rc;
      c.ULt[s] = nul;
      if (with_R) {
        double *nur = other(c.UR[s], c.URw[s]);
        if (sparse(c)) {
          rc = xq.add(expv_desc(c, c.UR[s], nur, n, +1.0, row, em, ep, true));
        } else {
          GemmDesc e = gemm_desc(c.Kinv, c.N, c.UR[s], n, nur, n, c.N, n, c.N);
          e.ks_field = row; e.ks_pos = em; e.ks_neg = ep;
          rc = q.add(e);
        }
        if (rc) return rc;
        c.UR[s] = nur;
      }
    }
  }
  int rc = q.flush();
  if (!rc) rc = xq.flush();
  for (int i = 0; i < b.n && !rc && with_R; ++i)
    if (gform(b[i])) rc = wrap_G(b[i], l, false);
  return rc;
}

// Initial stack of row-orthonormalised U_L and position-0 state (Sec. II B).
int build_state(const Walkers &b) {
  for (int i = 0; i < b.n; ++i) {
    pqmc_ctx &c = b[i];
    for (int s = 0; s < 2; ++s) {
      const int n = c.Ns[s];
      PQ_HIP_CHECK(copy_matrix(c.P[s], nullptr, n, slot(c.Lstack[s], c.nst, c, s), nullptr, n,
                               c.N, n, c.st));
      PQ_HIP_CHECK(copy_matrix(c.P[s], nullptr, n, slot(c.Rstack[s], 0, c, s), nullptr, n, c.N,
                               n, c.st));
      c.ULt[s] = slot(c.Lstack[s], c.nst, c, s);
    }
  }
  const pqmc_ctx &L = b.lead();
  for (int l = L.M; l >= 1; --l) {
    int rc = prop_backward(b, l, false);
    if (rc) return rc;
    if ((l - 1) % L.kt == 0) {
      const int j = (l - 1) / L.kt;
      double *src[kMaxMats], *tmp[kMaxMats], *dst[kMaxMats];
      for (int i = 0; i < b.n; ++i)
        for (int s = 0; s < 2; ++s) {
          src[2 * i + s] = b[i].ULt[s];
          tmp[2 * i + s] = other(b[i].ULt[s], b[i].ULw[s]);
          dst[2 * i + s] = slot(b[i].Lstack[s], j, b[i], s);
        }
      rc = orthonormalize(b, src, tmp, dst);
      if (rc) return rc;
      for (int i = 0; i < b.n; ++i)
        for (int s = 0; s < 2; ++s) b[i].ULt[s] = dst[2 * i + s];
    }
  }
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) b[i].UR[s] = slot(b[i].Rstack[s], 0, b[i], s);
  int rc = refresh_T(b);
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) {
    b[i].position = 0;
    b[i].windowed = false;
  }
  return PQMC_OK;
}

// Sparse propagation set-up: H0 qualifies when it has at most kExpMaxW
// nonzeros in every row, N <= kExpMaxN and ||dtau H0||_1 <= 1.  Its rows go
// to the workspace as ELL (zero-padded), and the Taylor degree J is the
// smallest for which the first dropped term, ||dtau H0||_1^(J+1) / (J+1)!,
// is at most 2^-60 (J = 13 at ||dtau H0||_1 = 0.2).
int setup_sparse(pqmc_ctx &c, const double *H, double norm1) {
  const int N = c.N;
  c.sparse_prop = false;
  int w = 0;
  for (int i = 0; i < N; ++i) {
    int nz = 0;
    for (int j = 0; j < N; ++j) nz += H[(size_t)i * N + j] != 0.0;
    w = std::max(w, nz);
  }
  if (w > kExpMaxW || N > kExpMaxN || !(norm1 <= 1.0)) return PQMC_OK;
  w = std::max(w, 1);
  std::vector<int> idx((size_t)N * w);
  std::vector<double> val((size_t)N * w);
  for (int i = 0; i < N; ++i) {
    int m = 0;
    for (int j = 0; j < N; ++j)
      if (H[(size_t)i * N + j] != 0.0) {
        idx[(size_t)i * w + m] = j;
        val[(size_t)i * w + m] = H[(size_t)i * N + j];
        ++m;
      }
    for (; m < w; ++m) {
      idx[(size_t)i * w + m] = i;
      val[(size_t)i * w + m] = 0.0;
    }
  }
  int J = 0;
  double term = 1.0;   // norm1^J / J!
  while (norm1 > 0.0 && term * norm1 / (J + 1) > std::ldexp(1.0, -60)) {
    ++J;
    term *= norm1 / J;
  }
  hipError_t e = hipMemcpyAsync(c.ell_idx, idx.data(), sizeof(int) * idx.size(),
                                hipMemcpyHostToDevice, c.st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c.ell_val, val.data(), sizeof(double) * val.size(),
                       hipMemcpyHostToDevice, c.st);
  if (e == hipSuccess) e = hipStreamSynchronize(c.st);   // the host vectors go away
  if (e != hipSuccess) return fail_device(e, "upload H0 rows", __FILE__, __LINE__);
  c.ell_w = w;
  c.taylor_J = J;
  c.sparse_prop = true;
  return PQMC_OK;
}

// e^{X} for X = sign * dtau * H0 (uploaded in Tay0 unscaled) by a degree-18
// Taylor series in Horner form after scaling by 2^-sq, then sq squarings.
int expm_taylor(pqmc_ctx &c, double scale, int sq, double *dst) {
  const int N = c.N;
  double *Y = dst, *Yn = c.Tay1;
  PQ_HIP_CHECK(set_identity_block(&Y, 1, N, N, 0, c.st));
  for (int j = 18; j >= 1; --j) {
    GemmBatch gb{};
    GemmDesc d = gemm_desc(c.Tay0, N, Y, N, Yn, N, N, N, N, scale / j);
    d.addI = 1;
    gb.d[gb.count++] = d;
    PQ_HIP_CHECK(gemm(gb, false, false, c.st));
    std::swap(Y, Yn);
  }
  for (int q = 0; q < sq; ++q) {
    GemmBatch gb{};
    gb.d[gb.count++] = gemm_desc(Y, N, Y, N, Yn, N, N, N, N);
    PQ_HIP_CHECK(gemm(gb, false, false, c.st));
    std::swap(Y, Yn);
  }
  if (Y != dst) PQ_HIP_CHECK(copy_matrix(Y, nullptr, N, dst, nullptr, N, N, N, c.st));
  return PQMC_OK;
}

SweepCtx sweep_ctx(pqmc_ctx &c, int l, int dir) {
  SweepCtx x{};
  x.key0 = c.seed;
  x.key1 = c.walker;
  x.sweep = c.sweep_index;
  x.slice_code = (uint64_t)dir * c.M + (l - 1);
  x.li = l - 1;
  x.N = c.N;
  x.fields = c.fields;
  for (int s = 0; s < 2; ++s) {
    x.dflip[s][0] = std::expm1(-2.0 * c.alpha * kSpin[s]);
    x.dflip[s][1] = std::expm1(2.0 * c.alpha * kSpin[s]);
    x.dremove[s][0] = std::expm1(-c.alpha * kSpin[s]);
    x.dremove[s][1] = std::expm1(c.alpha * kSpin[s]);
  }
  x.alpha = c.alpha;
  x.stats = c.stats;
  if (c.log_alloc && (c.opts.flags & PQMC_FLAG_LOG)) {
    x.log_meta = c.log_meta;
    x.log_margin = c.log_margin;
    x.hb_meta = c.hb_meta;
    x.hb_margin = c.hb_margin;
  }
  x.log_base = c.log_count;
  x.hb_base = c.hb_count;
  x.log_cap = c.log_cap;
  x.force = c.replaying ? c.replay + (size_t)x.slice_code * c.N : nullptr;
  x.sweep_dev = c.capturing ? c.sweep_dev : nullptr;
  return x;
}

int update_slice(const Walkers &b, int l, int dir) {
  pqmc_ctx &L = b.lead();
  SweepCtx x[kMaxBatch];
  SpinMats m[kMaxBatch];
  LocalBufs lb[kMaxBatch];
  GroupBufs gb[kMaxBatch];
  for (int i = 0; i < b.n; ++i) {
    pqmc_ctx &c = b[i];
    x[i] = sweep_ctx(c, l, dir);
    for (int s = 0; s < 2; ++s) {
      m[i].T[s] = c.T[s];
      m[i].T32[s] = c.T32[s];
      m[i].UR[s] = c.UR[s];
      m[i].ULt[s] = c.ULt[s];
      m[i].Ns[s] = c.Ns[s];
    }
    lb[i] = c.lb;
    gb[i] = c.gb;
  }
  const int N = L.N, nw = b.n;
  switch (L.opts.scheme) {
    case PQMC_LOCAL_G:
    case PQMC_LOCAL: {
      const bool gf = L.opts.scheme == PQMC_LOCAL_G;
      const bool persistent =
          gf || (nw == 1 && !(L.opts.flags & PQMC_FLAG_SITE_LAUNCHES) &&
                 local_persist_fits(L.Ns[0], L.Ns[1], N, false));
      if (persistent) {
        // one cooperative launch per walker and slice (walkers one after another)
        for (int w = 0; w < nw; ++w) {
          pqmc_ctx &c = b[w];
          LocalPersistArgs a{};
          a.m = m[w];
          a.c = x[w];
          a.g = GridSync{c.lp_sync, c.lp_sync + kLocalMaxGroups, 1u << 22};
          for (int s = 0; s < 2; ++s) {
            local_persist_grid(c.Ns[s], &a.pr[s], &a.pc[s]);
            a.P[s] = a.pr[s] * a.pc[s];
            a.ypart[s] = c.lp_y[s];
            a.xpart[s] = c.lp_x[s];
            a.spart[s] = c.lp_s[s];
            a.Gm[s] = c.G[s];
            a.grow_buf[s] = c.grow_buf[s];
          }
          a.grow = std::max(1, ceil_div(c.N, 256));
          KTimer kt(L, PQMC_K_LOCAL);
          PQ_HIP_CHECK(local_persist(a, gf, L.st));
        }
      } else {
        const int nt = ceil_div(std::max(L.Ns[0], L.Ns[1]), 64);
        for (int i = 0; i <= N; ++i) {
          KTimer kt(L, PQMC_K_LOCAL);
          PQ_HIP_CHECK(local_step(m, lb, x, nw, i, nt, L.st));
        }
      }
      for (int i = 0; i < nw; ++i) b[i].log_count += N;
      break;
    }
    case PQMC_DELAYED:
    default: {
      // Every walker's groups start at g0 = 0, k_b, 2 k_b, ... with
      // k_b = min(k, N_max); walker w's group at g0 has
      // kk[w] = min(k_b, N_w - g0) sites (0 once g0 >= N_w), which are the
      // groups it forms alone, since min(k, N_w) = min(k_b, N_w).
      const bool delayed = L.opts.scheme == PQMC_DELAYED;
      int Nmax = 0;
      bool fused = true;
      for (int i = 0; i < nw; ++i) {
        Nmax = std::max(Nmax, b[i].N);
        fused = fused && b[i].gmax <= 64;
      }
      const int k = std::min(delayed ? L.opts.delay_k : L.opts.block_b, Nmax);
      const int mode = delayed ? kUniDelayed : kUniBlock;
      const bool fp32 = fp32_form(L);
      long long bi = 0;
      int g_prev = 0, kk[kMaxBatch], kk_prev[kMaxBatch] = {};
      for (int g0 = 0; g0 < Nmax; g0 += k, ++bi) {
        for (int i = 0; i < nw; ++i) kk[i] = std::max(0, std::min(k, b[i].N - g0));
        if (fused) {
          {
            KTimer kt(L, PQMC_K_TILE);
            PQ_HIP_CHECK(group_tile(m, gb, nw, g_prev, kk_prev, g0, kk, fp32, L.st));
          }
          KTimer kt(L, PQMC_K_REDUCE);
          PQ_HIP_CHECK(group_reduce(m, gb, x, nw, mode, g0, kk, L.st));
        } else {
          PQ_HIP_CHECK(group_panels(m, gb, x, nw, mode, g0, kk, L.st));
        }
        {
          KTimer kt(L, PQMC_K_DECIDE);
          if (delayed) PQ_HIP_CHECK(delayed_decide(gb, x, nw, g0, kk, fused, L.st));
          else PQ_HIP_CHECK(block_decide(gb, x, nw, g0, kk, bi, fused, L.st));
        }
        if (fused) {
          g_prev = g0;
          for (int i = 0; i < nw; ++i) kk_prev[i] = kk[i];
        } else {
          PQ_HIP_CHECK(group_flush(m, gb, nw, g0, kk, L.st));
        }
      }
      if (fused && Nmax > 0) {
        const int none[kMaxBatch] = {};
        KTimer kt(L, PQMC_K_TILE);
        PQ_HIP_CHECK(group_tile(m, gb, nw, g_prev, kk_prev, 0, none, fp32, L.st));
      }
      if (fp32)
        for (int i = 0; i < nw; ++i) b[i].t32_ahead = true;
      for (int i = 0; i < nw; ++i) {
        if (delayed) {
          b[i].log_count += b[i].N;
        } else {
          b[i].log_count += ceil_div(b[i].N, k);
          b[i].hb_count += b[i].N;
        }
      }
      break;
    }
  }
  return PQMC_OK;
}

// Stabilisation drift: the largest change of G = 1 - U_R T U_L that a
// stabilisation makes, over kDriftCols sampled columns j (stride N / cols):
// Z_j = (U_R T U_L)[:, j] = U_R (T ULt[j, :]^T), formed from the running
// state before the QR and inverse (which = 0) and from the fresh state
// after (which = 1).  The identity cancels in the difference.
int drift_cols(const Walkers &b) { return std::min(kDriftCols, b.lead().N); }

int drift_columns(const Walkers &b, int which) {
  pqmc_ctx &L = b.lead();
  if (which == 0) {
    // the precision form's running T lives in float32
    const float *src[kMaxMats];
    double *dst[kMaxMats];
    long n[kMaxMats];
    int m = 0;
    for (int i = 0; i < b.n; ++i) {
      if (!(fp32_form(b[i]) && b[i].t32_ahead)) continue;
      for (int s = 0; s < 2; ++s) {
        src[m] = b[i].T32[s];
        dst[m] = b[i].T[s];
        n[m] = (long)b[i].Ns[s] * b[i].Ns[s];
        ++m;
      }
    }
    if (m) PQ_HIP_CHECK(widen_to_f64(src, dst, m, n, L.st));
  }
  GemmQueue qy{L.st, false, true};
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2 && !gform(b[i]); ++s) {
      pqmc_ctx &c = b[i];
      const int n = c.Ns[s], nc = std::min(kDriftCols, c.N), stride = c.N / nc;
      // Y^T (nc x n) = ULt[J, :] T^T
      int rc = qy.add(gemm_desc(c.ULt[s], (long)stride * n, c.T[s], n, c.drift_y[s], n, nc, n, n));
      if (rc) return rc;
    }
  int rc = qy.flush();
  if (rc) return rc;
  GemmQueue qz{L.st, false, true};
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2 && !gform(b[i]); ++s) {
      pqmc_ctx &c = b[i];
      const int n = c.Ns[s], nc = std::min(kDriftCols, c.N);
      // Z^T (nc x N) = Y^T U_R^T
      rc = qz.add(gemm_desc(c.drift_y[s], n, c.UR[s], n, c.drift_z[s][which], c.N, nc, c.N, n));
      if (rc) return rc;
    }
  rc = qz.flush();
  if (rc || which == 0) return rc;
  const double *za[kMaxMats], *zb[kMaxMats];
  unsigned long long *out[kMaxMats];
  long cnt[kMaxMats];
  int m = 0;
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      pqmc_ctx &c = b[i];
      if (gform(c)) {
        // G-form: the running G against the one rebuilt from the fresh state,
        // every entry; the fresh one is kept
        if (s == 0) {
          rc = assemble_G(c, c.Gw);
          if (rc) return rc;
        }
        za[m] = c.G[s];
        zb[m] = c.Gw[s];
        cnt[m] = (long)c.N * c.N;
      } else {
        za[m] = c.drift_z[s][0];
        zb[m] = c.drift_z[s][1];
        cnt[m] = (long)std::min(kDriftCols, c.N) * c.N;
      }
      out[m] = c.stats + kStDrift;
      ++m;
    }
  PQ_HIP_CHECK(max_abs_diff(za, zb, cnt, out, m, L.st));
  for (int i = 0; i < b.n; ++i)
    if (gform(b[i])) std::swap(b[i].G, b[i].Gw);
  return PQMC_OK;
}

int stab_forward(const Walkers &b, int l) {
  const int j = l / b.lead().kt;
  double *src[kMaxMats], *tmp[kMaxMats], *dst[kMaxMats];
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      src[2 * i + s] = b[i].UR[s];
      tmp[2 * i + s] = other(b[i].UR[s], b[i].URw[s]);
      dst[2 * i + s] = slot(b[i].Rstack[s], j, b[i], s);
    }
  int rc = drift_columns(b, 0);
  if (!rc) rc = orthonormalize(b, src, tmp, dst);
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      b[i].UR[s] = dst[2 * i + s];
      b[i].ULt[s] = slot(b[i].Lstack[s], j, b[i], s);
    }
  rc = refresh_T(b);
  if (!rc) rc = drift_columns(b, 1);
  return rc;
}

int stab_backward(const Walkers &b, int l) {
  const int j = (l - 1) / b.lead().kt;
  double *src[kMaxMats], *tmp[kMaxMats], *dst[kMaxMats];
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      src[2 * i + s] = b[i].ULt[s];
      tmp[2 * i + s] = other(b[i].ULt[s], b[i].ULw[s]);
      dst[2 * i + s] = slot(b[i].Lstack[s], j, b[i], s);
    }
  int rc = drift_columns(b, 0);
  if (!rc) rc = orthonormalize(b, src, tmp, dst);
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i)
    for (int s = 0; s < 2; ++s) {
      b[i].ULt[s] = dst[2 * i + s];
      b[i].UR[s] = slot(b[i].Rstack[s], j, b[i], s);
    }
  rc = refresh_T(b);
  if (!rc) rc = drift_columns(b, 1);
  return rc;
}

// phase timing: events recorded at boundaries, summed per phase at the end
struct PhaseTimer {
  pqmc_ctx &c;
  bool on;
  std::vector<std::pair<int, size_t>> marks;  // (phase, event index of start)
  size_t used = 0;
  explicit PhaseTimer(pqmc_ctx &cc)
      : c(cc), on((cc.opts.flags & PQMC_FLAG_TIMING) != 0 && !(cc.opts.flags & PQMC_FLAG_GRAPH)) {}
  int mark(int phase) {
    if (!on) return PQMC_OK;
    if (used == c.evs.size()) {
      hipEvent_t e;
      PQ_HIP_CHECK(hipEventCreate(&e));
      c.evs.push_back(e);
    }
    PQ_HIP_CHECK(hipEventRecord(c.evs[used], c.st));
    marks.push_back({phase, used});
    ++used;
    return PQMC_OK;
  }
  void totals(double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    if (!on) return;
    for (size_t k = 0; k + 1 < marks.size(); ++k) {
      float ms = 0.f;
      if (marks[k].first < 0) continue;
      if (hipEventElapsedTime(&ms, c.evs[marks[k].second], c.evs[marks[k + 1].second]) ==
          hipSuccess)
        out[marks[k].first] += ms * 1e-3;
    }
  }
};
enum { kPhUpdate = 0, kPhProp = 1, kPhStab = 2, kPhEnd = -1 };

int begin_call(pqmc_ctx &c) {
  PQ_HIP_CHECK(hipMemsetAsync(c.stats, 0, 16 * sizeof(unsigned long long), c.st));
  if (gform(c)) {
    int rc = assemble_G(c, c.G);
    if (rc) return rc;
    c.g_valid = true;
  } else {
    c.g_valid = false;
  }
  c.log_count = 0;
  c.hb_count = 0;
  c.kused = 0;
  c.kclass.clear();
  for (int k = 0; k < PQMC_K_COUNT; ++k) {
    c.kt_total[k] = 0.0;
    c.kt_count[k] = 0;
  }
  return PQMC_OK;
}

void resolve_kernel_times(pqmc_ctx &c) {
  for (size_t p = 0; p < c.kclass.size(); ++p) {
    const int k = c.kclass[p];
    if (k < 0 || k >= PQMC_K_COUNT) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.kevs[2 * p], c.kevs[2 * p + 1]) == hipSuccess) {
      c.kt_total[k] += ms * 1e-3;
      c.kt_count[k] += 1;
    }
  }
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Statistics of one walker after the batch's work has completed.
int finish_walker(pqmc_ctx &c, const double ph[3], double t_total, pqmc_stats *out) {
  int rc = sync_check(c);
  if (out) {
    unsigned long long h[16];
    PQ_HIP_CHECK(d2h(h, c.stats, sizeof h, c.st));
    std::memset(out, 0, sizeof *out);
    out->proposed = h[kStProposed];
    out->accepted = h[kStAccepted];
    out->flips = h[kStFlips];
    out->low_margin = h[kStLowMargin];
    out->negative = h[kStNegative];
    out->field_updates = h[kStFieldUpdates];
    out->t_total_s = t_total;
    out->t_update_s = ph[kPhUpdate];
    out->t_prop_s = ph[kPhProp];
    out->t_stab_s = ph[kPhStab];
    std::memcpy(&out->max_stab_drift, &h[kStDrift], sizeof(double));
  }
  c.hb_total = c.hb_count;
  return rc;
}

int finish_call(const Walkers &b, PhaseTimer &tm, double t0, pqmc_stats *out) {
  pqmc_ctx &L = b.lead();
  int rc = tm.mark(kPhEnd);
  if (rc) return rc;
  PQ_HIP_CHECK(hipStreamSynchronize(L.st));
  resolve_kernel_times(L);
  const double t1 = now_s();
  double ph[3];
  tm.totals(ph);
  for (int i = 0; i < b.n; ++i) {
    const int r = finish_walker(b[i], ph, t1 - t0, out ? out + i : nullptr);
    if (r && !rc) rc = r;
  }
  return rc;
}

int run_forward(const Walkers &b, int upto, PhaseTimer &tm) {
  const int kt = b.lead().kt;
  for (int l = 1; l <= upto; ++l) {
    int rc = tm.mark(kPhProp);
    if (!rc) rc = prop_forward(b, l);
    if (!rc) rc = tm.mark(kPhUpdate);
    if (!rc) rc = update_slice(b, l, 0);
    if (!rc && l % kt == 0) {
      rc = tm.mark(kPhStab);
      if (!rc) rc = stab_forward(b, l);
    }
    if (rc) return rc;
    for (int i = 0; i < b.n; ++i) b[i].position = l;
  }
  return PQMC_OK;
}

int run_backward(const Walkers &b, PhaseTimer &tm) {
  const int M = b.lead().M, kt = b.lead().kt;
  for (int l = M; l >= 1; --l) {
    int rc = tm.mark(kPhUpdate);
    if (!rc) rc = update_slice(b, l, 1);
    if (!rc) rc = tm.mark(kPhProp);
    if (!rc) rc = prop_backward(b, l, true);
    if (!rc && (l - 1) % kt == 0) {
      rc = tm.mark(kPhStab);
      if (!rc) rc = stab_backward(b, l);
    }
    if (rc) return rc;
    for (int i = 0; i < b.n; ++i) b[i].position = l - 1;
  }
  return PQMC_OK;
}

// Walkers run together must agree on everything that shapes the launches.
// The grouped schemes (delayed, block force bias) also run lattices of
// different sizes together: the batch walks the largest lattice's groups and
// a smaller walker sits out the groups beyond its own sites, so that each
// walker sees exactly the group boundaries it sees alone.
pqmc_status check_batch(pqmc_ctx *const *w, int n) {
  if (!w || n < 1 || n > kMaxBatch) return set_error(PQMC_EINVAL, "batch size must be 1..8");
  for (int i = 0; i < n; ++i) {
    if (!w[i]) return set_error(PQMC_EINVAL, "null context in batch");
    if ((w[i]->cx != nullptr) != (w[0]->cx != nullptr))
      return set_error(PQMC_EINVAL, "U < 0 and U >= 0 walkers cannot share a batch");
    if (w[i]->cx) continue;
    const pqmc_ctx &a = *w[0], &c = *w[i];
    if (c.M != a.M || c.kt != a.kt || c.opts.scheme != a.opts.scheme ||
        c.opts.delay_k != a.opts.delay_k || c.opts.block_b != a.opts.block_b || c.st != a.st ||
        fp32_form(c) != fp32_form(a) || (c.gmax <= 64) != (a.gmax <= 64))
      return set_error(PQMC_EINVAL,
                       "batched walkers need the same M, k_tau, scheme, k, b, precision form, "
                       "stream and group-size class (all k <= 64 or all above)");
    if (a.opts.scheme == PQMC_LOCAL &&
        (c.N != a.N || c.Ns[0] != a.Ns[0] || c.Ns[1] != a.Ns[1]))
      return set_error(PQMC_EINVAL, "the local scheme batches walkers of one N and N_sigma only");
    for (int j = 0; j < i; ++j)
      if (w[j] == w[i]) return set_error(PQMC_EINVAL, "a context appears twice in the batch");
    if (c.failed) return set_error(PQMC_ESTATE, "context failed; call pqmc_set_fields");
  }
  return PQMC_OK;
}

pqmc_status as_status(int rc) { return (pqmc_status)rc; }

// U < 0 walkers of a batch: the one-sector engine batches walkers of the
// same size, scheme and k; the others form batches of their own (in order of
// first appearance), run one after the other.
pqmc_status run_one_sector(pqmc_ctx *const *ctxs, int n, int n_sweeps, int n_slices,
                           pqmc_stats *out) {
  std::vector<bool> done(n, false);
  for (int i = 0; i < n; ++i) {
    if (done[i]) continue;
    pqmc_soc_ctx *grp[kMaxBatch];
    int pos[kMaxBatch], m = 0;
    for (int j = i; j < n; ++j)
      if (!done[j] && pq::soc::batch_compatible(ctxs[j]->cx, ctxs[i]->cx)) {
        grp[m] = ctxs[j]->cx;
        pos[m++] = j;
        done[j] = true;
      }
    pqmc_stats st[kMaxBatch];
    const pqmc_status v = pq::soc::batch_run(grp, m, n_sweeps, n_slices, out ? st : nullptr);
    if (v) return v;
    if (out)
      for (int j = 0; j < m; ++j) out[pos[j]] = st[j];
  }
  return PQMC_OK;
}

void drop_graph(pqmc_ctx &c) {
  if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
  if (c.graph) (void)hipGraphDestroy(c.graph);
  c.gexec = nullptr;
  c.graph = nullptr;
  c.gkey.clear();
  c.ggen.clear();
}

bool graph_mode(const Walkers &b) {
  for (int i = 0; i < b.n; ++i)
    if (!(b[i].opts.flags & PQMC_FLAG_GRAPH)) return false;
  const int sch = b.lead().opts.scheme;
  return sch == PQMC_DELAYED || sch == PQMC_BLOCK_FB;
}

// The batch's captured sweep: reused while the batch and every walker's
// generation are unchanged, captured (one forward and one backward pass,
// recorded but not run) otherwise.  Capturing leaves the host-side state
// where a real sweep leaves it, which is where it started.
int sweep_graph(const Walkers &b) {
  pqmc_ctx &L = b.lead();
  bool same = L.gexec && (int)L.gkey.size() == b.n;
  for (int i = 0; same && i < b.n; ++i)
    same = L.gkey[i] == &b[i] && L.ggen[i] == b[i].generation;
  if (same) return PQMC_OK;
  drop_graph(L);
  if (!L.st) return set_error(PQMC_EINVAL, "graph-captured sweeps need a non-null stream");
  for (int i = 0; i < b.n; ++i) b[i].capturing = true;
  PQ_HIP_CHECK(hipStreamBeginCapture(L.st, hipStreamCaptureModeRelaxed));
  PhaseTimer off(L);
  int rc = run_forward(b, L.M, off);
  if (!rc) rc = run_backward(b, off);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(L.st, &g);
  for (int i = 0; i < b.n; ++i) {
    // the host-side log positions the capture advanced are those every
    // launch of the graph fills; each call starts them again from zero
    b[i].capturing = false;
    b[i].glog = b[i].log_count;
    b[i].ghb = b[i].hb_count;
    b[i].log_count = 0;
    b[i].hb_count = 0;
  }
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail_device(e, "hipStreamEndCapture", __FILE__, __LINE__);
  L.graph = g;
  PQ_HIP_CHECK(hipGraphInstantiate(&L.gexec, g, nullptr, nullptr, 0));
  for (int i = 0; i < b.n; ++i) {
    L.gkey.push_back(&b[i]);
    L.ggen.push_back(b[i].generation);
  }
  return PQMC_OK;
}

// Device scratch of pqmc_get_green_static: X = U_R T and G, 32 MiB per GPU,
// held by every GPU the library runs on until the process ends.  Host code
// never uses the array's name as an address: its device address is looked
// up once per device (hipGetSymbolAddress, that device current) and kept.
constexpr size_t kStaticScratchDoubles = size_t(1) << 22;
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
// The device address of `scratch` on the current device.
int static_scratch(double **out) {
  int dev = 0;
  PQ_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(PQMC_EDEVICE, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    PQ_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(PQMC_EDEVICE, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return PQMC_OK;
}
}  // namespace

extern "C" {

const char *pqmc_last_error(void) { return g_last_error.c_str(); }

pqmc_status pqmc_workspace_bytes(const pqmc_problem *prob, const pqmc_update_opts *opts,
                                 size_t *bytes) {
  if (!bytes) return set_error(PQMC_EINVAL, "null bytes");
  if (prob && prob->U < 0) return pq::soc::one_sector_workspace_bytes(prob, opts, bytes);
  pqmc_status v = validate(prob, opts);
  if (v) return v;
  pqmc_ctx c;
  fill_problem(c, prob, opts);
  layout(c, nullptr, bytes);
  return PQMC_OK;
}

pqmc_status pqmc_create(const pqmc_problem *prob, const pqmc_update_opts *opts, void *hip_stream,
                        void *workspace, size_t workspace_bytes, pqmc_ctx **out) {
  if (!out) return set_error(PQMC_EINVAL, "null out");
  *out = nullptr;
  if (prob && prob->U < 0) {
    pqmc_ctx *c = new (std::nothrow) pqmc_ctx();
    if (!c) return set_error(PQMC_ENOMEM, "host allocation failed");
    pqmc_status st = pq::soc::one_sector_create(prob, opts, hip_stream, workspace,
                                                workspace_bytes, &c->cx);
    if (st) {
      delete c;
      return st;
    }
    pq::soc::one_sector_dims(c->cx, &c->N, &c->M);
    c->st = static_cast<hipStream_t>(hip_stream);
    c->opts = *opts;
    *out = c;
    return PQMC_OK;
  }
  pqmc_status v = validate(prob, opts);
  if (v) return v;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
    return set_error(PQMC_EINVAL, "workspace must be a 256-byte aligned device pointer");
  pqmc_ctx *c = new (std::nothrow) pqmc_ctx();
  if (!c) return set_error(PQMC_ENOMEM, "host allocation failed");
  fill_problem(*c, prob, opts);
  size_t need = 0;
  layout(*c, nullptr, &need);
  if (workspace_bytes < need) {
    delete c;
    return set_error(PQMC_ENOMEM, "workspace smaller than pqmc_workspace_bytes()");
  }
  layout(*c, static_cast<char *>(workspace), &need);
  c->st = static_cast<hipStream_t>(hip_stream);
  auto fail = [&](int rc) {
    delete c;
    return as_status(rc);
  };
  const int N = c->N;
  // host: trial states and H0 (scaled below) to the device
  int rc = PQMC_OK;
  {
    hipError_t e = hipMemcpyAsync(c->P[0], prob->trial_up, sizeof(double) * N * c->Ns[0],
                                  hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->P[1], prob->trial_dn, sizeof(double) * N * c->Ns[1],
                         hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->Tay0, prob->hopping, sizeof(double) * N * N, hipMemcpyHostToDevice,
                         c->st);
    if (e != hipSuccess) return fail(fail_device(e, "upload", __FILE__, __LINE__));
  }
  // scaling: ||dtau H0||_1 / 2^sq <= 1/2
  double norm1 = 0.0;
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += std::fabs(prob->hopping[(size_t)i * N + j]);
    norm1 = std::max(norm1, s);
  }
  norm1 *= prob->dtau;
  rc = setup_sparse(*c, prob->hopping, norm1);
  if (rc) return fail(rc);
  int sq = 0;
  while (norm1 / std::ldexp(1.0, sq) > 0.5) ++sq;
  const double sc = prob->dtau / std::ldexp(1.0, sq);
  rc = expm_taylor(*c, -sc, sq, c->K);
  if (!rc) rc = expm_taylor(*c, +sc, sq, c->Kinv);
  if (!rc) {
    hipError_t e = hipMemsetAsync(c->stats, 0, 16 * sizeof(unsigned long long), c->st);
    if (e != hipSuccess) rc = fail_device(e, "memset", __FILE__, __LINE__);
  }
  if (!rc) {
    hipError_t e = init_fields(c->fields, c->M, N, c->seed, c->walker, c->st);
    if (e != hipSuccess) rc = fail_device(e, "init_fields", __FILE__, __LINE__);
  }
  if (!rc) {
    pqmc_ctx *one[1] = {c};
    rc = build_state(Walkers{one, 1});
  }
  if (!rc) rc = sync_check(*c);
  if (rc) return fail(rc);
  *out = c;
  return PQMC_OK;
}

pqmc_status pqmc_set_opts(pqmc_ctx *c, const pqmc_update_opts *o) {
  if (!c || !o) return set_error(PQMC_EINVAL, "null argument");
  if (c->cx) {
    pqmc_status st = pq::soc::one_sector_set_opts(c->cx, o);
    if (!st) c->opts = *o;
    return st;
  }
  if (o->scheme < PQMC_LOCAL || o->scheme > PQMC_LOCAL_G) return set_error(PQMC_EINVAL, "scheme");
  if (o->scheme == PQMC_LOCAL_G && !c->gsized)
    return set_error(PQMC_EINVAL, "the G-form local update needs a context created with it");
  if (o->delay_k < 1 || std::min(o->delay_k, c->N) > c->gmax)
    return set_error(PQMC_EINVAL, "delay_k exceeds the workspace bound");
  if (o->block_b < 1 || o->block_b > 64 || std::min(o->block_b, c->N) > c->gmax)
    return set_error(PQMC_EINVAL, "block_b exceeds the workspace bound");
  if ((o->flags & PQMC_FLAG_LOG) && !c->log_alloc)
    return set_error(PQMC_EINVAL, "logging was not sized in the workspace");
  if (o->tile_chunks < 0) return set_error(PQMC_EINVAL, "tile_chunks must be >= 0");
  if ((o->flags & PQMC_FLAG_FP32) &&
      (o->scheme == PQMC_LOCAL || o->scheme == PQMC_LOCAL_G ||
       (o->scheme == PQMC_DELAYED ? o->delay_k : o->block_b) > 64))
    return set_error(PQMC_EINVAL, "the float32 form needs the delayed or block scheme, k, b <= 64");
  const bool was = fp32_form(*c), now = (o->flags & PQMC_FLAG_FP32) != 0;
  c->opts = *o;
  c->g_valid = false;
  ++c->generation;
  c->gb.chunks = o->tile_chunks > 0 ? o->tile_chunks : 2;
  // the current T moves to the representation the next call reads
  hipError_t e = hipSuccess;
  const long cnt[2] = {(long)c->Ns[0] * c->Ns[0], (long)c->Ns[1] * c->Ns[1]};
  if (now && !was) {
    const double *src[2] = {c->T[0], c->T[1]};
    float *dst[2] = {c->T32[0], c->T32[1]};
    e = round_to_f32(src, dst, 2, cnt, c->st);
  } else if (was && !now && c->t32_ahead) {
    const float *src[2] = {c->T32[0], c->T32[1]};
    double *dst[2] = {c->T[0], c->T[1]};
    e = widen_to_f64(src, dst, 2, cnt, c->st);
  }
  if (e != hipSuccess) return as_status(fail_device(e, "precision switch", __FILE__, __LINE__));
  c->t32_ahead = false;
  return PQMC_OK;
}

pqmc_status pqmc_set_fields(pqmc_ctx *c, const int8_t *fields) {
  if (!c || !fields) return set_error(PQMC_EINVAL, "null argument");
  if (c->cx) return pq::soc::one_sector_set_fields(c->cx, fields);
  const size_t n = (size_t)c->M * c->N;
  for (size_t e = 0; e < n; ++e)
    if (fields[e] != 1 && fields[e] != -1) return set_error(PQMC_EINVAL, "fields must be +-1");
  hipError_t e = hipMemcpyAsync(c->fields, fields, n, hipMemcpyHostToDevice, c->st);
  if (e != hipSuccess) return as_status(fail_device(e, "upload fields", __FILE__, __LINE__));
  e = hipMemsetAsync(c->stats, 0, 16 * sizeof(unsigned long long), c->st);
  if (e != hipSuccess) return as_status(fail_device(e, "memset", __FILE__, __LINE__));
  c->failed = false;
  c->g_valid = false;
  ++c->generation;
  pqmc_ctx *one[1] = {c};
  int rc = build_state(Walkers{one, 1});
  if (!rc) rc = sync_check(*c);
  return as_status(rc);
}

pqmc_status pqmc_get_fields(pqmc_ctx *c, int8_t *fields) {
  if (!c || !fields) return set_error(PQMC_EINVAL, "null argument");
  if (c->cx) return pqmc_soc_get_fields(c->cx, fields);
  hipError_t e = hipStreamSynchronize(c->st);
  if (e == hipSuccess)
    e = d2h(fields, c->fields, (size_t)c->M * c->N, c->st);
  if (e != hipSuccess) return as_status(fail_device(e, "download fields", __FILE__, __LINE__));
  return PQMC_OK;
}

pqmc_status pqmc_batch_sweep(pqmc_ctx *const *ctxs, int32_t n, int32_t n_sweeps,
                             pqmc_stats *out) {
  pqmc_status v = check_batch(ctxs, n);
  if (v) return v;
  if (n_sweeps < 0) return set_error(PQMC_EINVAL, "n_sweeps < 0");
  if (ctxs[0]->cx) return run_one_sector(ctxs, n, n_sweeps, -1, out);
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->windowed || ctxs[i]->position != 0)
      return set_error(PQMC_ESTATE, "walker is mid-sweep after pqmc_forward_window");
  const Walkers b{ctxs, n};
  const double t0 = now_s();
  int rc = PQMC_OK;
  for (int i = 0; i < n && !rc; ++i) rc = begin_call(b[i]);
  PhaseTimer tm(b.lead());
  if (!rc && n_sweeps > 0 && graph_mode(b)) {
    // one graph launch per sweep; the sweep counter goes to the device first
    rc = sweep_graph(b);
    for (int k = 0; k < n_sweeps && !rc; ++k) {
      uint64_t *ptr[kMaxBatch];
      uint64_t val[kMaxBatch];
      for (int i = 0; i < n; ++i) {
        ptr[i] = b[i].sweep_dev;
        val[i] = b[i].sweep_index;
      }
      hipError_t e = set_u64(ptr, val, n, b.lead().st);
      if (e == hipSuccess) e = hipGraphLaunch(b.lead().gexec, b.lead().st);
      if (e != hipSuccess) rc = fail_device(e, "hipGraphLaunch", __FILE__, __LINE__);
      if (!rc)
        for (int i = 0; i < n; ++i) {
          ++b[i].sweep_index;
          b[i].log_count = b[i].glog;
          b[i].hb_count = b[i].ghb;
        }
    }
  } else {
    for (int k = 0; k < n_sweeps && !rc; ++k) {
      rc = run_forward(b, b.lead().M, tm);
      if (!rc) rc = run_backward(b, tm);
      if (!rc)
        for (int i = 0; i < n; ++i) ++b[i].sweep_index;
    }
  }
  if (rc) {
    for (int i = 0; i < n; ++i) {
      b[i].failed = true;
      ++b[i].generation;
    }
    return as_status(rc);
  }
  return as_status(finish_call(b, tm, t0, out));
}

pqmc_status pqmc_multi_sweep(pqmc_ctx *const *ctxs, int32_t n, int32_t n_sweeps,
                             pqmc_stats *out) {
  constexpr int kMaxStreams = 16;
  if (!ctxs || n < 1 || n > kMaxStreams * kMaxBatch)
    return set_error(PQMC_EINVAL, "multi-stream sweep takes 1..128 contexts");
  if (n_sweeps < 0) return set_error(PQMC_EINVAL, "n_sweeps < 0");
  // one batch per stream, streams in order of first appearance
  std::vector<hipStream_t> streams;
  std::vector<std::vector<pqmc_ctx *>> grp;
  std::vector<std::vector<int>> pos;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return set_error(PQMC_EINVAL, "null context in batch");
    size_t g = 0;
    while (g < streams.size() && streams[g] != ctxs[i]->st) ++g;
    if (g == streams.size()) {
      if ((int)g == kMaxStreams) return set_error(PQMC_EINVAL, "more than 16 streams");
      streams.push_back(ctxs[i]->st);
      grp.emplace_back();
      pos.emplace_back();
    }
    grp[g].push_back(ctxs[i]);
    pos[g].push_back(i);
  }
  const int G = (int)grp.size();
  for (int g = 0; g < G; ++g) {
    pqmc_status v = check_batch(grp[g].data(), (int)grp[g].size());
    if (v) return v;
    for (pqmc_ctx *c : grp[g])
      if (c->windowed || c->position != 0)
        return set_error(PQMC_ESTATE, "walker is mid-sweep after pqmc_forward_window");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(PQMC_EDEVICE, "hipGetDevice failed");
  std::vector<std::vector<pqmc_stats>> st(G);
  std::vector<pqmc_status> rc(G, PQMC_OK);
  std::vector<std::string> msg(G);
  auto work = [&](int g, bool own_thread) {
    try {
      if (own_thread && hipSetDevice(dev) != hipSuccess) {
        rc[g] = PQMC_EDEVICE;
        msg[g] = "hipSetDevice failed in a worker thread";
        return;
      }
      st[g].resize(grp[g].size());
      rc[g] = pqmc_batch_sweep(grp[g].data(), (int)grp[g].size(), n_sweeps, st[g].data());
      if (rc[g]) msg[g] = g_last_error;
    } catch (...) {
      rc[g] = PQMC_ENOMEM;
      msg[g] = "host allocation failed in a multi-stream sweep";
    }
  };
  // batch 0 on the calling thread, the others on their own threads; a
  // thread that cannot be started runs its batch afterwards on this one
  std::vector<std::thread> th;
  std::vector<int> inline_g;
  for (int g = 1; g < G; ++g) {
    try {
      th.emplace_back(work, g, true);
    } catch (...) {
      inline_g.push_back(g);
    }
  }
  work(0, false);
  for (std::thread &t : th) t.join();
  for (int g : inline_g) work(g, false);
  for (int g = 0; g < G; ++g)
    if (rc[g]) return set_error(rc[g], msg[g]);
  if (out)
    for (int g = 0; g < G; ++g)
      for (size_t j = 0; j < pos[g].size(); ++j) out[pos[g][j]] = st[g][j];
  return PQMC_OK;
}

pqmc_status pqmc_sweep(pqmc_ctx *c, int32_t n_sweeps, pqmc_stats *out) {
  if (!c) return set_error(PQMC_EINVAL, "null context");
  pqmc_ctx *one[1] = {c};
  return pqmc_batch_sweep(one, 1, n_sweeps, out);
}

pqmc_status pqmc_replay(pqmc_ctx *c, const int8_t *flips, pqmc_stats *out) {
  if (!c || !flips) return set_error(PQMC_EINVAL, "null argument");
  if (c->cx) return pq::soc::one_sector_replay(c->cx, flips, out);
  if (c->failed) return set_error(PQMC_ESTATE, "context failed; call pqmc_set_fields");
  if (c->windowed || c->position != 0)
    return set_error(PQMC_ESTATE, "walker is mid-sweep after pqmc_forward_window");
  const size_t n = (size_t)2 * c->M * c->N;
  hipError_t e = hipMemcpyAsync(c->replay, flips, n, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);   // the host array may go away
  if (e != hipSuccess) return as_status(fail_device(e, "upload replay", __FILE__, __LINE__));
  c->replaying = true;
  ++c->generation;
  pqmc_ctx *one[1] = {c};
  const pqmc_status st = pqmc_batch_sweep(one, 1, 1, out);
  c->replaying = false;
  ++c->generation;
  return st;
}

pqmc_status pqmc_batch_forward_window(pqmc_ctx *const *ctxs, int32_t n, int32_t n_slices,
                                      pqmc_stats *out) {
  pqmc_status v = check_batch(ctxs, n);
  if (v) return v;
  if (n_slices < 0 || n_slices > ctxs[0]->M) return set_error(PQMC_EINVAL, "n_slices out of range");
  if (ctxs[0]->cx) return run_one_sector(ctxs, n, 0, n_slices, out);
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->windowed || ctxs[i]->position != 0)
      return set_error(PQMC_ESTATE, "walker is mid-sweep");
  const Walkers b{ctxs, n};
  const double t0 = now_s();
  int rc = PQMC_OK;
  for (int i = 0; i < n && !rc; ++i) rc = begin_call(b[i]);
  PhaseTimer tm(b.lead());
  if (!rc) rc = run_forward(b, n_slices, tm);
  for (int i = 0; i < n; ++i) {
    b[i].windowed = true;
    ++b[i].generation;
  }
  if (rc) {
    for (int i = 0; i < n; ++i) b[i].failed = true;
    return as_status(rc);
  }
  return as_status(finish_call(b, tm, t0, out));
}

pqmc_status pqmc_forward_window(pqmc_ctx *c, int32_t n_slices, pqmc_stats *out) {
  if (!c) return set_error(PQMC_EINVAL, "null context");
  pqmc_ctx *one[1] = {c};
  return pqmc_batch_forward_window(one, 1, n_slices, out);
}

// G^s = 1 - U_R T U_L into the host array out, with X = U_R T (N x N_s) and
// G (N x N) formed in the device scratch X, Gd.
static pqmc_status green_into(pqmc_ctx *c, int spin, double *X, double *Gd, double *out) {
  const int N = c->N, n = c->Ns[spin];
  if (gform(*c)) {
    // the G-form's state: G itself (at position 0 of a fresh context, or
    // before any G-form call, it is assembled first)
    hipError_t e = hipSuccess;
    if (!c->g_valid) {
      if (assemble_G(*c, c->G)) return PQMC_EDEVICE;
      c->g_valid = true;
    }
    e = hipStreamSynchronize(c->st);
    if (e == hipSuccess)
      e = d2h(out, c->G[spin], sizeof(double) * N * N, c->st);
    if (e != hipSuccess) return as_status(fail_device(e, "green", __FILE__, __LINE__));
    return PQMC_OK;
  }
  if (fp32_form(*c) && c->t32_ahead) {
    // flushes since the last stabilisation live in the float32 copy only
    const float *src[1] = {c->T32[spin]};
    double *dst[1] = {c->T[spin]};
    const long cnt[1] = {(long)n * n};
    hipError_t e = widen_to_f64(src, dst, 1, cnt, c->st);
    if (e != hipSuccess) return as_status(fail_device(e, "green", __FILE__, __LINE__));
  }
  GemmBatch a{};
  a.d[a.count++] = gemm_desc(c->UR[spin], n, c->T[spin], n, X, n, N, n, n);
  hipError_t e = gemm(a, false, false, c->st);
  GemmBatch b{};
  GemmDesc d = gemm_desc(X, n, c->ULt[spin], n, Gd, N, N, N, n, -1.0);
  d.addI = 1;
  b.d[b.count++] = d;
  if (e == hipSuccess) e = gemm(b, false, true, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e == hipSuccess) e = d2h(out, Gd, sizeof(double) * N * N, c->st);
  if (e != hipSuccess) return as_status(fail_device(e, "green", __FILE__, __LINE__));
  return PQMC_OK;
}

pqmc_status pqmc_get_green(pqmc_ctx *c, int32_t spin, double *out) {
  if (!c || !out || spin < 0 || spin > 1) return set_error(PQMC_EINVAL, "bad argument");
  if (c->cx) return pq::soc::one_sector_green(c->cx, spin, out);
  return green_into(c, spin, c->xtmp, c->gtmp, out);
}

pqmc_status pqmc_get_green_static(pqmc_ctx *c, int32_t spin, double *out) {
  if (!c || !out || spin < 0 || spin > 1) return set_error(PQMC_EINVAL, "bad argument");
  if (c->cx) return set_error(PQMC_EINVAL, "pqmc_get_green_static: U < 0 is not supported");
  const size_t N = c->N, n = c->Ns[spin];
  const size_t xs = (N * n + 31) / 32 * 32;   // G starts 256-byte aligned
  if (xs + N * N > kStaticScratchDoubles)
    return set_error(PQMC_EINVAL, "pqmc_get_green_static: N (N + N_sigma) exceeds the static "
                                  "scratch of 4194304 doubles (32 MiB)");
  double *ptr = nullptr;
  const int rc = static_scratch(&ptr);
  if (rc) return as_status(rc);
  return green_into(c, spin, ptr, ptr + xs, out);
}

static pqmc_status copy_log(pqmc_ctx *c, const int32_t *dmeta, const double *dmargin,
                            long long count, int32_t *meta, double *margin, size_t cap,
                            size_t *n) {
  if (!c || !n) return set_error(PQMC_EINVAL, "null argument");
  if (!c->log_alloc) return set_error(PQMC_EINVAL, "logging was not enabled at creation");
  const size_t cnt = (size_t)std::min<long long>(count, c->log_cap);
  *n = cnt;
  const size_t m = std::min(cnt, cap);
  hipError_t e = hipStreamSynchronize(c->st);
  if (e == hipSuccess && m && meta)
    e = d2h(meta, dmeta, 3 * sizeof(int32_t) * m, c->st);
  if (e == hipSuccess && m && margin)
    e = d2h(margin, dmargin, sizeof(double) * m, c->st);
  if (e != hipSuccess) return as_status(fail_device(e, "log copy", __FILE__, __LINE__));
  return PQMC_OK;
}

pqmc_status pqmc_get_decisions(pqmc_ctx *c, int32_t *meta, double *margin, size_t cap,
                               size_t *n) {
  if (!c) return set_error(PQMC_EINVAL, "null context");
  if (c->cx) return pqmc_soc_get_decisions(c->cx, meta, margin, cap, n);
  return copy_log(c, c->log_meta, c->log_margin, c->log_count, meta, margin, cap, n);
}

pqmc_status pqmc_get_heat_bath(pqmc_ctx *c, int32_t *meta, double *margin, size_t cap,
                               size_t *n) {
  if (!c) return set_error(PQMC_EINVAL, "null context");
  if (c->cx) return set_error(PQMC_EINVAL, "heat-bath draws are not logged for U < 0");
  return copy_log(c, c->hb_meta, c->hb_margin, c->hb_total, meta, margin, cap, n);
}

pqmc_status pqmc_get_kernel_times(pqmc_ctx *c, double *totals, uint64_t *counts) {
  if (!c || !totals || !counts) return set_error(PQMC_EINVAL, "null argument");
  for (int k = 0; k < PQMC_K_COUNT; ++k) {
    totals[k] = c->kt_total[k];
    counts[k] = c->kt_count[k];
  }
  return PQMC_OK;
}

pqmc_status pqmc_destroy(pqmc_ctx *c) {
  if (!c) return PQMC_OK;
  if (c->cx) {
    pqmc_soc_destroy(c->cx);
    delete c;
    return PQMC_OK;
  }
  (void)hipStreamSynchronize(c->st);
  drop_graph(*c);
  for (hipEvent_t e : c->evs) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->kevs) (void)hipEventDestroy(e);
  delete c;
  return PQMC_OK;
}

}  // extern "C"
