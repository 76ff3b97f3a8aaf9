// C ABI of the spin-orbit coupled Hubbard path (pqmc_soc_*): one walker per
// context, one complex sector of dimension 2N (Appendix A of the paper).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pqmc.h"
#include "engine.hpp"
#include "soc.hpp"

using namespace pq;
using namespace pq::soc;

struct pqmc_soc_ctx {
  // w: orbitals per site in the sector.  2: the spin-orbit coupled model
  // (rows i and N + i, 2 x 2 rotations).  1: the paper's U < 0 model of
  // Sec. II B, one complex spin-up sector with diagonal phases (spin down is
  // its complex conjugate and is never stored).
  int w = 2;
  int N = 0, n2 = 0, ne = 0, M = 0, kt = 0, nst = 0, k = 1;
  double U = 0, dtau = 0, gamma = 0, c1 = 1, s1 = 0, dd = 0, doff = 0;
  uint64_t seed = 0, walker = 0;
  pqmc_update_opts opts{};
  hipStream_t st = nullptr;
  // device buffers (complex128 unless noted)
  double2 *K = nullptr, *Kinv = nullptr, *P = nullptr;
  double2 *Lstack = nullptr, *Rstack = nullptr;     // (nst + 1) slots of n2 x ne
  double2 *Rw[2] = {nullptr, nullptr}, *Lw[2] = {nullptr, nullptr}, *Xtmp = nullptr;
  double2 *UR = nullptr, *ULt = nullptr;            // current (a slot or a work buffer)
  double2 *E = nullptr;                             // ne x 2ne: [U_L U_R | I] -> [I | T]
  double2 *T = nullptr;                             // = E (left half), leading dim 2 ne
  long ldT = 0;
  double2 *gjB = nullptr;                           // Gauss-Jordan block rows and Z
  int *gjP = nullptr;                               // Gauss-Jordan pivot order
  double2 *P2 = nullptr, *P1 = nullptr, *W0 = nullptr, *D = nullptr, *Q = nullptr;
  double2 *P2part = nullptr, *P1part = nullptr, *W0part = nullptr;   // split-K slices
  int ksplit = 0;                                   // depth per slice (0: no split)
  double2 *Tay0 = nullptr, *Tay1 = nullptr;         // n2 x n2 (set-up, then G)
  // H0 in ELL form (n2 x kCexpMaxW) for the Taylor propagation, its degree J;
  // sparse_prop when H0 qualifies (at most kCexpMaxW entries a row, dtau ||H0|| <= 1)
  int *ell_idx = nullptr;
  double2 *ell_val = nullptr;
  int ell_w = 0, taylor_J = 0;
  bool sparse_prop = false;
  int *nflush = nullptr;
  int *accx = nullptr;                              // accepted sites' old fields (decide)
  int8_t *fields = nullptr;
  int8_t *replay = nullptr;                         // 2 M x N forced outcomes (w = 1)
  bool replaying = false;
  unsigned long long *stats = nullptr;
  int32_t *log_meta = nullptr;
  double *log_margin = nullptr;
  long long log_cap = 0, log_count = 0;
  uint64_t sweep_index = 0;
  int position = 0;
  bool windowed = false, failed = false;
  bool block = false;   // block force bias: one decision per group of k sites
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace {

constexpr unsigned kSocFlags = PQMC_FLAG_LOG | PQMC_FLAG_TIMING | PQMC_FLAG_DENSE_PROP;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

pqmc_status err(pqmc_status st, const char *msg) { return (pqmc_status)api_error(st, msg); }

pqmc_status validate(const pqmc_soc_problem *p, const pqmc_update_opts *o) {
  if (!p || !o) return err(PQMC_EINVAL, "null problem or options");
  if (p->n_sites < 1) return err(PQMC_EINVAL, "n_sites must be >= 1");
  if (p->n_e < 1 || p->n_e > 2 * p->n_sites) return err(PQMC_EINVAL, "need 1 <= n_e <= 2 n_sites");
  if (p->n_e > 1024) return err(PQMC_EINVAL, "n_e above 1024 is not supported");
  if (!p->hopping || !p->trial) return err(PQMC_EINVAL, "null input");
  if (!(p->dtau > 0) || !std::isfinite(p->dtau)) return err(PQMC_EINVAL, "dtau must be > 0");
  if (!std::isfinite(p->U) || p->U > 0)
    return err(PQMC_EINVAL, "the spin-s^y decoupling needs a finite U <= 0");
  if (p->n_slices < 1 || p->stab_every < 1 || p->n_slices % p->stab_every)
    return err(PQMC_EINVAL, "stab_every must divide n_slices");
  if (o->scheme != PQMC_LOCAL && o->scheme != PQMC_DELAYED && o->scheme != PQMC_BLOCK_FB)
    return err(PQMC_EINVAL, "unknown scheme");
  if (o->scheme == PQMC_DELAYED && (o->delay_k < 1 || o->delay_k > kSocMaxK))
    return err(PQMC_EINVAL, "delay_k in [1, 32] for the SOC path");
  if (o->scheme == PQMC_BLOCK_FB && (o->block_b < 1 || o->block_b > kSocMaxK))
    return err(PQMC_EINVAL, "block_b in [1, 32] for the SOC path");
  if (o->flags & ~kSocFlags) return err(PQMC_EINVAL, "flags: only LOG, TIMING and DENSE_PROP");
  const long n2 = 2L * p->n_sites;
  double asym = 0.0, amax = 0.0;
  for (long i = 0; i < n2; ++i)
    for (long j = 0; j < n2; ++j) {
      const double *a = p->hopping + 2 * (i * n2 + j), *b = p->hopping + 2 * (j * n2 + i);
      if (!std::isfinite(a[0]) || !std::isfinite(a[1]))
        return err(PQMC_EINVAL, "non-finite hopping matrix");
      asym = std::max(asym, std::fabs(a[0] - b[0]) + std::fabs(a[1] + b[1]));
      amax = std::max(amax, std::fabs(a[0]) + std::fabs(a[1]));
    }
  if (asym > 1e-12 * std::max(1.0, amax)) return err(PQMC_EINVAL, "hopping matrix not Hermitian");
  return PQMC_OK;
}

void fill(pqmc_soc_ctx &c, const pqmc_soc_problem *p, const pqmc_update_opts *o) {
  c.N = p->n_sites;
  c.n2 = 2 * p->n_sites;
  c.ne = p->n_e;
  c.M = p->n_slices;
  c.kt = p->stab_every;
  c.nst = c.M / c.kt;
  c.U = p->U;
  c.dtau = p->dtau;
  c.gamma = std::acos(std::exp(p->dtau * p->U / 2.0));
  c.c1 = std::cos(c.gamma);
  c.s1 = std::sin(c.gamma);
  // delta = A(-x)^2 - 1 = [[c^2 - s^2 - 1, -x 2cs], [x 2cs, c^2 - s^2 - 1]]
  c.dd = (c.c1 * c.c1 - c.s1 * c.s1) - 1.0;
  c.doff = 2.0 * c.c1 * c.s1;
  c.seed = p->seed;
  c.walker = p->walker_id;
  c.opts = *o;
  c.k = o->scheme == PQMC_DELAYED    ? std::min(o->delay_k, c.N)
        : o->scheme == PQMC_BLOCK_FB ? std::min(o->block_b, c.N)
                                     : 1;
  c.block = o->scheme == PQMC_BLOCK_FB;
  // panels over the depth N_e in at most 8 slices of >= 64 (none below 128)
  c.ksplit = c.ne <= 128 ? 0 : std::max(64, ((c.ne + 7) / 8 + 15) / 16 * 16);
}

struct Carve {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = (off + 255) / 256 * 256;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

void layout(pqmc_soc_ctx &c, char *base, size_t *bytes) {
  Carve cv{base};
  const size_t n2 = c.n2, ne = c.ne, kn = 2 * (size_t)kSocMaxK;
  c.K = cv.take<double2>(n2 * n2);
  c.Kinv = cv.take<double2>(n2 * n2);
  c.Tay0 = cv.take<double2>(n2 * n2);
  c.Tay1 = cv.take<double2>(n2 * n2);
  c.ell_idx = cv.take<int>(n2 * kCexpMaxW);
  c.ell_val = cv.take<double2>(n2 * kCexpMaxW);
  c.P = cv.take<double2>(n2 * ne);
  c.Lstack = cv.take<double2>((c.nst + 1) * n2 * ne);
  c.Rstack = cv.take<double2>((c.nst + 1) * n2 * ne);
  for (int i = 0; i < 2; ++i) {
    c.Rw[i] = cv.take<double2>(n2 * ne);
    c.Lw[i] = cv.take<double2>(n2 * ne);
  }
  c.Xtmp = cv.take<double2>(n2 * ne);
  c.E = cv.take<double2>(ne * 2 * ne);
  c.T = c.E;
  c.ldT = 2L * (long)ne;
  c.gjB = cv.take<double2>(gj_scratch_complex(ne));
  c.gjP = cv.take<int>(gj_scratch_int(ne));
  c.P2 = cv.take<double2>(kn * ne);
  c.P1 = cv.take<double2>(ne * kn);
  c.W0 = cv.take<double2>(kn * kn);
  c.D = cv.take<double2>(kn * kn);
  c.Q = cv.take<double2>(ne * kn);
  if (c.ksplit > 0) {
    const size_t ns = (ne + c.ksplit - 1) / c.ksplit;
    c.P2part = cv.take<double2>(ns * kn * ne);
    c.P1part = cv.take<double2>(ns * ne * kn);
    c.W0part = cv.take<double2>(ns * kn * kn);
  }
  c.nflush = cv.take<int>(4);
  c.accx = cv.take<int>(2 * kSocMaxK);
  c.fields = cv.take<int8_t>((size_t)c.M * c.N);
  if (c.w == 1) c.replay = cv.take<int8_t>((size_t)2 * c.M * c.N);
  c.stats = cv.take<unsigned long long>(16);
  if (c.opts.flags & PQMC_FLAG_LOG) {
    c.log_cap = 2LL * c.M * c.N;
    c.log_meta = cv.take<int32_t>(3 * (size_t)c.log_cap);
    c.log_margin = cv.take<double>((size_t)c.log_cap);
  }
  *bytes = cv.off;
}

double2 *slot(double2 *stack, int j, const pqmc_soc_ctx &c) {
  return stack + (size_t)j * c.n2 * c.ne;
}
double2 *other(const double2 *cur, double2 *const w[2]) { return cur == w[0] ? w[1] : w[0]; }

int gemm1(const CgemmDesc &d, int opA, int opB, hipStream_t st) {
  CgemmBatch b{};
  b.d[0] = d;
  b.count = 1;
  PQ_HIP_CHECK(cgemm(b, opA, opB, st));
  return PQMC_OK;
}

// dst = e^{scale H0}: Taylor series of degree 18 in Horner form for the
// scaled exponent, then sq squarings.  H0 sits in Tay0 (kept); Tay1 is scratch.
int expm(pqmc_soc_ctx &c, double scale, int sq, double2 *dst) {
  const int n = c.n2;
  double2 *Y = dst, *Yn = c.Tay1;
  PQ_HIP_CHECK(set_identity(Y, n, n, 0, c.st));
  for (int j = 18; j >= 1; --j) {
    CgemmDesc d = cdesc(c.Tay0, n, Y, n, Yn, n, n, n, n);
    d.alpha = make_double2(scale / j, 0.0);
    d.addI = 1;
    int rc = gemm1(d, kOpN, kOpN, c.st);
    if (rc) return rc;
    std::swap(Y, Yn);
  }
  for (int q = 0; q < sq; ++q) {
    int rc = gemm1(cdesc(Y, n, Y, n, Yn, n, n, n, n), kOpN, kOpN, c.st);
    if (rc) return rc;
    std::swap(Y, Yn);
  }
  if (Y != dst)
    PQ_HIP_CHECK(hipMemcpyAsync(dst, Y, sizeof(double2) * (size_t)n * n,
                                hipMemcpyDeviceToDevice, c.st));
  return PQMC_OK;
}

// The walkers of one call: one, or a batch that shares n2, n_e, M, k_tau, the
// scheme, k, the width w and the stream.  Every launch of the engine serves
// all of them: the complex GEMMs take one descriptor per walker and matrix,
// the decisions and the eliminations one workgroup (row) per walker.  A
// walker's results do not depend on its batch partners.
struct SocWalkers {
  pqmc_soc_ctx *const *w;
  int n;
  pqmc_soc_ctx &operator[](int i) const { return *w[i]; }
  pqmc_soc_ctx &lead() const { return *w[0]; }
};

struct CgemmQueue {
  hipStream_t st;
  int opA, opB;
  CgemmBatch cur{};
  int add(const CgemmDesc &d) {
    cur.d[cur.count++] = d;
    return cur.count == kCgemmMaxBatch ? flush() : PQMC_OK;
  }
  int flush() {
    if (cur.count == 0) return PQMC_OK;
    hipError_t e = cgemm(cur, opA, opB, st);
    cur.count = 0;
    if (e != hipSuccess) return fail_device(e, "cgemm", __FILE__, __LINE__);
    return PQMC_OK;
  }
};

struct CexpvQueue {
  hipStream_t st;
  CexpvBatch cur{};
  int add(const CexpvDesc &d) {
    cur.d[cur.count++] = d;
    return cur.count == kCexpvMaxBatch ? flush() : PQMC_OK;
  }
  int flush() {
    if (cur.count == 0) return PQMC_OK;
    hipError_t e = cexpv(cur, st);
    cur.count = 0;
    if (e != hipSuccess) return fail_device(e, "cexpv", __FILE__, __LINE__);
    return PQMC_OK;
  }
};

// the Taylor propagation applies (H0 qualified and the dense form not asked for)
bool sparse(const pqmc_soc_ctx &c) {
  return c.sparse_prop && !(c.opts.flags & PQMC_FLAG_DENSE_PROP);
}

// Y = e^{a M} X for M = H0 (conj = 0) or H0^T = conj(H0) (conj = 1)
CexpvDesc cexpv_desc(const pqmc_soc_ctx &c, const double2 *X, double2 *Y, double a, int conj) {
  return CexpvDesc{X, c.ne, Y, c.ne, c.n2, c.ne, c.ell_idx, c.ell_val, c.ell_w, c.taylor_J, a,
                   conj};
}

struct CsumQueue {
  hipStream_t st;
  CsumBatch cur{};
  int add(const CsumDesc &d) {
    cur.d[cur.count++] = d;
    return cur.count == kCgemmMaxBatch ? flush() : PQMC_OK;
  }
  int flush() {
    if (cur.count == 0) return PQMC_OK;
    hipError_t e = csum(cur, st);
    cur.count = 0;
    if (e != hipSuccess) return fail_device(e, "csum", __FILE__, __LINE__);
    return PQMC_OK;
  }
};

SocElimBatch elim_batch(const SocWalkers &b) {
  SocElimBatch e{};
  for (int i = 0; i < b.n; ++i) {
    e.E[i] = b[i].E;
    e.B[i] = b[i].gjB;
    e.piv[i] = b[i].gjP;
    e.stats[i] = b[i].stats;
  }
  e.n = b.n;
  return e;
}

// dst[i] = A[i] R^{-1} with A^H A = R^H R (A: n2 x ne): columns orthonormalised.
// E serves as scratch: [A^H A | I] -> R^{-1} in the left half.
int orthonormalize(const SocWalkers &b, const double2 *const *A, double2 *const *dst) {
  pqmc_soc_ctx &L = b.lead();
  const int n2 = L.n2, ne = L.ne;
  const long ld = 2L * ne;
  CgemmQueue gram{L.st, kOpH, kOpN};
  for (int i = 0; i < b.n; ++i) {
    int rc = gram.add(cdesc(A[i], ne, A[i], ne, b[i].E, ld, ne, ne, n2));
    if (rc) return rc;
  }
  int rc = gram.flush();
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) PQ_HIP_CHECK(set_identity(b[i].E, ld, ne, ne, L.st));
  PQ_HIP_CHECK(chol_inverse(elim_batch(b), ld, ne, L.st));
  CgemmQueue out{L.st, kOpN, kOpN};
  for (int i = 0; i < b.n; ++i) {
    rc = out.add(cdesc(A[i], ne, b[i].E, ld, dst[i], ne, n2, ne, ne));
    if (rc) return rc;
  }
  return out.flush();
}

// T = (U_L U_R)^{-1} = (ULt^T UR)^{-1}, in the left half of E
int refresh_T(const SocWalkers &b) {
  pqmc_soc_ctx &L = b.lead();
  const int n2 = L.n2, ne = L.ne;
  CgemmQueue q{L.st, kOpT, kOpN};
  for (int i = 0; i < b.n; ++i) {
    int rc = q.add(cdesc(b[i].ULt, ne, b[i].UR, ne, b[i].E, 2L * ne, ne, ne, n2));
    if (rc) return rc;
  }
  int rc = q.flush();
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) PQ_HIP_CHECK(set_identity(b[i].E, 2L * ne, ne, ne, L.st));
  PQ_HIP_CHECK(gj_inverse(elim_batch(b), 2L * ne, ne, L.st));
  return PQMC_OK;
}

// position l-1 -> l: U_R <- e^{H_I(x_l)} K U_R; U_L <- U_L K^{-1} e^{-H_I(x_l)},
// i.e. ULt <- [e^{-H_I}]^T K^{-T} ULt, whose 2x2 blocks are A(x).
int prop_forward(const SocWalkers &b, int l) {
  pqmc_soc_ctx &L = b.lead();
  const int n2 = L.n2, ne = L.ne;
  CgemmQueue qr{L.st, kOpN, kOpN}, ql{L.st, kOpT, kOpN};
  CexpvQueue qx{L.st};
  for (int i = 0; i < b.n; ++i) {
    pqmc_soc_ctx &c = b[i];
    int rc;
    if (sparse(c)) {   // K = e^{-dtau H0}; K^{-T} = e^{dtau H0^T}
      rc = qx.add(cexpv_desc(c, c.UR, other(c.UR, c.Rw), -c.dtau, 0));
      if (!rc) rc = qx.add(cexpv_desc(c, c.ULt, other(c.ULt, c.Lw), c.dtau, 1));
    } else {
      rc = qr.add(cdesc(c.K, n2, c.UR, ne, other(c.UR, c.Rw), ne, n2, ne, n2));
      if (!rc) rc = ql.add(cdesc(c.Kinv, n2, c.ULt, ne, other(c.ULt, c.Lw), ne, n2, ne, n2));
    }
    if (rc) return rc;
  }
  int rc = qr.flush();
  if (!rc) rc = ql.flush();
  if (!rc) rc = qx.flush();
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) {
    pqmc_soc_ctx &c = b[i];
    const int8_t *x = c.fields + (size_t)(l - 1) * c.N;
    double2 *nur = other(c.UR, c.Rw), *nul = other(c.ULt, c.Lw);
    if (c.w == 1) {
      // U_R <- diag(e^{i gamma x}) K U_R; ULt <- diag(e^{-i gamma x}) K^{-T} ULt
      PQ_HIP_CHECK(phase_rows(nur, ne, nur, ne, ne, c.N, x, c.c1, c.s1, 1.0, c.st));
      PQ_HIP_CHECK(phase_rows(nul, ne, nul, ne, ne, c.N, x, c.c1, c.s1, -1.0, c.st));
    } else {
      PQ_HIP_CHECK(rotate_rows(nur, ne, nur, ne, ne, c.N, x, c.c1, c.s1, 1.0, c.st));
      PQ_HIP_CHECK(rotate_rows(nul, ne, nul, ne, ne, c.N, x, c.c1, c.s1, 1.0, c.st));
    }
    c.UR = nur;
    c.ULt = nul;
  }
  return PQMC_OK;
}

// position l -> l-1: U_L <- U_L e^{H_I(x_l)} K, i.e. ULt <- K^T [e^{H_I}]^T ULt
// (blocks A(-x)); U_R <- K^{-1} e^{-H_I(x_l)} U_R (blocks A(-x)).  The
// rotations go to a scratch buffer: the current matrices may be stack slots.
int prop_backward(const SocWalkers &b, int l, bool with_R) {
  pqmc_soc_ctx &L = b.lead();
  const int n2 = L.n2, ne = L.ne;
  // ULt <- K^T diag(e^{i gamma x}) ULt; U_R <- K^{-1} diag(e^{-i gamma x}) U_R (w = 1)
  CgemmQueue ql{L.st, kOpT, kOpN};
  CexpvQueue qx{L.st};
  for (int i = 0; i < b.n; ++i) {
    pqmc_soc_ctx &c = b[i];
    const int8_t *x = c.fields + (size_t)(l - 1) * c.N;
    if (c.w == 1)
      PQ_HIP_CHECK(phase_rows(c.ULt, ne, c.Xtmp, ne, ne, c.N, x, c.c1, c.s1, 1.0, c.st));
    else
      PQ_HIP_CHECK(rotate_rows(c.ULt, ne, c.Xtmp, ne, ne, c.N, x, c.c1, c.s1, -1.0, c.st));
    const int rc = sparse(c)   // K^T = e^{-dtau H0^T}
                       ? qx.add(cexpv_desc(c, c.Xtmp, other(c.ULt, c.Lw), -c.dtau, 1))
                       : ql.add(cdesc(c.K, n2, c.Xtmp, ne, other(c.ULt, c.Lw), ne, n2, ne, n2));
    if (rc) return rc;
  }
  int rc = ql.flush();
  if (!rc) rc = qx.flush();
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) b[i].ULt = other(b[i].ULt, b[i].Lw);
  if (!with_R) return PQMC_OK;
  CgemmQueue qr{L.st, kOpN, kOpN};
  CexpvQueue qy{L.st};
  for (int i = 0; i < b.n; ++i) {
    pqmc_soc_ctx &c = b[i];
    const int8_t *x = c.fields + (size_t)(l - 1) * c.N;
    if (c.w == 1)
      PQ_HIP_CHECK(phase_rows(c.UR, ne, c.Xtmp, ne, ne, c.N, x, c.c1, c.s1, -1.0, c.st));
    else
      PQ_HIP_CHECK(rotate_rows(c.UR, ne, c.Xtmp, ne, ne, c.N, x, c.c1, c.s1, -1.0, c.st));
    rc = sparse(c)   // K^{-1} = e^{dtau H0}
             ? qy.add(cexpv_desc(c, c.Xtmp, other(c.UR, c.Rw), c.dtau, 0))
             : qr.add(cdesc(c.Kinv, n2, c.Xtmp, ne, other(c.UR, c.Rw), ne, n2, ne, n2));
    if (rc) return rc;
  }
  rc = qr.flush();
  if (!rc) rc = qy.flush();
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) b[i].UR = other(b[i].UR, b[i].Rw);
  return PQMC_OK;
}

int build_state(pqmc_soc_ctx &c) {
  const size_t mat = (size_t)c.n2 * c.ne;
  pqmc_soc_ctx *one[1] = {&c};
  const SocWalkers b{one, 1};
  // U_L = P^+ at position M: ULt = conj(P)
  PQ_HIP_CHECK(conj_copy(c.P, slot(c.Lstack, c.nst, c), (long)mat, c.st));
  PQ_HIP_CHECK(hipMemcpyAsync(slot(c.Rstack, 0, c), c.P, sizeof(double2) * mat,
                              hipMemcpyDeviceToDevice, c.st));
  c.ULt = slot(c.Lstack, c.nst, c);
  c.UR = slot(c.Rstack, 0, c);
  for (int l = c.M; l >= 1; --l) {
    int rc = prop_backward(b, l, false);
    if (rc) return rc;
    if ((l - 1) % c.kt == 0) {
      double2 *dst = slot(c.Lstack, (l - 1) / c.kt, c);
      const double2 *src[1] = {c.ULt};
      double2 *dd[1] = {dst};
      rc = orthonormalize(b, src, dd);
      if (rc) return rc;
      c.ULt = dst;
    }
  }
  c.UR = slot(c.Rstack, 0, c);
  c.position = 0;
  c.windowed = false;
  return refresh_T(b);
}

int timer_mark(pqmc_soc_ctx &c) {
  if (!(c.opts.flags & PQMC_FLAG_TIMING)) return PQMC_OK;
  if (c.ev_used == c.ev.size()) {
    hipEvent_t e;
    PQ_HIP_CHECK(hipEventCreate(&e));
    c.ev.push_back(e);
  }
  PQ_HIP_CHECK(hipEventRecord(c.ev[c.ev_used++], c.st));
  return PQMC_OK;
}

// Field update of slice l (direction dir): groups of k sites (k = 1: the
// local update), each: panels P2 = W_g T, P1 = T U_L[:, g], W0' = P2 U_L[:, g],
// the decisions in 2k x 2k space (one decision per site, or one block
// force-bias decision per group), then T -= (P1 D) P2; every step one launch
// for the whole batch.
int update_slice(const SocWalkers &b, int l, int dir) {
  pqmc_soc_ctx &L = b.lead();
  const int N = L.N, ne = L.ne, li = l - 1;
  for (int i = 0; i < b.n; ++i) {
    int rc = timer_mark(b[i]);
    if (rc) return rc;
  }
  int nblk = 0;
  for (int g0 = 0; g0 < N; g0 += L.k, ++nblk) {
    const int kk = std::min(L.k, N - g0), n = L.w * kk;
    // P2 = W_g T; then P1 = T U_L[:, g] and W0' = P2 U_L[:, g].  Over a deep
    // N_e the products run as split-K slices, added in order by csum.
    const bool split = L.ksplit > 0;
    const int ns = split ? (ne + L.ksplit - 1) / L.ksplit : 1;
    const long s2 = (long)n * ne, s1 = (long)ne * n, sw = (long)n * n;
    CgemmQueue qa{L.st, kOpN, kOpN};
    for (int i = 0; i < b.n; ++i) {
      pqmc_soc_ctx &c = b[i];
      double2 *p2 = split ? c.P2part : c.P2;
      const double2 *ur0 = c.UR + (size_t)g0 * ne, *ur1 = c.UR + (size_t)(N + g0) * ne;
      CgemmDesc d0 = cdesc(ur0, ne, c.T, c.ldT, p2, ne, kk, ne, ne);
      CgemmDesc d1 = cdesc(ur1, ne, c.T, c.ldT, p2 + (size_t)kk * ne, ne, kk, ne, ne);
      if (split) {
        d0.ksplit = d1.ksplit = c.ksplit;
        d0.csplit = d1.csplit = s2;
      }
      int rc = qa.add(d0);
      if (!rc && c.w == 2) rc = qa.add(d1);
      if (rc) return rc;
    }
    int rc = qa.flush();
    if (rc) return rc;
    if (split) {
      CsumQueue r{L.st};
      for (int i = 0; i < b.n && !rc; ++i)
        rc = r.add(CsumDesc{b[i].P2part, s2, ne, b[i].P2, ne, n, ne, ns});
      if (!rc) rc = r.flush();
      if (rc) return rc;
    }
    CgemmQueue qb{L.st, kOpN, kOpT};
    for (int i = 0; i < b.n; ++i) {
      pqmc_soc_ctx &c = b[i];
      double2 *p1 = split ? c.P1part : c.P1, *w0 = split ? c.W0part : c.W0;
      const double2 *ul0 = c.ULt + (size_t)g0 * ne, *ul1 = c.ULt + (size_t)(N + g0) * ne;
      CgemmDesc d[4];
      int m = 0;
      d[m++] = cdesc(c.T, c.ldT, ul0, ne, p1, n, ne, kk, ne);
      if (c.w == 2) d[m++] = cdesc(c.T, c.ldT, ul1, ne, p1 + kk, n, ne, kk, ne);
      const int np1 = m;
      d[m++] = cdesc(c.P2, ne, ul0, ne, w0, n, n, kk, ne);
      if (c.w == 2) d[m++] = cdesc(c.P2, ne, ul1, ne, w0 + kk, n, n, kk, ne);
      for (int j = 0; j < m; ++j) {
        if (split) {
          d[j].ksplit = c.ksplit;
          d[j].csplit = j < np1 ? s1 : sw;
        }
        rc = qb.add(d[j]);
        if (rc) return rc;
      }
    }
    rc = qb.flush();
    if (rc) return rc;
    if (split) {
      CsumQueue r{L.st};
      for (int i = 0; i < b.n && !rc; ++i) {
        rc = r.add(CsumDesc{b[i].P1part, s1, n, b[i].P1, n, ne, n, ns});
        if (!rc) rc = r.add(CsumDesc{b[i].W0part, sw, n, b[i].W0, n, n, n, ns});
      }
      if (!rc) rc = r.flush();
      if (rc) return rc;
    }
    SocDecideArgs da[kSocMaxBatch];
    for (int i = 0; i < b.n; ++i) {
      pqmc_soc_ctx &c = b[i];
      SocDecideArgs d{};
      d.W0p = c.W0;
      d.D = c.D;
      d.UR = c.UR;
      d.nflush = c.nflush;
      d.accx = c.accx;
      d.fields = c.fields;
      d.li = li;
      d.N = N;
      d.ne = ne;
      d.g0 = g0;
      d.kk = kk;
      d.dd = c.dd;
      d.doff = c.doff;
      d.c1 = c.c1;
      d.s1 = c.s1;
      d.gamma = c.gamma;
      d.key0 = c.seed;
      d.key1 = c.walker;
      d.sweep = c.sweep_index;
      d.slice_code = (uint64_t)dir * c.M + li;
      d.stats = c.stats;
      d.log_meta = c.log_meta;
      d.log_margin = c.log_margin;
      d.log_base = c.block ? c.log_count + nblk : c.log_count;
      d.log_cap = c.log_cap;
      d.force = c.replaying ? c.replay + ((size_t)dir * c.M + li) * N : nullptr;
      da[i] = d;
    }
    if (L.block && L.w == 1) {
      PQ_HIP_CHECK(block_decide1(da, b.n, L.st));
    } else {
      PQ_HIP_CHECK(L.block ? block_decide(da, b.n, L.st)
                           : (L.w == 1 ? decide1(da, b.n, L.st) : decide(da, b.n, L.st)));
      PQ_HIP_CHECK(rotate_accepted(da, b.n, L.w, L.st));
    }
    CgemmQueue qq{L.st, kOpN, kOpN};
    for (int i = 0; i < b.n && !rc; ++i) {
      CgemmDesc q = cdesc(b[i].P1, n, b[i].D, n, b[i].Q, n, ne, n, n);
      q.Kdev = b[i].nflush;
      rc = qq.add(q);
    }
    if (!rc) rc = qq.flush();
    if (rc) return rc;
    CgemmQueue qu{L.st, kOpN, kOpN};
    for (int i = 0; i < b.n && !rc; ++i) {
      pqmc_soc_ctx &c = b[i];
      CgemmDesc u = cdesc(c.Q, n, c.P2, ne, c.T, c.ldT, ne, ne, n);
      u.alpha = make_double2(-1.0, 0.0);
      u.beta = make_double2(1.0, 0.0);
      u.Cin = c.T;
      u.ldcin = c.ldT;
      u.Kdev = c.nflush;
      rc = qu.add(u);
    }
    if (!rc) rc = qu.flush();
    if (rc) return rc;
  }
  for (int i = 0; i < b.n; ++i) {
    b[i].log_count += L.block ? nblk : N;
    int rc = timer_mark(b[i]);
    if (rc) return rc;
  }
  return PQMC_OK;
}

int stab_forward(const SocWalkers &b, int l) {
  const int j = l / b.lead().kt;
  const double2 *src[kSocMaxBatch];
  double2 *dst[kSocMaxBatch];
  for (int i = 0; i < b.n; ++i) {
    src[i] = b[i].UR;
    dst[i] = slot(b[i].Rstack, j, b[i]);
  }
  int rc = orthonormalize(b, src, dst);
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) {
    b[i].UR = dst[i];
    b[i].ULt = slot(b[i].Lstack, j, b[i]);
  }
  return refresh_T(b);
}

int stab_backward(const SocWalkers &b, int l) {
  const int j = (l - 1) / b.lead().kt;
  const double2 *src[kSocMaxBatch];
  double2 *dst[kSocMaxBatch];
  for (int i = 0; i < b.n; ++i) {
    src[i] = b[i].ULt;
    dst[i] = slot(b[i].Lstack, j, b[i]);
  }
  int rc = orthonormalize(b, src, dst);
  if (rc) return rc;
  for (int i = 0; i < b.n; ++i) {
    b[i].ULt = dst[i];
    b[i].UR = slot(b[i].Rstack, j, b[i]);
  }
  return refresh_T(b);
}

int begin_call(pqmc_soc_ctx &c) {
  PQ_HIP_CHECK(hipMemsetAsync(c.stats, 0, sizeof(unsigned long long) * 16, c.st));
  c.log_count = 0;
  c.ev_used = 0;
  return PQMC_OK;
}

int finish_call(pqmc_soc_ctx &c, double t0, pqmc_stats *out) {
  PQ_HIP_CHECK(hipStreamSynchronize(c.st));
  unsigned long long h[16];
  PQ_HIP_CHECK(d2h(h, c.stats, sizeof h, c.st));
  if (h[kStError] & kErrSingular) {
    c.failed = true;
    return api_error(PQMC_ESINGULAR, "a stabilisation factorisation broke down");
  }
  if (h[kStError] & kErrNonFinite) {
    c.failed = true;
    return api_error(PQMC_ENONFINITE, "a determinant ratio was not finite");
  }
  if (out) {
    std::memset(out, 0, sizeof *out);
    out->proposed = h[kStProposed];
    out->accepted = h[kStAccepted];
    out->flips = h[kStFlips];
    out->low_margin = h[kStLowMargin];
    out->negative = h[kStNegative];
    out->field_updates = h[kStFieldUpdates];
    out->t_total_s = now_s() - t0;
    double upd = 0.0;
    for (size_t i = 0; i + 1 < c.ev_used; i += 2) {
      float ms = 0.f;
      PQ_HIP_CHECK(hipEventElapsedTime(&ms, c.ev[i], c.ev[i + 1]));
      upd += ms * 1e-3;
    }
    out->t_update_s = upd;
  }
  return PQMC_OK;
}

int sync_check(pqmc_soc_ctx &c) {
  PQ_HIP_CHECK(hipStreamSynchronize(c.st));
  unsigned long long h[16];
  PQ_HIP_CHECK(d2h(h, c.stats, sizeof h, c.st));
  if (h[kStError] & kErrSingular)
    return api_error(PQMC_ESINGULAR, "a factorisation broke down while building the state");
  return PQMC_OK;
}

}  // namespace

extern "C" {

pqmc_status pqmc_soc_workspace_bytes(const pqmc_soc_problem *prob, const pqmc_update_opts *opts,
                                     size_t *bytes) {
  if (!bytes) return err(PQMC_EINVAL, "null bytes");
  pqmc_status v = validate(prob, opts);
  if (v) return v;
  pqmc_soc_ctx c;
  fill(c, prob, opts);
  layout(c, nullptr, bytes);
  return PQMC_OK;
}

// Set-up shared by both widths: workspace checks, H0 (n2 x n2 complex,
// interleaved) and the trial state to the device, e^{-+dtau H0}, Philox
// fields, the L-stack and the position-0 state.  Takes ownership of c.
static pqmc_status create_common(pqmc_soc_ctx *c, const double *hopping, const double *trial,
                                 void *hip_stream, void *workspace, size_t workspace_bytes,
                                 pqmc_soc_ctx **out) {
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
    delete c;
    return err(PQMC_EINVAL, "workspace must be a 256-byte aligned device pointer");
  }
  c->st = (hipStream_t)hip_stream;
  size_t need = 0;
  layout(*c, nullptr, &need);
  if (need > workspace_bytes) {
    delete c;
    return err(PQMC_ENOMEM, "workspace too small");
  }
  layout(*c, (char *)workspace, &need);
  auto fail = [&](int rc) {
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
    return (pqmc_status)rc;
  };
  const size_t n2 = c->n2, ne = c->ne;
  // H0 scaled into Tay0, P into place; host inputs are copied here
  double norm = 0.0;
  for (size_t i = 0; i < n2; ++i) {
    double row = 0.0;
    for (size_t j = 0; j < n2; ++j)
      row += std::hypot(hopping[2 * (i * n2 + j)], hopping[2 * (i * n2 + j) + 1]);
    norm = std::max(norm, row);
  }
  hipError_t e = hipMemcpyAsync(c->Tay0, hopping, sizeof(double2) * n2 * n2,
                                hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->P, trial, sizeof(double2) * n2 * ne, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipMemsetAsync(c->stats, 0, sizeof(unsigned long long) * 16, c->st);
  // the uploads read pageable host memory: finish them before the caller's
  // (possibly temporary) arrays can go away
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return fail(fail_device(e, "upload", __FILE__, __LINE__));
  const double x = c->dtau * norm;
  // H0 in ELL form for the Taylor propagation when it is sparse enough; the
  // degree J is the smallest whose first dropped term x^{J+1} / (J+1)! is at
  // most 2^-60 (x = dtau ||H0|| <= 1, ||H0|| the largest absolute row sum)
  {
    int w = 0;
    for (size_t i = 0; i < n2; ++i) {
      int nz = 0;
      for (size_t j = 0; j < n2; ++j)
        nz += (hopping[2 * (i * n2 + j)] != 0.0 || hopping[2 * (i * n2 + j) + 1] != 0.0);
      w = std::max(w, nz);
    }
    if (w <= kCexpMaxW && (int)n2 <= kCexpMaxN && x <= 1.0) {
      w = std::max(w, 1);
      std::vector<int> idx(n2 * w);
      std::vector<double2> val(n2 * w);
      for (size_t i = 0; i < n2; ++i) {
        int m = 0;
        for (size_t j = 0; j < n2; ++j) {
          const double re = hopping[2 * (i * n2 + j)], im = hopping[2 * (i * n2 + j) + 1];
          if (re != 0.0 || im != 0.0) {
            idx[i * w + m] = (int)j;
            val[i * w + m] = make_double2(re, im);
            ++m;
          }
        }
        for (; m < w; ++m) {
          idx[i * w + m] = (int)i;
          val[i * w + m] = make_double2(0.0, 0.0);
        }
      }
      int J = 0;
      double term = 1.0;   // x^J / J!
      while (x > 0.0 && term * x / (J + 1) > std::ldexp(1.0, -60)) {
        ++J;
        term *= x / J;
      }
      hipError_t ee = hipMemcpyAsync(c->ell_idx, idx.data(), sizeof(int) * idx.size(),
                                     hipMemcpyHostToDevice, c->st);
      if (ee == hipSuccess)
        ee = hipMemcpyAsync(c->ell_val, val.data(), sizeof(double2) * val.size(),
                            hipMemcpyHostToDevice, c->st);
      if (ee == hipSuccess) ee = hipStreamSynchronize(c->st);   // the host vectors go away
      if (ee != hipSuccess) return fail(fail_device(ee, "upload H0 rows", __FILE__, __LINE__));
      c->ell_w = w;
      c->taylor_J = J;
      c->sparse_prop = true;
    }
  }
  const int sq = x > 0.5 ? (int)std::ceil(std::log2(x / 0.5)) : 0;
  const double scale = c->dtau / std::ldexp(1.0, sq);
  int rc = expm(*c, -scale, sq, c->K);
  if (!rc) rc = expm(*c, scale, sq, c->Kinv);
  if (!rc) {
    e = init_fields(c->fields, c->M, c->N, c->seed, c->walker, c->st);
    if (e != hipSuccess) rc = fail_device(e, "init_fields", __FILE__, __LINE__);
  }
  if (!rc) rc = build_state(*c);
  if (!rc) rc = sync_check(*c);
  if (rc) return fail(rc);
  *out = c;
  return PQMC_OK;
}

pqmc_status pqmc_soc_create(const pqmc_soc_problem *prob, const pqmc_update_opts *opts,
                            void *hip_stream, void *workspace, size_t workspace_bytes,
                            pqmc_soc_ctx **out) {
  if (!out) return err(PQMC_EINVAL, "null out");
  *out = nullptr;
  pqmc_status v = validate(prob, opts);
  if (v) return v;
  pqmc_soc_ctx *c = new (std::nothrow) pqmc_soc_ctx;
  if (!c) return err(PQMC_ENOMEM, "host allocation failed");
  fill(*c, prob, opts);
  return create_common(c, prob->hopping, prob->trial, hip_stream, workspace, workspace_bytes, out);
}

}  // extern "C"

namespace pq {
namespace soc {

bool batch_compatible(const pqmc_soc_ctx *c, const pqmc_soc_ctx *a) {
  return c->N == a->N && c->ne == a->ne && c->M == a->M && c->kt == a->kt && c->k == a->k &&
         c->block == a->block && c->w == a->w && c->st == a->st &&
         c->opts.scheme == a->opts.scheme;
}

// n sweeps (n_slices < 0) or one forward window of n_slices slice visits for
// a batch of walkers (out: one entry per walker, or null).
pqmc_status batch_run(pqmc_soc_ctx *const *cs, int n, int n_sweeps, int n_slices,
                      pqmc_stats *out) {
  if (!cs || n < 1 || n > kSocMaxBatch) return err(PQMC_EINVAL, "batch size must be 1..8");
  for (int i = 0; i < n; ++i) {
    const pqmc_soc_ctx *c = cs[i];
    if (!c) return err(PQMC_EINVAL, "null context");
    if (!batch_compatible(c, cs[0]))
      return err(PQMC_EINVAL,
                 "batched SOC walkers need the same lattice, N_e, M, k_tau, scheme, k and "
                 "stream");
    for (int j = 0; j < i; ++j)
      if (cs[j] == c) return err(PQMC_EINVAL, "a context appears twice in the batch");
    if (c->failed) return err(PQMC_ESTATE, "context failed");
    if (c->windowed || c->position != 0) return err(PQMC_ESTATE, "walker is mid-sweep");
  }
  const SocWalkers b{cs, n};
  pqmc_soc_ctx &L = b.lead();
  const double t0 = now_s();
  int rc = PQMC_OK;
  for (int i = 0; i < n && !rc; ++i) rc = begin_call(b[i]);
  if (n_slices >= 0) {   // one forward window
    for (int l = 1; l <= n_slices && !rc; ++l) {
      rc = prop_forward(b, l);
      if (!rc) rc = update_slice(b, l, 0);
      if (!rc && l % L.kt == 0) rc = stab_forward(b, l);
    }
    for (int i = 0; i < n; ++i) {
      b[i].position = n_slices;
      b[i].windowed = true;
    }
  } else {
    for (int s = 0; s < n_sweeps && !rc; ++s) {
      for (int l = 1; l <= L.M && !rc; ++l) {
        rc = prop_forward(b, l);
        if (!rc) rc = update_slice(b, l, 0);
        if (!rc && l % L.kt == 0) rc = stab_forward(b, l);
      }
      for (int l = L.M; l >= 1 && !rc; --l) {
        rc = update_slice(b, l, 1);
        if (!rc) rc = prop_backward(b, l, true);
        if (!rc && (l - 1) % L.kt == 0) rc = stab_backward(b, l);
      }
      if (!rc)
        for (int i = 0; i < n; ++i) ++b[i].sweep_index;
    }
  }
  int first = rc;
  for (int i = 0; i < n; ++i) {
    const int r = rc ? rc : finish_call(b[i], t0, out ? out + i : nullptr);
    if (r) {
      b[i].failed = true;
      if (!first) first = r;
    }
  }
  return (pqmc_status)first;
}

}  // namespace soc
}  // namespace pq

extern "C" {

pqmc_status pqmc_soc_sweep(pqmc_soc_ctx *c, int32_t n_sweeps, pqmc_stats *out) {
  if (n_sweeps < 0) return err(PQMC_EINVAL, "n_sweeps < 0");
  pqmc_soc_ctx *one[1] = {c};
  return batch_run(one, 1, n_sweeps, -1, out);
}

pqmc_status pqmc_soc_forward_window(pqmc_soc_ctx *c, int32_t n_slices, pqmc_stats *out) {
  if (c && (n_slices < 0 || n_slices > c->M)) return err(PQMC_EINVAL, "n_slices out of range");
  pqmc_soc_ctx *one[1] = {c};
  return batch_run(one, 1, 0, n_slices, out);
}

pqmc_status pqmc_soc_batch_sweep(pqmc_soc_ctx *const *ctxs, int32_t n, int32_t n_sweeps,
                                 pqmc_stats *out) {
  if (n_sweeps < 0) return err(PQMC_EINVAL, "n_sweeps < 0");
  return batch_run(ctxs, n, n_sweeps, -1, out);
}

pqmc_status pqmc_soc_batch_forward_window(pqmc_soc_ctx *const *ctxs, int32_t n, int32_t n_slices,
                                          pqmc_stats *out) {
  if (ctxs && n >= 1 && ctxs[0] && (n_slices < 0 || n_slices > ctxs[0]->M))
    return err(PQMC_EINVAL, "n_slices out of range");
  return batch_run(ctxs, n, 0, n_slices, out);
}

pqmc_status pqmc_soc_get_green(pqmc_soc_ctx *c, double *out) {
  if (!c || !out) return err(PQMC_EINVAL, "null argument");
  const int n2 = c->n2, ne = c->ne;
  // Y = U_R T (n2 x ne, in Xtmp), G = 1 - Y ULt^T (n2 x n2, in Tay1)
  int rc = gemm1(cdesc(c->UR, ne, c->T, c->ldT, c->Xtmp, ne, n2, ne, ne), kOpN, kOpN, c->st);
  if (!rc) {
    CgemmDesc d = cdesc(c->Xtmp, ne, c->ULt, ne, c->Tay1, n2, n2, n2, ne);
    d.alpha = make_double2(-1.0, 0.0);
    d.addI = 1;
    rc = gemm1(d, kOpN, kOpT, c->st);
  }
  if (rc) return (pqmc_status)rc;
  hipError_t e = hipMemcpyAsync(out, c->Tay1, sizeof(double2) * (size_t)n2 * n2,
                                hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return (pqmc_status)fail_device(e, "green", __FILE__, __LINE__);
  return PQMC_OK;
}

pqmc_status pqmc_soc_get_fields(pqmc_soc_ctx *c, int8_t *out) {
  if (!c || !out) return err(PQMC_EINVAL, "null argument");
  hipError_t e = hipMemcpyAsync(out, c->fields, (size_t)c->M * c->N, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return (pqmc_status)fail_device(e, "fields", __FILE__, __LINE__);
  return PQMC_OK;
}

pqmc_status pqmc_soc_get_decisions(pqmc_soc_ctx *c, int32_t *meta, double *margin, size_t cap,
                                   size_t *n) {
  if (!c || !n) return err(PQMC_EINVAL, "null argument");
  if (!c->log_meta) return err(PQMC_EINVAL, "the context was created without PQMC_FLAG_LOG");
  const size_t cnt = (size_t)std::min(c->log_count, c->log_cap);
  *n = cnt;
  if (!meta || !margin || cap == 0) return PQMC_OK;
  const size_t m = std::min(cnt, cap);
  hipError_t e = hipMemcpyAsync(meta, c->log_meta, sizeof(int32_t) * 3 * m,
                                hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(margin, c->log_margin, sizeof(double) * m, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return (pqmc_status)fail_device(e, "log copy", __FILE__, __LINE__);
  return PQMC_OK;
}

pqmc_status pqmc_soc_destroy(pqmc_soc_ctx *c) {
  if (!c) return PQMC_OK;
  (void)hipStreamSynchronize(c->st);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
  return PQMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// The paper's U < 0 model (Sec. II B, Eqs. (13)-(14)) behind the spin-
// decoupled calls: one complex spin-up sector (w = 1) of N orbitals with
// N_up = N_dn fermions and P_dn = P_up, alpha = i gamma,
// gamma = arccos(e^{dtau U/2}); spin down is the complex conjugate.
// ------------------------------------------------------------------------
namespace pq {
namespace soc {

namespace {
constexpr unsigned kOneFlags = PQMC_FLAG_LOG | PQMC_FLAG_TIMING | PQMC_FLAG_DENSE_PROP;

pqmc_status one_check_opts(const pqmc_update_opts *o) {
  if (o->scheme != PQMC_LOCAL && o->scheme != PQMC_DELAYED && o->scheme != PQMC_BLOCK_FB)
    return err(PQMC_EINVAL, "U < 0 runs the local, delayed and block force-bias schemes");
  if (o->scheme == PQMC_DELAYED && (o->delay_k < 1 || o->delay_k > 2 * kSocMaxK))
    return err(PQMC_EINVAL, "delay_k in [1, 64] for U < 0");
  if (o->scheme == PQMC_BLOCK_FB && (o->block_b < 1 || o->block_b > 2 * kSocMaxK))
    return err(PQMC_EINVAL, "block_b in [1, 64] for U < 0");
  if (o->flags & ~kOneFlags)
    return err(PQMC_EINVAL, "flags for U < 0: only LOG, TIMING and DENSE_PROP");
  return PQMC_OK;
}

pqmc_status one_validate(const pqmc_problem *p, const pqmc_update_opts *o) {
  if (!p || !o) return err(PQMC_EINVAL, "null problem or options");
  if (p->n_sites < 1) return err(PQMC_EINVAL, "n_sites must be >= 1");
  if (p->n_up < 1 || p->n_up > p->n_sites || p->n_up > 1024)
    return err(PQMC_EINVAL, "need 1 <= n_up <= min(n_sites, 1024)");
  if (!p->hopping || !p->trial_up || !p->trial_dn) return err(PQMC_EINVAL, "null input");
  if (p->n_dn != p->n_up ||
      std::memcmp(p->trial_up, p->trial_dn, sizeof(double) * p->n_sites * p->n_up) != 0)
    return err(PQMC_EINVAL, "U < 0 simulates the spin-up sector only: it needs n_dn = n_up "
                            "and trial_dn = trial_up");
  if (!(p->dtau > 0) || !std::isfinite(p->dtau)) return err(PQMC_EINVAL, "dtau must be > 0");
  if (!std::isfinite(p->U) || !(p->U < 0)) return err(PQMC_EINVAL, "U must be finite and < 0");
  if (p->n_slices < 1 || p->stab_every < 1 || p->n_slices % p->stab_every)
    return err(PQMC_EINVAL, "stab_every must divide n_slices");
  const size_t NN = (size_t)p->n_sites * p->n_sites;
  for (size_t e = 0; e < NN; ++e)
    if (!std::isfinite(p->hopping[e])) return err(PQMC_EINVAL, "non-finite hopping matrix");
  return one_check_opts(o);
}

void one_set_scheme(pqmc_soc_ctx &c, const pqmc_update_opts *o) {
  c.opts = *o;
  c.k = o->scheme == PQMC_DELAYED    ? std::min(o->delay_k, c.N)
        : o->scheme == PQMC_BLOCK_FB ? std::min(o->block_b, c.N)
                                     : 1;
  c.block = o->scheme == PQMC_BLOCK_FB;
}

void one_fill(pqmc_soc_ctx &c, const pqmc_problem *p, const pqmc_update_opts *o) {
  c.w = 1;
  c.N = p->n_sites;
  c.n2 = p->n_sites;
  c.ne = p->n_up;
  c.M = p->n_slices;
  c.kt = p->stab_every;
  c.nst = c.M / c.kt;
  c.U = p->U;
  c.dtau = p->dtau;
  c.gamma = std::acos(std::exp(p->dtau * p->U / 2.0));
  c.c1 = std::cos(c.gamma);
  c.s1 = std::sin(c.gamma);
  c.dd = std::cos(2.0 * c.gamma) - 1.0;   // delta(x) = e^{-2 i gamma x} - 1 = (dd, -x doff)
  c.doff = std::sin(2.0 * c.gamma);
  c.seed = p->seed;
  c.walker = p->walker_id;
  one_set_scheme(c, o);
  c.ksplit = c.ne <= 128 ? 0 : std::max(64, ((c.ne + 7) / 8 + 15) / 16 * 16);
}
}  // namespace

pqmc_status one_sector_workspace_bytes(const pqmc_problem *p, const pqmc_update_opts *o,
                                       size_t *bytes) {
  pqmc_status v = one_validate(p, o);
  if (v) return v;
  pqmc_soc_ctx c;
  one_fill(c, p, o);
  layout(c, nullptr, bytes);
  return PQMC_OK;
}

pqmc_status one_sector_create(const pqmc_problem *p, const pqmc_update_opts *o,
                              void *hip_stream, void *workspace, size_t workspace_bytes,
                              pqmc_soc_ctx **out) {
  *out = nullptr;
  pqmc_status v = one_validate(p, o);
  if (v) return v;
  pqmc_soc_ctx *c = new (std::nothrow) pqmc_soc_ctx;
  if (!c) return err(PQMC_ENOMEM, "host allocation failed");
  one_fill(*c, p, o);
  // the real H0 and P as complex128
  const size_t N = c->N, ne = c->ne;
  std::vector<double> h(2 * N * N, 0.0), t(2 * N * ne, 0.0);
  for (size_t e = 0; e < N * N; ++e) h[2 * e] = p->hopping[e];
  for (size_t e = 0; e < N * ne; ++e) t[2 * e] = p->trial_up[e];
  return create_common(c, h.data(), t.data(), hip_stream, workspace, workspace_bytes, out);
}

pqmc_status one_sector_set_opts(pqmc_soc_ctx *c, const pqmc_update_opts *o) {
  pqmc_status v = one_check_opts(o);
  if (v) return v;
  if ((o->flags & PQMC_FLAG_LOG) && !c->log_meta)
    return err(PQMC_EINVAL, "logging was not sized in the workspace");
  one_set_scheme(*c, o);
  return PQMC_OK;
}

pqmc_status one_sector_set_fields(pqmc_soc_ctx *c, const int8_t *fields) {
  const size_t n = (size_t)c->M * c->N;
  for (size_t e = 0; e < n; ++e)
    if (fields[e] != 1 && fields[e] != -1) return err(PQMC_EINVAL, "fields must be +-1");
  hipError_t e = hipMemcpyAsync(c->fields, fields, n, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e == hipSuccess) e = hipMemsetAsync(c->stats, 0, 16 * sizeof(unsigned long long), c->st);
  if (e != hipSuccess) return (pqmc_status)fail_device(e, "upload fields", __FILE__, __LINE__);
  c->failed = false;
  int rc = build_state(*c);
  if (!rc) rc = sync_check(*c);
  if (rc) c->failed = true;
  return (pqmc_status)rc;
}

pqmc_status one_sector_replay(pqmc_soc_ctx *c, const int8_t *flips, pqmc_stats *out) {
  if (c->failed) return err(PQMC_ESTATE, "context failed; call pqmc_set_fields");
  if (c->windowed || c->position != 0) return err(PQMC_ESTATE, "walker is mid-sweep");
  const size_t n = (size_t)2 * c->M * c->N;
  hipError_t e = hipMemcpyAsync(c->replay, flips, n, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return (pqmc_status)fail_device(e, "upload replay", __FILE__, __LINE__);
  c->replaying = true;
  const pqmc_status st = pqmc_soc_sweep(c, 1, out);
  c->replaying = false;
  return st;
}

// G of spin 0 (N x N complex128 interleaved); spin 1 is its complex conjugate
pqmc_status one_sector_green(pqmc_soc_ctx *c, int spin, double *out) {
  pqmc_status st = pqmc_soc_get_green(c, out);
  if (st || spin == 0) return st;
  const size_t n = (size_t)c->N * c->N;
  for (size_t e = 0; e < n; ++e) out[2 * e + 1] = -out[2 * e + 1];
  return PQMC_OK;
}

int one_sector_dims(const pqmc_soc_ctx *c, int *N, int *M) {
  *N = c->N;
  *M = c->M;
  return c->w;
}

}  // namespace soc
}  // namespace pq
