// Internal interface between the C ABI (capi.cpp) and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.hpp"

namespace pq {

int fail_device(hipError_t e, const char *expr, const char *file, int line);
// sets the calling thread's pqmc_last_error message; returns st
int api_error(int st, const char *msg);

// ------------------------------------------------------------------ GEMM
// C = alpha * rs(i) cs(j) * sum_k op(A)(i,k) ks(k) op(B)(k,j) + beta * Cin(i,j) + [addI && i == j]
// Row-major storage; op(A) is M x K (A stored K x M when transA), op(B) K x N.
// rs / ks: optional diagonal scalings read from a field row: x > 0 -> pos, else neg.
// Split-K: when ksplit > 0, z-slice s of the grid handles k in [s*ksplit, (s+1)*ksplit)
// and writes C + s*csplit (beta, Cin, addI ignored).
struct GemmDesc {
  const double *A, *B, *Cin;
  double *C;
  long lda, ldb, ldcin, ldc;
  int M, N, K;
  const int *Kdev;                // if set: K = min(K, *Kdev)
  const int8_t *rs_field;
  double rs_pos, rs_neg;
  const int8_t *ks_field;
  double ks_pos, ks_neg;
  const int8_t *cs_field;         // optional scaling of the output columns (epilogue)
  double cs_pos, cs_neg;
  double alpha, beta;
  int addI;
  int ksplit;
  long csplit;
};
constexpr int kGemmMaxBatch = 8;
struct GemmBatch {
  GemmDesc d[kGemmMaxBatch];
  int count;
};
GemmDesc gemm_desc(const double *A, long lda, const double *B, long ldb, double *C, long ldc,
                   int M, int N, int K, double alpha = 1.0, double beta = 0.0,
                   const double *Cin = nullptr, long ldcin = 0);
hipError_t gemm(const GemmBatch &b, bool transA, bool transB, hipStream_t st);

// ------------------------------------------------------- sparse propagation
// Y = rs * e^{a H0} (ks * X) for an N x n row-major X (leading dim ldx), H0
// given as ELL rows of w (column, value) pairs (zero-padded), the Taylor
// series of degree J in Horner form; the field diagonal (x > 0 -> pos, else
// neg) scales X's rows first when pre, Y's rows last otherwise (none when
// field is null).  X and Y must not overlap.
struct ExpvDesc {
  const double *X;
  long ldx;
  double *Y;
  long ldy;
  int N, n;
  const int *idx;
  const double *val;
  int w, J;
  double a;
  const int8_t *field;
  double pos, neg;
  int pre;
};
constexpr int kExpvMaxBatch = 16;
constexpr int kExpMaxN = 4096;   // LDS: two iterates of N x 2 doubles
constexpr int kExpMaxW = 8;      // nonzeros per row of H0
struct ExpvBatch {
  ExpvDesc d[kExpvMaxBatch];
  int count;
};
hipError_t expv(const ExpvBatch &b, hipStream_t st);

// ------------------------------------------------------------- dense LA
constexpr int kNB = 32;   // panel width of the blocked eliminations
struct ElimSpin {
  double *E;       // n x w augmented matrix [M | I], row-major, leading dim ld, w = 2 n
  long ld;
  int n, w;
  double *Z;       // kNB x kNB: inverse of the current panel's pivot block
  int *prow;       // n: pivot row chosen for column c (Gauss-Jordan)
  int *slot;       // n: pivot column of row r, -1 while unused (Gauss-Jordan)
  double *BR;      // 2 x kNB x w: new block rows of the last two passes (Gauss-Jordan)
  double *F;       // n x n: rows of R^{-T} (Cholesky)
  unsigned long long *stats;   // error flags of the owning walker
};
// Up to kMaxMats matrices of the same size per call (two spin sectors of up
// to kMaxBatch walkers).
constexpr int kMaxMats = 16;
// out[i] = M_i^{-1} (n x n, leading dim ldo) for E_i = [M_i | I], n <= 1024,
// by Gauss-Jordan elimination with partial pivoting.  E_i is overwritten.
hipError_t gj_invert(const ElimSpin *s, int nmat, double *const *out, long ldo, hipStream_t st);
// Forward elimination normalised by the Cholesky factor of each diagonal
// block on E_i = [S_i | I], S_i SPD: F_i receives R_i^{-T}, S_i = R_i^T R_i.
hipError_t chol_eliminate(const ElimSpin *s, int nmat, hipStream_t st);
// E_i[r, col0 + c] = (r == c) for r, c < n, i < nmat.
hipError_t set_identity_block(double *const *E, int nmat, long ld, int n, int col0,
                              hipStream_t st);
hipError_t copy_matrix(const double *src0, const double *src1, long lds, double *dst0,
                       double *dst1, long ldd, int rows, int cols, hipStream_t st);
// dst_i = (float) src_i, dst_i = (double) src_i (n[i] elements, up to kMaxMats pairs)
hipError_t round_to_f32(const double *const *src, float *const *dst, int nmat, const long *n,
                        hipStream_t st);
hipError_t widen_to_f64(const float *const *src, double *const *dst, int nmat, const long *n,
                        hipStream_t st);
hipError_t init_fields(int8_t *fields, int M, int N, uint64_t k0, uint64_t k1, hipStream_t st);
// *p[i] = v[i], i < n (a kernel: safe inside captured graphs)
hipError_t set_u64(uint64_t *const *p, const uint64_t *v, int n, hipStream_t st);
// *out[i] = max(*out[i], max_e |a_i[e] - b_i[e]|), e < n[i], stored as the bits
// of a non-negative double (atomicMax on the integer pattern)
hipError_t max_abs_diff(const double *const *a, const double *const *b, const long *n,
                        unsigned long long *const *out, int nmat, hipStream_t st);

// ---------------------------------------------------------- field updates
// Batched launches: every update kernel takes one argument record per walker
// (blockIdx.z, or blockIdx.x for the single-workgroup decision kernels), so
// kMaxBatch independent walkers of the same shape share each launch.
constexpr int kMaxBatch = 8;
// Device-to-host copy on the caller's own stream, waited for.  Copies are
// never made on the legacy (null) stream: another thread of the process may be
// capturing a graph on a blocking stream, which a legacy-stream copy would
// have to wait for.
inline hipError_t d2h(void *dst, const void *src, size_t bytes, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

template <class T>
struct Batch {
  T w[kMaxBatch];
};

struct SpinMats {
  double *T[2];          // Ns x Ns
  float *T32[2];         // Ns x Ns, the precision form's T (null otherwise)
  double *UR[2];         // N x Ns (rows = u_i^T)
  const double *ULt[2];  // N x Ns (rows = columns of U_L)
  int Ns[2];
};
struct LocalBufs {       // fused local-step partials, double-buffered by site parity
  double *ypart[2][2];   // [spin][parity]: ntr x Ns
  double *tpart[2][2];   // ntc x Ns
  double *spart[2][2];   // ntr x ntc
  double *delta[2];      // [parity]: Delta of the pending site, per spin
};
// One launch per site i = 0..N: applies site i-1's decision and rank-1
// upgrade, then forms the partial ratio products of site i.
hipError_t local_step(const SpinMats *m, const LocalBufs *b, const SweepCtx *c, int nw, int i,
                      int nt_max, hipStream_t st);

struct GroupBufs {
  double *P2part[2], *P1part[2];   // split-K partials
  double *P2[2], *P1[2];           // kmax x Ns, Ns x kmax
  double *W0part[2];               // nt^2 x kmax x kmax: per-tile partials of W0
  double *W0[2];                   // kmax x kmax: W0 = U_g T L_g (partials in fixed order)
  double *uni;                     // kmax + 1: the group's Metropolis / heat-bath uniforms
  // Result of a decision over the group's kk sites, with A the accepted
  // (delayed) or flipped (block force bias) set:
  //   Mc = diag(Delta_A) (E_AA)^{-1} spread to kk x kk (zero outside A x A),
  //   sc = 1 + Delta on A and 1 elsewhere (the U_R row scale),
  // so that the flush is T <- T - P1 Mc P2 (Eqs. (30), (36)).
  double *Mc[2];                   // kmax x kmax
  double *sc[2];                   // kmax
  double *Q[2];                    // Ns x kmax: P1 Mc (flush without the tile kernel)
  int *nA;                         // 2: |A|, and the flush rank (kk, or 0 when A is empty)
  int *alist;                      // kmax: the sites of A in increasing order (|A| of them)
  int kmax;
  int Ns[2];                       // particles per spin
  int chunks;                      // tile kernel: column chunks asked per row strip
};
// Uniforms drawn by the reduce kernel for the decision that follows it.
enum UniMode { kUniNone = 0, kUniDelayed = 1, kUniBlock = 2 };
// Group launches over a batch: every walker's group starts at site g0 and
// has kk[w] sites (0: the walker has no group here, its lattice is smaller).
hipError_t group_panels(const SpinMats *m, const GroupBufs *g, const SweepCtx *c, int nw,
                        int mode, int g0, const int *kk, hipStream_t st);
// panels: the launch also sums the group's split-K panel partials (the fused
// path, whose reduce kernel leaves them for the decision launch)
hipError_t delayed_decide(const GroupBufs *g, const SweepCtx *c, int nw, int g0, const int *kk,
                          bool panels, hipStream_t st);
hipError_t block_decide(const GroupBufs *g, const SweepCtx *c, int nw, int g0, const int *kk,
                        long long block_index, bool panels, hipStream_t st);
hipError_t group_flush(const SpinMats *m, const GroupBufs *g, int nw, int g0, const int *kk,
                       hipStream_t st);
// Fused path (kmax <= 64): one tile kernel per group applies the previous
// group's flush and forms this group's split-K panel partials; group_reduce
// sums those of W0 and the decision launch (panels = true) those of P1, P2.
// fp32: the precision form, T in float32 (SpinMats::T32) and the products
// on FP32 MFMA with FP32 accumulation.
// The pending group of walker w (flushed by this launch) starts at g0_prev
// and has kk_prev[w] sites (0: nothing pending).
hipError_t group_tile(const SpinMats *m, const GroupBufs *g, int nw, int g0_prev,
                      const int *kk_prev, int g0, const int *kk, bool fp32, hipStream_t st);
hipError_t group_reduce(const SpinMats *m, const GroupBufs *g, const SweepCtx *c, int nw,
                        int mode, int g0, const int *kk, hipStream_t st);

// ------------------------------------------------- persistent local updates
// Grid-wide barrier of a cooperative launch: one epoch flag per workgroup
// (flags[kLocalMaxGroups], zeroed before the launch), bounded wait; *abort
// set when a wait exceeds spin_limit polls, and then every workgroup leaves
// the kernel.
constexpr int kLocalMaxGroups = 256;
struct GridSync {
  unsigned *flags;
  unsigned *abort;
  unsigned spin_limit;
};
struct LocalPersistArgs {
  SpinMats m;
  SweepCtx c;
  GridSync g;
  // T-form: per spin pr x pc blocks (P = pr pc workgroups) and the partial
  // buffers of one site, double-buffered by site parity:
  //   ypart[s]: 2 x pr x Ns, xpart[s]: 2 x pc x Ns, spart[s]: 2 x P
  int P[2], pr[2], pc[2];
  double *ypart[2], *xpart[2], *spart[2];
  // G-form: G_s (N x N), the published rows (2 x N per spin), rows per workgroup
  double *Gm[2];
  double *grow_buf[2];
  int grow;
};
// T-form blocks of at most 64 x 128 (pr = ceil(n / 64), pc = ceil(n / 128))
void local_persist_grid(int n, int *pr, int *pc);
// whether the persistent kernel holds this problem (at most 256 workgroups)
bool local_persist_fits(int n_up, int n_dn, int N, bool gform);
// one slice of the local update (gform: on G) as one cooperative launch
hipError_t local_persist(const LocalPersistArgs &a, bool gform, hipStream_t st);
constexpr int kLocalGRows = 8;   // G-form rows per workgroup (upper bound)

}  // namespace pq
