// Internal interface of the spin-orbit coupled (complex, one 2N sector) path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pq {
namespace soc {

enum { kOpN = 0, kOpT = 1, kOpH = 2 };   // op(X) = X, X^T, X^H

// C = alpha op(A) op(B) + beta Cin (+ I when addI), op(A) M x K, op(B) K x N;
// row-major complex128.  Kdev (optional): K = min(K, *Kdev), and a product
// with K = 0, beta = 1, Cin = C does nothing.
// Split-K: when ksplit > 0, slice s of the depth, [s ksplit, (s + 1) ksplit),
// is written raw (no alpha, beta, I) to C + s csplit; csum adds the slices.
struct CgemmDesc {
  const double2 *A, *B, *Cin;
  double2 *C;
  long lda, ldb, ldcin, ldc;
  int M, N, K;
  const int *Kdev;
  double2 alpha, beta;
  int addI;
  int ksplit;
  long csplit;
};
constexpr int kCgemmMaxBatch = 8;
struct CgemmBatch {
  CgemmDesc d[kCgemmMaxBatch];
  int count;
};
// dst[r][c] = sum_{s < ns} part[s csplit + r ldp + c], slices added in order
struct CsumDesc {
  const double2 *part;
  long csplit, ldp;
  double2 *dst;
  long ldd;
  int M, N, ns;
};
struct CsumBatch {
  CsumDesc d[kCgemmMaxBatch];
  int count;
};
hipError_t csum(const CsumBatch &b, hipStream_t st);
CgemmDesc cdesc(const double2 *A, long lda, const double2 *B, long ldb, double2 *C, long ldc,
                int M, int N, int K);
// op pairs supported: (N, N), (N, T), (T, N), (H, N)
hipError_t cgemm(const CgemmBatch &b, int opA, int opB, hipStream_t st);

// Y = e^{a M} X for a sparse complex M (M = H0, or H0^T = conj(H0) when conj
// is set: H0 is Hermitian, so both share H0's pattern), X and Y n2 x n
// row-major (leading dims ldx, ldy; X != Y): the Taylor series of degree J
// in Horner form, Z <- X + (a M Z) / j for j = J .. 1.  M in ELL form: row r
// has w entries idx[r w + e], val[r w + e] (padded with zero values).
constexpr int kCexpMaxN = 4096, kCexpMaxW = 8, kCexpvMaxBatch = 16;
struct CexpvDesc {
  const double2 *X;
  long ldx;
  double2 *Y;
  long ldy;
  int n2, n;
  const int *idx;
  const double2 *val;
  int w, J;
  double a;
  int conj;
};
struct CexpvBatch {
  CexpvDesc d[kCexpvMaxBatch];
  int count;
};
hipError_t cexpv(const CexpvBatch &b, hipStream_t st);

// rows (i, N+i) of Y <- A(sign x_i) rows (i, N+i) of X (X == Y allowed),
// A(y) = [[cos gamma y, sin gamma y], [-sin gamma y, cos gamma y]];
// c = cos gamma, s = sin gamma.
hipError_t rotate_rows(const double2 *X, long ldx, double2 *Y, long ldy, int ncols, int N,
                       const int8_t *xrow, double c, double s, double sign, hipStream_t st);
// Y = conj(X), n elements
hipError_t conj_copy(const double2 *X, double2 *Y, long n, hipStream_t st);
// E[r][off + c] = (r == c), r, c < n
hipError_t set_identity(double2 *E, long ld, int n, int off, hipStream_t st);
// Walkers of one SOC batch: all share n2, n_e, M, k_tau, the scheme and k.
constexpr int kSocMaxBatch = 8;
// Pivots per panel of the blocked Gauss-Jordan inverse.
constexpr int kGjNb = 16;
// complex128 scratch of one walker's blocked eliminations of order n (block
// rows kGjNb x 2n, then two kGjNb x kGjNb blocks), and the int scratch of
// the Gauss-Jordan inverse (pivot row of each column, pivot column of each row)
inline size_t gj_scratch_complex(size_t n) { return kGjNb * 2 * n + 2 * kGjNb * kGjNb; }
inline size_t gj_scratch_int(size_t n) { return 2 * n; }
// The matrices of a batched elimination, one per walker: E (n x 2n or
// n x n, leading dim ld), the Gauss-Jordan scratch and error flags.
struct SocElimBatch {
  double2 *E[kSocMaxBatch];
  double2 *B[kSocMaxBatch];   // gj_scratch_complex(n)
  int *piv[kSocMaxBatch];     // gj_scratch_int(n)
  unsigned long long *stats[kSocMaxBatch];
  int n;
};
// each E[w] = [S | I] (n x 2n, leading dim ld), S Hermitian positive
// definite: the left half <- R^{-1} with S = R^H R, R upper triangular with
// a positive diagonal, by blocked Cholesky-normalised forward elimination
// (kGjNb columns a panel, three launches per panel for the whole batch; the
// right half ends as R^{-H}); n <= 1024
hipError_t chol_inverse(const SocElimBatch &b, long ld, int n, hipStream_t st);
// each E[w] = [M | I] (n x 2n, leading dim ld): the left half <- M^{-1} by
// blocked Gauss-Jordan elimination with partial pivoting (kGjNb pivots per
// panel, three launches per panel for the whole batch; the right half is
// left overwritten); n <= 1024
hipError_t gj_inverse(const SocElimBatch &b, long ld, int n, hipStream_t st);

constexpr int kSocMaxK = 32;   // group size of the decision kernel (2k x 2k in LDS)
struct SocDecideArgs {
  const double2 *W0p;      // 2kk x 2kk
  double2 *D;              // 2kk x 2kk out
  double2 *UR;             // 2N x ne
  int *nflush;             // out: 2kk or 0
  int *accx;               // out (delayed and local): per site of the group, its field
                           // before the flip if accepted, else 0 (2 kSocMaxK ints)
  int8_t *fields;          // M x N
  int li, N, ne, g0, kk;
  double dd, doff;         // delta = [[dd, -x doff], [x doff, dd]]
  double c1, s1, gamma;    // cos gamma, sin gamma, gamma (block force bias)
  uint64_t key0, key1, sweep, slice_code;
  unsigned long long *stats;
  int32_t *log_meta;
  double *log_margin;
  long long log_base, log_cap;
  const int8_t *force;     // replay: forced outcomes of the slice visit (or null)
};
// one workgroup per walker: a[0..nb) (nb <= kSocMaxBatch), all with the same kk
struct SocDecideBatch {
  SocDecideArgs a[kSocMaxBatch];
};
hipError_t decide(const SocDecideArgs *a, int nb, hipStream_t st);
// after decide / decide1: the U_R rows of the accepted sites (accx) rotated
// by 1 + delta (w = 2: the row pairs (site, N + site); w = 1: the phase of
// row site), one workgroup per (256 columns, site, walker)
hipError_t rotate_accepted(const SocDecideArgs *a, int nb, int w, hipStream_t st);
// The one-sector model (U < 0 of Sec. II B, w = 1): rows scaled by the
// phases e^{i sign gamma x_i}; decisions of kk <= 64 sites with a scalar
// flip delta per site (delayed / local, and block force bias).
hipError_t phase_rows(const double2 *X, long ldx, double2 *Y, long ldy, int ncols, int N,
                      const int8_t *xrow, double c, double s, double sign, hipStream_t st);
hipError_t decide1(const SocDecideArgs *a, int nb, hipStream_t st);
hipError_t block_decide1(const SocDecideArgs *a, int nb, hipStream_t st);
// block force bias over the kk sites of the group (log entry at log_base)
hipError_t block_decide(const SocDecideArgs *a, int nb, hipStream_t st);

}  // namespace soc
}  // namespace pq

// The paper's U < 0 model behind the spin-decoupled calls (soc_capi.cpp):
// one complex spin-up sector run by the width-one form of this engine.
#include "../../include/pqmc.h"
namespace pq {
namespace soc {
pqmc_status one_sector_workspace_bytes(const pqmc_problem *p, const pqmc_update_opts *o,
                                       size_t *bytes);
pqmc_status one_sector_create(const pqmc_problem *p, const pqmc_update_opts *o,
                              void *hip_stream, void *workspace, size_t workspace_bytes,
                              pqmc_soc_ctx **out);
pqmc_status one_sector_set_opts(pqmc_soc_ctx *c, const pqmc_update_opts *o);
pqmc_status one_sector_set_fields(pqmc_soc_ctx *c, const int8_t *fields);
pqmc_status one_sector_replay(pqmc_soc_ctx *c, const int8_t *flips, pqmc_stats *out);
pqmc_status one_sector_green(pqmc_soc_ctx *c, int spin, double *out);
int one_sector_dims(const pqmc_soc_ctx *c, int *N, int *M);
// Sweeps (n_slices < 0) or one forward window of a batch of SOC or one-sector
// contexts (soc_capi.cpp); batch_compatible: a and b may share a batch.
pqmc_status batch_run(pqmc_soc_ctx *const *cs, int n, int n_sweeps, int n_slices,
                      pqmc_stats *out);
bool batch_compatible(const pqmc_soc_ctx *a, const pqmc_soc_ctx *b);
}  // namespace soc
}  // namespace pq
