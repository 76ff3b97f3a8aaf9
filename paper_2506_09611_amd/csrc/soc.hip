// Spin-orbit coupled Hubbard model (Appendix A of the paper): one complex
// sector of dimension 2N, N_e fermions, spin-s^y decoupling with 2x2 real
// rotations A(x) = e^{gamma x i sigma_y} on the row pairs (i, N + i).
//
// Kernels:
//   cgemm_kernel     C = alpha op(A) op(B) + beta Cin (+ I), op in {N, T, H},
//                    64 x 64 complex tiles through LDS on FP64 MFMA, up to 8
//                    products per launch
//   rotate_kernel    rows (i, N+i) of an n2 x ncols matrix mixed by A(s x_i)
//   ch_panel_kernel, ch_rows_kernel  R^{-1} for S = R^H R (S Hermitian
//                    positive definite) by blocked Cholesky-normalised forward
//                    elimination on [S | I], the trailing update by cgemm
//   gj_panel_kernel, gj_rows_kernel  blocked Gauss-Jordan inverse with partial
//                    pivoting on [M | I], 16 pivots a panel, the trailing
//                    rank-16 update by cgemm
//   soc_decide_kernel  the decisions of one group of k sites in 2k x 2k space
//                    (rank-two blocks, Eqs. (A7)-(A9) and the delayed update)
//   soc_block_decide_kernel  one block force-bias update of b sites in 2b x 2b
//                    space (Sec. III B with the spin-s^y force bias)
// All matrices are row-major complex128 (interleaved re, im).
#include <hip/hip_runtime.h>
#include <math.h>
#include "common.hpp"
#include "soc.hpp"
#include "mfma.hpp"

namespace pq {
namespace soc {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// acc += a b
__device__ __forceinline__ void cfma(double2 &acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// ------------------------------------------------------------------ GEMM
constexpr int BM = 64, BN = 64, BK = 16;

template <int OP>
__device__ __forceinline__ double2 op_load(const double2 *A, long ld, int r, int k) {
  // element (r, k) of op(A): N -> A[r][k], T -> A[k][r], H -> conj(A[k][r])
  if (OP == kOpN) return A[(long)r * ld + k];
  const double2 v = A[(long)k * ld + r];
  return OP == kOpH ? cconj(v) : v;
}

template <int OPA, int OPB>
__global__ __launch_bounds__(256) void cgemm_kernel(CgemmBatch b, int ns) {
  const CgemmDesc &g = b.d[blockIdx.z / ns];
  const int split = blockIdx.z % ns;
  int K = g.K;
  if (g.Kdev) K = min(K, *g.Kdev);
  const int M = g.M, N = g.N;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (m0 >= M || n0 >= N) return;
  int kbeg = 0, kend = K;
  if (g.ksplit > 0) {
    kbeg = split * g.ksplit;
    kend = min(K, kbeg + g.ksplit);
    if (kbeg >= K) return;   // this product has fewer slices
  } else if (split > 0) {
    return;
  }
  if (K <= 0 && g.Kdev && g.beta.x == 1.0 && g.beta.y == 0.0 && g.Cin == g.C && !g.addI) return;
  // Two LDS buffers: the next depth slice is loaded into registers while the
  // current one is multiplied, then stored to the other buffer.  Loads are
  // unconditional (clamped in-range addresses) so that they issue together;
  // the conjugation and the zeroing of the depth tail are applied when the
  // slice is stored.  Rows and columns past M and N only reach outputs that
  // are not stored.
  //
  // The products run on FP64 MFMA (16 x 16 x 4): wave w owns the 32 x 32
  // quadrant (w / 2, w % 2) of the 64 x 64 tile as 2 x 2 blocks, each with a
  // real and an imaginary accumulator; per depth step of 4 a block takes
  // four MFMAs, re += a_re b_re - a_im b_im and im += a_re b_im + a_im b_re,
  // with a and b read from LDS as complex pairs in the A and B operand
  // layouts (lane l: row l % 16, depth l / 16; depth l / 16, column l % 16).
  __shared__ double2 As[2][BK][BM];
  __shared__ double2 Bs[2][BK][BN];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave >> 1, wn = wave & 1, li = lane & 15, lk = lane >> 4;
  dbl4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  double2 ra[4], rb[4];
  auto a_index = [&](int p, int &r, int &kk) {
    const int e = t + 256 * p;
    if (OPA == kOpN) { r = e >> 4; kk = e & 15; } else { kk = e >> 6; r = e & 63; }
  };
  auto b_index = [&](int p, int &c, int &kb) {
    const int e = t + 256 * p;
    if (OPB == kOpN) { kb = e >> 6; c = e & 63; } else { c = e >> 4; kb = e & 15; }
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int r, kk, c, kb;
      a_index(p, r, kk);
      const int gr = min(m0 + r, M - 1), gk = min(k0 + kk, kend - 1);
      ra[p] = OPA == kOpN ? g.A[(long)gr * g.lda + gk] : g.A[(long)gk * g.lda + gr];
      b_index(p, c, kb);
      const int gc = min(n0 + c, N - 1), gkb = min(k0 + kb, kend - 1);
      // element (k, c) of op(B): N -> B[k][c], T -> B[c][k], H -> conj(B[c][k])
      rb[p] = OPB == kOpN ? g.B[(long)gkb * g.ldb + gc] : g.B[(long)gc * g.ldb + gkb];
    }
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int r, kk, c, kb;
      a_index(p, r, kk);
      const double m = k0 + kk < kend ? 1.0 : 0.0;
      As[buf][kk][r] = make_double2(ra[p].x * m, (OPA == kOpH ? -ra[p].y : ra[p].y) * m);
      b_index(p, c, kb);
      Bs[buf][kb][c] = OPB == kOpH ? cconj(rb[p]) : rb[p];
    }
  };
  if (kbeg < kend) {
    load(kbeg);
    store(0, kbeg);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
#pragma unroll
    for (int q = 0; q < BK; q += 4) {
      double2 a[2], bb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[buf][q + lk][wm * 32 + 16 * i + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = Bs[buf][q + lk][wn * 32 + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, bb[j].x, accR[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i].y, bb[j].y, accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, bb[j].y, accI[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, bb[j].x, accI[i][j], 0, 0, 0);
        }
    }
    // the other buffer was last read before the previous barrier
    if (more) store(buf ^ 1, k0 + BK);
    __syncthreads();
    buf ^= 1;
  }
  // register e of lane l holds element (l / 16 + 4 e, l % 16) of a block
  double2 *C = g.ksplit > 0 ? g.C + (long)split * g.csplit : g.C;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = m0 + wm * 32 + 16 * i + lk + 4 * e, c = n0 + wn * 32 + 16 * j + li;
        if (r >= M || c >= N) continue;
        double2 v = make_double2(accR[i][j][e], accI[i][j][e]);
        if (g.ksplit <= 0) {
          v = cmul(g.alpha, v);
          if (g.Cin && (g.beta.x != 0.0 || g.beta.y != 0.0))
            v = cadd(v, cmul(g.beta, g.Cin[(long)r * g.ldcin + c]));
          if (g.addI && r == c) v.x += 1.0;
        }
        C[(long)r * g.ldc + c] = v;
      }
}

__global__ __launch_bounds__(256) void csum_kernel(CsumBatch b) {
  const CsumDesc &d = b.d[blockIdx.y];
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)d.M * d.N) return;
  const int r = (int)(e / d.N), c = (int)(e % d.N);
  double2 s = make_double2(0.0, 0.0);
  for (int q = 0; q < d.ns; ++q) s = cadd(s, d.part[q * d.csplit + (long)r * d.ldp + c]);
  d.dst[(long)r * d.ldd + c] = s;
}

// ------------------------------------------------------- propagation
// One workgroup of 512 threads owns one column of one product for all n2
// rows: both Horner iterates in LDS (2 x n2 complex), the thread's R rows of
// X and of a M (ELL, WD entries a row) in registers.  Each step reads the
// neighbour rows from LDS and ends on a barrier; X is read once and Y
// written once.  XCD-aware: consecutive workgroup ids go round-robin to the
// 8 XCDs, so XCD x takes the contiguous range [x per, (x + 1) per) of
// columns, and the eight columns of a cache line of X and Y share one L2.
constexpr int kCexpThreads = 512;

// The matrix values stay in registers when R <= 4 and R WD <= 32; above that (n2 > 2048
// rows) they are read at every step (cached, shared by
// every workgroup) so that the kernel does not spill.
template <int R, int WD>
__global__ __launch_bounds__(kCexpThreads) void cexpv_kernel(CexpvBatch B) {
  constexpr bool kRegVal = R * WD <= 32 && R <= 4;
  constexpr int RV = kRegVal ? R : 1;
  const CexpvDesc &d = B.d[blockIdx.y];
  const int per = (int)(gridDim.x >> 3);   // the grid is a multiple of 8
  const int col = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (col >= d.n) return;
  extern __shared__ double2 czs[];
  double2 *Za = czs, *Zb = czs + d.n2;
  const int t = threadIdx.x, n2 = d.n2;
  const double cs = d.conj ? -1.0 : 1.0;
  // a M entry e of row r (zero past the row's w entries)
  auto mval = [&](int r, int e) {
    const int rr = min(r, n2 - 1), ec = min(e, d.w - 1);
    const double2 v = d.val[(long)rr * d.w + ec];
    const double m = (r < n2 && e < d.w) ? d.a : 0.0;
    return make_double2(v.x * m, cs * v.y * m);
  };
  double2 x[R];
  int idx[R][WD];
  double2 val[RV][WD];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = t + kCexpThreads * i;
    const int rr = min(r, n2 - 1);
#pragma unroll
    for (int e = 0; e < WD; ++e) {
      idx[i][e] = d.idx[(long)rr * d.w + min(e, d.w - 1)];
      if constexpr (kRegVal) val[i][e] = mval(r, e);
    }
    x[i] = d.X[(long)rr * d.ldx + col];
    if (r < n2) Za[r] = x[i];
  }
  __syncthreads();
  for (int j = d.J; j >= 1; --j) {
    const double inv = 1.0 / (double)j;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = t + kCexpThreads * i;
      if (r < n2) {
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int e = 0; e < WD; ++e) {
          if constexpr (kRegVal) cfma(s, val[i][e], Za[idx[i][e]]);
          else cfma(s, mval(r, e), Za[idx[i][e]]);
        }
        Zb[r] = make_double2(fma(s.x, inv, x[i].x), fma(s.y, inv, x[i].y));
      }
    }
    __syncthreads();
    double2 *tmp = Za;
    Za = Zb;
    Zb = tmp;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = t + kCexpThreads * i;
    if (r < n2) d.Y[(long)r * d.ldy + col] = Za[r];
  }
}

template <int R, int WD>
hipError_t launch_cexpv(const CexpvBatch &b, int nmax, int n2max, hipStream_t st) {
  const size_t lds = sizeof(double2) * 2 * (size_t)n2max;
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)cexpv_kernel<R, WD>, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(sizeof(double2) * 2 * kCexpMaxN));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((cexpv_kernel<R, WD>), dim3((nmax + 7) / 8 * 8, b.count), dim3(kCexpThreads),
                     lds, st, b);
  return hipGetLastError();
}

template <int R>
hipError_t launch_cexpv_w(const CexpvBatch &b, int nmax, int n2max, int wmax, hipStream_t st) {
  if (wmax <= 4) return launch_cexpv<R, 4>(b, nmax, n2max, st);
  return launch_cexpv<R, 8>(b, nmax, n2max, st);
}

// ------------------------------------------------------------- rotations
// rows (i, N+i) of Y <- A(sign x_i) rows (i, N+i) of X (n2 x ncols, leading
// dims ldx, ldy; X == Y allowed), A(y) = [[cos gamma y, sin gamma y],
// [-sin gamma y, cos gamma y]]; x = +-1 so cos(gamma x) = c, sin(gamma x) = x s.
__global__ __launch_bounds__(256) void rotate_kernel(const double2 *X, long ldx, double2 *Y,
                                                     long ldy, int ncols, int N,
                                                     const int8_t *xrow, double c, double s,
                                                     double sign) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)N * ncols) return;
  const int i = (int)(e / ncols), col = (int)(e % ncols);
  const double sn = sign * (double)xrow[i] * s;
  const double2 a = X[(long)i * ldx + col], b = X[(long)(N + i) * ldx + col];
  Y[(long)i * ldy + col] = make_double2(c * a.x + sn * b.x, c * a.y + sn * b.y);
  Y[(long)(N + i) * ldy + col] = make_double2(-sn * a.x + c * b.x, -sn * a.y + c * b.y);
}

// Y = conj(X) (n elements)
__global__ __launch_bounds__(256) void conj_kernel(const double2 *X, double2 *Y, long n) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e < n) Y[e] = cconj(X[e]);
}

// E[r][off + c] = (r == c) for r, c < n (leading dim ld)
__global__ __launch_bounds__(256) void ident_kernel(double2 *E, long ld, int n, int off) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  E[(long)r * ld + off + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
}

// ------------------------------------------------------------ dense LA

// ------------------------------------------ blocked Cholesky elimination
// E = [S | I] (n x 2n, leading dim ld), S Hermitian positive definite.
// Panel kb (nbp columns), with S11 = C C^H (C lower triangular, positive
// diagonal) the current diagonal block:
//   ch_panel_kernel  Z = C^{-1} and W = S11^{-1} = Z^H Z (one workgroup a
//                    matrix, in LDS);
//   ch_rows_kernel   the block rows become Z E[b, c], and Bk = W E[b, c], for
//                    the live columns c in [kb + nbp, n + kb + nbp);
//   cgemm            E[i, c] -= E[i, panel] Bk[:, c] for the rows below.
// Row operations only add multiples of earlier rows, so the right half ends
// as the lower triangular G with G S = R: G = R^{-H}.  During panel kb the
// right-half entries of the block rows at columns >= n + kb + nbp are still
// the identity's zeros, which bounds the live columns.  ch_adjoint_kernel
// finally writes R^{-1} = G^H into the left half.
__global__ __launch_bounds__(256) void ch_panel_kernel(SocElimBatch B, long ld, int n, int kb) {
  const int w = blockIdx.x;
  const double2 *E = B.E[w];
  double2 *Zg = B.B[w] + (size_t)kGjNb * 2 * n;   // Z, then W
  const int nbp = min(kGjNb, n - kb);
  const int t = threadIdx.x, ra = t >> 4, cb = t & 15;
  static_assert(kGjNb * kGjNb == 256, "one block entry a thread");
  __shared__ double2 S[kGjNb][kGjNb];   // the block, then C in its lower triangle
  __shared__ double2 X[kGjNb][kGjNb];   // Z = C^{-1}
  S[ra][cb] = (ra < nbp && cb < nbp) ? E[(long)(kb + ra) * ld + kb + cb]
                                     : make_double2(ra == cb ? 1.0 : 0.0, 0.0);
  __syncthreads();
  // right-looking: column j of C, then the trailing block loses C_:j C_:j^H
  bool bad = false;
  for (int j = 0; j < nbp; ++j) {
    const double d = S[j][j].x;
    bad = bad || !(d > 0.0) || !isfinite(d);
    const double2 sij = S[ra][j], skj = S[cb][j], x = S[ra][cb];
    __syncthreads();
    const double cj = sqrt(d), ic = 1.0 / cj, id = 1.0 / d;
    if (cb == j && ra >= j)
      S[ra][j] = ra == j ? make_double2(cj, 0.0) : make_double2(sij.x * ic, sij.y * ic);
    else if (ra > j && cb > j) {
      const double2 p = cmul(sij, cconj(skj));
      S[ra][cb] = make_double2(x.x - p.x * id, x.y - p.y * id);
    }
    __syncthreads();
  }
  // Z = C^{-1} by forward substitution, one row of Z a step
  for (int i = 0; i < kGjNb; ++i) {
    if (ra == i) {
      double2 acc = make_double2(0.0, 0.0);
      for (int k = cb; k < i; ++k) cfma(acc, S[i][k], X[k][cb]);
      const double ici = 1.0 / S[i][i].x;
      X[i][cb] = cb > i    ? make_double2(0.0, 0.0)
                 : cb == i ? make_double2(ici, 0.0)
                           : make_double2(-acc.x * ici, -acc.y * ici);
    }
    __syncthreads();
  }
  double2 wv = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < kGjNb; ++k) cfma(wv, cconj(X[k][ra]), X[k][cb]);
  const bool in = ra < nbp && cb < nbp;
  Zg[t] = in ? X[ra][cb] : make_double2(0.0, 0.0);
  Zg[kGjNb * kGjNb + t] = in ? wv : make_double2(0.0, 0.0);
  if (bad && t == 0) B.stats[w][kStError] |= kErrSingular;
}

// Block rows E[kb + a][c] <- (Z x)_a and Bk[a][c] = (W x)_a with x = E[kb .. kb
// + nbp)[c], for c in [kb + nbp, n + kb + nbp); 64 columns a workgroup, four
// output rows a thread.  The block rows are staged in LDS, so every read of
// a column precedes (by a barrier) its rewrite.
__global__ __launch_bounds__(256) void ch_rows_kernel(SocElimBatch B, long ld, int n, int kb) {
  const int w = blockIdx.y;
  double2 *E = B.E[w];
  const double2 *Zg = B.B[w] + (size_t)kGjNb * 2 * n;
  double2 *Bk = B.B[w];
  const int nbp = min(kGjNb, n - kb), c0 = kb + nbp, c1 = n + c0, n2 = 2 * n;
  const int t = threadIdx.x, g = t >> 6, lc = t & 63;
  const int col = c0 + (int)blockIdx.x * 64 + lc;
  __shared__ double2 Zs[kGjNb][kGjNb], Ws[kGjNb][kGjNb], Xs[kGjNb][64];
  Zs[t >> 4][t & 15] = Zg[t];
  Ws[t >> 4][t & 15] = Zg[kGjNb * kGjNb + t];
  const int cc = min(col, c1 - 1);
#pragma unroll
  for (int q = 0; q < kGjNb / 4; ++q)
    Xs[g + 4 * q][lc] = E[(long)(kb + min(g + 4 * q, nbp - 1)) * ld + cc];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kGjNb / 4; ++q) {
    const int a = g + 4 * q;
    double2 y = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < kGjNb; ++b) {
      const double2 xb = Xs[b][lc];
      cfma(y, Zs[a][b], xb);
      cfma(v, Ws[a][b], xb);
    }
    if (a < nbp && col < c1) {
      E[(long)(kb + a) * ld + col] = y;
      Bk[(long)a * n2 + col] = v;
    }
  }
}

// left half <- (right half)^H, 16 x 16 tiles through LDS
__global__ __launch_bounds__(256) void ch_adjoint_kernel(SocElimBatch B, long ld, int n) {
  double2 *E = B.E[blockIdx.z];
  __shared__ double2 tile[16][17];
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
  // read G[r0 + i][c0 + j] (right half), write conj into left [c0 + i][r0 + j]
  if (r0 + i < n && c0 + j < n) tile[i][j] = E[(long)(r0 + i) * ld + n + c0 + j];
  __syncthreads();
  if (c0 + i < n && r0 + j < n) E[(long)(c0 + i) * ld + r0 + j] = cconj(tile[j][i]);
}

// ------------------------------------------------ blocked Gauss-Jordan
// E = [M | I] (n x 2n, leading dim ld) is inverted in panels of kGjNb pivot
// columns kb .. kb + nbp - 1, three launches per panel for the whole batch:
//   gj_panel_kernel  one workgroup per matrix holds the panel's columns of
//                    every row in registers and takes the panel's pivots by
//                    partial pivoting on the Schur complement among the rows
//                    not used yet (no rows are moved), then inverts the pivot
//                    block D = E[R, panel] (rows R in pivot order): Z = D^{-1};
//   gj_rows_kernel   the new block rows B = Z E[R, c] for the live columns
//                    c >= kb + nbp;
//   cgemm            E[:, c] -= E[:, panel] B[:, c] for every row (MFMA).
// The pivot rows must become B itself: the panel kernel subtracts 1 from
// their pivot entries E[R_a, kb + a] (the panel's columns are not read
// again), so that the same rank-nbp product leaves E[R_a] - (D - I)_a B = B_a.
// After the last panel row prow[c] holds (e_c | row c of M^{-1}), and
// gj_gather_kernel writes M^{-1} into the left half.  Row r counts as used
// once piv[n + r] = c < kb with piv[c] = r, so the scratch needs no clearing
// between inversions (a stale entry fails the test).
constexpr int kGjThreads = 512;   // panel kernel: rows t and t + 512 (n <= 1024)

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const int lo = __shfl_xor((int)(unsigned)v, m, 64);
  const int hi = __shfl_xor((int)(unsigned)(v >> 32), m, 64);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
}

__global__ __launch_bounds__(kGjThreads) void gj_panel_kernel(SocElimBatch B, long ld, int n,
                                                              int kb) {
  const int w = blockIdx.x;
  double2 *E = B.E[w];
  int *prow = B.piv[w], *slot = B.piv[w] + n;
  double2 *Z = B.B[w] + (size_t)kGjNb * 2 * n;
  const int nbp = min(kGjNb, n - kb);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int kWaves = kGjThreads / 64;
  __shared__ unsigned long long wkey[2][kWaves];
  __shared__ double2 wrow[2][kWaves][kGjNb];
  __shared__ double2 D[kGjNb][2 * kGjNb];
  __shared__ int rows[kGjNb];

  // the panel's entries of rows t and t + 512 (clamped addresses, all loads
  // in flight together), and whether each row is still unused
  double2 a[2][kGjNb];
  int r[2], sl[2];
  bool live[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    r[i] = t + kGjThreads * i;
    const int rc = min(r[i], n - 1);
#pragma unroll
    for (int j = 0; j < kGjNb; ++j) a[i][j] = E[(long)rc * ld + kb + min(j, nbp - 1)];
    sl[i] = slot[rc];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const bool cand = sl[i] >= 0 && sl[i] < kb;
    const int pr = prow[cand ? sl[i] : 0];
    live[i] = r[i] < n && !(cand && pr == r[i]);
  }

  // per column: the largest |entry|^2 among unused rows wins; the key packs
  // its IEEE bits (a non-negative double orders like its bit pattern) with
  // 2047 - row in the low 11 bits, so ties go to the smaller row and the
  // reduction is an integer max.  Each wave's winner puts its key and its
  // panel row in LDS (double-buffered by column parity: one barrier a column).
  // The register rows are shifted one column left after each column, so the
  // current column is always a[i][0] and no register is indexed by j.
  bool singular = false;
  for (int j = 0; j < nbp; ++j) {
    const int bf = j & 1;
    unsigned long long best = 0;
    int bi = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double m = a[i][0].x * a[i][0].x + a[i][0].y * a[i][0].y;
      const unsigned long long key = ((unsigned long long)__double_as_longlong(m) & ~0x7FFull) |
                                     (unsigned long long)(2047 - r[i]);
      if (live[i] && key > best) {
        best = key;
        bi = i;
      }
    }
    unsigned long long wb = best;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
      const unsigned long long o = shfl_xor_u64(wb, m);
      wb = o > wb ? o : wb;
    }
    // (two stores with constant register indices: a select between the rows
    // would index the register array at run time and move it to scratch)
    if (wb != 0 && best == wb) {
      wkey[bf][wave] = wb;
      if (bi == 0) {
#pragma unroll
        for (int c = 0; c < kGjNb; ++c) wrow[bf][wave][c] = a[0][c];
      } else {
#pragma unroll
        for (int c = 0; c < kGjNb; ++c) wrow[bf][wave][c] = a[1][c];
      }
    }
    if (wb == 0 && lane == 0) wkey[bf][wave] = 0;
    __syncthreads();
    unsigned long long kmax = 0;
    int wv = 0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) {
      const unsigned long long k = wkey[bf][v];
      if (k > kmax) {
        kmax = k;
        wv = v;
      }
    }
    // an unused row always exists, so kmax >= 1024 names one (the clamp
    // only keeps the indices in range should that ever fail)
    const int p = min(2047 - (int)(kmax & 0x7FF), n - 1);
    const double2 d = wrow[bf][wv][0];
    const double dm = d.x * d.x + d.y * d.y;
    singular = singular || kmax < 1024 || !(dm > 0.0) || !isfinite(dm);
    const double2 inv = make_double2(d.x / dm, -d.y / dm);
    if (t == 0) {
      prow[kb + j] = p;
      slot[p] = kb + j;
      rows[j] = p;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (r[i] == p) live[i] = false;
      if (live[i]) {
        const double2 f = cmul(a[i][0], inv);
#pragma unroll
        for (int c = 1; c < kGjNb; ++c) a[i][c] = csub(a[i][c], cmul(f, wrow[bf][wv][c]));
      }
#pragma unroll
      for (int c = 0; c + 1 < kGjNb; ++c) a[i][c] = a[i][c + 1];
      a[i][kGjNb - 1] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  // [D | I] in LDS, D extended by the identity to kGjNb x kGjNb; its
  // elimination needs no pivoting (D's rows are in the order of the pivots
  // just taken), one thread per entry of the 16 x 32 block
  const int ra = t >> 5, cb = t & 31;
  {
    double2 v;
    if (cb < kGjNb && ra < nbp && cb < nbp)
      v = E[(long)rows[ra] * ld + kb + cb];
    else
      v = make_double2((cb & (kGjNb - 1)) == ra ? 1.0 : 0.0, 0.0);
    D[ra][cb] = v;
  }
  __syncthreads();
  for (int s = 0; s < nbp; ++s) {
    const double2 x = D[ra][cb], das = D[ra][s], dsb = D[s][cb], ps = D[s][s];
    __syncthreads();
    const double pm = ps.x * ps.x + ps.y * ps.y;
    const double2 rowv = cmul(dsb, make_double2(ps.x / pm, -ps.y / pm));
    D[ra][cb] = ra == s ? rowv : csub(x, cmul(das, rowv));
    __syncthreads();
  }
  if (cb >= kGjNb)
    Z[ra * kGjNb + cb - kGjNb] =
        (ra < nbp && cb - kGjNb < nbp) ? D[ra][cb] : make_double2(0.0, 0.0);
  if (t < nbp) E[(long)rows[t] * ld + kb + t].x -= 1.0;
  if (singular && t == 0) B.stats[w][kStError] |= kErrSingular;
}

// B[a][c] = sum_b Z[a][b] E[R_b][c] for a < nbp and the live columns
// c >= kb + nbp; 64 columns a workgroup, four rows of B a thread.
__global__ __launch_bounds__(256) void gj_rows_kernel(SocElimBatch B, long ld, int n, int kb) {
  const int w = blockIdx.y;
  const double2 *E = B.E[w];
  const int *prow = B.piv[w];
  const double2 *Z = B.B[w] + (size_t)kGjNb * 2 * n;
  double2 *Bk = B.B[w];
  const int nbp = min(kGjNb, n - kb), c0 = kb + nbp, n2 = 2 * n;
  const int t = threadIdx.x, g = t >> 6;
  const int col = c0 + (int)blockIdx.x * 64 + (t & 63);
  __shared__ double2 Zs[kGjNb][kGjNb];
  static_assert(kGjNb * kGjNb == 256, "one Z entry a thread");
  Zs[t >> 4][t & 15] = Z[t];
  __syncthreads();
  const int cc = min(col, n2 - 1);
  double2 x[kGjNb];
#pragma unroll
  for (int b = 0; b < kGjNb; ++b) x[b] = E[(long)prow[kb + min(b, nbp - 1)] * ld + cc];
#pragma unroll
  for (int q = 0; q < kGjNb / 4; ++q) {
    const int ar = g + 4 * q;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < kGjNb; ++b) cfma(acc, Zs[ar][b], x[b]);
    if (ar < nbp && col < n2) Bk[(long)ar * n2 + col] = acc;
  }
}

// left half row c <- right half of row prow[c] (= row c of M^{-1})
__global__ __launch_bounds__(256) void gj_gather_kernel(SocElimBatch B, long ld, int n) {
  double2 *E = B.E[blockIdx.y];
  const int c = blockIdx.x;
  const double2 *src = E + (long)B.piv[blockIdx.y][c] * ld + n;
  double2 *dst = E + (long)c * ld;
  for (int j = threadIdx.x; j < n; j += 256) dst[j] = src[j];
}

// --------------------------------------------------------------- decisions
// One workgroup decides the kk sites g0 .. g0 + kk - 1 of one group.
// n = 2 kk, index a < kk: the up row of site g0 + a, a >= kk: the down row.
// In: W0p (n x n) = W_g T0 U_L[:, g] (without the flip blocks), the fields.
// Out: D (n x n) = delta_bd Mc, Mc = (1 + W0_AA)^{-1} spread to n x n (zero
// outside the accepted set A), so that T = T0 - (T0 U_L[:, g]) D (W_g T0);
// *nflush = n if A is not empty, else 0; accepted sites' fields flipped and
// accx[j] = their old field (rotate_accepted then turns their U_R rows).
//
// The decisions sweep pivots out of E = 1 + W0 (W0 = W0p with each site's
// flip block on its column pair).  Once the 2 x 2 pivot blocks of the
// accepted sites are swept (principal pivot transform), every unswept pivot
// block E_JJ, J = (j, kk + j), is its Schur complement given A: the current
// 1 + W_j T V_j, whose determinant is site j's ratio (Eqs. (A7)-(A9)); and
// the swept block E_AA is -(1 + W0_AA)^{-1}.  Accepting site j sweeps J with
// S = E_JJ:
//   E_rc -= E_rJ S^{-1} E_Jc,  E_rJ <- E_rJ S^{-1},  E_Jc <- S^{-1} E_Jc,
//   E_JJ <- -S^{-1}            (r, c outside J).
// All four cases are one formula, E_rc -= e_r g_c, with e_r = E_rJ - [r in J]
// (the unit row of r's place in J), g_c = S^{-1} E_Jc for c outside J and
// g_c = u_c - S^{-1} u_c for c in J, and -2 on the two diagonal entries of
// J.  E lives in registers (thread t: column t % 64, rows t / 64 + 4 i); per
// site the owners of J's two rows and two columns publish them in LDS
// (double-buffered by site parity: one barrier a site), every thread reads
// the pivot block and takes the same decision, and a rejected site changes
// nothing.
constexpr int kDecThreads = 256;

__global__ __launch_bounds__(kDecThreads) void soc_decide_kernel(SocDecideBatch B) {
  const SocDecideArgs &a = B.a[blockIdx.x];   // one workgroup per walker
  extern __shared__ double2 Ms[];      // n x (n + 1): Mc at the end
  const int kk = a.kk, n = 2 * kk;
  const int ld = n + 1;
  __shared__ double xs[64];
  __shared__ double us[64];            // the group's Metropolis uniforms (independent of decisions)
  __shared__ int accm[64];
  __shared__ double2 colJ[2][2][64];   // [site parity][J place][row]
  __shared__ double2 rowJ[2][2][64];   // [site parity][J place][column]
  const int t = threadIdx.x, c = t & 63, rq = t >> 6;
  int n_low = 0, n_neg = 0, n_acc = 0;   // thread 0's counters (n_acc: every thread's)
  bool nonfinite = false;
  int8_t *xrow = a.fields + (long)a.li * a.N + a.g0;
  for (int j = t; j < kk; j += kDecThreads) {
    xs[j] = (double)xrow[j];
    us[j] = philox_uniform(a.key0, a.key1, a.sweep, a.slice_code, (uint64_t)(a.g0 + j),
                           kPurposeMH);
  }
  __syncthreads();
  // this thread's entries of E = 1 + W0: the flip block delta = [[dd, -x do],
  // [x do, dd]] (dd = cos 2gamma - 1, do = sin 2gamma) of site cs on the
  // column pair (cs, kk + cs); zero outside n x n
  const bool cv = c < n;
  const int cs = cv ? (c < kk ? c : c - kk) : 0;
  const bool up = c < kk;
  double2 e[16];
  {
    const double x = xs[cs];
    const double da = up ? a.dd : -x * a.doff, db = up ? x * a.doff : a.dd;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = rq + 4 * i;
      const int rr = min(r, n - 1);
      const double2 w0 = a.W0p[(long)rr * n + cs], w1 = a.W0p[(long)rr * n + kk + cs];
      double2 v = make_double2(w0.x * da + w1.x * db, w0.y * da + w1.y * db);
      if (r == c) v.x += 1.0;
      e[i] = (r < n && cv) ? v : make_double2(0.0, 0.0);
    }
  }
  for (int j = 0; j < kk; ++j) {
    const int p = j & 1, c0 = j, c1 = kk + j;
    // publish J's columns (their owners) and rows (selected from the registers)
    if (c == c0 || c == c1) {
      const int q = c == c1 ? 1 : 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) colJ[p][q][rq + 4 * i] = e[i];
    }
    {
      double v0x = 0.0, v0y = 0.0, v1x = 0.0, v1y = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = rq + 4 * i;
        v0x = r == c0 ? e[i].x : v0x;
        v0y = r == c0 ? e[i].y : v0y;
        v1x = r == c1 ? e[i].x : v1x;
        v1y = r == c1 ? e[i].y : v1y;
      }
      if (rq == (c0 & 3)) rowJ[p][0][c] = make_double2(v0x, v0y);
      if (rq == (c1 & 3)) rowJ[p][1][c] = make_double2(v1x, v1y);
    }
    __syncthreads();
    const double2 S00 = rowJ[p][0][c0], S01 = rowJ[p][0][c1];
    const double2 S10 = rowJ[p][1][c0], S11 = rowJ[p][1][c1];
    const double2 R = csub(cmul(S00, S11), cmul(S01, S10));
    const double absR = hypot(R.x, R.y);
    const double uu = us[j];
    const bool finite = !isnan(absR);
    const bool acc = __builtin_amdgcn_readfirstlane((finite && uu < absR) ? 1 : 0) != 0;
    if (t == 0) {
      const int site = a.g0 + j;
      const double margin = absR - uu;
      // counters kept in registers, added to memory once per group
      if (fabs(margin) < 1e-12) ++n_low;
      if (R.x < 0.0) ++n_neg;
      if (!finite) nonfinite = true;
      const long long idx = a.log_base + site;
      if (a.log_meta && idx < a.log_cap) {
        a.log_meta[3 * idx + 0] = (int32_t)a.slice_code;
        a.log_meta[3 * idx + 1] = site;
        a.log_meta[3 * idx + 2] = acc ? 1 : 0;
        a.log_margin[idx] = margin;
      }
      if (acc) xrow[j] = (int8_t)(xs[j] > 0.0 ? -1 : 1);
      accm[j] = acc ? 1 : 0;
    }
    if (!acc) continue;
    ++n_acc;
    const double2 iR = cdiv(make_double2(1.0, 0.0), R);
    const double2 I00 = cmul(S11, iR), I01 = cmul(make_double2(-S01.x, -S01.y), iR);
    const double2 I10 = cmul(make_double2(-S10.x, -S10.y), iR), I11 = cmul(S00, iR);
    // g for this column
    const double2 ej0 = rowJ[p][0][c], ej1 = rowJ[p][1][c];
    double2 g0 = cmul(I00, ej0), g1 = cmul(I10, ej0);
    cfma(g0, I01, ej1);
    cfma(g1, I11, ej1);
    const bool k0 = c == c0, k1 = c == c1;
    g0.x = k0 ? 1.0 - I00.x : (k1 ? -I01.x : g0.x);
    g0.y = k0 ? -I00.y : (k1 ? -I01.y : g0.y);
    g1.x = k0 ? -I10.x : (k1 ? 1.0 - I11.x : g1.x);
    g1.y = k0 ? -I10.y : (k1 ? -I11.y : g1.y);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = rq + 4 * i;
      double2 e0 = colJ[p][0][r], e1 = colJ[p][1][r];
      e0.x -= r == c0 ? 1.0 : 0.0;
      e1.x -= r == c1 ? 1.0 : 0.0;
      double2 v = csub(e[i], cmul(e0, g0));
      v = csub(v, cmul(e1, g1));
      v.x -= (r == c && (k0 || k1)) ? 2.0 : 0.0;
      e[i] = v;
    }
  }
  // Mc = -E on A x A, zero elsewhere, to LDS; the accepted sites' old fields
  __syncthreads();   // accm visible
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = rq + 4 * i;
    if (r < n && cv) {
      const bool in = accm[r < kk ? r : r - kk] && accm[cs];
      Ms[r * ld + c] = in ? make_double2(-e[i].x, -e[i].y) : make_double2(0.0, 0.0);
    }
  }
  for (int j = t; j < kk; j += kDecThreads) a.accx[j] = accm[j] ? (int)xs[j] : 0;
  __syncthreads();
  // D = delta_bd Mc (rows (j, kk + j) of Mc mixed by the pre-flip delta_j)
  for (int e2 = t; e2 < kk * n; e2 += kDecThreads) {
    const int j = e2 / n, q = e2 % n;
    const double x = xs[j];
    const double d00 = a.dd, d01 = -x * a.doff, d10 = x * a.doff, d11 = a.dd;
    const double2 m0 = Ms[j * ld + q], m1 = Ms[(kk + j) * ld + q];
    a.D[(long)j * n + q] = make_double2(d00 * m0.x + d01 * m1.x, d00 * m0.y + d01 * m1.y);
    a.D[(long)(kk + j) * n + q] =
        make_double2(d10 * m0.x + d11 * m1.x, d10 * m0.y + d11 * m1.y);
  }
  if (t == 0) {
    *a.nflush = n_acc > 0 ? n : 0;
    a.stats[kStProposed] += kk;
    a.stats[kStFieldUpdates] += kk;
    a.stats[kStAccepted] += n_acc;
    a.stats[kStFlips] += n_acc;
    if (n_low) a.stats[kStLowMargin] += n_low;
    if (n_neg) a.stats[kStNegative] += n_neg;
    if (nonfinite) a.stats[kStError] |= kErrNonFinite;
  }
}

// U_R rows of the sites accepted by decide / decide1 <- (1 + delta) rows:
// w = 2, rows (site, N + site) by the 2 x 2 block of the old field; w = 1,
// row site by the phase factor.  Grid (256-column slices, kk, walkers).
__global__ __launch_bounds__(256) void rotate_accepted_kernel(SocDecideBatch B, int w) {
  const SocDecideArgs &a = B.a[blockIdx.z];
  const int j = blockIdx.y;
  if (j >= a.kk) return;
  const int xo = a.accx[j];
  const int q = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (xo == 0 || q >= a.ne) return;
  const double x = (double)xo;
  double2 *p0 = a.UR + (long)(a.g0 + j) * a.ne + q;
  if (w == 1) {
    *p0 = cmul(make_double2(1.0 + a.dd, -x * a.doff), *p0);
    return;
  }
  double2 *p1 = a.UR + (long)(a.N + a.g0 + j) * a.ne + q;
  const double d00 = 1.0 + a.dd, d01 = -x * a.doff, d10 = x * a.doff, d11 = 1.0 + a.dd;
  const double2 r0 = *p0, r1 = *p1;
  *p0 = make_double2(d00 * r0.x + d01 * r1.x, d00 * r0.y + d01 * r1.y);
  *p1 = make_double2(d10 * r0.x + d11 * r1.x, d10 * r0.y + d11 * r1.y);
}

// Gauss-Jordan elimination with partial pivoting of the n x n left part of
// A (n rows, ncols columns, leading dim ld; n <= 64) in LDS, by one
// workgroup: A <- [I | A_left^{-1} A_right] up to rounding, *det <- det(A_left)
// (thread 0; 0 if singular).  All threads call it.
__device__ void gj_lds(double2 *A, int n, int ncols, int ld, double2 *det, int *ok) {
  __shared__ int pv;
  __shared__ double2 pd;          // the pivot value, published with its row
  __shared__ double2 fcol[64];    // each row's multiplier of the pivot row
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) {
    *det = make_double2(1.0, 0.0);
    *ok = 1;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double bv = -1.0;
    int bi = n;
    if (wave == 0) {
      const int r = j + lane;
      if (r < n) {
        bv = hypot(A[r * ld + j].x, A[r * ld + j].y);
        bi = r;
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(bv, off, 64);
        const int oi = __shfl_down(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (lane == 0) {
        const bool good = bv > 0.0 && isfinite(bv);
        pv = good ? bi : -1;
        if (good) pd = A[bi * ld + j];
        if (!good) {
          *ok = 0;
          *det = make_double2(0.0, 0.0);
        }
      }
    }
    __syncthreads();
    const int p = pv;
    if (p < 0) return;
    // One phase: swap rows j and p, scale the new row j by 1/d and keep the
    // multipliers (column j after the swap, before the scaling).  Only rows
    // j and p are written, so the other rows' column j is read freely; the
    // thread of column j hands row p its multiplier, the old A[j][j].
    const double2 d = pd;
    const double2 inv = cdiv(make_double2(1.0, 0.0), d);
    if (t < n && t != j && t != p) fcol[t] = A[t * ld + j];
    for (int c = t; c < ncols; c += kDecThreads) {
      const double2 aj = A[j * ld + c], ap = A[p * ld + c];
      A[j * ld + c] = cmul(ap, inv);
      if (p != j) {
        A[p * ld + c] = aj;
        if (c == j) fcol[p] = aj;
      }
    }
    if (t == 0) {
      double2 dt = cmul(*det, d);
      if (p != j) dt = make_double2(-dt.x, -dt.y);
      *det = dt;
    }
    __syncthreads();
    // rows wave + 4 q, columns lane and lane + 64 (n <= 64, ncols <= 128):
    // the entries and multipliers of four rows a wave loaded before any of
    // their stores, one LDS round trip per four rows (no integer division)
    {
      const int wv = t >> 6;
      double2 ajc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) ajc[h] = A[j * ld + min(lane + 64 * h, ncols - 1)];
      // four rows a wave at a time, their loads issued together
      auto upd = [&](int r, double2 f, double2 v0, double2 v1) {
        if (r < n && r != j) {
          if (lane < ncols && lane >= j) A[r * ld + lane] = csub(v0, cmul(f, ajc[0]));
          if (lane + 64 < ncols && lane + 64 >= j) A[r * ld + lane + 64] = csub(v1, cmul(f, ajc[1]));
        }
      };
      const int c0 = min(lane, ncols - 1), c1 = min(lane + 64, ncols - 1);
      for (int r0 = wv; r0 < n; r0 += 16) {
        const int ra = r0, rb = r0 + 4, rc = r0 + 8, rd = r0 + 12;
        const int pa = min(ra, n - 1), pb = min(rb, n - 1), pc = min(rc, n - 1), pd = min(rd, n - 1);
        const double2 fa = fcol[pa], fb = fcol[pb], fc = fcol[pc], fd = fcol[pd];
        const double2 a0 = A[pa * ld + c0], a1 = A[pa * ld + c1];
        const double2 b0 = A[pb * ld + c0], b1 = A[pb * ld + c1];
        const double2 d0 = A[pc * ld + c0], d1 = A[pc * ld + c1];
        const double2 e0 = A[pd * ld + c0], e1 = A[pd * ld + c1];
        upd(ra, fa, a0, a1);
        upd(rb, fb, b0, b1);
        upd(rc, fc, d0, d1);
        upd(rd, fd, e0, e1);
      }
    }
    __syncthreads();
  }
}

// Block force-bias decision for the kk sites g0 .. g0 + kk - 1 (n = 2 kk,
// index a < kk: the up row of site g0 + a, a >= kk: the down row).
// In: W0p = W_b T U_L[:, b] (n x n, no flip blocks).  Steps: force bias
// s_j = gamma <O_j> with the block's fields removed from the small matrix
// M = A_bd W0p (1 + Db W0p)^{-1} (A_bd = blocks A(-x_j), Db = A_bd - 1);
// heat-bath fields x'_j; flip set F; R = det(1 + W0p_FF delta_F),
// prior = prod_F e^{2 s_j x_j}; accept iff u < |R prior| (u at site g0).
// Out: D = delta_F (1 + W0p_FF delta_F)^{-1} spread to n x n, *nflush,
// fields and U_R row pairs of F when accepted.
__global__ __launch_bounds__(kDecThreads) void soc_block_decide_kernel(SocDecideBatch B) {
  const SocDecideArgs &a = B.a[blockIdx.x];   // one workgroup per walker
  extern __shared__ double2 lds[];
  const int kk = a.kk, n = 2 * kk;
  const int ld = 2 * n + 1;
  double2 *Aug = lds;                // n x ld
  __shared__ double xs[64], sv[64];
  __shared__ int flip[64], fidx[64], nf_s, acc_s, ok_s;
  __shared__ double2 det_s;
  const int t = threadIdx.x;
  int8_t *xrow = a.fields + (long)a.li * a.N + a.g0;
  for (int j = t; j < kk; j += kDecThreads) xs[j] = (double)xrow[j];
  __syncthreads();
  // [E^T | W0p^T] with E = 1 + Db W0p: row r of E^T is column r of E
  for (int e = t; e < n * n; e += kDecThreads) {
    const int r = e / n, c = e - r * n;   // Aug[r][c] = E[c][r], Aug[r][n + c] = W0p[c][r]
    const int jc = c < kk ? c : c - kk;
    const double x = xs[jc];
    // row c of Db W0p: Db rows (jc, kk + jc) = A(-x) - 1 = [[cg - 1, -x sg], [x sg, cg - 1]]
    const double d0 = c < kk ? a.c1 - 1.0 : x * a.s1;    // coefficient of W0p[jc][r]
    const double d1 = c < kk ? -x * a.s1 : a.c1 - 1.0;   // coefficient of W0p[kk + jc][r]
    const double2 w0 = a.W0p[(long)jc * n + r], w1 = a.W0p[(long)(kk + jc) * n + r];
    double2 v = make_double2(d0 * w0.x + d1 * w1.x, d0 * w0.y + d1 * w1.y);
    if (r == c) v.x += 1.0;
    Aug[r * ld + c] = v;
    Aug[r * ld + n + c] = a.W0p[(long)c * n + r];
  }
  __syncthreads();
  gj_lds(Aug, n, 2 * n, ld, &det_s, &ok_s);
  // Y = W0p E^{-1}: Y[a][b] = Aug[b][n + a]; M rows of site j = A(-x_j) Y rows
  if (t < kk) {
    const int j = t;
    const double x = xs[j];
    const double2 yjj = Aug[j * ld + n + j], ydj = Aug[j * ld + n + kk + j];
    const double2 yjd = Aug[(kk + j) * ld + n + j], ydd = Aug[(kk + j) * ld + n + kk + j];
    // <c+_up c_dn> = M[kk + j][j] = x sg Y[j][j] + cg Y[kk + j][j]
    // <c+_dn c_up> = M[j][kk + j] = cg Y[j][kk + j] - x sg Y[kk + j][kk + j]
    const double up_dn = x * a.s1 * yjj.x + a.c1 * ydj.x;
    const double dn_up = a.c1 * yjd.x - x * a.s1 * ydd.x;
    sv[j] = ok_s ? a.gamma * (up_dn - dn_up) : 0.0;
  }
  __syncthreads();
  // heat bath and the flip set
  if (t == 0) {
    int nf = 0;
    for (int j = 0; j < kk; ++j) {
      const double pu = 1.0 / (1.0 + exp(-2.0 * sv[j]));
      const double u = philox_uniform(a.key0, a.key1, a.sweep, a.slice_code,
                                      (uint64_t)(a.g0 + j), kPurposeHB);
      const double xn = u < pu ? 1.0 : -1.0;
      flip[j] = xn != xs[j];
      if (flip[j]) fidx[nf++] = j;
    }
    nf_s = nf;
    if (!ok_s) a.stats[kStError] |= kErrSingular;
  }
  __syncthreads();
  const int nf = nf_s, m = 2 * nf;
  // [S_F | I], S_F = 1 + W0p[pF, pF] delta_F, pF = (up rows of F, down rows of F)
  const int ldf = 2 * m + 1;
  for (int e = t; e < m * m; e += kDecThreads) {
    const int r = e / m, c = e - r * m;
    const int jr = fidx[r < nf ? r : r - nf], jc = fidx[c < nf ? c : c - nf];
    const int ar = r < nf ? jr : kk + jr;
    const double x = xs[jc];
    // column c of W0p[pF, pF] delta_F: delta = [[dd, -x do], [x do, dd]] on (jc, kk + jc)
    const double2 wu = a.W0p[(long)ar * n + jc], wd = a.W0p[(long)ar * n + kk + jc];
    const double q0 = c < nf ? a.dd : -x * a.doff;       // delta[0][cc]
    const double q1 = c < nf ? x * a.doff : a.dd;        // delta[1][cc]
    double2 v = make_double2(wu.x * q0 + wd.x * q1, wu.y * q0 + wd.y * q1);
    if (r == c) v.x += 1.0;
    Aug[r * ldf + c] = v;
    Aug[r * ldf + m + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (nf > 0) gj_lds(Aug, m, 2 * m, ldf, &det_s, &ok_s);
  if (t == 0) {
    double2 R = nf > 0 ? det_s : make_double2(1.0, 0.0);
    double pe = 0.0;
    for (int q = 0; q < nf; ++q) pe += 2.0 * sv[fidx[q]] * xs[fidx[q]];
    const double prior = exp(pe);
    const double absA = hypot(R.x, R.y) * prior;
    const double u = philox_uniform(a.key0, a.key1, a.sweep, a.slice_code, (uint64_t)a.g0,
                                    kPurposeMH);
    const bool finite = !isnan(absA);
    const bool acc = finite && u < absA && (nf == 0 || ok_s);
    const double margin = absA - u;
    a.stats[kStProposed] += 1;
    a.stats[kStFieldUpdates] += kk;
    if (acc) {
      a.stats[kStAccepted] += 1;
      a.stats[kStFlips] += nf;
    }
    if (fabs(margin) < 1e-12) a.stats[kStLowMargin] += 1;
    if (R.x < 0.0) a.stats[kStNegative] += 1;
    if (!finite) a.stats[kStError] |= kErrNonFinite;
    const long long idx = a.log_base;
    if (a.log_meta && idx < a.log_cap) {
      a.log_meta[3 * idx + 0] = (int32_t)a.slice_code;
      a.log_meta[3 * idx + 1] = a.g0;
      a.log_meta[3 * idx + 2] = acc ? 1 : 0;
      a.log_margin[idx] = margin;
    }
    acc_s = acc && nf > 0;
    *a.nflush = (acc && nf > 0) ? n : 0;
  }
  __syncthreads();
  // D = delta_F S_F^{-1} spread to the block's n x n (zero elsewhere)
  for (int e = t; e < n * n; e += kDecThreads) a.D[e] = make_double2(0.0, 0.0);
  if (!acc_s)
    for (int j = t; j < kk; j += kDecThreads) a.accx[j] = 0;   // no rows to turn
  __syncthreads();
  if (!acc_s) return;
  for (int e = t; e < m * m; e += kDecThreads) {
    const int r = e / m, c = e - r * m;
    const int q = r < nf ? r : r - nf;
    const int j = fidx[q];
    const double x = xs[j];
    // rows (q, nf + q) of S_F^{-1} mixed by delta_j
    const double2 m0 = Aug[q * ldf + m + c], m1 = Aug[(nf + q) * ldf + m + c];
    const double e0 = r < nf ? a.dd : x * a.doff;
    const double e1 = r < nf ? -x * a.doff : a.dd;
    const int jc = fidx[c < nf ? c : c - nf];
    const int ar = r < nf ? j : kk + j, ac = c < nf ? jc : kk + jc;
    a.D[(long)ar * n + ac] = make_double2(e0 * m0.x + e1 * m1.x, e0 * m0.y + e1 * m1.y);
  }
  // fields of the flip set, and its old fields for rotate_accepted (which
  // turns the U_R row pairs)
  for (int j = t; j < kk; j += kDecThreads) {
    if (flip[j]) xrow[j] = (int8_t)(xs[j] > 0.0 ? -1 : 1);
    a.accx[j] = flip[j] ? (int)xs[j] : 0;
  }
}

// ---------------------------------------------------- one sector (w = 1)
// The paper's own U < 0 model (Sec. II B, Eqs. (13)-(14)): the imaginary
// coupling alpha = i gamma gives B_dn = conj(B_up), so only the spin-up
// sector (N orbitals, N_up fermions) is propagated and every ratio is
// R = r_up r_dn = |r_up|^2.  The field of site i multiplies row i by the
// phase e^{i gamma x_i}; a flip x -> -x is the scalar
// delta(x) = e^{-2 i gamma x} - 1 = (dd, -x doff) with dd = cos 2 gamma - 1,
// doff = sin 2 gamma (the same numbers as the rank-two path's delta block).

// Y[i, :] = e^{i sign gamma x_i} X[i, :] (X == Y allowed); c = cos gamma, s = sin gamma
__global__ __launch_bounds__(256) void phase_kernel(const double2 *X, long ldx, double2 *Y,
                                                    long ldy, int ncols, int N,
                                                    const int8_t *xrow, double c, double s,
                                                    double sign) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)N * ncols) return;
  const int i = (int)(e / ncols), col = (int)(e % ncols);
  const double sn = sign * (double)xrow[i] * s;
  const double2 v = X[(long)i * ldx + col];
  Y[(long)i * ldy + col] = make_double2(c * v.x - sn * v.y, c * v.y + sn * v.x);
}

__device__ __forceinline__ double2 flip_delta(const SocDecideArgs &a, double x) {
  return make_double2(a.dd, -x * a.doff);
}

// Delayed (and, with kk = 1, local) decisions of one group of kk <= 64 sites
// of the one-sector model.  In: W0p = U_g T0 U_L[:, g] (kk x kk).  With
// W0 = W0p diag(delta) and Mc = (1 + W0_AA)^{-1} spread to kk x kk (zero
// outside the accepted set A), site j's ratio is the Schur complement
// r = 1 + W0_jj - W0_j,: Mc W0_:,j (the recursion of Eq. (28)) and the test
// is u < |r|^2.  As in the rank-two kernel, E = 1 + W0 is swept, in
// registers: the unswept diagonal entry E_jj is r; accepting j sweeps pivot j
//   E_rc -= E_rj E_jc / r,  E_rj <- E_rj / r,  E_jc <- E_jc / r,  E_jj <- -1 / r,
// as one formula E_rc -= e_r g_c with e_r = E_rj - [r = j], g_c = E_jc / r
// (c != j), g_j = 1 - 1 / r, and -2 on E_jj; the swept block ends as
// E_AA = -Mc.  Out: D = diag(delta) Mc, so that T = T0 - (T0 U_L[:, g]) D
// (U_g T0) (Eq. (30)); accx as the rank-two kernel.
__global__ __launch_bounds__(kDecThreads) void cplx_decide_kernel(SocDecideBatch B) {
  const SocDecideArgs &a = B.a[blockIdx.x];   // one workgroup per walker
  extern __shared__ double2 Ms[];      // n x (n + 1): Mc at the end
  const int n = a.kk;
  const int ld = n + 1;
  __shared__ double xs[64], us[64];
  __shared__ int accm[64];
  __shared__ double2 colJ[2][64], rowJ[2][64];   // [site parity][row / column]
  const int t = threadIdx.x, c = t & 63, rq = t >> 6;
  int n_low = 0, n_acc = 0;
  bool nonfinite = false;
  int8_t *xrow = a.fields + (long)a.li * a.N + a.g0;
  for (int j = t; j < n; j += kDecThreads) {
    xs[j] = (double)xrow[j];
    us[j] = a.force ? (a.force[a.g0 + j] ? -0.0 : __builtin_inf())
                    : philox_uniform(a.key0, a.key1, a.sweep, a.slice_code,
                                     (uint64_t)(a.g0 + j), kPurposeMH);
  }
  __syncthreads();
  const bool cv = c < n;
  double2 e[16];
  {
    const double2 dl = flip_delta(a, xs[cv ? c : 0]);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = rq + 4 * i;
      double2 v = cmul(a.W0p[(long)min(r, n - 1) * n + (cv ? c : 0)], dl);
      if (r == c) v.x += 1.0;
      e[i] = (r < n && cv) ? v : make_double2(0.0, 0.0);
    }
  }
  for (int j = 0; j < n; ++j) {
    const int p = j & 1;
    if (c == j) {
#pragma unroll
      for (int i = 0; i < 16; ++i) colJ[p][rq + 4 * i] = e[i];
    }
    {
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        vx = rq + 4 * i == j ? e[i].x : vx;
        vy = rq + 4 * i == j ? e[i].y : vy;
      }
      if (rq == (j & 3)) rowJ[p][c] = make_double2(vx, vy);
    }
    __syncthreads();
    const double2 r = rowJ[p][j];
    const double R = r.x * r.x + r.y * r.y;   // r_up r_dn with r_dn = conj(r_up)
    const double uu = us[j];
    const bool finite = !isnan(R);
    const bool acc = __builtin_amdgcn_readfirstlane((finite && uu < R) ? 1 : 0) != 0;
    if (t == 0) {
      const double margin = R - uu;
      if (fabs(margin) < 1e-12) ++n_low;
      if (!finite) nonfinite = true;
      const int site = a.g0 + j;
      const long long idx = a.log_base + site;
      if (a.log_meta && idx < a.log_cap) {
        a.log_meta[3 * idx + 0] = (int32_t)a.slice_code;
        a.log_meta[3 * idx + 1] = site;
        a.log_meta[3 * idx + 2] = acc ? 1 : 0;
        a.log_margin[idx] = margin;
      }
      if (acc) xrow[j] = (int8_t)(xs[j] > 0.0 ? -1 : 1);
      accm[j] = acc ? 1 : 0;
    }
    if (!acc) continue;
    ++n_acc;
    const double2 ir = cdiv(make_double2(1.0, 0.0), r);
    double2 g = cmul(rowJ[p][c], ir);
    const bool kj = c == j;
    g.x = kj ? 1.0 - ir.x : g.x;
    g.y = kj ? -ir.y : g.y;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int rw = rq + 4 * i;
      double2 er = colJ[p][rw];
      er.x -= rw == j ? 1.0 : 0.0;
      double2 v = csub(e[i], cmul(er, g));
      v.x -= (rw == c && kj) ? 2.0 : 0.0;
      e[i] = v;
    }
  }
  __syncthreads();   // accm visible
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = rq + 4 * i;
    if (r < n && cv) {
      const bool in = accm[r] && accm[c];
      Ms[r * ld + c] = in ? make_double2(-e[i].x, -e[i].y) : make_double2(0.0, 0.0);
    }
  }
  for (int j = t; j < n; j += kDecThreads) a.accx[j] = accm[j] ? (int)xs[j] : 0;
  __syncthreads();
  // D = diag(delta) Mc
  for (int e2 = t; e2 < n * n; e2 += kDecThreads) {
    const int j = e2 / n, q = e2 - j * n;
    a.D[(long)j * n + q] = cmul(flip_delta(a, xs[j]), Ms[j * ld + q]);
  }
  if (t == 0) {
    *a.nflush = n_acc > 0 ? n : 0;
    a.stats[kStProposed] += n;
    a.stats[kStFieldUpdates] += n;
    a.stats[kStAccepted] += n_acc;
    a.stats[kStFlips] += n_acc;
    if (n_low) a.stats[kStLowMargin] += n_low;
    if (nonfinite) a.stats[kStError] |= kErrNonFinite;
  }
}

// Block force-bias decision for kk <= 64 sites of the one-sector model
// (Sec. III B).  Force bias with the block's fields removed,
// Db = diag(e^{-i gamma x} - 1): nbar_j = (1 + Db_j) [W0p (1 + Db W0p)^{-1}]_jj
// for spin up, nbar_dn = conj(nbar_up), so s_j = alpha (nbar_up - nbar_dn)
// = -2 gamma Im nbar_j.  Heat bath, flip set F, r = det(1 + W0p_FF delta_F),
// prior prod_F e^{2 s_j x_j}, accept iff u < |r|^2 prior.  Out as the
// rank-two kernel: D = delta_F (1 + W0p_FF delta_F)^{-1} spread to kk x kk.
__global__ __launch_bounds__(kDecThreads) void cplx_block_decide_kernel(SocDecideBatch B) {
  const SocDecideArgs &a = B.a[blockIdx.x];   // one workgroup per walker
  extern __shared__ double2 lds[];
  const int n = a.kk;
  const int ld = 2 * n + 1;
  double2 *Aug = lds;                // n x ld
  __shared__ double xs[64], sv[64];
  __shared__ int fidx[64], nf_s, acc_s, ok_s;
  __shared__ double2 det_s;
  const int t = threadIdx.x;
  int8_t *xrow = a.fields + (long)a.li * a.N + a.g0;
  for (int j = t; j < n; j += kDecThreads) xs[j] = (double)xrow[j];
  __syncthreads();
  // [E^T | W0p^T], E = 1 + Db W0p
  for (int e = t; e < n * n; e += kDecThreads) {
    const int r = e / n, c = e - r * n;
    const double2 db = make_double2(a.c1 - 1.0, -xs[c] * a.s1);
    double2 v = cmul(db, a.W0p[(long)c * n + r]);
    if (r == c) v.x += 1.0;
    Aug[r * ld + c] = v;
    Aug[r * ld + n + c] = a.W0p[(long)c * n + r];
  }
  __syncthreads();
  gj_lds(Aug, n, 2 * n, ld, &det_s, &ok_s);
  if (t < n) {
    const int j = t;
    const double2 nb = cmul(make_double2(a.c1, -xs[j] * a.s1), Aug[j * ld + n + j]);
    sv[j] = ok_s ? -2.0 * a.gamma * nb.y : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    int nf = 0;
    for (int j = 0; j < n; ++j) {
      const double pu = 1.0 / (1.0 + exp(-2.0 * sv[j]));
      double u;
      if (a.force) {
        const double xt = a.force[a.g0 + j] ? -xs[j] : xs[j];
        u = xt > 0.0 ? -0.0 : __builtin_inf();
      } else {
        u = philox_uniform(a.key0, a.key1, a.sweep, a.slice_code, (uint64_t)(a.g0 + j),
                           kPurposeHB);
      }
      const double xn = u < pu ? 1.0 : -1.0;
      if (xn != xs[j]) fidx[nf++] = j;
    }
    nf_s = nf;
    if (!ok_s) a.stats[kStError] |= kErrSingular;
  }
  __syncthreads();
  const int nf = nf_s, m = nf;
  const int ldf = 2 * m + 1;
  for (int e = t; e < m * m; e += kDecThreads) {
    const int r = e / m, c = e - r * m;
    double2 v = cmul(a.W0p[(long)fidx[r] * n + fidx[c]], flip_delta(a, xs[fidx[c]]));
    if (r == c) v.x += 1.0;
    Aug[r * ldf + c] = v;
    Aug[r * ldf + m + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (nf > 0) gj_lds(Aug, m, 2 * m, ldf, &det_s, &ok_s);
  if (t == 0) {
    const double2 r = nf > 0 ? det_s : make_double2(1.0, 0.0);
    double pe = 0.0;
    for (int q = 0; q < nf; ++q) pe += 2.0 * sv[fidx[q]] * xs[fidx[q]];
    const double prior = exp(pe);
    const double absA = (r.x * r.x + r.y * r.y) * prior;
    const double u = a.force ? -0.0
                             : philox_uniform(a.key0, a.key1, a.sweep, a.slice_code,
                                              (uint64_t)a.g0, kPurposeMH);
    const bool finite = !isnan(absA);
    const bool acc = finite && u < absA && (nf == 0 || ok_s);
    const double margin = absA - u;
    a.stats[kStProposed] += 1;
    a.stats[kStFieldUpdates] += n;
    if (acc) {
      a.stats[kStAccepted] += 1;
      a.stats[kStFlips] += nf;
    }
    if (fabs(margin) < 1e-12) a.stats[kStLowMargin] += 1;
    if (!finite) a.stats[kStError] |= kErrNonFinite;
    const long long idx = a.log_base;
    if (a.log_meta && idx < a.log_cap) {
      a.log_meta[3 * idx + 0] = (int32_t)a.slice_code;
      a.log_meta[3 * idx + 1] = a.g0;
      a.log_meta[3 * idx + 2] = acc ? 1 : 0;
      a.log_margin[idx] = margin;
    }
    acc_s = acc && nf > 0;
    *a.nflush = (acc && nf > 0) ? n : 0;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += kDecThreads) a.D[e] = make_double2(0.0, 0.0);
  __syncthreads();
  if (!acc_s) return;
  for (int e = t; e < m * m; e += kDecThreads) {
    const int r = e / m, c = e - r * m;
    a.D[(long)fidx[r] * n + fidx[c]] = cmul(flip_delta(a, xs[fidx[r]]), Aug[r * ldf + m + c]);
  }
  for (int q = 0; q < nf; ++q) {
    const int j = fidx[q];
    const double2 f = make_double2(1.0 + a.dd, -xs[j] * a.doff);
    double2 *p0 = a.UR + (long)(a.g0 + j) * a.ne;
    for (int c = t; c < a.ne; c += kDecThreads) p0[c] = cmul(f, p0[c]);
    if (t == 0) xrow[j] = (int8_t)(xs[j] > 0.0 ? -1 : 1);
  }
}

}  // namespace

// ------------------------------------------------------------------- host
hipError_t cgemm(const CgemmBatch &b, int opA, int opB, hipStream_t st) {
  if (b.count <= 0) return hipSuccess;
  if (b.count > kCgemmMaxBatch) return hipErrorInvalidValue;
  int mt = 0, nt = 0;
  for (int i = 0; i < b.count; ++i) {
    mt = max(mt, (b.d[i].M + BM - 1) / BM);
    nt = max(nt, (b.d[i].N + BN - 1) / BN);
  }
  if (mt == 0 || nt == 0) return hipSuccess;
  int ns = 1;
  for (int i = 0; i < b.count; ++i)
    if (b.d[i].ksplit > 0) ns = max(ns, (b.d[i].K + b.d[i].ksplit - 1) / b.d[i].ksplit);
  const dim3 grid(nt, mt, b.count * ns);
#define PQ_CG(A_, B_)                                                                  \
  if (opA == A_ && opB == B_) {                                                        \
    hipLaunchKernelGGL((cgemm_kernel<A_, B_>), grid, dim3(256), 0, st, b, ns);          \
    return hipGetLastError();                                                          \
  }
  PQ_CG(kOpN, kOpN)
  PQ_CG(kOpN, kOpT)
  PQ_CG(kOpT, kOpN)
  PQ_CG(kOpH, kOpN)
#undef PQ_CG
  return hipErrorInvalidValue;
}

hipError_t csum(const CsumBatch &b, hipStream_t st) {
  if (b.count <= 0) return hipSuccess;
  if (b.count > kCgemmMaxBatch) return hipErrorInvalidValue;
  long mx = 0;
  for (int i = 0; i < b.count; ++i) mx = max(mx, (long)b.d[i].M * b.d[i].N);
  if (mx == 0) return hipSuccess;
  hipLaunchKernelGGL(csum_kernel, dim3((unsigned)((mx + 255) / 256), b.count), dim3(256), 0, st, b);
  return hipGetLastError();
}

CgemmDesc cdesc(const double2 *A, long lda, const double2 *B, long ldb, double2 *C, long ldc,
                int M, int N, int K) {
  CgemmDesc d{};
  d.A = A; d.B = B; d.C = C;
  d.lda = lda; d.ldb = ldb; d.ldc = ldc;
  d.M = M; d.N = N; d.K = K;
  d.alpha = make_double2(1.0, 0.0);
  d.beta = make_double2(0.0, 0.0);
  return d;
}

hipError_t cexpv(const CexpvBatch &b, hipStream_t st) {
  if (b.count < 1 || b.count > kCexpvMaxBatch) return hipErrorInvalidValue;
  int nmax = 0, n2max = 0, wmax = 1;
  for (int i = 0; i < b.count; ++i) {
    const CexpvDesc &d = b.d[i];
    if (d.n2 < 1 || d.n2 > kCexpMaxN || d.w < 1 || d.w > kCexpMaxW || d.n < 1 || d.J < 0 ||
        d.X == d.Y)
      return hipErrorInvalidValue;
    nmax = max(nmax, d.n);
    n2max = max(n2max, d.n2);
    wmax = max(wmax, d.w);
  }
  const int R = (n2max + kCexpThreads - 1) / kCexpThreads;
  if (R <= 1) return launch_cexpv_w<1>(b, nmax, n2max, wmax, st);
  if (R <= 2) return launch_cexpv_w<2>(b, nmax, n2max, wmax, st);
  if (R <= 4) return launch_cexpv_w<4>(b, nmax, n2max, wmax, st);
  return launch_cexpv_w<8>(b, nmax, n2max, wmax, st);
}

hipError_t rotate_rows(const double2 *X, long ldx, double2 *Y, long ldy, int ncols, int N,
                       const int8_t *xrow, double c, double s, double sign, hipStream_t st) {
  const long tot = (long)N * ncols;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(rotate_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, ldx,
                     Y, ldy, ncols, N, xrow, c, s, sign);
  return hipGetLastError();
}

hipError_t conj_copy(const double2 *X, double2 *Y, long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(conj_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, Y, n);
  return hipGetLastError();
}

hipError_t set_identity(double2 *E, long ld, int n, int off, hipStream_t st) {
  const long tot = (long)n * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(ident_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, E, ld, n,
                     off);
  return hipGetLastError();
}

hipError_t chol_inverse(const SocElimBatch &b, long ld, int n, hipStream_t st) {
  if (n < 1 || n > 1024 || b.n < 1 || b.n > kSocMaxBatch) return hipErrorInvalidValue;
  for (int kb = 0; kb < n; kb += kGjNb) {
    const int nbp = min(kGjNb, n - kb), c0 = kb + nbp;
    hipLaunchKernelGGL(ch_panel_kernel, dim3(b.n), dim3(256), 0, st, b, ld, n, kb);
    hipLaunchKernelGGL(ch_rows_kernel, dim3((n + 63) / 64, b.n), dim3(256), 0, st, b, ld, n, kb);
    if (c0 >= n) continue;
    CgemmBatch g{};
    for (int w = 0; w < b.n; ++w) {
      CgemmDesc d = cdesc(b.E[w] + (long)c0 * ld + kb, ld, b.B[w] + c0, 2L * n,
                          b.E[w] + (long)c0 * ld + c0, ld, n - c0, n, nbp);
      d.Cin = d.C;
      d.ldcin = ld;
      d.alpha = make_double2(-1.0, 0.0);
      d.beta = make_double2(1.0, 0.0);
      g.d[g.count++] = d;
    }
    const hipError_t e = cgemm(g, kOpN, kOpN, st);
    if (e != hipSuccess) return e;
  }
  const int nt = (n + 15) / 16;
  hipLaunchKernelGGL(ch_adjoint_kernel, dim3(nt, nt, b.n), dim3(256), 0, st, b, ld, n);
  return hipGetLastError();
}

hipError_t gj_inverse(const SocElimBatch &b, long ld, int n, hipStream_t st) {
  if (n < 1 || n > 1024 || b.n < 1 || b.n > kSocMaxBatch) return hipErrorInvalidValue;
  for (int kb = 0; kb < n; kb += kGjNb) {
    const int nbp = min(kGjNb, n - kb), c0 = kb + nbp;
    hipLaunchKernelGGL(gj_panel_kernel, dim3(b.n), dim3(kGjThreads), 0, st, b, ld, n, kb);
    hipLaunchKernelGGL(gj_rows_kernel, dim3((2 * n - c0 + 63) / 64, b.n), dim3(256), 0, st, b, ld,
                       n, kb);
    CgemmBatch g{};
    for (int w = 0; w < b.n; ++w) {
      CgemmDesc d = cdesc(b.E[w] + kb, ld, b.B[w] + c0, 2L * n, b.E[w] + c0, ld, n, 2 * n - c0,
                          nbp);
      d.Cin = b.E[w] + c0;
      d.ldcin = ld;
      d.alpha = make_double2(-1.0, 0.0);
      d.beta = make_double2(1.0, 0.0);
      g.d[g.count++] = d;
    }
    const hipError_t e = cgemm(g, kOpN, kOpN, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gj_gather_kernel, dim3(n, b.n), dim3(256), 0, st, b, ld, n);
  return hipGetLastError();
}

namespace {
// one decision workgroup per walker of the batch (all with the same kk)
template <class F>
hipError_t launch_decide(F kernel, const SocDecideArgs *a, int nb, size_t lds, hipStream_t st,
                         const hipError_t &attr) {
  if (nb < 1 || nb > kSocMaxBatch) return hipErrorInvalidValue;
  if (attr != hipSuccess) return attr;
  SocDecideBatch B{};
  for (int i = 0; i < nb; ++i) B.a[i] = a[i];
  hipLaunchKernelGGL(kernel, dim3(nb), dim3(kDecThreads), lds, st, B);
  return hipGetLastError();
}
}  // namespace

hipError_t block_decide(const SocDecideArgs *a, int nb, hipStream_t st) {
  if (a[0].kk < 1 || a[0].kk > kSocMaxK) return hipErrorInvalidValue;
  const int n = 2 * a[0].kk;
  const size_t lds = sizeof(double2) * (size_t)n * (2 * n + 1);
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)soc_block_decide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(sizeof(double2) * 64 * 129));
  return launch_decide(soc_block_decide_kernel, a, nb, lds, st, attr);
}

hipError_t phase_rows(const double2 *X, long ldx, double2 *Y, long ldy, int ncols, int N,
                      const int8_t *xrow, double c, double s, double sign, hipStream_t st) {
  const long tot = (long)N * ncols;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(phase_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, ldx,
                     Y, ldy, ncols, N, xrow, c, s, sign);
  return hipGetLastError();
}

hipError_t decide1(const SocDecideArgs *a, int nb, hipStream_t st) {
  if (a[0].kk < 1 || a[0].kk > 2 * kSocMaxK) return hipErrorInvalidValue;
  const int n = a[0].kk;
  const size_t lds = sizeof(double2) * (size_t)n * (n + 1);
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)cplx_decide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(sizeof(double2) * 64 * 65));
  return launch_decide(cplx_decide_kernel, a, nb, lds, st, attr);
}

hipError_t block_decide1(const SocDecideArgs *a, int nb, hipStream_t st) {
  if (a[0].kk < 1 || a[0].kk > 2 * kSocMaxK) return hipErrorInvalidValue;
  const int n = a[0].kk;
  const size_t lds = sizeof(double2) * (size_t)n * (2 * n + 1);
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)cplx_block_decide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(sizeof(double2) * 64 * 129));
  return launch_decide(cplx_block_decide_kernel, a, nb, lds, st, attr);
}

hipError_t rotate_accepted(const SocDecideArgs *a, int nb, int w, hipStream_t st) {
  if (nb < 1 || nb > kSocMaxBatch || a[0].kk < 1 || a[0].kk > 2 * kSocMaxK) return hipErrorInvalidValue;
  SocDecideBatch B{};
  for (int i = 0; i < nb; ++i) B.a[i] = a[i];
  hipLaunchKernelGGL(rotate_accepted_kernel, dim3((a[0].ne + 255) / 256, a[0].kk, nb), dim3(256),
                     0, st, B, w);
  return hipGetLastError();
}

hipError_t decide(const SocDecideArgs *a, int nb, hipStream_t st) {
  if (a[0].kk < 1 || a[0].kk > kSocMaxK) return hipErrorInvalidValue;
  const int n = 2 * a[0].kk;
  const size_t lds = sizeof(double2) * (size_t)n * (n + 1);
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)soc_decide_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(sizeof(double2) * 64 * 65));
  return launch_decide(soc_decide_kernel, a, nb, lds, st, attr);
}

}  // namespace soc
}  // namespace pq
