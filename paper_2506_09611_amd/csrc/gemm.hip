// FP64 GEMM on gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// One 256-thread workgroup computes a 64x32 tile of C; its four waves each
// own a 32x16 block held as 2x1 MFMA accumulators (4 doubles per lane per
// 16x16 block).  A and B tiles of depth 16 are staged through two LDS
// buffers: the next depth slice is loaded into registers while the current
// one is multiplied, then stored to the other buffer, one barrier per slice.  The same kernel serves the B-matrix propagation (diagonal
// field scalings fused into the operand load or the epilogue), the Taylor
// series of e^{-dtau H0}, the Gram and product matrices of the
// stabilisation, the split-K panel products of the delayed and block
// updates, the rank-n_A flush of T and the Green's function assembly.
//
// MFMA f64 16x16x4 operand layout (lane l of 64):
//   A (16x4):  A[l % 16][l / 16]        B (4x16): B[l / 16][l % 16]
//   D (16x16): lane l, register j holds D[l / 16 + 4 * j][l % 16]
#include "engine.hpp"

namespace pq {

namespace {
// Tile shape chosen by measurement on MI355X at the propagation shape
// (4 x [1600 x 1600] x [1600 x 800]): 64 x 32 tiles of 4 waves (32 x 16
// each) reached 40-42 TFLOP/s, against 28 for 64 x 64 single-buffered,
// 37 for 64 x 64 double-buffered, 27 for 128 x 64 and 44 for the vendor
// library without the fused scaling.
constexpr int BM = 64, BN = 32, WM = 32, WN = 16, BK = 16;
constexpr int PA = BM + 4, PB = BN + 4;   // padded LDS rows
constexpr int MI = WM / 16, NI = WN / 16, WGM = BM / WM;
constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmBatch batch, int nsplit) {
  const int bz = blockIdx.z / nsplit;
  const int split = blockIdx.z % nsplit;
  if (bz >= batch.count) return;
  const GemmDesc &g = batch.d[bz];
  const int M = g.M, N = g.N;
  int K = g.K;
  if (g.Kdev) K = min(K, *g.Kdev);
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (m0 >= M || n0 >= N) return;
  int kbeg = 0, kend = K;
  if (g.ksplit > 0) {
    kbeg = split * g.ksplit;
    kend = min(K, kbeg + g.ksplit);
    if (kbeg >= K) return;   // beyond this product's depth: it has fewer partials
  } else if (split > 0) {
    return;
  }
  if (g.ksplit <= 0 && K <= 0 && g.Kdev && g.beta == 1.0 && g.Cin == g.C && !g.addI) return;

  // two depth slices in flight: one being multiplied, the next being stored
  __shared__ double As[2][BK][PA];
  __shared__ double Bs[2][BK][PB];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  const double *A = g.A, *B = g.B;
  const long lda = g.lda, ldb = g.ldb;

  // Loads are unconditional (clamped in-range addresses) and issue together;
  // the depth tail is zeroed and the field scaling applied when the slice is
  // stored to LDS, after the current slice's products, so that no load is
  // waited for early.  Rows and columns past M and N only reach outputs that
  // are not stored.
  const int8_t *ksf = g.ks_field;
  const double ks_pos = g.ks_pos, ks_neg = g.ks_neg;
  double ra[NA], rb[NB];
  int8_t fb[NB];
  int kload = 0;   // depth offset of the slice in ra / rb
  auto load = [&](int k0) {
    kload = k0;
#pragma unroll
    for (int p = 0; p < NA; ++p) {
      int mm, kk;
      if (!TA) { kk = t % BK; mm = t / BK + (256 / BK) * p; }
      else     { mm = t % BM; kk = t / BM + (256 / BM) * p; }
      const int gi = min(m0 + mm, M - 1), gk = min(k0 + kk, kend - 1);
      ra[p] = TA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
    }
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      int nn, kk;
      if (!TB) { nn = t % BN; kk = t / BN + (256 / BN) * p; }
      else     { kk = t % BK; nn = t / BK + (256 / BK) * p; }
      const int gj = min(n0 + nn, N - 1), gk = min(k0 + kk, kend - 1);
      rb[p] = TB ? B[(long)gj * ldb + gk] : B[(long)gk * ldb + gj];
      fb[p] = ksf ? ksf[gk] : (int8_t)1;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < NA; ++p) {
      int mm, kk;
      if (!TA) { kk = t % BK; mm = t / BK + (256 / BK) * p; }
      else     { mm = t % BM; kk = t / BM + (256 / BM) * p; }
      As[buf][kk][mm] = ra[p] * (kload + kk < kend ? 1.0 : 0.0);
    }
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      int nn, kk;
      if (!TB) { nn = t % BN; kk = t / BN + (256 / BN) * p; }
      else     { kk = t % BK; nn = t / BK + (256 / BK) * p; }
      Bs[buf][kk][nn] = rb[p] * (fb[p] > 0 ? ks_pos : ks_neg);
    }
  };

  // fields of the output rows (epilogue scaling), loaded before the depth loop
  const int8_t *rsf = g.rs_field;
  int rf[MI][4];   // one register each: packing bytes would wait for every load
  if (rsf) {
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        rf[mi][j] = rsf[min(m0 + wm * WM + mi * 16 + (lane >> 4) + 4 * j, M - 1)];
  } else {
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int j = 0; j < 4; ++j) rf[mi][j] = 1;
  }

  // fields of the output columns (epilogue column scaling)
  const int8_t *csf = g.cs_field;
  int cf[NI];
#pragma unroll
  for (int ni = 0; ni < NI; ++ni)
    cf[ni] = csf ? csf[min(n0 + wn * WN + ni * 16 + (lane & 15), N - 1)] : 1;

  dbl4 acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double a[MI], b[NI];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = As[buf][kk][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kk][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  double *C = g.C;
  if (g.ksplit > 0) C += (long)split * g.csplit;
  const bool split_out = g.ksplit > 0;
  const double rs_pos = g.rs_pos, rs_neg = g.rs_neg, alpha = g.alpha, beta = g.beta;
  // the epilogue's Cin operands are loaded together first
  double cin[MI][NI][4];
  const bool use_cin = !split_out && beta != 0.0;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = min(m0 + wm * WM + mi * 16 + (lane >> 4) + 4 * j, M - 1);
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        const int col = min(n0 + wn * WN + ni * 16 + (lane & 15), N - 1);
        cin[mi][ni][j] = use_cin ? g.Cin[(long)row * g.ldcin + col] : 0.0;
      }
    }
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = m0 + wm * WM + mi * 16 + (lane >> 4) + 4 * j;
        const int col = n0 + wn * WN + ni * 16 + (lane & 15);
        if (row < M && col < N) {
          double v = alpha * acc[mi][ni][j];
          if (rsf) v *= (rf[mi][j] > 0) ? rs_pos : rs_neg;
          if (csf) v *= (cf[ni] > 0) ? g.cs_pos : g.cs_neg;
          if (!split_out) {
            if (use_cin) v += beta * cin[mi][ni][j];
            if (g.addI && row == col) v += 1.0;
          }
          C[(long)row * g.ldc + col] = v;
        }
      }
}
}  // namespace

GemmDesc gemm_desc(const double *A, long lda, const double *B, long ldb, double *C, long ldc,
                   int M, int N, int K, double alpha, double beta, const double *Cin,
                   long ldcin) {
  GemmDesc d{};
  d.A = A; d.B = B; d.C = C; d.Cin = Cin ? Cin : C;
  d.lda = lda; d.ldb = ldb; d.ldc = ldc; d.ldcin = Cin ? ldcin : ldc;
  d.M = M; d.N = N; d.K = K;
  d.alpha = alpha; d.beta = beta;
  d.rs_pos = d.rs_neg = d.ks_pos = d.ks_neg = d.cs_pos = d.cs_neg = 1.0;
  return d;
}

hipError_t gemm(const GemmBatch &b, bool transA, bool transB, hipStream_t st) {
  if (b.count <= 0) return hipSuccess;
  int mt = 0, nt = 0, ns = 1;
  for (int i = 0; i < b.count; ++i) {
    mt = max(mt, (b.d[i].M + BM - 1) / BM);
    nt = max(nt, (b.d[i].N + BN - 1) / BN);
    if (b.d[i].ksplit > 0) ns = max(ns, (b.d[i].K + b.d[i].ksplit - 1) / b.d[i].ksplit);
  }
  if (mt == 0 || nt == 0) return hipSuccess;
  dim3 grid(nt, mt, b.count * ns);
  if (!transA && !transB) hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, dim3(256), 0, st, b, ns);
  else if (transA && !transB) hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, dim3(256), 0, st, b, ns);
  else if (!transA && transB) hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, dim3(256), 0, st, b, ns);
  else hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, dim3(256), 0, st, b, ns);
  return hipGetLastError();
}

}  // namespace pq
