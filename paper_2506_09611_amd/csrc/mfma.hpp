// FP64 MFMA building blocks for gfx950 (v_mfma_f64_16x16x4f64).
//
// Operand layout of one 16x16x4 step: lane l supplies A(l % 16, k0 + l / 16)
// and B(k0 + l / 16, l % 16).  Accumulator layout (measured on the device):
// lane l, register j holds D(l / 16 + 4 j, l % 16).
#pragma once
#include <hip/hip_runtime.h>

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

namespace pq {

// One 16x16x4 MFMA step in float64 or float32.  Operand layout as above for
// both; the accumulator layouts differ (both measured on the device):
//   f64 (v_mfma_f64_16x16x4f64): lane l, register j holds D(l / 16 + 4 j, l % 16)
//   f32 (v_mfma_f32_16x16x4f32): lane l, register j holds D(4 (l / 16) + j, l % 16)
template <class R>
struct Mma;
template <>
struct Mma<double> {
  typedef dbl4 acc;
  __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};
template <>
struct Mma<float> {
  typedef flt4 acc;
  __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};

// One 16x16 tile: A (16 x K) B (K x 16), K a multiple of 4, with
// A(i, k) = Am[i * lda + k] and B(k, j) = Bm[k * ldb + j] (TB: Bm[j * ldb + k]).
template <bool TB>
__device__ __forceinline__ dbl4 mma16(const double *Am, int lda, const double *Bm, int ldb,
                                      int K, int lane) {
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const int i = lane & 15, kq = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + kq;
    const double a = Am[i * lda + k];
    const double b = TB ? Bm[i * ldb + k] : Bm[k * ldb + i];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// acc (this wave's 32x32 quadrant (wm, wn) of a 64x64 result) += A (64 x K)
// B (K x 64) with A, B in LDS; TB: B(k, j) = Bm[j * ldb + k].  Operand
// entries with k >= K read as zero, so K need not be a multiple of 4.
// Quadrants whose rows are >= mrows or columns >= ncols are skipped.
template <bool TB>
__device__ __forceinline__ void lds_mma(dbl4 (&acc)[2][2], const double *A, int lda,
                                        const double *B, int ldb, int K, int mrows, int ncols,
                                        int wm, int wn, int lane) {
  if (wm * 32 >= mrows || wn * 32 >= ncols) return;
  const int i0 = wm * 32 + (lane & 15);
  const int j0 = wn * 32 + (lane & 15);
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    const bool kv = kk < K;
    const double a0 = kv ? A[i0 * lda + kk] : 0.0;
    const double a1 = kv ? A[(i0 + 16) * lda + kk] : 0.0;
    double b0, b1;
    if (!TB) {
      b0 = kv ? B[kk * ldb + j0] : 0.0;
      b1 = kv ? B[kk * ldb + j0 + 16] : 0.0;
    } else {
      b0 = kv ? B[j0 * ldb + kk] : 0.0;
      b1 = kv ? B[(j0 + 16) * ldb + kk] : 0.0;
    }
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// (row, col) of accumulator element [mi][ni][j] of wave (wm, wn) in a 64x64 tile
__device__ __forceinline__ int acc_row(int wm, int mi, int lane, int j) {
  return wm * 32 + mi * 16 + (lane >> 4) + 4 * j;
}
__device__ __forceinline__ int acc_col(int wn, int ni, int lane) {
  return wn * 32 + ni * 16 + (lane & 15);
}

}  // namespace pq
