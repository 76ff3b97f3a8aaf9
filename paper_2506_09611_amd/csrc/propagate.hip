// Propagation by the sparse hopping matrix: Y = e^{a H0} X for the N x n
// row-major walker matrices of a slice step (Eq. (9)), a = -dtau (K) or
// +dtau (K^{-1}), with the slice's field diagonal applied before or after.
//
// H0 of a lattice model has a few nonzeros per row (four on the square
// lattice), so e^{a H0} X is formed from its Taylor series in Horner form,
//   Z <- X;  Z <- X + (a H0 Z) / j  for j = J, ..., 1,
// with J fixed at set-up so that the first dropped term is below 2^-60 of the
// kept ones (||a H0||_1 <= 1 is required).  This replaces the dense K X
// product (2 N^2 n flops) by 2 J nnz n flops, and keeps the propagator exact
// to rounding.
//
// One workgroup of 512 threads owns two columns of one product for all N
// rows: both Horner iterates live in LDS (2 x N x 2 doubles), the thread's
// rows of X and of H0 (ELL: WD entries per row, zero-padded) in registers.
// Each Horner step reads the neighbour rows' two columns from LDS (16 bytes a
// row) and ends on a barrier.  Global memory is read once (X) and written
// once (Y).
#include "engine.hpp"

namespace pq {
namespace {

constexpr int kExpThreads = 512;

template <int R, int WD>
__global__ __launch_bounds__(kExpThreads) void expv_kernel(ExpvBatch B) {
  const ExpvDesc &d = B.d[blockIdx.y];
  // XCD-aware: consecutive workgroup ids go round-robin to the 8 XCDs, so
  // XCD x takes the contiguous range [x per, (x + 1) per) of column pairs;
  // the pairs that share a cache line of X and Y then share one L2
  const int per = gridDim.x >> 3;   // the grid is a multiple of 8
  const int N = d.N, n = d.n, c0 = 2 * ((int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3));
  if (c0 >= n) return;
  const bool two = c0 + 1 < n;
  extern __shared__ double zs[];
  double *Za = zs, *Zb = zs + 2 * (long)N;
  const int t = threadIdx.x;
  double x0[R], x1[R];
  int idx[R][WD];
  double val[R][WD];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = t + kExpThreads * i;
    const bool in = r < N;
    const int rr = in ? r : 0;
#pragma unroll
    for (int e = 0; e < WD; ++e) {
      idx[i][e] = in ? d.idx[(long)rr * d.w + min(e, d.w - 1)] : 0;
      val[i][e] = (in && e < d.w) ? d.a * d.val[(long)rr * d.w + e] : 0.0;
    }
    double v0 = 0.0, v1 = 0.0;
    if (in) {
      v0 = d.X[(long)r * d.ldx + c0];
      v1 = two ? d.X[(long)r * d.ldx + c0 + 1] : 0.0;
      if (d.field && d.pre) {
        const double sc = d.field[r] > 0 ? d.pos : d.neg;
        v0 *= sc;
        v1 *= sc;
      }
      Za[2 * r] = v0;
      Za[2 * r + 1] = v1;
    }
    x0[i] = v0;
    x1[i] = v1;
  }
  __syncthreads();
  for (int j = d.J; j >= 1; --j) {
    const double inv = 1.0 / (double)j;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = t + kExpThreads * i;
      if (r < N) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int e = 0; e < WD; ++e) {
          const double2 z = *reinterpret_cast<const double2 *>(Za + 2 * idx[i][e]);
          s0 = fma(val[i][e], z.x, s0);
          s1 = fma(val[i][e], z.y, s1);
        }
        double2 o;
        o.x = fma(s0, inv, x0[i]);
        o.y = fma(s1, inv, x1[i]);
        *reinterpret_cast<double2 *>(Zb + 2 * r) = o;
      }
    }
    __syncthreads();
    double *tmp = Za;
    Za = Zb;
    Zb = tmp;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = t + kExpThreads * i;
    if (r < N) {
      double y0 = Za[2 * r], y1 = Za[2 * r + 1];
      if (d.field && !d.pre) {
        const double sc = d.field[r] > 0 ? d.pos : d.neg;
        y0 *= sc;
        y1 *= sc;
      }
      d.Y[(long)r * d.ldy + c0] = y0;
      if (two) d.Y[(long)r * d.ldy + c0 + 1] = y1;
    }
  }
}

template <int R, int WD>
hipError_t launch_expv(const ExpvBatch &b, int nmax, int Nmax, hipStream_t st) {
  const size_t lds = sizeof(double) * 4 * (size_t)Nmax;
  if (lds > 64 * 1024) {
    static const hipError_t attr = hipFuncSetAttribute(
        (const void *)expv_kernel<R, WD>, hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)(sizeof(double) * 4 * kExpMaxN));
    if (attr != hipSuccess) return attr;
  }
  const int pairs = (nmax + 1) / 2;
  hipLaunchKernelGGL((expv_kernel<R, WD>), dim3((pairs + 7) / 8 * 8, b.count), dim3(kExpThreads),
                     lds, st, b);
  return hipGetLastError();
}

template <int R>
hipError_t launch_expv_w(const ExpvBatch &b, int nmax, int Nmax, int wmax, hipStream_t st) {
  if (wmax <= 4) return launch_expv<R, 4>(b, nmax, Nmax, st);
  if (wmax <= 8) return launch_expv<R, 8>(b, nmax, Nmax, st);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t expv(const ExpvBatch &b, hipStream_t st) {
  if (b.count < 1 || b.count > kExpvMaxBatch) return hipErrorInvalidValue;
  int nmax = 0, Nmax = 0, wmax = 1;
  for (int i = 0; i < b.count; ++i) {
    const ExpvDesc &d = b.d[i];
    if (d.N < 1 || d.N > kExpMaxN || d.w < 1 || d.w > kExpMaxW || d.n < 1 || d.J < 0)
      return hipErrorInvalidValue;
    nmax = max(nmax, d.n);
    Nmax = max(Nmax, d.N);
    wmax = max(wmax, d.w);
  }
  const int R = (Nmax + kExpThreads - 1) / kExpThreads;
  if (R <= 1) return launch_expv_w<1>(b, nmax, Nmax, wmax, st);
  if (R <= 2) return launch_expv_w<2>(b, nmax, Nmax, wmax, st);
  if (R <= 4) return launch_expv_w<4>(b, nmax, Nmax, wmax, st);
  if (R <= 8) return launch_expv_w<8>(b, nmax, Nmax, wmax, st);
  return hipErrorInvalidValue;
}

}  // namespace pq
