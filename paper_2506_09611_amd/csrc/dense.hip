// Dense FP64 linear algebra for the stabilisation step (Sec. II B): the
// inverse T = (U_L U_R)^{-1} and the re-orthonormalisation of U_R / U_L.
//
// Both run one blocked elimination engine over an augmented row-major
// matrix E = [M | I] (n x 2n), panel width kNB = 32:
//   * Gauss-Jordan with partial pivoting (T): a single workgroup factors the
//     panel E[kb:n, kb:kb+nb] with row pivoting on a private register copy,
//     returning the pivots and Z = inverse of the pivoted diagonal block;
//     the pivots are applied to whole rows, the block row is replaced by
//     Z * (block row), and every other row gets a rank-nb GEMM update.
//     The right half ends as M^{-1}.
//   * Cholesky-normalised forward elimination (QR): the diagonal block's
//     Cholesky factor C gives Z1 = C^{-1} for the block row and
//     Z2 = Z1^T Z1 for the rank-nb update of the rows below.  E = [S | I]
//     with S = A^T A ends as [R | R^{-T}], so Q = A R^{-1} (CholQR).
#include "engine.hpp"

namespace pq {

namespace {

constexpr int kPanelThreads = 1024;
// rows per row group (template): panels up to 32 * MAXQ rows

struct PanelArgs {
  ElimSpin s[2];
  int nspin;
  int kb;
  unsigned long long *stats;
};

// LU with partial pivoting of the panel E[kb:n, kb:kb+nb] (register copy),
// then Z = U11^{-1} L11^{-1}.  Thread (rg, c): column c, rows rg + 32 q.
template <int kPanelMaxQ>
__global__ __launch_bounds__(kPanelThreads) void gj_panel_kernel(PanelArgs a) {
  const ElimSpin &S = a.s[blockIdx.x];
  const int kb = a.kb;
  const int nb = min(kNB, S.n - kb);
  const int R = S.n - kb;
  const int t = threadIdx.x, c = t & 31, rg = t >> 5;
  const int lane = t & 63;
  double v[kPanelMaxQ];
#pragma unroll
  for (int q = 0; q < kPanelMaxQ; ++q) {
    const int r = rg + 32 * q;
    v[q] = (r < R && c < nb) ? S.E[(long)(kb + r) * S.ld + kb + c] : 0.0;
  }
  __shared__ double red_v[32];
  __shared__ int red_i[32];
  __shared__ double rowj[32], rowp[32];
  __shared__ int s_p;
  __shared__ double LU[32][33];
  __shared__ double Li[32][33], Ui[32][33];

  for (int j = 0; j < nb; ++j) {
    if (c == j) {
      double best = -1.0;
      int bi = -1;
#pragma unroll
      for (int q = 0; q < kPanelMaxQ; ++q) {
        const int r = rg + 32 * q;
        if (r >= j && r < R) {
          const double av = fabs(v[q]);
          if (av > best) { best = av; bi = r; }
        }
      }
      red_v[rg] = best;
      red_i[rg] = bi;
    }
    __syncthreads();
    // argmax over the 32 row groups in wave 0 (ties: smallest row)
    if (t < 64) {
      double bv = (t < 32 && red_i[t] >= 0) ? red_v[t] : -1.0;
      int bix = (t < 32 && red_i[t] >= 0) ? red_i[t] : 0x7fffffff;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bix, o, 64);
        const bool take = (ov > bv) || (ov == bv && oi < bix);
        bv = take ? ov : bv;
        bix = take ? oi : bix;
      }
      if (t == 0) {
        int bi = bix;
        if (!(bv > 0.0) || bi == 0x7fffffff) {
          a.stats[kStError] |= kErrSingular;
          bi = j;
        }
        s_p = bi;
        S.piv[j] = kb + bi;
      }
    }
    __syncthreads();
    const int p = s_p;
    // swap local rows j (row group j, q = 0) and p (row group p % 32, q = p / 32)
    if (rg == j) rowj[c] = v[0];
    if (rg == (p & 31)) {
#pragma unroll
      for (int q = 0; q < kPanelMaxQ; ++q)
        if (q == (p >> 5)) rowp[c] = v[q];
    }
    __syncthreads();
    if (p != j) {
      if (rg == (p & 31)) {
#pragma unroll
        for (int q = 0; q < kPanelMaxQ; ++q)
          if (q == (p >> 5)) v[q] = rowj[c];
      }
      if (rg == j) v[0] = rowp[c];
    }
    // pivot row is now rowp (old row p)
    const double d = rowp[j];
    const double pr = rowp[c];
#pragma unroll
    for (int q = 0; q < kPanelMaxQ; ++q) {
      const int r = rg + 32 * q;
      const double arj = __shfl(v[q], (lane & 32) | j, 64);
      if (r > j && r < R) {
        const double l = (d != 0.0) ? arj / d : 0.0;
        if (c > j) v[q] -= l * pr;
        else if (c == j) v[q] = l;
      }
    }
    __syncthreads();
  }
  // L11 (unit lower) and U11 sit in rows 0..nb-1 = row groups 0..nb-1, q = 0.
  if (rg < 32) LU[rg][c] = (rg < nb && c < nb) ? v[0] : (rg == c ? 1.0 : 0.0);
  __syncthreads();
  if (t < 32) {
    const int col = t;
    // column col of L^{-1} (unit lower) by forward substitution
    double x[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < 32; ++m)
        if (m < i) s -= LU[i][m] * x[m];
      x[i] = s;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) Li[i][col] = x[i];
  } else if (t >= 64 && t < 96) {
    const int col = t - 64;
    // column col of U^{-1} by back substitution
    double x[32];
#pragma unroll
    for (int ii = 0; ii < 32; ++ii) {
      const int i = 31 - ii;
      double s = (i == col) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < 32; ++m)
        if (m > i) s -= LU[i][m] * x[m];
      const double dd = LU[i][i];
      x[i] = (dd != 0.0) ? s / dd : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) Ui[i][col] = x[i];
  }
  __syncthreads();
  {
    const int i = t >> 5, cc = t & 31;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 32; ++m) s += Ui[i][m] * Li[m][cc];
    if (i < nb && cc < nb) {
      S.Z[i * kNB + cc] = s;
      S.Z[kNB * kNB + i * kNB + cc] = s;
    }
  }
}

// Cholesky of the nb x nb diagonal block (current Schur complement), then
// Z1 = C^{-1} (lower) and Z2 = Z1^T Z1.
__global__ __launch_bounds__(kPanelThreads) void chol_panel_kernel(PanelArgs a) {
  const ElimSpin &S = a.s[blockIdx.x];
  const int kb = a.kb;
  const int nb = min(kNB, S.n - kb);
  const int t = threadIdx.x, i = t >> 5, j = t & 31;
  __shared__ double A[32][33];
  __shared__ double Ci[32][33];
  __shared__ int bad;
  if (t == 0) bad = 0;
  A[i][j] = (i < nb && j < nb) ? S.E[(long)(kb + i) * S.ld + kb + j] : (i == j ? 1.0 : 0.0);
  __syncthreads();
  for (int k = 0; k < 32; ++k) {
    if (t == 0) {
      const double d = A[k][k];
      if (!(d > 0.0)) { bad = 1; A[k][k] = 1.0; }
      else A[k][k] = sqrt(d);
    }
    __syncthreads();
    if (j == k && i > k) A[i][k] /= A[k][k];
    __syncthreads();
    if (i > k && j > k && j <= i) A[i][j] -= A[i][k] * A[j][k];
    __syncthreads();
  }
  if (t == 0 && bad) a.stats[kStError] |= kErrSingular;
  if (t < 32) {
    const int col = t;
    double x[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      double s = (r == col) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < 32; ++m)
        if (m < r) s -= A[r][m] * x[m];
      x[r] = s / A[r][r];
    }
#pragma unroll
    for (int r = 0; r < 32; ++r) Ci[r][col] = x[r];
  }
  __syncthreads();
  double z2 = 0.0;
#pragma unroll
  for (int m = 0; m < 32; ++m) z2 += Ci[m][i] * Ci[m][j];
  if (i < nb && j < nb) {
    S.Z[i * kNB + j] = (j <= i) ? Ci[i][j] : 0.0;
    S.Z[kNB * kNB + i * kNB + j] = z2;
  }
}

struct ColArgs {
  ElimSpin s[2];
  int kb;
  int c0[2], c1[2];   // column range per spin
};

// Apply the panel's row interchanges to columns [c0, c1).
__global__ void swap_rows_kernel(ColArgs a) {
  const ElimSpin &S = a.s[blockIdx.y];
  const int col = a.c0[blockIdx.y] + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= a.c1[blockIdx.y]) return;
  const int nb = min(kNB, S.n - a.kb);
  for (int j = 0; j < nb; ++j) {
    const int p = S.piv[j];
    const int r = a.kb + j;
    if (p != r) {
      const double x = S.E[(long)r * S.ld + col];
      S.E[(long)r * S.ld + col] = S.E[(long)p * S.ld + col];
      S.E[(long)p * S.ld + col] = x;
    }
  }
}

// Block row: E[b, c] <- Z1 E[b, c]; optionally R2[:, c] <- Z2 E_old[b, c].
__global__ void block_row_kernel(ColArgs a, int with_r2) {
  const ElimSpin &S = a.s[blockIdx.y];
  const int nb = min(kNB, S.n - a.kb);
  __shared__ double z1[kNB * kNB], z2[kNB * kNB];
  for (int e = threadIdx.x; e < kNB * kNB; e += blockDim.x) {
    z1[e] = S.Z[e];
    z2[e] = S.Z[kNB * kNB + e];
  }
  __syncthreads();
  const int col = a.c0[blockIdx.y] + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= a.c1[blockIdx.y]) return;
  double x[kNB];
#pragma unroll
  for (int m = 0; m < kNB; ++m) x[m] = (m < nb) ? S.E[(long)(a.kb + m) * S.ld + col] : 0.0;
#pragma unroll
  for (int i = 0; i < kNB; ++i) {
    if (i < nb) {
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int m = 0; m < kNB; ++m) {
        s1 += z1[i * kNB + m] * x[m];
        s2 += z2[i * kNB + m] * x[m];
      }
      S.E[(long)(a.kb + i) * S.ld + col] = s1;
      if (with_r2) S.R2[(long)i * S.w + col] = s2;
    }
  }
}

__global__ void set_identity_kernel(double *E0, double *E1, long ld, int n, int col0) {
  double *E = blockIdx.z ? E1 : E0;
  const int r = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) E[(long)r * ld + col0 + c] = (r == c) ? 1.0 : 0.0;
}

__global__ void copy_kernel(const double *s0, const double *s1, long lds, double *d0, double *d1,
                            long ldd, int rows, int cols) {
  const double *s = blockIdx.z ? s1 : s0;
  double *d = blockIdx.z ? d1 : d0;
  const int r = blockIdx.y;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x)
    d[(long)r * ldd + c] = s[(long)r * lds + c];
}

__global__ void init_fields_kernel(int8_t *f, int M, int N, uint64_t k0, uint64_t k1) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  const int li = (int)(e / N), i = (int)(e % N);
  const double u = philox_uniform(k0, k1, 0, (uint64_t)li, (uint64_t)i, kPurposeInit);
  f[e] = (u < 0.5) ? (int8_t)1 : (int8_t)-1;
}

hipError_t run_elimination(const ElimSpin *s, int nspin, unsigned long long *stats,
                           hipStream_t st, bool pivoted) {
  const int n = s[0].n;
  for (int i = 1; i < nspin; ++i)
    if (s[i].n != n) return hipErrorInvalidValue;
  for (int kb = 0; kb < n; kb += kNB) {
    const int nb = min(kNB, n - kb);
    PanelArgs pa{};
    for (int i = 0; i < nspin; ++i) pa.s[i] = s[i];
    pa.nspin = nspin;
    pa.kb = kb;
    pa.stats = stats;
    ColArgs ca{};
    for (int i = 0; i < nspin; ++i) ca.s[i] = s[i];
    ca.kb = kb;
    if (pivoted) {
      const int rows = n - kb;
      if (rows <= 32 * 8)
        hipLaunchKernelGGL(gj_panel_kernel<8>, dim3(nspin), dim3(kPanelThreads), 0, st, pa);
      else if (rows <= 32 * 16)
        hipLaunchKernelGGL(gj_panel_kernel<16>, dim3(nspin), dim3(kPanelThreads), 0, st, pa);
      else if (rows <= 32 * 32)
        hipLaunchKernelGGL(gj_panel_kernel<32>, dim3(nspin), dim3(kPanelThreads), 0, st, pa);
      else
        hipLaunchKernelGGL(gj_panel_kernel<64>, dim3(nspin), dim3(kPanelThreads), 0, st, pa);
      // interchange whole rows: panel and everything right of it
      int maxc = 0;
      for (int i = 0; i < nspin; ++i) {
        ca.c0[i] = kb;
        ca.c1[i] = s[i].w;
        maxc = max(maxc, ca.c1[i] - ca.c0[i]);
      }
      hipLaunchKernelGGL(swap_rows_kernel, dim3((maxc + 255) / 256, nspin), dim3(256), 0, st, ca);
    } else {
      hipLaunchKernelGGL(chol_panel_kernel, dim3(nspin), dim3(kPanelThreads), 0, st, pa);
    }
    // columns carrying nonzeros of the block row: without pivoting, the
    // right half is lower triangular so far; with pivoting, everything.
    int maxc = 0;
    for (int i = 0; i < nspin; ++i) {
      ca.c0[i] = kb + nb;
      ca.c1[i] = pivoted ? s[i].w : min(s[i].w, n + kb + nb);
      maxc = max(maxc, ca.c1[i] - ca.c0[i]);
    }
    if (maxc > 0)
      hipLaunchKernelGGL(block_row_kernel, dim3((maxc + 127) / 128, nspin), dim3(128), 0, st, ca,
                         pivoted ? 0 : 1);
    GemmBatch gb{};
    gb.count = 0;
    for (int i = 0; i < nspin; ++i) {
      const ElimSpin &S = s[i];
      const int c0 = kb + nb, c1 = ca.c1[i];
      if (c1 <= c0) continue;
      const double *R2 = pivoted ? S.E + (long)kb * S.ld : S.R2;
      const long ldr = pivoted ? S.ld : S.w;
      // rows below the block
      if (kb + nb < n) {
        gb.d[gb.count++] = gemm_desc(S.E + (long)(kb + nb) * S.ld + kb, S.ld, R2 + c0, ldr,
                                     S.E + (long)(kb + nb) * S.ld + c0, S.ld, n - kb - nb,
                                     c1 - c0, nb, -1.0, 1.0);
      }
      // rows above the block (Gauss-Jordan only)
      if (pivoted && kb > 0) {
        gb.d[gb.count++] = gemm_desc(S.E + kb, S.ld, R2 + c0, ldr, S.E + c0, S.ld, kb, c1 - c0,
                                     nb, -1.0, 1.0);
      }
    }
    hipError_t e = gemm(gb, false, false, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t gj_invert(const ElimSpin *s, int nspin, unsigned long long *stats, hipStream_t st) {
  return run_elimination(s, nspin, stats, st, true);
}

hipError_t chol_eliminate(const ElimSpin *s, int nspin, unsigned long long *stats,
                          hipStream_t st) {
  return run_elimination(s, nspin, stats, st, false);
}

hipError_t set_identity_block(double *E0, double *E1, long ld, int n, int col0, hipStream_t st) {
  dim3 grid((n + 255) / 256, n, E1 ? 2 : 1);
  hipLaunchKernelGGL(set_identity_kernel, grid, dim3(256), 0, st, E0, E1, ld, n, col0);
  return hipGetLastError();
}

hipError_t copy_matrix(const double *src0, const double *src1, long lds, double *dst0,
                       double *dst1, long ldd, int rows, int cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid(min((cols + 255) / 256, 8), rows, dst1 ? 2 : 1);
  hipLaunchKernelGGL(copy_kernel, grid, dim3(256), 0, st, src0, src1, lds, dst0, dst1, ldd, rows,
                     cols);
  return hipGetLastError();
}

hipError_t init_fields(int8_t *fields, int M, int N, uint64_t k0, uint64_t k1, hipStream_t st) {
  const long tot = (long)M * N;
  hipLaunchKernelGGL(init_fields_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     fields, M, N, k0, k1);
  return hipGetLastError();
}

}  // namespace pq
