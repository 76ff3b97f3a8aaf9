// Dense FP64 linear algebra for the stabilisation step (Sec. II B): the
// inverse T = (U_L U_R)^{-1} and the re-orthonormalisation of U_R / U_L.
//
// Both run one blocked elimination over an augmented row-major matrix
// E = [M | I] (n x 2n, n <= 1024), panel width kNB = 32, with two launches
// per panel:
//   * a panel kernel factors the panel's pivot block and returns
//     Z = (pivot block)^{-1} (Gauss-Jordan) or the inverse Cholesky factor;
//   * an update kernel tiles the live columns: it forms the new block rows
//     Z E[block rows, :] on MFMA and subtracts their rank-kNB product from
//     every other row, reading each tile of E once.
// Gauss-Jordan (T = M^{-1}) pivots implicitly: the panel kernel picks, for
// each column, the largest remaining entry among rows not yet used as pivots
// (partial pivoting on the Schur complement), and records the chosen rows;
// no rows are moved.  The new block rows of a pass go to a side buffer
// (the rows are still being read by other workgroups of that pass) and are
// taken from there by the next pass, so each pass updates E in place.  At
// the end the right half holds P M^{-1} for the recorded pivot order P, and
// T is gathered row by row.
// Cholesky-normalised forward elimination (CholQR) on E = [S | I], S SPD:
// the diagonal block's Cholesky factor C gives the block row C^{-1} E_b and
// the update of the rows below with multipliers E[i, panel] C^{-T}.  The
// right half ends as R^{-T} with S = R^T R, collected block row by block
// row in F, so that Q = A R^{-1} = A F^T.
#include "engine.hpp"

namespace pq {

namespace {

struct ElimArgs {
  ElimSpin s[kMaxMats];
  int kb, nb, pass;
};

// Value of v in lane src (src uniform).
__device__ __forceinline__ double lane_value(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// In-place inverse of a lower-triangular kNB x kNB matrix X (LDS, entries
// above the diagonal zero) by doubling: once the diagonal blocks A, C of
// size b hold their inverses, the block B below A becomes -C^{-1} B A^{-1}.
// unit: X has a unit diagonal.  Tm is scratch.  All threads of the block
// take part; every thread must call it.
__device__ void tri_lower_inverse(double (*X)[kNB + 1], double (*Tm)[kNB + 1], bool unit) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int i = t; i < kNB; i += nt) X[i][i] = unit ? 1.0 : 1.0 / X[i][i];
  __syncthreads();
  for (int b = 1; b < kNB; b <<= 1) {
    const int ne = (kNB / (2 * b)) * b * b;
    for (int e = t; e < ne; e += nt) {
      const int q = e / (b * b), i = (e / b) % b, j = e % b, p0 = 2 * b * q;
      double s = 0.0;
      for (int m = j; m < b; ++m) s += X[p0 + b + i][p0 + m] * X[p0 + m][p0 + j];
      Tm[p0 + b + i][p0 + j] = s;
    }
    __syncthreads();
    for (int e = t; e < ne; e += nt) {
      const int q = e / (b * b), i = (e / b) % b, j = e % b, p0 = 2 * b * q;
      double s = 0.0;
      for (int m = 0; m <= i; ++m) s += X[p0 + b + i][p0 + b + m] * Tm[p0 + b + m][p0 + j];
      X[p0 + b + i][p0 + j] = -s;
    }
    __syncthreads();
  }
}

// Gauss-Jordan panel E[:, kb:kb+nb) with implicit partial pivoting.
// Thread t holds rows t and t + 512 of the panel in registers (staged
// through LDS so that the global loads are coalesced).  Per column the
// largest |entry| among the rows not yet used as pivots wins; the key packs
// the magnitude's bits (an IEEE double >= 0 orders like its bit pattern)
// with the row index in the low 11 bits, so ties go to the smaller row and
// the reduction is an integer max.  Each wave's winner writes its row to LDS
// with its key, so one barrier per column suffices.  Columns are taken in
// blocks of 8, the register rows shifted by 8 after each block, so the
// column loop need not be unrolled in full.  No global memory is touched
// inside the column loop.  Outputs: prow[kb + j], slot[row] = kb + j, and
// Z = D^{-1} for the pivot block D (rows in pivot order) from D = L U:
// with U from the elimination, L = D U^{-1} and Z = U^{-1} L^{-1}.
constexpr int kLuThreads = 512;
constexpr int kLuWaves = kLuThreads / 64;
constexpr int kLuChunk = 256;   // rows staged through LDS at a time
constexpr int kLuLoads = kLuChunk * kNB / kLuThreads;   // loads in flight per thread

__device__ __forceinline__ unsigned long long pivot_key(double x, int r) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(x));
  return (b & ~2047ull) | (unsigned long long)(2047 - r);
}

__global__ __launch_bounds__(kLuThreads) void lu_panel_kernel(ElimArgs a) {
  const ElimSpin &S = a.s[blockIdx.x];
  const int kb = a.kb, nb = a.nb, n = S.n;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int rr0 = t, rr1 = t + kLuThreads;
  __shared__ double rowbuf[2][kLuWaves][kNB];
  __shared__ unsigned long long kbuf[2][kLuWaves];
  __shared__ double shm[kLuChunk * (kNB + 1)];
  __shared__ double Ut[kNB][kNB + 1];
  __shared__ int prs[kNB];
  __shared__ int bad;
  double (*stage)[kNB + 1] = reinterpret_cast<double (*)[kNB + 1]>(shm);
  double (*Lm)[kNB + 1] = reinterpret_cast<double (*)[kNB + 1]>(shm);
  double (*Tm)[kNB + 1] = reinterpret_cast<double (*)[kNB + 1]>(shm + kNB * (kNB + 1));
  if (t == 0) bad = 0;
  for (int e = t; e < kNB * kNB; e += kLuThreads) {
    const int i = e / kNB, j = e % kNB;
    Ut[i][j] = (i == j && j >= nb) ? 1.0 : 0.0;
  }
  bool cand0 = rr0 < n && S.slot[rr0] < 0;
  bool cand1 = rr1 < n && S.slot[rr1] < 0;
  double v0[kNB], v1[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) v0[c] = v1[c] = 0.0;
  for (int c0 = 0; c0 < n; c0 += kLuChunk) {
    // all of a chunk's loads in flight together: clamped in-range addresses,
    // the panel's columns past nb zeroed when staged (rows past n are never
    // read back)
    double sv[kLuLoads];
#pragma unroll
    for (int q = 0; q < kLuLoads; ++q) {
      const int e = t + q * kLuThreads;
      const int i = e / kNB, c = e % kNB, row = min(c0 + i, n - 1);
      sv[q] = S.E[(long)row * S.ld + kb + min(c, nb - 1)];
    }
#pragma unroll
    for (int q = 0; q < kLuLoads; ++q) {
      const int e = t + q * kLuThreads;
      const int i = e / kNB, c = e % kNB;
      stage[i][c] = sv[q] * (c < nb ? 1.0 : 0.0);
    }
    __syncthreads();
    const bool in0 = cand0 && rr0 >= c0 && rr0 < c0 + kLuChunk;
    const bool in1 = cand1 && rr1 >= c0 && rr1 < c0 + kLuChunk;
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
      if (in0) v0[c] = stage[rr0 - c0][c];
      if (in1) v1[c] = stage[rr1 - c0][c];
    }
    __syncthreads();
  }
  int pos0 = -1, pos1 = -1;
  for (int jb = 0; jb < nb; jb += 8) {
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int j = jb + jj;
      if (j < nb) {   // uniform
        const int par = jj & 1;
        const unsigned long long k0 = cand0 ? pivot_key(v0[jj], rr0) : 0ull;
        const unsigned long long k1 = cand1 ? pivot_key(v1[jj], rr1) : 0ull;
        unsigned long long key = k0 > k1 ? k0 : k1;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const unsigned long long ok = __shfl_xor(key, o, 64);
          key = ok > key ? ok : key;
        }
        if (key != 0ull) {
          const int rw = 2047 - (int)(key & 2047ull);
          if (rw == rr0) {
#pragma unroll
            for (int c = 0; c < kNB; ++c) rowbuf[par][wave][c] = v0[c];
          } else if (rw == rr1) {
#pragma unroll
            for (int c = 0; c < kNB; ++c) rowbuf[par][wave][c] = v1[c];
          }
        }
        if (lane == 0) kbuf[par][wave] = key;
        __syncthreads();
        unsigned long long best = 0ull;
#pragma unroll
        for (int w = 0; w < kLuWaves; ++w) {
          const unsigned long long kv = kbuf[par][w];
          best = kv > best ? kv : best;
        }
        const int brow = __builtin_amdgcn_readfirstlane(2047 - (int)(best & 2047ull));
        const int bw = (brow & (kLuThreads - 1)) >> 6;
        const double *prw = rowbuf[par][bw];
        const double d = prw[jj];
        const bool okp = fabs(d) > 0.0;
        if (t == 0 && !okp) bad = 1;
        const double invd = okp ? 1.0 / d : 0.0;
        // row j of U (columns >= j), stored transposed
        if (t >= jj && t < kNB - jb) Ut[jb + t][j] = prw[t];
        if (t == 0) prs[j] = brow;
        if (rr0 == brow) {
          cand0 = false;
          pos0 = j;
        }
        if (rr1 == brow) {
          cand1 = false;
          pos1 = j;
        }
        const double l0 = v0[jj] * invd, l1 = v1[jj] * invd;
#pragma unroll
        for (int c = jj + 1; c < kNB; ++c) {
          const double pc = prw[c];
          if (cand0) v0[c] -= l0 * pc;
          if (cand1) v1[c] -= l1 * pc;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
      v0[c] = (c + 8 < kNB) ? v0[c + 8] : 0.0;
      v1[c] = (c + 8 < kNB) ? v1[c + 8] : 0.0;
    }
  }
  if (pos0 >= 0) {
    S.slot[rr0] = kb + pos0;
    S.prow[kb + pos0] = rr0;
  }
  if (pos1 >= 0) {
    S.slot[rr1] = kb + pos1;
    S.prow[kb + pos1] = rr1;
  }
  __syncthreads();
  if (t == 0 && bad) atomicOr(&S.stats[kStError], (unsigned long long)kErrSingular);
  // (U^T)^{-1}, in place
  tri_lower_inverse(Ut, Tm, false);
  // D (pivot rows in order, original entries) into Lm
  for (int e = t; e < kNB * kNB; e += kLuThreads) {
    const int i = e / kNB, c = e % kNB;
    Lm[i][c] = (i < nb && c < nb) ? S.E[(long)prs[i] * S.ld + kb + c] : (i == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // L = D U^{-1}, strictly lower part, unit diagonal; U^{-1}(m, j) = Ut(j, m)
  for (int e = t; e < kNB * kNB; e += kLuThreads) {
    const int i = e / kNB, j = e % kNB;
    double s = 0.0;
    if (j < i) {
#pragma unroll 8
      for (int m = 0; m < kNB; ++m) s += Lm[i][m] * Ut[j][m];
    }
    Tm[i][j] = (j < i) ? s : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  tri_lower_inverse(Tm, Lm, true);
  for (int e = t; e < kNB * kNB; e += kLuThreads) {
    const int i = e / kNB, j = e % kNB;
    double s = 0.0;
#pragma unroll 8
    for (int m = 0; m < kNB; ++m) s += Ut[m][i] * Tm[m][j];
    if (i < nb && j < nb) S.Z[i * kNB + j] = s;
  }
}

// Cholesky panel: C C^T = E[kb:kb+nb, kb:kb+nb) (the current Schur
// complement), Z = C^{-1} (lower).  Wave 0 factors the block with lane i
// holding row i and cross-lane reads (no barriers); then the workgroup
// inverts C.
constexpr int kCholThreads = 256;

__global__ __launch_bounds__(kCholThreads) void chol_panel_kernel(ElimArgs a) {
  const ElimSpin &S = a.s[blockIdx.x];
  const int kb = a.kb, nb = a.nb;
  const int t = threadIdx.x;
  __shared__ double C[kNB][kNB + 1], Tm[kNB][kNB + 1];
  for (int e = t; e < kNB * kNB; e += kCholThreads) {
    const int i = e / kNB, c = e % kNB;
    C[i][c] = (i < nb && c < nb) ? S.E[(long)(kb + i) * S.ld + kb + c] : (i == c ? 1.0 : 0.0);
  }
  __syncthreads();
  if (t < 64) {
    const int i = t;
    double v[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) v[c] = (i < kNB) ? C[i][c] : 0.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
      const double dk = lane_value(v[k], k);
      const bool ok = dk > 0.0;
      bad = bad || !ok;
      const double ck = ok ? sqrt(dk) : 1.0;
      const double ick = 1.0 / ck;
      const double l = (i > k) ? v[k] * ick : 0.0;
      v[k] = (i == k) ? ck : ((i > k) ? l : v[k]);
#pragma unroll
      for (int j = k + 1; j < kNB; ++j) {
        const double lj = lane_value(l, j);
        if (i >= j) v[j] -= l * lj;
      }
    }
    if (i < kNB) {
#pragma unroll
      for (int c = 0; c < kNB; ++c) C[i][c] = (c <= i) ? v[c] : 0.0;
    }
    if (i == 0 && bad) atomicOr(&S.stats[kStError], (unsigned long long)kErrSingular);
  }
  __syncthreads();
  tri_lower_inverse(C, Tm, false);
  for (int e = t; e < kNB * kNB; e += kCholThreads) {
    const int rr = e / kNB, cc = e % kNB;
    if (rr < nb && cc < nb) S.Z[rr * kNB + cc] = C[rr][cc];
  }
}

// One 64 x 64 tile (rows r0.., live columns c0..) of a pass.
//   block rows:  B = Z E[b, :]  (Gauss-Jordan: to the side buffer BR;
//                Cholesky: their right-half entries to F)
//   other rows:  E[i, :] -= L_i B with L_i = E[i, panel] (Gauss-Jordan) or
//                E[i, panel] Z^T (Cholesky).
// Gauss-Jordan rows that were block rows of the previous pass are read from
// BR.  Rows < kb are final in the Cholesky mode and are not visited.
template <bool GJ>
__global__ __launch_bounds__(256) void elim_update_kernel(ElimArgs a) {
  const ElimSpin &S = a.s[blockIdx.z];
  const int n = S.n, w = S.w, kb = a.kb, nb = a.nb;
  const long ld = S.ld;
  const int r0 = (GJ ? 0 : kb) + blockIdx.x * 64;
  const int c0 = kb + nb + blockIdx.y * 64;
  const int c1 = GJ ? w : min(w, n + kb + nb);
  if (r0 >= n || c0 >= c1) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, wm = wave >> 1, wn = wave & 1;
  constexpr int LZ = kNB + 1, LB = 65;
  __shared__ double Zs[kNB * LZ];
  __shared__ double EB[kNB * LB];
  __shared__ double NBs[kNB * LB];
  __shared__ double Lp[64 * LZ];
  __shared__ const double *rsrc[64];
  __shared__ int rcur[64];

  if (t < 64) {
    const int r = r0 + t;
    const double *p = nullptr;
    int cur = -1;
    if (r < n) {   // rows past n keep p = nullptr (read as row 0, never stored)
      p = S.E + (long)r * ld;
      if (GJ) {
        const int sl = S.slot[r];
        if (sl >= kb && sl < kb + nb) {
          cur = sl - kb;
        } else if (kb > 0 && sl >= kb - kNB && sl < kb) {
          p = S.BR + (long)((a.pass - 1) & 1) * kNB * w + (long)(sl - (kb - kNB)) * w;
        }
      } else if (r < kb + nb) {
        cur = r - kb;
      }
    }
    rsrc[t] = p;
    rcur[t] = cur;
  }
  // Loads are unconditional so that they issue together: clamped addresses
  // inside the data the guarded reads would touch (written, finite), with the
  // entries outside the panel zeroed when stored (a multiply: a select would
  // become a branch around the load and a wait).
  constexpr int QZ = kNB * kNB / 256, QE = kNB * 64 / 256;
  double zv[QZ], ev[QE];
  int prw[QE];
#pragma unroll
  for (int q = 0; q < QE; ++q) {
    const int b = (t + 256 * q) >> 6;
    prw[q] = GJ ? S.prow[kb + min(b, nb - 1)] : kb + min(b, nb - 1);
  }
  // Z holds only its leading nb x nb block: read inside it
#pragma unroll
  for (int q = 0; q < QZ; ++q) {
    const int e = t + 256 * q, i = e / kNB, j = e % kNB;
    zv[q] = S.Z[min(i, nb - 1) * kNB + min(j, nb - 1)];
  }
#pragma unroll
  for (int q = 0; q < QE; ++q) {
    const int cc = (t + 256 * q) & 63;
    ev[q] = S.E[(long)prw[q] * ld + min(c0 + cc, c1 - 1)];
  }
#pragma unroll
  for (int q = 0; q < QZ; ++q) {
    const int e = t + 256 * q, i = e / kNB, j = e % kNB;
    Zs[i * LZ + j] = zv[q] * ((i < nb && j < nb) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int q = 0; q < QE; ++q) {
    const int e = t + 256 * q, b = e >> 6, cc = e & 63;
    EB[b * LB + cc] = ev[q] * ((b < nb && c0 + cc < c1) ? 1.0 : 0.0);
  }
  __syncthreads();
  constexpr int QL = 64 * kNB / 256;
  double lv[QL];
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int e = t + 256 * q, rr = e / kNB, b = e % kNB;
    const double *p = rsrc[rr];
    lv[q] = (p ? p : S.E)[kb + min(b, nb - 1)];
  }
  dbl4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = acc_row(wm, mi, lane, j), c = c0 + acc_col(wn, ni, lane);
        const double *p = rsrc[rr];
        acc[mi][ni][j] = (p ? p : S.E)[min(c, c1 - 1)];
      }
#pragma unroll
  for (int q = 0; q < QL; ++q) {
    const int e = t + 256 * q, rr = e / kNB, b = e % kNB;
    const double v = lv[q] * ((rsrc[rr] && b < nb) ? 1.0 : 0.0);
    Lp[rr * LZ + b] = GJ ? -v : v;
  }
  __syncthreads();
  // block rows B = Z EB: 2 x 4 tiles of 16 x 16, two per wave
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int tt = wave + 4 * u, mt = tt >> 2, ct = tt & 3;
    const dbl4 q = mma16<false>(Zs + mt * 16 * LZ, LZ, EB + ct * 16, LB, kNB, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      NBs[(mt * 16 + (lane >> 4) + 4 * j) * LB + ct * 16 + (lane & 15)] = q[j];
  }
  if (!GJ) {
    // multipliers -(E[i, panel] Z^T): wave w owns rows [16 w, 16 w + 16) and
    // overwrites them after both of its tiles are formed
    const dbl4 q0 = mma16<true>(Lp + wave * 16 * LZ, LZ, Zs, LZ, kNB, lane);
    const dbl4 q1 = mma16<true>(Lp + wave * 16 * LZ, LZ, Zs + 16 * LZ, LZ, kNB, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = wave * 16 + (lane >> 4) + 4 * j;
      Lp[rr * LZ + (lane & 15)] = -q0[j];
      Lp[rr * LZ + 16 + (lane & 15)] = -q1[j];
    }
  }
  __syncthreads();
  lds_mma<false>(acc, Lp, LZ, NBs, LB, kNB, 64, 64, wm, wn, lane);
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = acc_row(wm, mi, lane, j), cc = acc_col(wn, ni, lane);
        const int r = r0 + rr, c = c0 + cc;
        if (r >= n || c >= c1) continue;
        const int cur = rcur[rr];
        if (cur >= 0) {
          const double v = NBs[cur * LB + cc];
          if (GJ) S.BR[(long)(a.pass & 1) * kNB * w + (long)cur * w + c] = v;
          else if (c >= n) S.F[(long)r * n + (c - n)] = v;
        } else {
          S.E[(long)r * ld + c] = acc[mi][ni][j];
        }
      }
}

// T[c, :] = (right half of row prow[c]) after the last Gauss-Jordan pass
struct GatherArgs {
  ElimSpin s[kMaxMats];
  double *out[kMaxMats];
  long ldo;
  int kb_last, pass_last;
};

__global__ void gj_gather_kernel(GatherArgs a) {
  const ElimSpin &S = a.s[blockIdx.z];
  const int n = S.n, c = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || j >= n) return;
  const int r = S.prow[c];
  const int sl = S.slot[r];
  const double *src = (sl >= a.kb_last)
                          ? S.BR + (long)(a.pass_last & 1) * kNB * S.w + (long)(sl - a.kb_last) * S.w
                          : S.E + (long)r * S.ld;
  a.out[blockIdx.z][(long)c * a.ldo + j] = src[n + j];
}

struct FillArgs {
  int *ip[kMaxMats];
  double *dp[kMaxMats];
};

__global__ void fill_int_kernel(FillArgs f, long count, int value) {
  int *p = f.ip[blockIdx.y];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x)
    p[e] = value;
}

__global__ void zero_kernel(FillArgs f, long count) {
  double *p = f.dp[blockIdx.y];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x)
    p[e] = 0.0;
}

struct IdentArgs {
  double *E[kMaxMats];
};

__global__ void set_identity_kernel(IdentArgs a, long ld, int n, int col0) {
  double *E = a.E[blockIdx.z];
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

struct ConvArgs {
  const void *src[kMaxMats];
  void *dst[kMaxMats];
  long n[kMaxMats];    // elements of each pair
};

__global__ void round_kernel(ConvArgs a) {
  const double *s = static_cast<const double *>(a.src[blockIdx.y]);
  float *d = static_cast<float *>(a.dst[blockIdx.y]);
  const long n = a.n[blockIdx.y];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    d[e] = (float)s[e];
}

__global__ void widen_kernel(ConvArgs a) {
  const float *s = static_cast<const float *>(a.src[blockIdx.y]);
  double *d = static_cast<double *>(a.dst[blockIdx.y]);
  const long n = a.n[blockIdx.y];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    d[e] = (double)s[e];
}

struct SetArgs {
  uint64_t *p[kMaxMats];
  uint64_t v[kMaxMats];
};
__global__ void set_u64_kernel(SetArgs a, int n) {
  if ((int)threadIdx.x < n) *a.p[threadIdx.x] = a.v[threadIdx.x];
}

struct DiffArgs {
  const double *a[kMaxMats], *b[kMaxMats];
  unsigned long long *out[kMaxMats];
  long n[kMaxMats];
};

// *out = max(*out, max_e |a[e] - b[e]|) as the bit pattern of a non-negative
// double (whose integer order is its numeric order; a NaN difference wins).
__global__ __launch_bounds__(256) void max_abs_diff_kernel(DiffArgs d) {
  const int m = blockIdx.y;
  double v = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < d.n[m]; e += (long)gridDim.x * 256) {
    const double x = fabs(d.a[m][e] - d.b[m][e]);
    v = (x > v || x != x) ? x : v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(v, o, 64);
    v = (x > v || x != x) ? x : v;
  }
  if ((threadIdx.x & 63) == 0)
    atomicMax(d.out[m], (unsigned long long)__double_as_longlong(v));
}

__global__ void init_fields_kernel(int8_t *f, int M, int N, uint64_t k0, uint64_t k1) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  const int li = (int)(e / N), i = (int)(e % N);
  const double u = philox_uniform(k0, k1, 0, (uint64_t)li, (uint64_t)i, kPurposeInit);
  f[e] = (u < 0.5) ? (int8_t)1 : (int8_t)-1;
}

}  // namespace

hipError_t gj_invert(const ElimSpin *s, int nmat, double *const *out, long ldo, hipStream_t st) {
  if (nmat < 1 || nmat > kMaxMats) return hipErrorInvalidValue;
  const int n = s[0].n;
  for (int i = 1; i < nmat; ++i)
    if (s[i].n != n || s[i].w != s[0].w) return hipErrorInvalidValue;
  if (n < 1 || n > 2 * kLuThreads) return hipErrorInvalidValue;
  const int w = s[0].w;
  FillArgs fa{};
  for (int i = 0; i < nmat; ++i) fa.ip[i] = s[i].slot;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256, nmat), dim3(256), 0, st, fa, (long)n,
                     -1);
  ElimArgs ea{};
  for (int i = 0; i < nmat; ++i) ea.s[i] = s[i];
  int pass = 0, kb = 0;
  for (; kb < n; kb += kNB, ++pass) {
    ea.kb = kb;
    ea.nb = min(kNB, n - kb);
    ea.pass = pass;
    hipLaunchKernelGGL(lu_panel_kernel, dim3(nmat), dim3(kLuThreads), 0, st, ea);
    const int cols = w - kb - ea.nb;
    hipLaunchKernelGGL(elim_update_kernel<true>, dim3((n + 63) / 64, (cols + 63) / 64, nmat),
                       dim3(256), 0, st, ea);
  }
  GatherArgs ga{};
  for (int i = 0; i < nmat; ++i) {
    ga.s[i] = s[i];
    ga.out[i] = out[i];
  }
  ga.ldo = ldo;
  ga.kb_last = kb - kNB;
  ga.pass_last = pass - 1;
  hipLaunchKernelGGL(gj_gather_kernel, dim3((n + 255) / 256, n, nmat), dim3(256), 0, st, ga);
  return hipGetLastError();
}

hipError_t chol_eliminate(const ElimSpin *s, int nmat, hipStream_t st) {
  if (nmat < 1 || nmat > kMaxMats) return hipErrorInvalidValue;
  const int n = s[0].n;
  for (int i = 1; i < nmat; ++i)
    if (s[i].n != n || s[i].w != s[0].w) return hipErrorInvalidValue;
  if (n < 1 || s[0].w < 2 * n) return hipErrorInvalidValue;
  const int w = s[0].w;
  FillArgs fa{};
  for (int i = 0; i < nmat; ++i) fa.dp[i] = s[i].F;
  hipLaunchKernelGGL(zero_kernel, dim3(256, nmat), dim3(256), 0, st, fa, (long)n * n);
  ElimArgs ea{};
  for (int i = 0; i < nmat; ++i) ea.s[i] = s[i];
  for (int kb = 0, pass = 0; kb < n; kb += kNB, ++pass) {
    ea.kb = kb;
    ea.nb = min(kNB, n - kb);
    ea.pass = pass;
    hipLaunchKernelGGL(chol_panel_kernel, dim3(nmat), dim3(kCholThreads), 0, st, ea);
    const int cols = min(w, n + kb + ea.nb) - kb - ea.nb;
    hipLaunchKernelGGL(elim_update_kernel<false>,
                       dim3((n - kb + 63) / 64, (cols + 63) / 64, nmat), dim3(256), 0, st, ea);
  }
  return hipGetLastError();
}

hipError_t set_identity_block(double *const *E, int nmat, long ld, int n, int col0,
                              hipStream_t st) {
  if (nmat < 1 || nmat > kMaxMats) return hipErrorInvalidValue;
  IdentArgs a{};
  for (int i = 0; i < nmat; ++i) a.E[i] = E[i];
  dim3 grid((n + 255) / 256, n, nmat);
  hipLaunchKernelGGL(set_identity_kernel, grid, dim3(256), 0, st, a, ld, n, col0);
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

hipError_t round_to_f32(const double *const *src, float *const *dst, int nmat, const long *n,
                        hipStream_t st) {
  if (nmat < 1 || nmat > kMaxMats) return hipErrorInvalidValue;
  ConvArgs a{};
  for (int i = 0; i < nmat; ++i) {
    a.src[i] = src[i];
    a.dst[i] = dst[i];
    a.n[i] = n[i];
  }
  hipLaunchKernelGGL(round_kernel, dim3(256, nmat), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t widen_to_f64(const float *const *src, double *const *dst, int nmat, const long *n,
                        hipStream_t st) {
  if (nmat < 1 || nmat > kMaxMats) return hipErrorInvalidValue;
  ConvArgs a{};
  for (int i = 0; i < nmat; ++i) {
    a.src[i] = src[i];
    a.dst[i] = dst[i];
    a.n[i] = n[i];
  }
  hipLaunchKernelGGL(widen_kernel, dim3(256, nmat), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t set_u64(uint64_t *const *p, const uint64_t *v, int n, hipStream_t st) {
  if (n < 1 || n > kMaxMats) return hipErrorInvalidValue;
  SetArgs a{};
  for (int i = 0; i < n; ++i) {
    a.p[i] = p[i];
    a.v[i] = v[i];
  }
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, st, a, n);
  return hipGetLastError();
}

hipError_t max_abs_diff(const double *const *a, const double *const *b, const long *n,
                        unsigned long long *const *out, int nmat, hipStream_t st) {
  if (nmat < 1 || nmat > kMaxMats) return hipErrorInvalidValue;
  DiffArgs d{};
  for (int i = 0; i < nmat; ++i) {
    d.a[i] = a[i];
    d.b[i] = b[i];
    d.n[i] = n[i];
    d.out[i] = out[i];
  }
  hipLaunchKernelGGL(max_abs_diff_kernel, dim3(16, nmat), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t init_fields(int8_t *fields, int M, int N, uint64_t k0, uint64_t k1, hipStream_t st) {
  const long tot = (long)M * N;
  hipLaunchKernelGGL(init_fields_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     fields, M, N, k0, k1);
  return hipGetLastError();
}

}  // namespace pq
