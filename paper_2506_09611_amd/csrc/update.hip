// Field-update kernels of one time slice (Secs. II D, III A, III B).
//
// Local update: one launch per site.  The launch for site i first applies
// the pending decision of site i-1 -- the Metropolis test on
// r_up r_dn with r_s = 1 + y^T v (Eq. (20)) and, on acceptance, the rank-1
// upgrade T <- T - x y^T with x = T v / r (Eq. (21)) -- and then forms the
// partial products of site i (y^T = u_i^T T, T v_i and u_i^T T v_i) from
// the freshly updated tile.  Each 256-thread workgroup owns one 64x64 tile
// of T for the launch; cross-tile sums use per-tile partial buffers that
// every workgroup reduces in the same fixed order, so all of them take the
// same decision without atomics.
//
// Delayed and block force-bias updates work on a group of kk consecutive
// sites.  With U_g the group's rows of U_R and L_g its columns of U_L:
//   P2 = U_g T (kk x Ns), P1 = T L_g (Ns x kk), W0 = U_g T L_g (kk x kk)
// are formed by split-K MFMA GEMMs and a reduction.  A single workgroup
// then takes all decisions of the group on kk x kk matrices:
//   delayed: E = 1 + W0 diag(Delta); the ratio of site j given the accepted
//            set A is the Schur complement E_jj - E_jA E_AA^{-1} E_Aj, i.e.
//            the diagonal entry after sweeping the pivots in A (principal
//            pivot transform).  This equals the recursion of Eq. (28).
//   block:   E = 1 + diag(Delta_b) W0 gives the force bias of Eq. (35),
//            nbar_i = (1 + Delta_b,i) [W0 E^{-1}]_ii; heat-bath proposal;
//            det[1 + W0_FF diag(Delta'_F)] by sweeping the flipped pivots.
// After the sweep the accepted block holds -(E_AA)^{-1}, so the flush
// T <- T - P1_A diag(Delta_A) (E_AA)^{-1} P2_A is Eq. (30) (delayed) or
// Eq. (36) (block), done as a rank-n_A MFMA GEMM.
#include "engine.hpp"

namespace pq {

namespace {

// ------------------------------------------------------------------------
// local update
// ------------------------------------------------------------------------
struct LocalArgs {
  SpinMats m;
  LocalBufs b;
  SweepCtx c;
  int i;
};

__device__ __forceinline__ void record_decision(const SweepCtx &c, long long idx, int site,
                                                bool acc, double margin) {
  if (c.log_meta && idx < c.log_cap) {
    c.log_meta[3 * idx + 0] = (int32_t)c.slice_code;
    c.log_meta[3 * idx + 1] = site;
    c.log_meta[3 * idx + 2] = acc ? 1 : 0;
    c.log_margin[idx] = margin;
  }
}

__global__ __launch_bounds__(256) void local_step_kernel(LocalArgs a) {
  const int s = blockIdx.y;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int tile = blockIdx.x;
  const int rb = tile / nt, cb = tile % nt;
  if (rb >= nt) return;
  const int t = threadIdx.x, c = t & 63, rq = t >> 6;
  const int lane = t & 63;
  const int row0 = rb * 64, col0 = cb * 64;
  const int col = col0 + c;
  const bool colok = col < Ns;
  double *T = a.m.T[s];
  const bool designated = (s == 0 && tile == 0);
  const int i = a.i;
  const SweepCtx &C = a.c;

  __shared__ double red[4][64];
  __shared__ double sred[4];
  __shared__ double s_r[2];
  __shared__ double xs[64], ys[64];

  double tv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = row0 + rq + 4 * q;
    tv[q] = (r < Ns && colok) ? T[(long)r * Ns + col] : 0.0;
  }
  bool dirty = false;

  if (i > 0) {
    const int par = (i - 1) & 1;
    // r_s = 1 + sum over tiles of u^T T_tile v, same order in every workgroup
    if (rq < 2) {
      const int ss = rq;
      const int nts = (a.m.Ns[ss] + 63) / 64;
      const int ntot = nts * nts;
      double p = 0.0;
      for (int e = lane; e < ntot; e += 64) p += a.b.spart[ss][par][e];
      p = wave_sum(p);
      if (lane == 0) s_r[ss] = 1.0 + p;
    }
    __syncthreads();
    const double r0 = s_r[0], r1 = s_r[1];
    const double R = r0 * r1;
    const double absA = fabs(R);
    const double u = philox_uniform(C.key0, C.key1, C.sweep, C.slice_code, (uint64_t)(i - 1),
                                    kPurposeMH);
    const bool finite = !isnan(absA);
    // every lane computes the same value; make it an explicit scalar
    const bool acc = __builtin_amdgcn_readfirstlane((finite && (u < absA)) ? 1 : 0) != 0;
    const double rs = s ? r1 : r0;
    if (acc) {
      // x_r = (T v)_r / r over all column tiles (threads 0..63), y_c over all
      // row tiles (threads 64..127), then the rank-1 upgrade of this tile
      if (t < 64) {
        const int r = row0 + t;
        xs[t] = (r < Ns) ? sum_strided(a.b.tpart[s][par] + r, Ns, nt) / rs : 0.0;
      } else if (t < 128) {
        const int cc = col0 + (t - 64);
        ys[t - 64] = (cc < Ns) ? sum_strided(a.b.ypart[s][par] + cc, Ns, nt) : 0.0;
      }
      __syncthreads();
      const double yc = ys[c];
#pragma unroll
      for (int q = 0; q < 16; ++q) tv[q] -= xs[rq + 4 * q] * yc;
      dirty = true;
    }
    if (designated) {
      const double d0 = a.b.delta[par][0], d1 = a.b.delta[par][1];
      if (t == 0) {
        const double margin = absA - u;
        C.stats[kStProposed] += 1;
        C.stats[kStFieldUpdates] += 1;
        if (acc) { C.stats[kStAccepted] += 1; C.stats[kStFlips] += 1; }
        if (fabs(margin) < 1e-12) C.stats[kStLowMargin] += 1;
        if (R < 0.0) C.stats[kStNegative] += 1;
        if (!finite) C.stats[kStError] |= kErrNonFinite;
        record_decision(C, C.log_base + (i - 1), i - 1, acc, margin);
        if (acc) C.fields[(long)C.li * C.N + (i - 1)] = (int8_t)(-C.fields[(long)C.li * C.N + (i - 1)]);
      }
      if (acc) {
        for (int ss = 0; ss < 2; ++ss) {
          const int n = a.m.Ns[ss];
          const double f = 1.0 + (ss ? d1 : d0);
          double *row = a.m.UR[ss] + (long)(i - 1) * n;
          for (int e = t; e < n; e += 256) row[e] *= f;
        }
      }
    }
  }

  if (i < C.N) {
    const int par = i & 1;
    const int8_t x = C.fields[(long)C.li * C.N + i];
    const double dl = C.dflip[s][x > 0 ? 0 : 1];
    const double vc = colok ? dl * a.m.ULt[s][(long)i * Ns + col] : 0.0;
    double ur[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = row0 + rq + 4 * q;
      ur[q] = (r < Ns) ? a.m.UR[s][(long)i * Ns + r] : 0.0;
    }
    // y partial (column c, this tile's rows) and (T v) partial (rows, this tile's columns)
    double yp = 0.0, sp = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      yp += ur[q] * tv[q];
      const double trow = wave_sum(tv[q] * vc);
      sp += ur[q] * trow;
      if (lane == 0) {
        const int r = row0 + rq + 4 * q;
        if (r < Ns) a.b.tpart[s][par][(long)cb * Ns + r] = trow;
      }
    }
    red[rq][c] = yp;
    if (lane == 0) sred[rq] = sp;
    __syncthreads();
    if (rq == 0) {
      const double y = red[0][c] + red[1][c] + red[2][c] + red[3][c];
      if (colok) a.b.ypart[s][par][(long)rb * Ns + col] = y;
      if (t == 0) a.b.spart[s][par][rb * nt + cb] = sred[0] + sred[1] + sred[2] + sred[3];
    }
    if (designated && t == 0) {
      a.b.delta[par][0] = C.dflip[0][x > 0 ? 0 : 1];
      a.b.delta[par][1] = C.dflip[1][x > 0 ? 0 : 1];
    }
  }

  if (dirty) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = row0 + rq + 4 * q;
      if (r < Ns && colok) T[(long)r * Ns + col] = tv[q];
    }
  }
}

// ------------------------------------------------------------------------
// group panels: reduce split-K partials, form W0 partials per column strip
// ------------------------------------------------------------------------
struct ReduceArgs {
  SpinMats m;
  GroupBufs g;
  int g0, kk;
};

constexpr int kRedThreads = 1024;

__global__ __launch_bounds__(kRedThreads) void group_reduce_kernel(ReduceArgs a) {
  const int s = blockIdx.y;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int strip = blockIdx.x;
  if (strip >= nt) return;
  const int kk = a.kk, kmax = a.g.kmax;
  const int t = threadIdx.x;
  const int c0 = strip * 64;
  const int w = min(64, Ns - c0);
  extern __shared__ double dyn_lds[];
  double (*p2s)[65] = reinterpret_cast<double (*)[65]>(dyn_lds);
  double (*lgs)[65] = reinterpret_cast<double (*)[65]>(dyn_lds + (size_t)kk * 65);
  // P2[:, strip] and the group's rows of U_L^T over the strip
  for (int e = t; e < kk * 64; e += kRedThreads) {
    const int mrow = e >> 6, cc = e & 63;
    double v = 0.0, l = 0.0;
    if (cc < w) {
      const long off = (long)mrow * Ns + c0 + cc;
      v = sum_strided(a.g.P2part[s] + off, (long)kmax * Ns, nt);
      a.g.P2[s][off] = v;
      l = a.m.ULt[s][(long)(a.g0 + mrow) * Ns + c0 + cc];
    }
    p2s[mrow][cc] = v;
    lgs[mrow][cc] = l;
  }
  // P1[strip rows, :]
  for (int e = t; e < 64 * kk; e += kRedThreads) {
    const int rr = e / kk, mcol = e % kk;
    if (rr < w) {
      const long off = (long)(c0 + rr) * kmax + mcol;
      a.g.P1[s][off] = sum_strided(a.g.P1part[s] + off, (long)Ns * kmax, nt);
    }
  }
  __syncthreads();
  // W0 partial over this strip: sum_c P2[m1][c] L_g[m2][c]
  for (int e = t; e < kk * kk; e += kRedThreads) {
    const int m1 = e / kk, m2 = e % kk;
    double v = 0.0;
#pragma unroll 8
    for (int cc = 0; cc < 64; ++cc) v += p2s[m1][cc] * lgs[m2][cc];
    a.g.W0part[s][(long)strip * kmax * kmax + m1 * kmax + m2] = v;
  }
  // the last strip to finish sums the partials in strip order into W0
  // (deterministic; the ticket counter is reset for the next launch)
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (t == 0) s_last = (atomicAdd(&a.g.ticket[s], 1) == nt - 1) ? 1 : 0;
  __syncthreads();
  if (s_last) {
    __threadfence();
    for (int e = t; e < kk * kk; e += kRedThreads) {
      const int m1 = e / kk, m2 = e % kk;
      a.g.W0[s][m1 * kmax + m2] =
          sum_strided(a.g.W0part[s] + m1 * kmax + m2, (long)kmax * kmax, nt);
    }
    if (t == 0) a.g.ticket[s] = 0;
  }
}

// ------------------------------------------------------------------------
// decision kernels (one workgroup of 1024 threads)
// ------------------------------------------------------------------------

struct DecideArgs {
  GroupBufs g;
  SweepCtx c;
  int g0, kk;
  long long block_index;
};

// W0 = U_g T L_g for element (a, b), as summed by the reduce kernel
__device__ __forceinline__ double w0_elem(const DecideArgs &A, int s, int a, int b) {
  return A.g.W0[s][a * A.g.kmax + b];
}

// kDecThreads lanes, kDecQ = ceil(kk * kk / kDecThreads) elements of each
// spin's E per lane (kk <= kDecThreads).
template <int kDecThreads, int kDecQ>
__global__ __launch_bounds__(kDecThreads) void delayed_decide_kernel(DecideArgs A) {
  const int kk = A.kk;
  const int t = threadIdx.x;
  const SweepCtx &C = A.c;
  __shared__ double colb[2][2][128], rowb[2][2][128];
  __shared__ double uni[128];
  __shared__ double dl[2][128];
  __shared__ int acc_s[128];
  __shared__ int pos[128];

  if (t < kk) {
    const int site = A.g0 + t;
    const int8_t x = C.fields[(long)C.li * C.N + site];
    dl[0][t] = C.dflip[0][x > 0 ? 0 : 1];
    dl[1][t] = C.dflip[1][x > 0 ? 0 : 1];
    uni[t] = philox_uniform(C.key0, C.key1, C.sweep, C.slice_code, (uint64_t)site, kPurposeMH);
  }
  __syncthreads();
  // owned elements of E_s = 1 + W0_s diag(Delta_s); (row, column) per element
  double e0[kDecQ], e1[kDecQ];
  int ra[kDecQ], cb_[kDecQ];
#pragma unroll
  for (int q = 0; q < kDecQ; ++q) {
    const int e = t + kDecThreads * q;
    e0[q] = e1[q] = 0.0;
    ra[q] = (e < kk * kk) ? e / kk : 1 << 20;
    cb_[q] = (e < kk * kk) ? e % kk : 1 << 20;
    if (e < kk * kk) {
      const int ia = ra[q], ib = cb_[q];
      e0[q] = (ia == ib ? 1.0 : 0.0) + w0_elem(A, 0, ia, ib) * dl[0][ib];
      e1[q] = (ia == ib ? 1.0 : 0.0) + w0_elem(A, 1, ia, ib) * dl[1][ib];
      if (ib == 0) { colb[0][0][ia] = e0[q]; colb[1][0][ia] = e1[q]; }
      if (ia == 0) { rowb[0][0][ib] = e0[q]; rowb[1][0][ib] = e1[q]; }
    }
  }
  __syncthreads();
  // lane 0 keeps the statistics in registers and writes them once
  unsigned long long n_acc = 0, n_low = 0, n_neg = 0;
  bool any_nan = false;
  for (int j = 0; j < kk; ++j) {
    const int par = j & 1, nxt = par ^ 1;
    const double p0 = colb[0][par][j], p1 = colb[1][par][j];
    const double R = p0 * p1;
    const double absA = fabs(R);
    const bool finite = !isnan(absA);
    // every lane computes the same value; make it an explicit scalar
    const bool acc = __builtin_amdgcn_readfirstlane((finite && (uni[j] < absA)) ? 1 : 0) != 0;
    if (t == 0) {
      const double margin = absA - uni[j];
      n_acc += acc ? 1 : 0;
      n_low += (fabs(margin) < 1e-12) ? 1 : 0;
      n_neg += (R < 0.0) ? 1 : 0;
      any_nan = any_nan || !finite;
      record_decision(C, C.log_base + A.g0 + j, A.g0 + j, acc, margin);
      acc_s[j] = acc ? 1 : 0;
    }
    const double ip0 = 1.0 / p0, ip1 = 1.0 / p1;
#pragma unroll
    for (int q = 0; q < kDecQ; ++q) {
      const int ia = ra[q], ib = cb_[q];
      if (ia < kk) {
        if (acc) {
          // principal pivot transform on pivot j, both spins (branch-free)
          const bool rj = ia == j, cj = ib == j;
          const double ca0 = colb[0][par][ia] * ip0, rb0 = rowb[0][par][ib];
          const double ca1 = colb[1][par][ia] * ip1, rb1 = rowb[1][par][ib];
          double v0 = e0[q] - ca0 * rb0, v1 = e1[q] - ca1 * rb1;
          v0 = rj ? rb0 * ip0 : v0;
          v1 = rj ? rb1 * ip1 : v1;
          v0 = cj ? ca0 : v0;
          v1 = cj ? ca1 : v1;
          v0 = (rj && cj) ? -ip0 : v0;
          v1 = (rj && cj) ? -ip1 : v1;
          e0[q] = v0;
          e1[q] = v1;
        }
        if (j + 1 < kk) {
          if (ib == j + 1) { colb[0][nxt][ia] = e0[q]; colb[1][nxt][ia] = e1[q]; }
          if (ia == j + 1) { rowb[0][nxt][ib] = e0[q]; rowb[1][nxt][ib] = e1[q]; }
        }
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    C.stats[kStProposed] += kk;
    C.stats[kStFieldUpdates] += kk;
    C.stats[kStAccepted] += n_acc;
    C.stats[kStFlips] += n_acc;
    C.stats[kStLowMargin] += n_low;
    C.stats[kStNegative] += n_neg;
    if (any_nan) C.stats[kStError] |= kErrNonFinite;
  }
  // compaction of the accepted set, one lane per site (no single-lane loops)
  if (t < kk) {
    int before = 0;
    for (int m = 0; m < t; ++m) before += acc_s[m];
    const int mine = acc_s[t];
    pos[t] = mine ? before : -1;
    if (mine) {
      A.g.Alist[before] = t;
      A.g.Dsel[0][before] = dl[0][t];
      A.g.Dsel[1][before] = dl[1][t];
      C.fields[(long)C.li * C.N + A.g0 + t] = (int8_t)(-C.fields[(long)C.li * C.N + A.g0 + t]);
    }
    if (t == kk - 1) *A.g.nA = before + mine;
  }
  __syncthreads();
  // M^{-1} = (E_AA)^{-1} = -(swept E)_AA, compacted
  const int kmax = A.g.kmax;
#pragma unroll
  for (int q = 0; q < kDecQ; ++q) {
    const int ia = ra[q], ib = cb_[q];
    if (ia < kk) {
      const int pa = pos[ia], pb = pos[ib];
      if (pa >= 0 && pb >= 0) {
        A.g.Minv[0][pa * kmax + pb] = -e0[q];
        A.g.Minv[1][pa * kmax + pb] = -e1[q];
      }
    }
  }
}

// In-place inverse of the n x n matrix A (LDS, row-major, stride ld, n <= 64)
// by Gauss-Jordan elimination with partial pivoting; returns det(A).  Every
// lane of the workgroup takes part and gets the same result.
template <int NT>
__device__ double lds_gj_inverse(double *A, int ld, int n, double *colk, double *rowk, int *ipiv,
                                 int *s_piv) {
  const int t = threadIdx.x;
  double det = 1.0;
  for (int k = 0; k < n; ++k) {
    if (t < 64) {
      double bv = (t >= k && t < n) ? fabs(A[t * ld + k]) : -1.0;
      int bi = (t >= k && t < n) ? t : 0x7fffffff;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        const bool take = (ov > bv) || (ov == bv && oi < bi);
        bv = take ? ov : bv;
        bi = take ? oi : bi;
      }
      if (t == 0) {
        *s_piv = (bi < n) ? bi : k;
        ipiv[k] = (bi < n) ? bi : k;
      }
    }
    __syncthreads();
    const int p = __builtin_amdgcn_readfirstlane(*s_piv);
    if (p != k)
      for (int j = t; j < n; j += NT) {
        const double x = A[k * ld + j];
        A[k * ld + j] = A[p * ld + j];
        A[p * ld + j] = x;
      }
    __syncthreads();
    const double piv = A[k * ld + k];
    det *= (p != k) ? -piv : piv;
    const double ip = 1.0 / piv;
    for (int i = t; i < n; i += NT) {
      colk[i] = A[i * ld + k];
      rowk[i] = A[k * ld + i] * ip;
    }
    __syncthreads();
    for (int e = t; e < n * n; e += NT) {
      const int i = e / n, j = e % n;
      double v;
      if (i == k) v = (j == k) ? ip : rowk[j];
      else v = (j == k) ? -colk[i] * ip : A[i * ld + j] - colk[i] * rowk[j];
      A[i * ld + j] = v;
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = __builtin_amdgcn_readfirstlane(ipiv[k]);
    if (p != k)
      for (int i = t; i < n; i += NT) {
        const double x = A[i * ld + k];
        A[i * ld + k] = A[i * ld + p];
        A[i * ld + p] = x;
      }
    __syncthreads();
  }
  return det;
}

// Block force-bias decision for kk <= 64 sites (one workgroup of NT lanes):
// force bias from B = 1 + diag(Delta_b) W0 (Eq. (35)), heat-bath proposal,
// det[1 + W0_FF diag(Delta'_F)] per spin and the Metropolis test with the
// prior ratio (Sec. III B).  Both small inversions use partial pivoting.
template <int NT>
__global__ __launch_bounds__(NT) void block_decide_kernel(DecideArgs A) {
  const int kk = A.kk;
  const int t = threadIdx.x;
  const SweepCtx &C = A.c;
  const int kmax = A.g.kmax;
  constexpr int LD = 65;
  extern __shared__ double blds[];
  double *M0 = blds;              // 64 x 65
  double *M1 = blds + 64 * LD;    // 64 x 65
  __shared__ double colk[64], rowk[64];
  __shared__ int ipiv[64];
  __shared__ int s_piv;
  __shared__ double db[2][64], nbar[2][64], sval[64], dp[2][64], hbm[64];
  __shared__ int xold[64], xnew[64], flist[64];
  __shared__ int s_nF;

  if (t < kk) {
    const int8_t x = C.fields[(long)C.li * C.N + A.g0 + t];
    xold[t] = x > 0 ? 1 : -1;
    db[0][t] = C.dremove[0][x > 0 ? 0 : 1];
    db[1][t] = C.dremove[1][x > 0 ? 0 : 1];
  }
  __syncthreads();
  for (int s = 0; s < 2; ++s) {
    // M1 = W0 (kept for the force-bias product), M0 = 1 + diag(Delta_b) W0
    for (int e = t; e < kk * kk; e += NT) {
      const int ia = e / kk, ib = e % kk;
      const double w = w0_elem(A, s, ia, ib);
      M1[ia * LD + ib] = w;
      M0[ia * LD + ib] = (ia == ib ? 1.0 : 0.0) + db[s][ia] * w;
    }
    __syncthreads();
    lds_gj_inverse<NT>(M0, LD, kk, colk, rowk, ipiv, &s_piv);
    if (t < kk) {
      double v = 0.0;
      for (int m = 0; m < kk; ++m) v += M1[t * LD + m] * M0[m * LD + t];
      nbar[s][t] = (1.0 + db[s][t]) * v;     // [UU_R (U_L UU_R)^{-1} U_L]_ii
    }
    __syncthreads();
  }
  // heat-bath proposal x'_i, P(+1) = 1 / (1 + e^{-2 s_i}), s_i = alpha (nbar_up - nbar_dn)
  if (t < kk) {
    const int site = A.g0 + t;
    const double sv = C.alpha * (nbar[0][t] - nbar[1][t]);
    sval[t] = sv;
    const double pp = 1.0 / (1.0 + exp(-2.0 * sv));
    const double u = philox_uniform(C.key0, C.key1, C.sweep, C.slice_code, (uint64_t)site,
                                    kPurposeHB);
    xnew[t] = (u < pp) ? 1 : -1;
    const double margin = pp - u;
    hbm[t] = margin;
    if (C.hb_meta) {
      const long long idx = C.hb_base + site;
      if (idx < C.log_cap) {
        C.hb_meta[3 * idx + 0] = (int32_t)C.slice_code;
        C.hb_meta[3 * idx + 1] = site;
        C.hb_meta[3 * idx + 2] = xnew[t];
        C.hb_margin[idx] = margin;
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    unsigned long long low = 0;
    for (int j = 0; j < kk; ++j) low += (fabs(hbm[j]) < 1e-12) ? 1ull : 0ull;
    C.stats[kStLowMargin] += low;
  }
  // flip set F in site order, one lane per site
  if (t < kk) {
    int before = 0;
    for (int m = 0; m < t; ++m) before += (xnew[m] != xold[m]) ? 1 : 0;
    const int mine = (xnew[t] != xold[t]) ? 1 : 0;
    if (mine) flist[before] = t;
    if (t == kk - 1) s_nF = before + mine;
  }
  __syncthreads();
  const int nF = __builtin_amdgcn_readfirstlane(s_nF);
  const double u_mh = philox_uniform(C.key0, C.key1, C.sweep, C.slice_code, (uint64_t)A.g0,
                                     kPurposeMH);
  if (nF == 0) {
    if (t == 0) {
      C.stats[kStProposed] += 1;
      C.stats[kStAccepted] += 1;
      C.stats[kStFieldUpdates] += kk;
      const double margin = 1.0 - u_mh;
      if (fabs(margin) < 1e-12) C.stats[kStLowMargin] += 1;
      record_decision(C, C.log_base + A.block_index, A.g0, true, margin);
      *A.g.nA = 0;
    }
    return;
  }
  // E'_s = 1 + W0_FF diag(Delta'_F), Delta'_i = e^{-2 alpha f_s x_i} - 1
  if (t < nF) {
    const int j = flist[t];
    dp[0][t] = C.dflip[0][xold[j] > 0 ? 0 : 1];
    dp[1][t] = C.dflip[1][xold[j] > 0 ? 0 : 1];
  }
  __syncthreads();
  for (int e = t; e < nF * nF; e += NT) {
    const int ia = e / nF, ib = e % nF;
    const int fa = flist[ia], fb = flist[ib];
    M0[ia * LD + ib] = (ia == ib ? 1.0 : 0.0) + A.g.W0[0][fa * kmax + fb] * dp[0][ib];
    M1[ia * LD + ib] = (ia == ib ? 1.0 : 0.0) + A.g.W0[1][fa * kmax + fb] * dp[1][ib];
  }
  __syncthreads();
  const double r0 = lds_gj_inverse<NT>(M0, LD, nF, colk, rowk, ipiv, &s_piv);
  const double r1 = lds_gj_inverse<NT>(M1, LD, nF, colk, rowk, ipiv, &s_piv);
  // prior ratio P(X'->X)/P(X->X') and the test, evaluated identically in every lane
  double lp = 0.0;
  for (int a = 0; a < nF; ++a) {
    const int j = flist[a];
    lp += sval[j] * (double)(xold[j] - xnew[j]);
  }
  const double prior = exp(lp);
  const double Rb = r0 * r1;
  const double absAb = fabs(Rb * prior);
  const bool nan_b = isnan(absAb);
  const bool acc_b = __builtin_amdgcn_readfirstlane((!nan_b && (u_mh < absAb)) ? 1 : 0) != 0;
  if (t == 0) {
    const double margin = absAb - u_mh;
    C.stats[kStProposed] += 1;
    C.stats[kStFieldUpdates] += kk;
    if (acc_b) { C.stats[kStAccepted] += 1; C.stats[kStFlips] += nF; }
    if (fabs(margin) < 1e-12) C.stats[kStLowMargin] += 1;
    if (Rb < 0.0) C.stats[kStNegative] += 1;
    if (nan_b) C.stats[kStError] |= kErrNonFinite;
    record_decision(C, C.log_base + A.block_index, A.g0, acc_b, margin);
    *A.g.nA = acc_b ? nF : 0;
  }
  if (acc_b) {
    if (t < nF) {
      const int j = flist[t];
      A.g.Alist[t] = j;
      A.g.Dsel[0][t] = dp[0][t];
      A.g.Dsel[1][t] = dp[1][t];
      C.fields[(long)C.li * C.N + A.g0 + j] = (int8_t)xnew[j];
    }
    for (int e = t; e < nF * nF; e += NT) {
      const int ia = e / nF, ib = e % nF;
      A.g.Minv[0][ia * kmax + ib] = M0[ia * LD + ib];
      A.g.Minv[1][ia * kmax + ib] = M1[ia * LD + ib];
    }
  }
}

// ------------------------------------------------------------------------
// flush: Q = P1_A diag(Delta_A) Minv, P2c = P2_A, U_R rows of accepted sites
// ------------------------------------------------------------------------
struct QArgs {
  SpinMats m;
  GroupBufs g;
  int g0;
};

__global__ __launch_bounds__(256) void group_q_kernel(QArgs a) {
  const int s = blockIdx.y;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int strip = blockIdx.x;
  if (strip >= nt) return;
  const int nA = *a.g.nA;
  if (nA == 0) return;
  const int kmax = a.g.kmax;
  const int t = threadIdx.x;
  const int r0 = strip * 64;
  const int w = min(64, Ns - r0);
  extern __shared__ double dyn_lds[];
  const int ldp = a.g.kmax + 1;
  for (int e = t; e < 64 * nA; e += 256) {
    const int rr = e / nA, m = e % nA;
    dyn_lds[rr * ldp + m] = (rr < w) ? a.g.P1[s][(long)(r0 + rr) * kmax + a.g.Alist[m]] * a.g.Dsel[s][m] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < 64 * nA; e += 256) {
    const int rr = e / nA, cc = e % nA;
    if (rr < w) {
      double v = 0.0;
      for (int m = 0; m < nA; ++m) v += dyn_lds[rr * ldp + m] * a.g.Minv[s][m * kmax + cc];
      a.g.Q[s][(long)(r0 + rr) * kmax + cc] = v;
    }
  }
  // compact P2 rows and scale the accepted rows of U_R over this column strip
  for (int e = t; e < nA * 64; e += 256) {
    const int m = e >> 6, cc = e & 63;
    if (cc < w) {
      const int j = a.g.Alist[m];
      a.g.P2c[s][(long)m * Ns + r0 + cc] = a.g.P2[s][(long)j * Ns + r0 + cc];
      a.m.UR[s][(long)(a.g0 + j) * Ns + r0 + cc] *= (1.0 + a.g.Dsel[s][m]);
    }
  }
}

// ------------------------------------------------------------------------
// fused group tile kernel: one 64x64 tile of T per workgroup, read once per
// group.  (1) applies the pending flush of the previous group,
//     T_tile -= (P1_A diag(Delta_A) M) P2_A,   M = (E_AA)^{-1}   (Eqs. (30)/(36)),
// and scales that group's accepted rows of U_R; (2) forms this tile's
// split-K contributions to the next group's panels P2 = U_g T and
// P1 = T L_g from the updated tile.  All products run on MFMA from LDS.
// ------------------------------------------------------------------------
struct TileArgs {
  SpinMats m;
  GroupBufs g;   // g.P1 / g.P2: panels of the pending (flushed) group
  int flush;     // apply the pending flush (its size is read from g.nA)
  int g0_prev;   // first site of the pending group
  int g0, kk;    // next group (kk == 0: flush only)
  int kpad;      // kmax rounded up to a multiple of 32
};

constexpr int kLdt = 65;   // padded LDS row stride

// acc (this wave's 32x32 quadrant of a 64x64 result) += A (64 x K) B (K x 64)
// with A, B in LDS; TB: B(k, j) = Bm[j * ldb + k].  Quadrants whose rows
// are >= mrows or columns >= ncols are skipped.
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

// (row, col) of accumulator element [mi][ni][j] in the 64x64 tile
__device__ __forceinline__ int acc_row(int wm, int mi, int lane, int j) {
  return wm * 32 + mi * 16 + (lane >> 4) + 4 * j;
}
__device__ __forceinline__ int acc_col(int wn, int ni, int lane) {
  return wn * 32 + ni * 16 + (lane & 15);
}

__device__ __forceinline__ void zero_acc(dbl4 (&a)[2][2]) {
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) a[mi][ni] = dbl4{0.0, 0.0, 0.0, 0.0};
}

constexpr int kPanMax = 16;   // panel elements per lane staged in registers (kpad <= 64)

__global__ __launch_bounds__(256) void group_tile_kernel(TileArgs a) {
  const int s = blockIdx.y;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int rb = blockIdx.x / nt, cb = blockIdx.x % nt;
  if (rb >= nt) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int row0 = rb * 64, col0 = cb * 64;
  const int kmax = a.g.kmax, kpad = a.kpad;
  const int kk = a.kk;
  double *T = a.m.T[s];
  extern __shared__ double lds[];
  double *X = lds;                       // 64 x kLdt
  double *Y = lds + 64 * kLdt;           // kpad x kLdt
  double *Z = Y + kpad * kLdt;           // kpad x kLdt
  __shared__ int al_s[64];
  __shared__ double dsel_s[64];

  // issue every independent load first: T tile, next group's panel rows, flush size
  dbl4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + acc_row(wm, mi, lane, j), c = col0 + acc_col(wn, ni, lane);
        acc[mi][ni][j] = (r < Ns && c < Ns) ? T[(long)r * Ns + c] : 0.0;
      }
  double ug[kPanMax], lg[kPanMax];
  if (kk > 0) {
    const double *UR = a.m.UR[s], *ULt = a.m.ULt[s];
#pragma unroll
    for (int i = 0; i < kPanMax; ++i) {
      const int e = t + 256 * i;
      const int m = e >> 6, c = e & 63;
      const bool ok = e < kpad * 64 && m < kk;
      ug[i] = (ok && row0 + c < Ns) ? UR[(long)(a.g0 + m) * Ns + row0 + c] : 0.0;
      lg[i] = (ok && col0 + c < Ns) ? ULt[(long)(a.g0 + m) * Ns + col0 + c] : 0.0;
    }
  }
  const int nA = a.flush ? __builtin_amdgcn_readfirstlane(*a.g.nA) : 0;

  if (nA > 0) {
    const double *P1 = a.g.P1[s], *P2 = a.g.P2[s], *Mi = a.g.Minv[s];
    if (t < nA) {
      al_s[t] = a.g.Alist[t];
      dsel_s[t] = a.g.Dsel[s][t];
    }
    __syncthreads();
    for (int e = t; e < 64 * kpad; e += 256) {
      const int r = e / kpad, m = e % kpad;
      X[r * kLdt + m] = (m < nA && row0 + r < Ns) ? -P1[(long)(row0 + r) * kmax + al_s[m]] * dsel_s[m] : 0.0;
    }
    for (int e = t; e < kpad * 64; e += 256) {
      const int m = e >> 6, c = e & 63;
      Y[m * kLdt + c] = (m < nA && c < nA) ? Mi[m * kmax + c] : 0.0;
      Z[m * kLdt + c] = (m < nA && col0 + c < Ns) ? P2[(long)al_s[m] * Ns + col0 + c] : 0.0;
    }
    __syncthreads();
    dbl4 q[2][2];
    zero_acc(q);
    lds_mma<false>(q, X, kLdt, Y, kLdt, nA, 64, nA, wm, wn, lane);   // Q = -P1_A D M
    __syncthreads();
    if (wn * 32 < nA) {
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            X[acc_row(wm, mi, lane, j) * kLdt + acc_col(wn, ni, lane)] = q[mi][ni][j];
    }
    __syncthreads();
    lds_mma<false>(acc, X, kLdt, Z, kLdt, nA, 64, 64, wm, wn, lane);  // T += Q P2_A
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = row0 + acc_row(wm, mi, lane, j), c = col0 + acc_col(wn, ni, lane);
          if (r < Ns && c < Ns) T[(long)r * Ns + c] = acc[mi][ni][j];
        }
    if (rb == 0) {
      // accepted rows of U_R over this tile's columns
      for (int e = t; e < nA * 64; e += 256) {
        const int m = e >> 6, c = col0 + (e & 63);
        if (c < Ns) a.m.UR[s][(long)(a.g0_prev + al_s[m]) * Ns + c] *= (1.0 + dsel_s[m]);
      }
    }
    __syncthreads();
  }

  if (kk <= 0) return;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        X[acc_row(wm, mi, lane, j) * kLdt + acc_col(wn, ni, lane)] = acc[mi][ni][j];
#pragma unroll
  for (int i = 0; i < kPanMax; ++i) {
    const int e = t + 256 * i;
    if (e < kpad * 64) {
      Y[(e >> 6) * kLdt + (e & 63)] = ug[i];
      Z[(e >> 6) * kLdt + (e & 63)] = lg[i];
    }
  }
  __syncthreads();
  dbl4 p[2][2];
  zero_acc(p);
  lds_mma<false>(p, Y, kLdt, X, kLdt, 64, kk, 64, wm, wn, lane);   // U_g[:, R] T_tile
  if (wm * 32 < kk) {
    double *out = a.g.P2part[s] + (long)rb * kmax * Ns;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = acc_row(wm, mi, lane, j), c = col0 + acc_col(wn, ni, lane);
          if (m < kk && c < Ns) out[(long)m * Ns + c] = p[mi][ni][j];
        }
  }
  zero_acc(p);
  lds_mma<true>(p, X, kLdt, Z, kLdt, 64, 64, kk, wm, wn, lane);    // T_tile L_g[C, :]
  if (wn * 32 < kk) {
    double *out = a.g.P1part[s] + (long)cb * Ns * kmax;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = row0 + acc_row(wm, mi, lane, j), m = acc_col(wn, ni, lane);
          if (r < Ns && m < kk) out[(long)r * kmax + m] = p[mi][ni][j];
        }
  }

}

}  // namespace

hipError_t local_step(const SpinMats &m, const LocalBufs &b, const SweepCtx &c, int i,
                      int nt_max, hipStream_t st) {
  LocalArgs a{m, b, c, i};
  hipLaunchKernelGGL(local_step_kernel, dim3(nt_max * nt_max, 2), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t group_panels(const SpinMats &m, const GroupBufs &g, int g0, int kk, hipStream_t st) {
  GemmBatch b2{}, b1{};
  for (int s = 0; s < 2; ++s) {
    const int Ns = m.Ns[s];
    GemmDesc d = gemm_desc(m.UR[s] + (long)g0 * Ns, Ns, m.T[s], Ns, g.P2part[s], Ns, kk, Ns, Ns);
    d.ksplit = 64;
    d.csplit = (long)g.kmax * Ns;
    b2.d[b2.count++] = d;
    GemmDesc e = gemm_desc(m.T[s], Ns, m.ULt[s] + (long)g0 * Ns, Ns, g.P1part[s], g.kmax, Ns, kk,
                           Ns);
    e.ksplit = 64;
    e.csplit = (long)Ns * g.kmax;
    b1.d[b1.count++] = e;
  }
  hipError_t err = gemm(b2, false, false, st);
  if (err != hipSuccess) return err;
  err = gemm(b1, false, true, st);
  if (err != hipSuccess) return err;
  const int nt = (max(m.Ns[0], m.Ns[1]) + 63) / 64;
  ReduceArgs ra{m, g, g0, kk};
  const size_t lds = sizeof(double) * 2 * 65 * (size_t)kk;
  static bool attr_set = false;
  if (!attr_set) {
    // up to 133 KB of LDS for kk = 128 (gfx950 has 160 KB per CU)
    hipError_t e = hipFuncSetAttribute((const void *)group_reduce_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * 2 * 65 * 128));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(group_reduce_kernel, dim3(nt, 2), dim3(kRedThreads), lds, st, ra);
  return hipGetLastError();
}

hipError_t delayed_decide(const GroupBufs &g, const SweepCtx &c, int g0, int kk,
                          hipStream_t st) {
  DecideArgs a{};
  a.g = g;
  a.c = c;
  a.g0 = g0;
  a.kk = kk;
  if (kk <= 8) hipLaunchKernelGGL((delayed_decide_kernel<64, 1>), dim3(1), dim3(64), 0, st, a);
  else if (kk <= 16) hipLaunchKernelGGL((delayed_decide_kernel<64, 4>), dim3(1), dim3(64), 0, st, a);
  else if (kk <= 32) hipLaunchKernelGGL((delayed_decide_kernel<256, 4>), dim3(1), dim3(256), 0, st, a);
  else if (kk <= 64) hipLaunchKernelGGL((delayed_decide_kernel<512, 8>), dim3(1), dim3(512), 0, st, a);
  else hipLaunchKernelGGL((delayed_decide_kernel<1024, 16>), dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t block_decide(const GroupBufs &g, const SweepCtx &c, int g0, int kk,
                        long long block_index, hipStream_t st) {
  DecideArgs a{};
  a.g = g;
  a.c = c;
  a.g0 = g0;
  a.kk = kk;
  a.block_index = block_index;
  const size_t lds = sizeof(double) * 2 * 64 * 65;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)block_decide_kernel<256>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)block_decide_kernel<64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (kk <= 16) hipLaunchKernelGGL((block_decide_kernel<64>), dim3(1), dim3(64), lds, st, a);
  else hipLaunchKernelGGL((block_decide_kernel<256>), dim3(1), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t group_tile(const SpinMats &m, const GroupBufs &g, bool flush, int g0_prev, int g0,
                      int kk, hipStream_t st) {
  TileArgs a{};
  a.m = m;
  a.g = g;
  a.flush = flush ? 1 : 0;
  a.g0_prev = g0_prev;
  a.g0 = g0;
  a.kk = kk;
  a.kpad = (g.kmax + 31) / 32 * 32;
  if (a.kpad > 64) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * kLdt * (64 + 2 * (size_t)a.kpad);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)group_tile_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * kLdt * (64 + 2 * 64)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int nt = (max(m.Ns[0], m.Ns[1]) + 63) / 64;
  hipLaunchKernelGGL(group_tile_kernel, dim3(nt * nt, 2), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t group_reduce(const SpinMats &m, const GroupBufs &g, int g0, int kk, hipStream_t st) {
  const int nt = (max(m.Ns[0], m.Ns[1]) + 63) / 64;
  ReduceArgs ra{m, g, g0, kk};
  const size_t lds = sizeof(double) * 2 * 65 * (size_t)kk;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)group_reduce_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * 2 * 65 * 128));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(group_reduce_kernel, dim3(nt, 2), dim3(kRedThreads), lds, st, ra);
  return hipGetLastError();
}

hipError_t group_flush(const SpinMats &m, const GroupBufs &g, int g0, int kk, hipStream_t st) {
  const int nt = (max(m.Ns[0], m.Ns[1]) + 63) / 64;
  QArgs qa{m, g, g0};
  const size_t lds = sizeof(double) * 64 * (size_t)(g.kmax + 1);
  hipLaunchKernelGGL(group_q_kernel, dim3(nt, 2), dim3(256), lds, st, qa);
  GemmBatch b{};
  for (int s = 0; s < 2; ++s) {
    const int Ns = m.Ns[s];
    GemmDesc d = gemm_desc(g.Q[s], g.kmax, g.P2c[s], Ns, m.T[s], Ns, Ns, Ns, kk, -1.0, 1.0,
                           m.T[s], Ns);
    d.Kdev = g.nA;
    b.d[b.count++] = d;
  }
  (void)kk;
  return gemm(b, false, false, st);
}

}  // namespace pq
