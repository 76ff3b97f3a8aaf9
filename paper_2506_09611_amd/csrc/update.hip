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
    const bool finite = isfinite(R);
    // every lane computes the same value; make it an explicit scalar
    const bool acc = __builtin_amdgcn_readfirstlane((finite && (u < absA)) ? 1 : 0) != 0;
    const double rs = s ? r1 : r0;
    if (acc) {
      // x_r = (T v)_r / r over all column tiles; y_c over all row tiles
      double yc = 0.0;
      if (colok)
        for (int b2 = 0; b2 < nt; ++b2) yc += a.b.ypart[s][par][(long)b2 * Ns + col];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int r = row0 + rq + 4 * q;
        if (r < Ns) {
          double xr = 0.0;
          for (int b2 = 0; b2 < nt; ++b2) xr += a.b.tpart[s][par][(long)b2 * Ns + r];
          tv[q] -= (xr / rs) * yc;
        }
      }
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

__global__ __launch_bounds__(256) void group_reduce_kernel(ReduceArgs a) {
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
  for (int e = t; e < kk * 64; e += 256) {
    const int mrow = e >> 6, cc = e & 63;
    double v = 0.0, l = 0.0;
    if (cc < w) {
      const long off = (long)mrow * Ns + c0 + cc;
      for (int sp = 0; sp < nt; ++sp) v += a.g.P2part[s][(long)sp * kmax * Ns + off];
      a.g.P2[s][off] = v;
      l = a.m.ULt[s][(long)(a.g0 + mrow) * Ns + c0 + cc];
    }
    p2s[mrow][cc] = v;
    lgs[mrow][cc] = l;
  }
  // P1[strip rows, :]
  for (int e = t; e < 64 * kk; e += 256) {
    const int rr = e / kk, mcol = e % kk;
    if (rr < w) {
      const long off = (long)(c0 + rr) * kmax + mcol;
      double v = 0.0;
      for (int sp = 0; sp < nt; ++sp) v += a.g.P1part[s][(long)sp * Ns * kmax + off];
      a.g.P1[s][off] = v;
    }
  }
  __syncthreads();
  // W0 partial over this strip: sum_c P2[m1][c] L_g[m2][c]
  for (int e = t; e < kk * kk; e += 256) {
    const int m1 = e / kk, m2 = e % kk;
    double v = 0.0;
    for (int cc = 0; cc < 64; ++cc) v += p2s[m1][cc] * lgs[m2][cc];
    a.g.W0part[s][(long)strip * kmax * kmax + m1 * kmax + m2] = v;
  }
}

// ------------------------------------------------------------------------
// decision kernels (one workgroup of 1024 threads)
// ------------------------------------------------------------------------
constexpr int kDecThreads = 1024;

struct DecideArgs {
  GroupBufs g;
  SweepCtx c;
  int g0, kk;
  long long block_index;
};

// sum of the W0 strip partials for element (a, b)
__device__ __forceinline__ double w0_elem(const DecideArgs &A, int s, int a, int b) {
  const int nt = (A.g.Ns[s] + 63) / 64;
  const int kmax = A.g.kmax;
  double v = 0.0;
  for (int sp = 0; sp < nt; ++sp) v += A.g.W0part[s][(long)sp * kmax * kmax + a * kmax + b];
  return v;
}

// kDecQ = ceil(kk * kk / 1024) elements of each spin's E per thread.
template <int kDecQ>
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
  // owned elements of E_s = 1 + W0_s diag(Delta_s)
  double e0[kDecQ], e1[kDecQ];
#pragma unroll
  for (int q = 0; q < kDecQ; ++q) {
    const int e = t + kDecThreads * q;
    e0[q] = e1[q] = 0.0;
    if (e < kk * kk) {
      const int ia = e / kk, ib = e % kk;
      e0[q] = (ia == ib ? 1.0 : 0.0) + w0_elem(A, 0, ia, ib) * dl[0][ib];
      e1[q] = (ia == ib ? 1.0 : 0.0) + w0_elem(A, 1, ia, ib) * dl[1][ib];
      if (ib == 0) { colb[0][0][ia] = e0[q]; colb[1][0][ia] = e1[q]; }
      if (ia == 0) { rowb[0][0][ib] = e0[q]; rowb[1][0][ib] = e1[q]; }
    }
  }
  __syncthreads();
  for (int j = 0; j < kk; ++j) {
    const int par = j & 1, nxt = par ^ 1;
    const double p0 = colb[0][par][j], p1 = colb[1][par][j];
    const double R = p0 * p1;
    const double absA = fabs(R);
    const bool finite = isfinite(R);
    const bool acc = __builtin_amdgcn_readfirstlane((finite && (uni[j] < absA)) ? 1 : 0) != 0;
    if (t == 0) {
      const double margin = absA - uni[j];
      C.stats[kStProposed] += 1;
      C.stats[kStFieldUpdates] += 1;
      if (acc) { C.stats[kStAccepted] += 1; C.stats[kStFlips] += 1; }
      if (fabs(margin) < 1e-12) C.stats[kStLowMargin] += 1;
      if (R < 0.0) C.stats[kStNegative] += 1;
      if (!finite) C.stats[kStError] |= kErrNonFinite;
      record_decision(C, C.log_base + A.g0 + j, A.g0 + j, acc, margin);
      acc_s[j] = acc ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < kDecQ; ++q) {
      const int e = t + kDecThreads * q;
      if (e < kk * kk) {
        const int ia = e / kk, ib = e % kk;
        if (acc) {
          // principal pivot transform on pivot j, both spins
          const double ca0 = colb[0][par][ia], rb0 = rowb[0][par][ib];
          const double ca1 = colb[1][par][ia], rb1 = rowb[1][par][ib];
          if (ia == j && ib == j) { e0[q] = -1.0 / p0; e1[q] = -1.0 / p1; }
          else if (ib == j) { e0[q] = ca0 / p0; e1[q] = ca1 / p1; }
          else if (ia == j) { e0[q] = rb0 / p0; e1[q] = rb1 / p1; }
          else { e0[q] -= ca0 * rb0 / p0; e1[q] -= ca1 * rb1 / p1; }
        }
        if (j + 1 < kk) {
          if (ib == j + 1) { colb[0][nxt][ia] = e0[q]; colb[1][nxt][ia] = e1[q]; }
          if (ia == j + 1) { rowb[0][nxt][ib] = e0[q]; rowb[1][nxt][ib] = e1[q]; }
        }
      }
    }
    __syncthreads();
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
    const int e = t + kDecThreads * q;
    if (e < kk * kk) {
      const int ia = e / kk, ib = e % kk;
      const int pa = pos[ia], pb = pos[ib];
      if (pa >= 0 && pb >= 0) {
        A.g.Minv[0][pa * kmax + pb] = -e0[q];
        A.g.Minv[1][pa * kmax + pb] = -e1[q];
      }
    }
  }
}

__global__ __launch_bounds__(kDecThreads) void block_decide_kernel(DecideArgs A) {
  const int kk = A.kk;
  const int t = threadIdx.x;
  const SweepCtx &C = A.c;
  const int kmax = A.g.kmax;
  __shared__ double colb[2][2][64], rowb[2][2][64];
  __shared__ double db[2][64];
  __shared__ double prod[64][65];
  __shared__ double nbar[2][64];
  __shared__ double sval[64];
  __shared__ int xold[64], xnew[64];
  __shared__ int flist[64];
  __shared__ int s_nF;
  __shared__ double dp[2][64];
  __shared__ double pivprod[2];
  __shared__ double hb_margin_s[64];

  if (t < kk) {
    const int8_t x = C.fields[(long)C.li * C.N + A.g0 + t];
    xold[t] = x > 0 ? 1 : -1;
    db[0][t] = C.dremove[0][x > 0 ? 0 : 1];
    db[1][t] = C.dremove[1][x > 0 ? 0 : 1];
  }
  __syncthreads();
  // W0 (reduced, kept in global scratch for the flipped submatrix later);
  // owned element e <-> (ia, ib) holds E_ab = delta_ab + Db_a W0_ab and the
  // transposed W0_ba for the force-bias product.
  double e0[4], e1[4], wt0[4], wt1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + kDecThreads * q;
    e0[q] = e1[q] = wt0[q] = wt1[q] = 0.0;
    if (e < kk * kk) {
      const int ia = e / kk, ib = e % kk;
      const double w0 = w0_elem(A, 0, ia, ib), w1 = w0_elem(A, 1, ia, ib);
      A.g.W0[0][ia * kmax + ib] = w0;
      A.g.W0[1][ia * kmax + ib] = w1;
      wt0[q] = w0_elem(A, 0, ib, ia);
      wt1[q] = w0_elem(A, 1, ib, ia);
      e0[q] = (ia == ib ? 1.0 : 0.0) + db[0][ia] * w0;
      e1[q] = (ia == ib ? 1.0 : 0.0) + db[1][ia] * w1;
      if (ib == 0) { colb[0][0][ia] = e0[q]; colb[1][0][ia] = e1[q]; }
      if (ia == 0) { rowb[0][0][ib] = e0[q]; rowb[1][0][ib] = e1[q]; }
    }
  }
  __syncthreads();
  // invert E by sweeping every pivot: afterwards e = -(E^{-1})_ab
  for (int j = 0; j < kk; ++j) {
    const int par = j & 1, nxt = par ^ 1;
    const double p0 = colb[0][par][j], p1 = colb[1][par][j];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + kDecThreads * q;
      if (e < kk * kk) {
        const int ia = e / kk, ib = e % kk;
        const double ca0 = colb[0][par][ia], rb0 = rowb[0][par][ib];
        const double ca1 = colb[1][par][ia], rb1 = rowb[1][par][ib];
        if (ia == j && ib == j) { e0[q] = -1.0 / p0; e1[q] = -1.0 / p1; }
        else if (ib == j) { e0[q] = ca0 / p0; e1[q] = ca1 / p1; }
        else if (ia == j) { e0[q] = rb0 / p0; e1[q] = rb1 / p1; }
        else { e0[q] -= ca0 * rb0 / p0; e1[q] -= ca1 * rb1 / p1; }
        if (j + 1 < kk) {
          if (ib == j + 1) { colb[0][nxt][ia] = e0[q]; colb[1][nxt][ia] = e1[q]; }
          if (ia == j + 1) { rowb[0][nxt][ib] = e0[q]; rowb[1][nxt][ib] = e1[q]; }
        }
      }
    }
    __syncthreads();
  }
  // nbar_b = (1 + Db_b) sum_a W0_ba (E^{-1})_ab, per spin (column sums of the products)
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + kDecThreads * q;
      if (e < kk * kk) {
        const int ia = e / kk, ib = e % kk;
        prod[ia][ib] = s ? (-e1[q] * wt1[q]) : (-e0[q] * wt0[q]);
      }
    }
    __syncthreads();
    if (t < kk) {
      double v = 0.0;
      for (int ia = 0; ia < kk; ++ia) v += prod[ia][t];
      nbar[s][t] = (1.0 + db[s][t]) * v;
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
    hb_margin_s[t] = margin;
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
    for (int j = 0; j < kk; ++j)
      if (fabs(hb_margin_s[j]) < 1e-12) ++low;
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
  // E' = 1 + W0_FF diag(Delta'_F), Delta'_i = e^{-2 alpha f_s x_i} - 1; det by pivot sweep
  if (t < nF) {
    const int j = flist[t];
    dp[0][t] = C.dflip[0][xold[j] > 0 ? 0 : 1];
    dp[1][t] = C.dflip[1][xold[j] > 0 ? 0 : 1];
  }
  if (t == 0) { pivprod[0] = 1.0; pivprod[1] = 1.0; }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = t + kDecThreads * q;
    e0[q] = e1[q] = 0.0;
    if (e < nF * nF) {
      const int ia = e / nF, ib = e % nF;
      const int fa = flist[ia], fb = flist[ib];
      e0[q] = (ia == ib ? 1.0 : 0.0) + A.g.W0[0][fa * kmax + fb] * dp[0][ib];
      e1[q] = (ia == ib ? 1.0 : 0.0) + A.g.W0[1][fa * kmax + fb] * dp[1][ib];
      if (ib == 0) { colb[0][0][ia] = e0[q]; colb[1][0][ia] = e1[q]; }
      if (ia == 0) { rowb[0][0][ib] = e0[q]; rowb[1][0][ib] = e1[q]; }
    }
  }
  __syncthreads();
  for (int j = 0; j < nF; ++j) {
    const int par = j & 1, nxt = par ^ 1;
    const double p0 = colb[0][par][j], p1 = colb[1][par][j];
    if (t == 0) { pivprod[0] *= p0; pivprod[1] *= p1; }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + kDecThreads * q;
      if (e < nF * nF) {
        const int ia = e / nF, ib = e % nF;
        const double ca0 = colb[0][par][ia], rb0 = rowb[0][par][ib];
        const double ca1 = colb[1][par][ia], rb1 = rowb[1][par][ib];
        if (ia == j && ib == j) { e0[q] = -1.0 / p0; e1[q] = -1.0 / p1; }
        else if (ib == j) { e0[q] = ca0 / p0; e1[q] = ca1 / p1; }
        else if (ia == j) { e0[q] = rb0 / p0; e1[q] = rb1 / p1; }
        else { e0[q] -= ca0 * rb0 / p0; e1[q] -= ca1 * rb1 / p1; }
        if (j + 1 < nF) {
          if (ib == j + 1) { colb[0][nxt][ia] = e0[q]; colb[1][nxt][ia] = e1[q]; }
          if (ia == j + 1) { rowb[0][nxt][ib] = e0[q]; rowb[1][nxt][ib] = e1[q]; }
        }
      }
    }
    __syncthreads();
  }
  // prior ratio P(X'->X)/P(X->X') and the test, evaluated identically in every lane
  double lp = 0.0;
  for (int a = 0; a < nF; ++a) {
    const int j = flist[a];
    lp += sval[j] * (double)(xold[j] - xnew[j]);
  }
  const double prior = exp(lp);
  const double Rb = pivprod[0] * pivprod[1];
  const double absAb = fabs(Rb * prior);
  const bool finite_b = isfinite(absAb);
  const bool acc_b = __builtin_amdgcn_readfirstlane((finite_b && (u_mh < absAb)) ? 1 : 0) != 0;
  if (t == 0) {
    const double margin = absAb - u_mh;
    C.stats[kStProposed] += 1;
    C.stats[kStFieldUpdates] += kk;
    if (acc_b) { C.stats[kStAccepted] += 1; C.stats[kStFlips] += nF; }
    if (fabs(margin) < 1e-12) C.stats[kStLowMargin] += 1;
    if (Rb < 0.0) C.stats[kStNegative] += 1;
    if (!finite_b) C.stats[kStError] |= kErrNonFinite;
    record_decision(C, C.log_base + A.block_index, A.g0, acc_b, margin);
    *A.g.nA = acc_b ? nF : 0;
  }
  if (acc_b && t < nF) {
    const int j = flist[t];
    A.g.Alist[t] = j;
    A.g.Dsel[0][t] = dp[0][t];
    A.g.Dsel[1][t] = dp[1][t];
    C.fields[(long)C.li * C.N + A.g0 + j] = (int8_t)xnew[j];
  }
  if (acc_b) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + kDecThreads * q;
      if (e < nF * nF) {
        const int ia = e / nF, ib = e % nF;
        A.g.Minv[0][ia * kmax + ib] = -e0[q];
        A.g.Minv[1][ia * kmax + ib] = -e1[q];
      }
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
  hipLaunchKernelGGL(group_reduce_kernel, dim3(nt, 2), dim3(256), lds, st, ra);
  return hipGetLastError();
}

hipError_t delayed_decide(const GroupBufs &g, const SweepCtx &c, int g0, int kk,
                          hipStream_t st) {
  DecideArgs a{};
  a.g = g;
  a.c = c;
  a.g0 = g0;
  a.kk = kk;
  const int q = (kk * kk + kDecThreads - 1) / kDecThreads;
  if (q <= 1) hipLaunchKernelGGL(delayed_decide_kernel<1>, dim3(1), dim3(kDecThreads), 0, st, a);
  else if (q <= 2) hipLaunchKernelGGL(delayed_decide_kernel<2>, dim3(1), dim3(kDecThreads), 0, st, a);
  else if (q <= 4) hipLaunchKernelGGL(delayed_decide_kernel<4>, dim3(1), dim3(kDecThreads), 0, st, a);
  else if (q <= 8) hipLaunchKernelGGL(delayed_decide_kernel<8>, dim3(1), dim3(kDecThreads), 0, st, a);
  else hipLaunchKernelGGL(delayed_decide_kernel<16>, dim3(1), dim3(kDecThreads), 0, st, a);
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
  hipLaunchKernelGGL(block_decide_kernel, dim3(1), dim3(kDecThreads), 0, st, a);
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
