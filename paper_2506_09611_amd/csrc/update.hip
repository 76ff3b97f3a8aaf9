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

#include <algorithm>

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

// One 256-thread workgroup per 64 x 64 tile of T (16 elements a thread); the
// flat grid covers (walker, spin, tile) with nt_max^2 tiles per matrix and is
// padded to a multiple of 8.  XCD-aware: consecutive workgroup ids go
// round-robin to the 8 XCDs, so XCD x takes the contiguous range
// [x per, (x + 1) per) of matrix tiles, and the split-K partials of one
// matrix, which all of its tiles read, are fetched into one L2 rather than
// eight.  At most 128 VGPRs: four workgroups per CU.
__global__ __launch_bounds__(256, 4) void local_step_kernel(Batch<LocalArgs> B, int nt2,
                                                            int total) {
  const int per = (int)(gridDim.x >> 3);
  const int lid = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (lid >= total) return;
  const int mat = lid / nt2;
  const LocalArgs &a = B.w[mat >> 1];
  const int s = mat & 1;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int tile = lid - mat * nt2;
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

  // unconditional loads from clamped addresses (all sixteen in flight), the
  // elements outside T zeroed afterwards
  double tv[16];
  const int colc = min(col, Ns - 1);
#pragma unroll
  for (int q = 0; q < 16; ++q) tv[q] = T[(long)min(row0 + rq + 4 * q, Ns - 1) * Ns + colc];
#pragma unroll
  for (int q = 0; q < 16; ++q) tv[q] = (row0 + rq + 4 * q < Ns && colok) ? tv[q] : 0.0;
  bool dirty = false;

  if (i > 0) {
    const int par = (i - 1) & 1;
    // r_s = 1 + sum over tiles of u^T T_tile v, same order in every workgroup
    if (rq < 2) {
      const int ss = rq;
      const int nts = (a.m.Ns[ss] + 63) / 64;
      const int ntot = nts * nts;
      // added in the order e = lane, lane + 64, ...; four loads in flight
      const double *sp = a.b.spart[ss][par];
      double p = 0.0;
      for (int e0 = lane; e0 < ntot; e0 += 256) {
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = sp[min(e0 + 64 * q, ntot - 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (e0 + 64 * q < ntot) p += v[q];
      }
      p = wave_sum(p);
      if (lane == 0) s_r[ss] = 1.0 + p;
    }
    __syncthreads();
    const double r0 = s_r[0], r1 = s_r[1];
    const double R = r0 * r1;
    const double absA = fabs(R);
    const double u = C.force ? forced_uniform(C.force[i - 1] != 0)
                             : philox_uniform(C.key0, C.key1, sweep_of(C.sweep, C.sweep_dev),
                                              C.slice_code,
                                              (uint64_t)(i - 1), kPurposeMH);
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
    const double *urow = a.m.UR[s] + (long)i * Ns;
#pragma unroll
    for (int q = 0; q < 16; ++q) ur[q] = urow[min(row0 + rq + 4 * q, Ns - 1)];
#pragma unroll
    for (int q = 0; q < 16; ++q) ur[q] = (row0 + rq + 4 * q < Ns) ? ur[q] : 0.0;
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
// group panels: sums of the split-K partials of P1, P2 and W0
// ------------------------------------------------------------------------
// Column chunks per row strip of the tile kernel (one P1 partial each) for a
// matrix of nt column strips when `want` chunks are asked for: the
// chunks are ceil(nt / c) strips wide, and only non-empty ones count.
__host__ __device__ inline int strip_chunk_width(int nt, int want) {
  const int c = min(max(want, 1), nt);
  return (nt + c - 1) / c;
}
__host__ __device__ inline int strip_chunks(int nt, int want) {
  const int per = strip_chunk_width(nt, want);
  return (nt + per - 1) / per;
}

struct ReduceArgs {
  SpinMats m;
  GroupBufs g;
  int g0, kk;
  int ntm_all;               // column strips of the launch (largest walker)
  int do_panels;             // sum the split-K partials of P1 and P2
  int w0_mode;               // W0 partials to add: 0 none, 1 from the tile kernel (nt x
                             // strip_chunks(nt, g.chunks), and P1 then has
                             // strip_chunks(nt, g.chunks)), 2 per strip (nt)
  int mode;                  // UniMode: uniforms drawn for the following decision
  uint64_t key0, key1, sweep, slice_code;
  const int8_t *force;       // replay: forced outcomes of the slice visit (or null)
  const int8_t *xrow;        // the slice's fields (forced heat-bath proposals)
  const uint64_t *sweep_dev; // graph-captured sweeps: the sweep counter on the device
};

constexpr int kRedThreads = 256;
constexpr int kRedParts = 4;       // panel workgroups per (column strip, spin)
constexpr int kRedChunk = 16;      // partials loaded together per element

// p[0] + p[stride] + ... + p[(n-1) stride], added in index order, for two
// independent elements at once so that all their loads are in flight together.
__device__ __forceinline__ void sum_pair(const double *p, const double *q, bool pv, bool qv,
                                         long stride, int n, double &sp, double &sq) {
  sp = 0.0;
  sq = 0.0;
  for (int b = 0; b < n; b += kRedChunk) {
    double vp[kRedChunk], vq[kRedChunk];
#pragma unroll
    for (int i = 0; i < kRedChunk; ++i) {
      const bool in = b + i < n;
      vp[i] = (pv && in) ? p[(long)(b + i) * stride] : 0.0;
      vq[i] = (qv && in) ? q[(long)(b + i) * stride] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kRedChunk; ++i) {
      if (b + i < n) {
        sp += vp[i];
        sq += vq[i];
      }
    }
  }
}

// Sums of the split-K partials of a group's panels over column strip
// `strip`, share `part` of kRedParts, by the NT threads of one workgroup:
// P2 rows [m0, m1) (one partial per row strip of T, added in order) and P1
// rows of the strip (np1 partials).  Every element is summed by one thread
// in a fixed order, so the sums do not depend on the launch that runs them.
template <int NT>
__device__ void panel_sums(const GroupBufs &g, int s, int kk, int strip, int part, int np1) {
  const int t = threadIdx.x;
  const int Ns = g.Ns[s], kmax = g.kmax;
  const int nt = (Ns + 63) / 64;
  if (strip >= nt) return;
  const int c0 = strip * 64;
  const int w = min(64, Ns - c0);
  const int mper = (kk + kRedParts - 1) / kRedParts;
  const int m0 = part * mper, m1 = min(kk, m0 + mper);
  const int r0 = part * (64 / kRedParts), r1 = min(w, r0 + 64 / kRedParts);
  // P2 rows [m0, m1) over the strip
  const int n2 = max(0, m1 - m0) * 64;
  for (int e = t; e < n2; e += 2 * NT) {
    const int e2 = e + NT;
    const int ma = m0 + (e >> 6), ca = e & 63;
    const int mb = m0 + (e2 >> 6), cb = e2 & 63;
    const bool va = ca < w, vb = e2 < n2 && cb < w;
    const long oa = (long)ma * Ns + c0 + ca, ob = (long)mb * Ns + c0 + cb;
    double sa, sb;
    sum_pair(g.P2part[s] + oa, g.P2part[s] + (vb ? ob : oa), va, vb, (long)kmax * Ns, nt, sa, sb);
    if (va) g.P2[s][oa] = sa;
    if (vb) g.P2[s][ob] = sb;
  }
  // P1 rows [c0 + r0, c0 + r1)
  const int n1 = max(0, r1 - r0) * kk;
  for (int e = t; e < n1; e += 2 * NT) {
    const int e2 = e + NT;
    const long oa = (long)(c0 + r0 + e / kk) * kmax + e % kk;
    const long ob = (long)(c0 + r0 + e2 / kk) * kmax + e2 % kk;
    const bool vb = e2 < n1;
    double sa, sb;
    sum_pair(g.P1part[s] + oa, g.P1part[s] + (vb ? ob : oa), true, vb, (long)Ns * kmax, np1, sa,
             sb);
    g.P1[s][oa] = sa;
    if (vb) g.P1[s][ob] = sb;
  }
}

// Grid (nP + nW + 1, 2 spins) with nP = nt * kRedParts panel workgroups and
// nW = kk W0 workgroups per spin.  Panel workgroup (strip, part) sums its
// share of the split-K partials of P2[:, strip] (rows of P2) and of
// P1[strip rows, :]; W0 workgroup m adds the partials of row m of W0 in a
// fixed order; the last workgroup (spin 0) draws the group's uniforms.  No
// workgroup depends on another.
__global__ __launch_bounds__(kRedThreads) void group_reduce_kernel(Batch<ReduceArgs> B) {
  const ReduceArgs &a = B.w[blockIdx.z];
  const int s = blockIdx.y;
  const int t = threadIdx.x;
  const int kk = a.kk, kmax = a.g.kmax;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int np1 = a.w0_mode == 1 ? strip_chunks(nt, a.g.chunks) : nt;   // P1 partials
  const int nP = a.do_panels ? a.ntm_all * kRedParts : 0;
  const int nW = a.w0_mode ? kk : 0;
  const int x = blockIdx.x;
  if (kk <= 0) return;   // this walker has no group here (uneven batch)
  if (x == (int)gridDim.x - 1) {
    if (s == 0 && a.mode != kUniNone && a.force) {
      // replay: delayed sites accepted iff listed; block proposals set to the
      // listed fields and the block's Metropolis test accepted
      if (t < kk) {
        const bool fl = a.force[a.g0 + t] != 0;
        const int x = a.xrow[a.g0 + t];
        a.g.uni[t] = a.mode == kUniDelayed ? forced_uniform(fl) : forced_uniform((fl ? -x : x) > 0);
      }
      if (a.mode == kUniBlock && t == kk) a.g.uni[kk] = forced_uniform(true);
    } else if (s == 0 && a.mode != kUniNone) {
      const uint64_t purpose = a.mode == kUniDelayed ? kPurposeMH : kPurposeHB;
      const uint64_t sw = sweep_of(a.sweep, a.sweep_dev);
      if (t < kk)
        a.g.uni[t] = philox_uniform(a.key0, a.key1, sw, a.slice_code, (uint64_t)(a.g0 + t),
                                    purpose);
      if (a.mode == kUniBlock && t == kk)
        a.g.uni[kk] = philox_uniform(a.key0, a.key1, sw, a.slice_code, (uint64_t)a.g0,
                                     kPurposeMH);
    }
    return;
  }
  if (x >= nP) {
    // ---- row m of W0: partials added with lane group q taking partials
    // q, q + 4, ... in order, then the four groups in order
    const int mrow = x - nP;
    if (mrow >= nW) return;
    __shared__ double red[4][64];
    const long stride = (long)kmax * kmax;
    // W0 partials: one per (row strip, column chunk) from the tile kernel,
    // one per column strip from the split-K GEMM
    const int np = a.w0_mode == 1 ? nt * strip_chunks(nt, a.g.chunks) : nt;
    const int q = t >> 6, ln = t & 63;
    for (int n0 = 0; n0 < kk; n0 += 64) {
      const int n = n0 + ln;
      const double *p = a.g.W0part[s] + mrow * kmax + n;
      double sum = 0.0;
      for (int b = q; b < np; b += 4 * kRedChunk) {
        double v[kRedChunk];
#pragma unroll
        for (int i = 0; i < kRedChunk; ++i) {
          const int pi = b + 4 * i;
          v[i] = (n < kk && pi < np) ? p[(long)pi * stride] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kRedChunk; ++i)
          if (b + 4 * i < np) sum += v[i];
      }
      red[q][ln] = sum;
      __syncthreads();
      if (q == 0 && n < kk)
        a.g.W0[s][mrow * kmax + n] = ((red[0][ln] + red[1][ln]) + red[2][ln]) + red[3][ln];
      __syncthreads();
    }
    return;
  }
  // ---- panel workgroup
  panel_sums<kRedThreads>(a.g, s, kk, x / kRedParts, x % kRedParts, np1);
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

// Rows y > 0 of a decision launch's grid sum the group's panel partials for
// the next flush (row y - 1 = 2 (strip kRedParts + part) + spin), beside the
// decisions of row 0, which need only W0.
template <int NT>
__device__ __forceinline__ bool decide_panel_block(const DecideArgs &A) {
  if (blockIdx.y == 0) return false;
  const int q = blockIdx.y - 1, s = q & 1, x = q >> 1;
  if (A.kk > 0)
    panel_sums<NT>(A.g, s, A.kk, x / kRedParts, x % kRedParts,
                   strip_chunks((A.g.Ns[s] + 63) / 64, A.g.chunks));
  return true;
}


// kDecThreads lanes, kDecQ = ceil(kk * kk / kDecThreads) elements of each
// spin's E per lane (kk <= kDecThreads).
template <int kDecThreads, int kDecQ>
__global__ __launch_bounds__(kDecThreads) void delayed_decide_kernel(Batch<DecideArgs> B) {
  const DecideArgs &A = B.w[blockIdx.x];
  if (decide_panel_block<kDecThreads>(A)) return;
  if (A.kk <= 0) return;   // no group for this walker (uneven batch)
  const int kk = A.kk;
  const int t = threadIdx.x;
  const SweepCtx &C = A.c;
  __shared__ double colb[2][2][128], rowb[2][2][128];
  __shared__ double uni[128];
  __shared__ double dl[2][128];
  __shared__ int acc_s[128];

  if (t < kk) {
    const int site = A.g0 + t;
    const int8_t x = C.fields[(long)C.li * C.N + site];
    dl[0][t] = C.dflip[0][x > 0 ? 0 : 1];
    dl[1][t] = C.dflip[1][x > 0 ? 0 : 1];
    uni[t] = A.g.uni[t];
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
      e0[q] = (ia == ib ? 1.0 : 0.0) + A.g.W0[0][ia * A.g.kmax + ib] * dl[0][ib];
      e1[q] = (ia == ib ? 1.0 : 0.0) + A.g.W0[1][ia * A.g.kmax + ib] * dl[1][ib];
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
  // row scales and flipped fields, one lane per site
  if (t < kk) {
    const int mine = acc_s[t];
    A.g.sc[0][t] = mine ? 1.0 + dl[0][t] : 1.0;
    A.g.sc[1][t] = mine ? 1.0 + dl[1][t] : 1.0;
    if (mine) C.fields[(long)C.li * C.N + A.g0 + t] = (int8_t)(-C.fields[(long)C.li * C.N + A.g0 + t]);
    if (mine) {   // the accepted sites in order
      int pos = 0;
      for (int m = 0; m < t; ++m) pos += acc_s[m];
      A.g.alist[pos] = t;
    }
  }
  if (t == 0) {
    A.g.nA[0] = (int)n_acc;
    A.g.nA[1] = n_acc ? kk : 0;
  }
  // Mc = diag(Delta_A) (E_AA)^{-1} = -diag(Delta_A) (swept E)_AA, zero elsewhere
  const int kmax = A.g.kmax;
#pragma unroll
  for (int q = 0; q < kDecQ; ++q) {
    const int ia = ra[q], ib = cb_[q];
    if (ia < kk) {
      const bool in = acc_s[ia] && acc_s[ib];
      A.g.Mc[0][ia * kmax + ib] = in ? -dl[0][ia] * e0[q] : 0.0;
      A.g.Mc[1][ia * kmax + ib] = in ? -dl[1][ia] * e1[q] : 0.0;
    }
  }
}

// Value of v in lane src (uniform src): the result is a wave-uniform scalar.
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1/p to full double precision for the pivots of the decision kernels:
// hardware reciprocal estimate refined by two Newton steps (p is a finite,
// nonzero pivot of an accepted proposal).
__device__ __forceinline__ double recip(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  return fma(r, fma(-p, r, 1.0), r);
}

// Delayed decision for kk <= KK <= 32 sites in a single wave.  The whole of
// E_s = 1 + W0_s diag(Delta_s), both spins, stays in registers: lane
// (ra, cb) = (lane / 8, lane % 8) holds rows ra + 8 i and columns cb + 8 j,
// i, j < KK / 8.  Each decision reads its pivot's row and column with
// cross-lane permutes and, when accepted, sweeps the pivot out of every
// element (principal pivot transform), so decisions follow one another
// without barriers or shared-memory round trips.
template <int KK>
__global__ __launch_bounds__(64) void delayed_decide_wave_kernel(Batch<DecideArgs> B) {
  const DecideArgs &A = B.w[blockIdx.x];
  if (decide_panel_block<64>(A)) return;
  if (A.kk <= 0) return;   // no group for this walker (uneven batch)
  constexpr int R = KK / 8;
  static_assert(KK % 8 == 0 && R >= 1 && R <= 4, "tile shape");
  const int kk = A.kk;
  const int lane = threadIdx.x;
  const int ra = lane >> 3, cb = lane & 7;
  const SweepCtx &C = A.c;
  const int kmax = A.g.kmax;
  const int8_t *xrow = C.fields + (long)C.li * C.N + A.g0;

  // the group's uniforms and field values, one lane per site
  const double ul = lane < kk ? A.g.uni[lane] : 0.0;
  const int8_t xl = lane < kk ? xrow[lane] : 1;
  double e0[R][R], e1[R][R];
  double da0[R], da1[R];   // Delta of this lane's rows, from the fields before any flip
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int a = ra + 8 * i;
    const int8_t xa = a < kk ? xrow[a] : 1;
    da0[i] = C.dflip[0][xa > 0 ? 0 : 1];
    da1[i] = C.dflip[1][xa > 0 ? 0 : 1];
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int a = ra + 8 * i, b = cb + 8 * j;
      const bool ok = a < kk && b < kk;
      const int8_t xb = ok ? xrow[b] : 1;
      const double w0 = ok ? A.g.W0[0][a * kmax + b] : 0.0;
      const double w1 = ok ? A.g.W0[1][a * kmax + b] : 0.0;
      e0[i][j] = (a == b ? 1.0 : 0.0) + w0 * C.dflip[0][xb > 0 ? 0 : 1];
      e1[i][j] = (a == b ? 1.0 : 0.0) + w1 * C.dflip[1][xb > 0 ? 0 : 1];
    }

  unsigned long long amask = 0;   // accepted sites (uniform)
  unsigned long long n_low = 0, n_neg = 0;
  bool any_nan = false;
  double my_margin = 0.0;         // lane j: the margin of site j (logged after the loop)
#pragma unroll
  for (int J = 0; J < R; ++J) {
    for (int jl = 0; jl < 8; ++jl) {
      const int j = 8 * J + jl;
      if (j >= kk) break;
      const int src_c = ra * 8 + jl, src_r = jl * 8 + cb;
      double c0[R], c1[R], r0[R], r1[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        c0[i] = __shfl(e0[i][J], src_c, 64);
        c1[i] = __shfl(e1[i][J], src_c, 64);
        r0[i] = __shfl(e0[J][i], src_r, 64);
        r1[i] = __shfl(e1[J][i], src_r, 64);
      }
      const double p0 = readlane_f64(e0[J][J], jl * 9), p1 = readlane_f64(e1[J][J], jl * 9);
      // used only on acceptance; computed here, off the decision's critical path
      const double ip0 = recip(p0), ip1 = recip(p1);
      asm volatile("" ::"v"(ip0), "v"(ip1));
      const double u = readlane_f64(ul, j);
      const double Rr = p0 * p1;
      const double absA = fabs(Rr);
      const bool finite = !isnan(absA);
      const bool acc = __builtin_amdgcn_readfirstlane((finite && (u < absA)) ? 1 : 0) != 0;
      const double margin = absA - u;
      n_low += (fabs(margin) < 1e-12) ? 1 : 0;
      n_neg += (Rr < 0.0) ? 1 : 0;
      any_nan = any_nan || !finite;
      my_margin = lane == j ? margin : my_margin;
      if (acc) {
        amask |= 1ull << j;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const double ci0 = c0[i] * ip0, ci1 = c1[i] * ip1;
#pragma unroll
          for (int jp = 0; jp < R; ++jp) {
            e0[i][jp] -= ci0 * r0[jp];
            e1[i][jp] -= ci1 * r1[jp];
          }
        }
        if (ra == jl) {   // pivot row: E_jb / p
#pragma unroll
          for (int jp = 0; jp < R; ++jp) {
            e0[J][jp] = r0[jp] * ip0;
            e1[J][jp] = r1[jp] * ip1;
          }
        }
        if (cb == jl) {   // pivot column: E_aj / p
#pragma unroll
          for (int i = 0; i < R; ++i) {
            e0[i][J] = c0[i] * ip0;
            e1[i][J] = c1[i] * ip1;
          }
        }
        if (lane == jl * 9) {
          e0[J][J] = -ip0;
          e1[J][J] = -ip1;
        }
      }
    }
  }
  const int n_acc = __popcll(amask);
  if (lane == 0) {
    C.stats[kStProposed] += kk;
    C.stats[kStFieldUpdates] += kk;
    C.stats[kStAccepted] += n_acc;
    C.stats[kStFlips] += n_acc;
    C.stats[kStLowMargin] += n_low;
    C.stats[kStNegative] += n_neg;
    if (any_nan) C.stats[kStError] |= kErrNonFinite;
    A.g.nA[0] = n_acc;
    A.g.nA[1] = n_acc ? kk : 0;
  }
  if (lane < kk)
    record_decision(C, C.log_base + A.g0 + lane, A.g0 + lane, (amask >> lane) & 1, my_margin);
  // row scales and flipped fields, one lane per site
  if (lane < kk) {
    const bool mine = (amask >> lane) & 1;
    A.g.sc[0][lane] = mine ? 1.0 + C.dflip[0][xl > 0 ? 0 : 1] : 1.0;
    A.g.sc[1][lane] = mine ? 1.0 + C.dflip[1][xl > 0 ? 0 : 1] : 1.0;
    if (mine) C.fields[(long)C.li * C.N + A.g0 + lane] = (int8_t)(-xl);
    if (mine) A.g.alist[__popcll(amask & ((1ull << lane) - 1))] = lane;   // A in order
  }
  // Mc = diag(Delta_A) (E_AA)^{-1} = -diag(Delta_A) (swept E)_AA, zero elsewhere
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int a = ra + 8 * i;
    if (a >= kk) continue;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int b = cb + 8 * j;
      if (b >= kk) continue;
      const bool in = ((amask >> a) & 1) && ((amask >> b) & 1);
      A.g.Mc[0][a * kmax + b] = in ? -da0[i] * e0[i][j] : 0.0;
      A.g.Mc[1][a * kmax + b] = in ? -da1[i] * e1[i][j] : 0.0;
    }
  }
}

// Delayed decision for kk <= KK <= 64 sites with one wave per spin sector.
// Wave s holds E_s = 1 + W0_s diag(Delta_s) in registers (lane (ra, cb) =
// (lane / 8, lane % 8) owns rows ra + 8 i and columns cb + 8 j, i, j < KK / 8)
// and sweeps accepted pivots out of it with cross-lane reads, as the
// single-wave kernel does for both spins; per site the two waves exchange
// their pivots through LDS (one barrier) and take the same decision.
template <int KK>
__global__ __launch_bounds__(128) void delayed_decide_spin_kernel(Batch<DecideArgs> B) {
  const DecideArgs &A = B.w[blockIdx.x];
  if (decide_panel_block<128>(A)) return;
  if (A.kk <= 0) return;   // no group for this walker (uneven batch)
  constexpr int R = KK / 8;
  static_assert(KK % 8 == 0 && R >= 1 && R <= 8, "tile shape");
  const int kk = A.kk;
  const int t = threadIdx.x, sp = t >> 6, lane = t & 63;
  const int ra = lane >> 3, cb = lane & 7;
  const SweepCtx &C = A.c;
  const int kmax = A.g.kmax;
  const int8_t *xrow = C.fields + (long)C.li * C.N + A.g0;
  __shared__ double piv[2][2];   // [site parity][spin]

  const double ul = lane < kk ? A.g.uni[lane] : 0.0;
  const int8_t xl = lane < kk ? xrow[lane] : 1;
  const double *W0 = A.g.W0[sp];
  double e[R][R];
  double da[R];   // Delta of this lane's rows, from the fields before any flip
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int a = ra + 8 * i;
    const int8_t xa = a < kk ? xrow[a] : 1;
    da[i] = C.dflip[sp][xa > 0 ? 0 : 1];
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int a = ra + 8 * i, b = cb + 8 * j;
      const bool ok = a < kk && b < kk;
      const int8_t xb = ok ? xrow[b] : 1;
      const double w = ok ? W0[a * kmax + b] : 0.0;
      e[i][j] = (a == b ? 1.0 : 0.0) + w * C.dflip[sp][xb > 0 ? 0 : 1];
    }

  unsigned long long amask = 0;   // accepted sites (uniform)
  unsigned long long n_low = 0, n_neg = 0;
  bool any_nan = false;
  double my_margin = 0.0;         // lane j: the margin of site j (logged after the loop)
#pragma unroll
  for (int J = 0; J < R; ++J) {
    for (int jl = 0; jl < 8; ++jl) {
      const int j = 8 * J + jl;
      if (j >= kk) break;
      const int src_c = ra * 8 + jl, src_r = jl * 8 + cb;
      double c[R], r[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        c[i] = __shfl(e[i][J], src_c, 64);
        r[i] = __shfl(e[J][i], src_r, 64);
      }
      const double p = readlane_f64(e[J][J], jl * 9);
      // used only on acceptance; computed here, while the pivots are exchanged
      const double ip = recip(p);
      asm volatile("" ::"v"(ip));
      if (lane == 0) piv[j & 1][sp] = p;
      __syncthreads();
      const double p0 = piv[j & 1][0], p1 = piv[j & 1][1];
      const double u = readlane_f64(ul, j);
      const double Rr = p0 * p1;
      const double absA = fabs(Rr);
      const bool finite = !isnan(absA);
      const bool acc = __builtin_amdgcn_readfirstlane((finite && (u < absA)) ? 1 : 0) != 0;
      const double margin = absA - u;
      n_low += (fabs(margin) < 1e-12) ? 1 : 0;
      n_neg += (Rr < 0.0) ? 1 : 0;
      any_nan = any_nan || !finite;
      my_margin = lane == j ? margin : my_margin;
      if (acc) {
        amask |= 1ull << j;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const double ci = c[i] * ip;
#pragma unroll
          for (int jp = 0; jp < R; ++jp) e[i][jp] -= ci * r[jp];
        }
        if (ra == jl) {   // pivot row: E_jb / p
#pragma unroll
          for (int jp = 0; jp < R; ++jp) e[J][jp] = r[jp] * ip;
        }
        if (cb == jl) {   // pivot column: E_aj / p
#pragma unroll
          for (int i = 0; i < R; ++i) e[i][J] = c[i] * ip;
        }
        if (lane == jl * 9) e[J][J] = -ip;
      }
    }
  }
  const int n_acc = __popcll(amask);
  if (t == 0) {
    C.stats[kStProposed] += kk;
    C.stats[kStFieldUpdates] += kk;
    C.stats[kStAccepted] += n_acc;
    C.stats[kStFlips] += n_acc;
    C.stats[kStLowMargin] += n_low;
    C.stats[kStNegative] += n_neg;
    if (any_nan) C.stats[kStError] |= kErrNonFinite;
    A.g.nA[0] = n_acc;
    A.g.nA[1] = n_acc ? kk : 0;
  }
  if (sp == 0 && lane < kk)
    record_decision(C, C.log_base + A.g0 + lane, A.g0 + lane, (amask >> lane) & 1, my_margin);
  // row scales of spin sp; wave 0 also flips the accepted fields
  if (lane < kk) {
    const bool mine = (amask >> lane) & 1;
    A.g.sc[sp][lane] = mine ? 1.0 + C.dflip[sp][xl > 0 ? 0 : 1] : 1.0;
    if (sp == 0 && mine) {
      C.fields[(long)C.li * C.N + A.g0 + lane] = (int8_t)(-xl);
      A.g.alist[__popcll(amask & ((1ull << lane) - 1))] = lane;   // A in order
    }
  }
  // Mc_s = diag(Delta_A) (E_AA)^{-1} = -diag(Delta_A) (swept E)_AA, zero elsewhere
  double *Mc = A.g.Mc[sp];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int a = ra + 8 * i;
    if (a >= kk) continue;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int b = cb + 8 * j;
      if (b >= kk) continue;
      const bool in = ((amask >> a) & 1) && ((amask >> b) & 1);
      Mc[a * kmax + b] = in ? -da[i] * e[i][j] : 0.0;
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
    // rows t / 64 + (NT / 64) q, columns t % 64 (n <= 64; no integer division)
    for (int i = t >> 6; i < n; i += NT / 64) {
      const int j = t & 63;
      if (j < n) {
        const double ci = colk[i];
        double v;
        if (i == k) v = (j == k) ? ip : rowk[j];
        else v = (j == k) ? -ci * ip : A[i * ld + j] - ci * rowk[j];
        A[i * ld + j] = v;
      }
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

// Wave-level synchronisation: the LDS operations of one wave complete in
// issue order, so a fence that keeps the compiler from moving memory
// operations across it is all that one wave's lanes need between writing
// and reading each other's LDS entries.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// In-place inverse of the n x n matrix A (n <= 16, LDS, row-major, stride ld)
// by Gauss-Jordan elimination with partial pivoting, by the 64 lanes of the
// calling wave alone (no workgroup barrier, so that two waves can invert two
// matrices at once); returns det(A) in every lane.  Lane (i, q) = (lane / 4,
// lane % 4) owns row i, columns q + 4 p.  Per column: the pivot (the largest
// |A_rk|, r >= k, by an integer max over keys that pack the magnitude's bits
// with 63 - r, so ties go to the smaller row), the row swap, then every
// entry's new value from loads issued before any store (a wave's LDS
// operations complete in order), so one LDS round trip a column.
__device__ __forceinline__ unsigned long long shfl_xor_key(unsigned long long v, int m) {
  const int lo = __shfl_xor((int)(unsigned)v, m, 64);
  const int hi = __shfl_xor((int)(unsigned)(v >> 32), m, 64);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
}

__device__ double wave_gj_inverse16(double *A, int ld, int n, int *ipiv) {
  const int lane = threadIdx.x & 63, i = lane >> 2, jq = lane & 3;
  const int ic = min(i, n - 1);
  double det = 1.0;
  for (int k = 0; k < n; ++k) {
    const double av = A[ic * ld + k];
    unsigned long long key =
        (i >= k && i < n)
            ? (((unsigned long long)__double_as_longlong(fabs(av)) & ~0x3Full) |
               (unsigned long long)(63 - i))
            : 0ull;
    // the four lanes of a row hold the same key: reduce over the rows only
#pragma unroll
    for (int m = 4; m < 64; m <<= 1) {
      const unsigned long long o = shfl_xor_key(key, m);
      key = o > key ? o : key;
    }
    const int p = __builtin_amdgcn_readfirstlane(min(63 - (int)(key & 0x3F), n - 1));
    if (lane == 0) ipiv[k] = p;
    if (p != k && lane < n) {
      const double x = A[k * ld + lane];
      A[k * ld + lane] = A[p * ld + lane];
      A[p * ld + lane] = x;
    }
    wave_sync();
    const double piv = A[k * ld + k];
    const double aik = A[ic * ld + k];
    double akj[4], aij[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jc = min(jq + 4 * q, n - 1);
      akj[q] = A[k * ld + jc];
      aij[q] = A[ic * ld + jc];
    }
    const double ip = 1.0 / piv;
    det *= (p != k) ? -piv : piv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = jq + 4 * q;
      if (i < n && j < n) {
        const double rk = akj[q] * ip;
        A[i * ld + j] = (i == k) ? ((j == k) ? ip : rk) : ((j == k) ? -aik * ip : aij[q] - aik * rk);
      }
    }
    wave_sync();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = __builtin_amdgcn_readfirstlane(ipiv[k]);
    if (p != k && lane < n) {
      const double x = A[lane * ld + k];
      A[lane * ld + k] = A[lane * ld + p];
      A[lane * ld + p] = x;
    }
    wave_sync();
  }
  return det;
}

// Block force-bias decision for kk <= 64 sites (one workgroup of NT lanes;
// NT = 128 for kk <= 16: wave s inverts spin s's matrices, both at once):
// force bias from B = 1 + diag(Delta_b) W0 (Eq. (35)), heat-bath proposal,
// det[1 + W0_FF diag(Delta'_F)] per spin and the Metropolis test with the
// prior ratio (Sec. III B).  Both small inversions use partial pivoting.
template <int NT>
__global__ __launch_bounds__(NT) void block_decide_kernel(Batch<DecideArgs> B) {
  const DecideArgs &A = B.w[blockIdx.x];
  if (decide_panel_block<NT>(A)) return;
  if (A.kk <= 0) return;   // no group for this walker (uneven batch)
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
  __shared__ double rdet[2];   // the two-wave form
  __shared__ int ipiv2[2][64];
  __shared__ double db[2][64], nbar[2][64], sval[64], dp[2][64], hbm[64];
  __shared__ int xold[64], xnew[64], flist[64], posF[64];
  __shared__ int s_nF;
  __shared__ double W0s[2][64 * LD];

  if (t < kk) {
    const int8_t x = C.fields[(long)C.li * C.N + A.g0 + t];
    xold[t] = x > 0 ? 1 : -1;
    db[0][t] = C.dremove[0][x > 0 ? 0 : 1];
    db[1][t] = C.dremove[1][x > 0 ? 0 : 1];
  }
  for (int e = t; e < kk * kk; e += NT) {
    W0s[0][(e / kk) * LD + e % kk] = A.g.W0[0][(e / kk) * kmax + e % kk];
    W0s[1][(e / kk) * LD + e % kk] = A.g.W0[1][(e / kk) * kmax + e % kk];
  }
  __syncthreads();
  if constexpr (NT == 128) {
    // wave s inverts spin s's 1 + diag(Delta_b) W0 (in M0 / M1), both at once
    const int sw = t >> 6, ln = t & 63;
    double *Mw = sw ? M1 : M0;
    for (int e = ln; e < kk * kk; e += 64) {
      const int ia = e / kk, ib = e % kk;
      Mw[ia * LD + ib] = (ia == ib ? 1.0 : 0.0) + db[sw][ia] * W0s[sw][ia * LD + ib];
    }
    wave_sync();
    wave_gj_inverse16(Mw, LD, kk, ipiv2[sw]);
    if (ln < kk) {
      double v = 0.0;
      for (int m = 0; m < kk; ++m) v += W0s[sw][ln * LD + m] * Mw[m * LD + ln];
      nbar[sw][ln] = (1.0 + db[sw][ln]) * v;     // [UU_R (U_L UU_R)^{-1} U_L]_ii
    }
    __syncthreads();
  } else {
    for (int s = 0; s < 2; ++s) {
      // M1 = W0 (kept for the force-bias product), M0 = 1 + diag(Delta_b) W0
      for (int e = t; e < kk * kk; e += NT) {
        const int ia = e / kk, ib = e % kk;
        const double w = W0s[s][ia * LD + ib];
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
  }
  // heat-bath proposal x'_i, P(+1) = 1 / (1 + e^{-2 s_i}), s_i = alpha (nbar_up - nbar_dn)
  if (t < kk) {
    const int site = A.g0 + t;
    const double sv = C.alpha * (nbar[0][t] - nbar[1][t]);
    sval[t] = sv;
    const double pp = 1.0 / (1.0 + exp(-2.0 * sv));
    const double u = A.g.uni[t];
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
    posF[t] = mine ? before : -1;
    if (t == kk - 1) s_nF = before + mine;
  }
  __syncthreads();
  const int nF = __builtin_amdgcn_readfirstlane(s_nF);
  const double u_mh = A.g.uni[kk];
  if (nF == 0) {
    if (t == 0) {
      C.stats[kStProposed] += 1;
      C.stats[kStAccepted] += 1;
      C.stats[kStFieldUpdates] += kk;
      const double margin = 1.0 - u_mh;
      if (fabs(margin) < 1e-12) C.stats[kStLowMargin] += 1;
      record_decision(C, C.log_base + A.block_index, A.g0, true, margin);
      A.g.nA[0] = 0;
      A.g.nA[1] = 0;
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
    M0[ia * LD + ib] = (ia == ib ? 1.0 : 0.0) + W0s[0][fa * LD + fb] * dp[0][ib];
    M1[ia * LD + ib] = (ia == ib ? 1.0 : 0.0) + W0s[1][fa * LD + fb] * dp[1][ib];
  }
  __syncthreads();
  double r0, r1;
  if constexpr (NT == 128) {
    // wave s: spin s's flip-set determinant and inverse, both at once
    const int sw = t >> 6;
    const double r = wave_gj_inverse16(sw ? M1 : M0, LD, nF, ipiv2[sw]);
    if ((t & 63) == 0) rdet[sw] = r;
    __syncthreads();
    r0 = rdet[0];
    r1 = rdet[1];
  } else {
    r0 = lds_gj_inverse<NT>(M0, LD, nF, colk, rowk, ipiv, &s_piv);
    r1 = lds_gj_inverse<NT>(M1, LD, nF, colk, rowk, ipiv, &s_piv);
  }
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
    A.g.nA[0] = acc_b ? nF : 0;
    A.g.nA[1] = acc_b ? kk : 0;
  }
  if (acc_b) {
    // Mc = diag(Delta'_F) (E'_FF)^{-1} spread to kk x kk, row scales, new fields
    if (t < nF) A.g.alist[t] = flist[t];   // F in site order
    if (t < kk) {
      const int pf = posF[t];
      A.g.sc[0][t] = pf >= 0 ? 1.0 + dp[0][pf] : 1.0;
      A.g.sc[1][t] = pf >= 0 ? 1.0 + dp[1][pf] : 1.0;
      if (pf >= 0) C.fields[(long)C.li * C.N + A.g0 + t] = (int8_t)xnew[t];
    }
    for (int e = t; e < kk * kk; e += NT) {
      const int a = e / kk, b = e % kk;
      const int pa = posF[a], pb = posF[b];
      const bool in = pa >= 0 && pb >= 0;
      A.g.Mc[0][a * kmax + b] = in ? dp[0][pa] * M0[pa * LD + pb] : 0.0;
      A.g.Mc[1][a * kmax + b] = in ? dp[1][pa] * M1[pa * LD + pb] : 0.0;
    }
  }
}

// ------------------------------------------------------------------------
// flush without the tile kernel (kmax > 64): Q = P1 Mc per row strip, and
// the accepted rows of U_R scaled; T -= Q P2 follows as a GEMM of rank kk
// (skipped on the device when nothing was accepted)
// ------------------------------------------------------------------------
struct QArgs {
  SpinMats m;
  GroupBufs g;
  int g0, kk;
};

__global__ __launch_bounds__(256) void group_q_kernel(Batch<QArgs> B) {
  const QArgs &a = B.w[blockIdx.z];
  const int s = blockIdx.y;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int strip = blockIdx.x;
  if (strip >= nt) return;
  if (a.kk <= 0 || a.g.nA[0] == 0) return;
  const int kmax = a.g.kmax, kk = a.kk;
  const int t = threadIdx.x;
  const int r0 = strip * 64;
  const int w = min(64, Ns - r0);
  extern __shared__ double dyn_lds[];
  const int ldp = kmax + 1;
  for (int e = t; e < 64 * kk; e += 256) {
    const int rr = e / kk, m = e % kk;
    dyn_lds[rr * ldp + m] = (rr < w) ? a.g.P1[s][(long)(r0 + rr) * kmax + m] : 0.0;
  }
  __syncthreads();
  const double *Mc = a.g.Mc[s];
  for (int e = t; e < 64 * kk; e += 256) {
    const int rr = e / kk, cc = e % kk;
    if (rr < w) {
      double v = 0.0;
      for (int m = 0; m < kk; ++m) v += dyn_lds[rr * ldp + m] * Mc[m * kmax + cc];
      a.g.Q[s][(long)(r0 + rr) * kmax + cc] = v;
    }
  }
  for (int e = t; e < kk * 64; e += 256) {
    const int j = e >> 6, cc = e & 63;
    if (cc < w) a.m.UR[s][(long)(a.g0 + j) * Ns + r0 + cc] *= a.g.sc[s][j];
  }
}

// ------------------------------------------------------------------------
// fused group tile kernel: one 64x64 tile of T per workgroup, read once per
// group.  (1) applies the pending flush of the previous group,
//     T_tile -= (P1 Mc) P2,   Mc = diag(Delta_A) (E_AA)^{-1}   (Eqs. (30)/(36)),
// and scales that group's accepted rows of U_R; (2) forms this tile's
// split-K contributions to the next group's panels P2 = U_g T and
// P1 = T L_g from the updated tile.  Every operand is loaded at the start,
// and all products run on MFMA from LDS.
// ------------------------------------------------------------------------
struct TileArgs {
  SpinMats m;
  GroupBufs g;   // pending group: panels P1, P2, its Mc, sc and nA
  int nmat, tpm; // matrices (2 spins x walkers) and (strip, chunk) slots per matrix
  int chm;       // column-chunk slots per strip
  int flush;     // a group is pending (its flush is skipped on the device if nA == 0)
  int g0_prev, kk_prev;
  int g0, kk;    // next group (kk == 0: flush only)
};

constexpr int kLdt = 65;   // padded LDS row stride
constexpr int kTileThreads = 512;

// T of spin s in the type the tile kernel works in
template <class R>
__device__ __forceinline__ R *tile_matrix(const SpinMats &m, int s);
template <>
__device__ __forceinline__ double *tile_matrix<double>(const SpinMats &m, int s) {
  return m.T[s];
}
template <>
__device__ __forceinline__ float *tile_matrix<float>(const SpinMats &m, int s) {
  return m.T32[s];
}

// KP: kmax rounded up to a multiple of 16 (16, 32 or 64).  R: the type T is
// kept in and multiplied in between stabilisations (double, or float for
// the precision form); the pending group's panels and Mc arrive in double
// and are rounded to R, and the partial panels leave in double.
//
// One workgroup of 512 threads (8 waves) per (matrix, row strip of 64 rows,
// column chunk).  It forms the pending group's -(P1 Mc) rows of the strip
// once, then walks the chunk's 64 x 64 tiles of T: applies the flush to the
// tile (wave w owns the 16 x 32 block at rows 16 (w / 2), columns 32 (w % 2),
// and the flush operand -(P1 Mc) is held in registers in the MFMA A layout),
// writes the tile back, writes the next group's P2 partial of the tile
// (P2 is split over row strips) and adds the tile's share of the strip's P1
// rows into accumulators.  P1 therefore has one partial per column chunk
// and W0 = U_g P1 one per (strip, chunk), instead of one per tile.
template <int KP, class R>
__global__ __launch_bounds__(kTileThreads, KP <= 32 ? 4 : 1) void group_tile_kernel(Batch<TileArgs> B) {
  typedef Mma<R> MM;
  constexpr int NT = kTileThreads, NW = kTileThreads / 64;
  constexpr int kPre = 64 * KP / NT;                 // per lane: a KP x 64 operand
  constexpr int kPreM = KP * KP >= NT ? KP * KP / NT : 1;     // per lane: KP x KP
  constexpr int kpad = KP;
  constexpr int QS = KP / 4;                         // depth steps of the flush
  // XCD-aware placement: consecutive workgroup ids go round-robin to the 8
  // XCDs, so XCD x receives ids x, x + 8, ...; giving it the contiguous range
  // [x per, (x + 1) per) of (matrix, strip, chunk) indices keeps the strips
  // that share panel operands (same matrix) in one L2.
  const int per = gridDim.x >> 3;   // the grid is a multiple of 8
  const int flat = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int spm = B.w[0].tpm;       // (strip, chunk) slots per matrix
  const int chm = B.w[0].chm;       // chunk slots per strip
  const int mat = flat / spm;
  if (mat >= B.w[0].nmat) return;
  const TileArgs &a = B.w[mat >> 1];
  const int s = mat & 1;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64, nch = strip_chunks(nt, a.g.chunks);
  const int slot = flat % spm;
  const int rb = slot / chm, ch = slot % chm;
  if (rb >= nt || ch >= nch) return;
  const int cper = strip_chunk_width(nt, a.g.chunks);
  const int cb0 = ch * cper, cb1 = min(nt, cb0 + cper);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;   // 16-row quarter, 32-column half
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = rb * 64;
  const int kmax = a.g.kmax;
  const int kk = a.kk, kkp = a.kk_prev;
  extern __shared__ double lds_raw[];
  const bool fl = a.flush && a.g.nA[0] > 0;
  // The flush has rank |A|: P1 Mc P2 only involves the accepted sites'
  // columns of P1 and rows of P2 (Mc is zero outside A x A), so they are
  // gathered by the pending group's site list and the flush runs at |A|
  // rounded to the MFMA depth instead of the group size.
  const int na = fl ? a.g.nA[0] : 0;
  const int kp = (na + 3) & ~3;
  __shared__ int al_s[KP];
  for (int e = t; e < KP; e += NT)
    al_s[e] = (e < na) ? a.g.alist[e] : (na > 0 ? a.g.alist[na - 1] : 0);
  __syncthreads();
  R *T = tile_matrix<R>(a.m, s);
  R *lds = reinterpret_cast<R *>(lds_raw);
  R *Y = lds;                      // KP x kLdt: U_g over the strip's rows (whole walk)
  R *X = Y + KP * kLdt;            // 64 x kLdt: the current tile of T
  R *Zb = X + 64 * kLdt;           // KP x kLdt: the tile's P2 columns, then its L_g columns

  // accepted rows of U_R over the chunk's columns, by the first strip
  if (fl && rb == 0) {
    const double *sc = a.g.sc[s];
    double *UR = a.m.UR[s];
    const int c0 = cb0 * 64, w = min(Ns, cb1 * 64) - c0;
    for (int e = t; e < kkp * w; e += NT) {
      const int m = e / w, c = c0 + e % w;
      UR[(long)(a.g0_prev + m) * Ns + c] *= sc[m];
    }
  }
  // U_g over the strip's rows (the next group's panels)
  if (kk > 0) {
    const double *UR = a.m.UR[s];
    for (int e = t; e < KP * 64; e += NT) {
      const int m = e >> 6, c = e & 63;
      Y[m * kLdt + c] = (m < kk && row0 + c < Ns) ? UR[(long)(a.g0 + m) * Ns + row0 + c] : 0.0;
    }
  }
  // -(P1 Mc) rows of the strip, then into registers in the A layout of the
  // flush: qa[q] = Q[wm 16 + li][4 q + lk]
  R qa[QS];
  if (fl) {
    const int ld1 = kpad + 1;
    R *A1 = X;                       // 64 x ld1 (aliases X and Zb before the walk)
    R *M1 = A1 + 64 * ld1;           // kpad x ld1
    const double *P1 = a.g.P1[s], *Mc = a.g.Mc[s];
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int e = t + NT * i;
      const int r = e / kpad, m = e % kpad;
      A1[r * ld1 + m] =
          (m < na && row0 + r < Ns) ? (R)P1[(long)(row0 + r) * kmax + al_s[m]] : (R)0.0;
    }
#pragma unroll
    for (int i = 0; i < kPreM; ++i) {
      const int e = t + NT * i;
      const int ma = e / kpad, mb = e % kpad;
      if (e < kpad * kpad)
        M1[ma * ld1 + mb] =
            (ma < na && mb < na) ? (R)Mc[al_s[ma] * kmax + al_s[mb]] : (R)0.0;
    }
    __syncthreads();
    {
      constexpr int QT = KP / 16, QV = (QT + 1) / 2;
      const int rq = wave & 3, uh = wave >> 2;
      typename MM::acc q[QV];
#pragma unroll
      for (int v = 0; v < QV; ++v) q[v] = MM::zero();
      for (int k0 = 0; k0 < kp; k0 += 4) {
        const R av = A1[(16 * rq + li) * ld1 + k0 + lk];
#pragma unroll
        for (int v = 0; v < QV; ++v) {
          const int u = uh + 2 * v;
          if (u < QT) q[v] = MM::op(av, M1[(k0 + lk) * ld1 + u * 16 + li], q[v]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int v = 0; v < QV; ++v) {
        const int u = uh + 2 * v;
        if (u < QT)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            A1[(16 * rq + MM::row(lane, j)) * ld1 + u * 16 + li] = -q[v][j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QS; ++q) qa[q] = A1[(wm * 16 + li) * ld1 + 4 * q + lk];
  }
  __syncthreads();   // Y staged; A1 / M1 free

  // accumulators of the strip's P1 rows over the chunk: 4 row tiles x mtk
  // column tiles of 16 x 16, round robin over the waves
  const int mtk = (kk + 15) >> 4;
  constexpr int U1 = (4 * (KP / 16) + NW - 1) / NW;
  typename MM::acc p1acc[U1];
  int rt1[U1], mt1[U1];
#pragma unroll
  for (int u = 0; u < U1; ++u) {
    const int tt = wave + NW * u;
    const bool v = tt < 4 * mtk;
    rt1[u] = v ? tt / mtk : 0;
    mt1[u] = v ? tt % mtk : 0;
    p1acc[u] = MM::zero();
  }
  constexpr int U2 = (4 * (KP / 16) + NW - 1) / NW;  // P2 tiles per wave and tile of T
  const double *P2 = a.g.P2[s];
  const double *ULt = a.m.ULt[s];
  double *o2 = a.g.P2part[s] + (long)rb * kmax * Ns;

  // this wave's 16 x 32 block of a tile (two 16 x 16 column tiles) and the
  // tile's L_g rows, into registers: for the first tile here, for the next
  // one while the current tile's panel products run
  typename MM::acc acc[2];
  R lg[kPre];
  // Loads are unconditional, so that all of a tile's loads are in flight
  // together: out-of-range elements read a clamped in-range address.  Such
  // elements of T and P2 are finite and only ever meet a zero factor (L_g
  // past N_s, U_g and -(P1 Mc) past the group) or a store that skips them;
  // L_g is masked to zero past N_s when it is stored to LDS (a multiply, so
  // that the load is not waited for early, nor sunk into a branch).
  auto load_tile = [&](int cb, typename MM::acc *acc, double *lg) {
    const int col0 = cb * 64;
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + wm * 16 + MM::row(lane, j), c = col0 + wn * 32 + ni * 16 + li;
        acc[ni][j] = T[(long)min(r, Ns - 1) * Ns + min(c, Ns - 1)];
      }
    if (kk > 0) {
#pragma unroll
      for (int i = 0; i < kPre; ++i) {
        const int e = t + NT * i;
        const int m = e >> 6, c = col0 + (e & 63);
        lg[i] = ULt[(long)(a.g0 + min(m, kk - 1)) * Ns + min(c, Ns - 1)];
      }
    }
  };
  // The walk over the chunk's tiles, one instantiation per (flush pending,
  // next group) case, so that the compiler's wait counts know where the
  // tile's registers come from.
  auto walk = [&](auto flc, auto nxc) {
    constexpr bool FL = decltype(flc)::value, NX = decltype(nxc)::value;
    // this wave's 16 x 32 block of a tile (two 16 x 16 column tiles) and the
    // tile's L_g rows: for the first tile here, for the next one while the
    // current tile's panel products run
    typename MM::acc acc[2];
    double lg[kPre];
    // the P2 columns of a tile, in registers from one tile to the next
    double pv[kPre];
    auto load_p2 = [&](int cb) {
#pragma unroll
      for (int i = 0; i < kPre; ++i) {
        const int e = t + NT * i;
        const int m = e >> 6, c = cb * 64 + (e & 63);
        pv[i] = P2[(long)al_s[min(m, KP - 1)] * Ns + min(c, Ns - 1)];
      }
    };
    load_tile(cb0, acc, lg);
    if (FL) load_p2(cb0);
    for (int cb = cb0; cb < cb1; ++cb) {
      const int col0 = cb * 64;
      const bool more = cb + 1 < cb1;
      if (FL) {
        // the tile's P2 columns into LDS, then the next tile's into registers
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
          const int e = t + NT * i;
          Zb[(e >> 6) * kLdt + (e & 63)] = (R)pv[i];
        }
        if (more) load_p2(cb + 1);
        __syncthreads();
        // acc (16 x 32) += -(P1 Mc) (strip rows x kp) P2 (kp x tile columns)
#pragma unroll
        for (int q = 0; q < QS; ++q) {
          if (4 * q < kp) {
            const R b0 = Zb[(4 * q + lk) * kLdt + wn * 32 + li];
            const R b1 = Zb[(4 * q + lk) * kLdt + wn * 32 + 16 + li];
            acc[0] = MM::op(qa[q], b0, acc[0]);
            acc[1] = MM::op(qa[q], b1, acc[1]);
          }
        }
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int r = row0 + wm * 16 + MM::row(lane, j), c = col0 + wn * 32 + ni * 16 + li;
            if (r < Ns && c < Ns) T[(long)r * Ns + c] = acc[ni][j];
          }
      }
      if (NX) {
        if (FL) __syncthreads();   // every wave is done with the P2 columns in Zb
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            X[(wm * 16 + MM::row(lane, j)) * kLdt + wn * 32 + ni * 16 + li] = acc[ni][j];
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
          const int e = t + NT * i;
          const int m = e >> 6, c = col0 + (e & 63);
          Zb[m * kLdt + (e & 63)] = (R)(lg[i] * ((m < kk && c < Ns) ? 1.0 : 0.0));
        }
        if (more) load_tile(cb + 1, acc, lg);
        __syncthreads();
        // P2 partial of the tile: U_g[:, strip rows] T_tile (kk x 64)
#pragma unroll
        for (int u = 0; u < U2; ++u) {
          const int tt = wave + NW * u;
          if (tt >= 4 * mtk) continue;
          const int mt2 = tt >> 2, ct2 = tt & 3;
          typename MM::acc p2t = MM::zero();
          for (int k0 = 0; k0 < 64; k0 += 4)
            p2t = MM::op(Y[(mt2 * 16 + li) * kLdt + k0 + lk], X[(k0 + lk) * kLdt + ct2 * 16 + li],
                         p2t);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int m = mt2 * 16 + MM::row(lane, j), c = col0 + ct2 * 16 + li;
            if (m < kk && c < Ns) o2[(long)m * Ns + c] = p2t[j];
          }
        }
        // P1 rows of the strip += T_tile L_g[tile columns, :]
#pragma unroll
        for (int u = 0; u < U1; ++u) {
          if (wave + NW * u >= 4 * mtk) continue;
          for (int k0 = 0; k0 < 64; k0 += 4)
            p1acc[u] = MM::op(X[(rt1[u] * 16 + li) * kLdt + k0 + lk],
                              Zb[(mt1[u] * 16 + li) * kLdt + k0 + lk], p1acc[u]);
        }
      } else if (more) {
        load_tile(cb + 1, acc, lg);
      }
      __syncthreads();   // X and Zb are free for the next tile
    }
  };
  if (fl && kk > 0) walk(std::true_type{}, std::true_type{});
  else if (kk > 0) walk(std::false_type{}, std::true_type{});
  else if (fl) walk(std::true_type{}, std::false_type{});
  if (kk <= 0) return;

  // P1 partial of this chunk, then W0 partial (strip, chunk) = U_g P1_chunk
  double *o1 = a.g.P1part[s] + (long)ch * Ns * kmax;
#pragma unroll
  for (int u = 0; u < U1; ++u) {
    if (wave + NW * u >= 4 * mtk) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = row0 + rt1[u] * 16 + MM::row(lane, j), m1 = mt1[u] * 16 + li;
      if (r < Ns && m1 < kk) o1[(long)r * kmax + m1] = p1acc[u][j];
      X[(rt1[u] * 16 + MM::row(lane, j)) * kLdt + mt1[u] * 16 + li] = p1acc[u][j];
    }
  }
  // columns m >= kk of X are never read below (the W0 tiles stop at kk)
  __syncthreads();
  constexpr int UW = (KP / 16 * KP / 16 + NW - 1) / NW;
  double *ow = a.g.W0part[s] + (long)(rb * nch + ch) * kmax * kmax;
#pragma unroll
  for (int u = 0; u < UW; ++u) {
    const int tt = wave + NW * u;
    if (tt >= mtk * mtk) continue;
    const int mw = tt / mtk, nw2 = tt % mtk;
    typename MM::acc w0 = MM::zero();
    for (int k0 = 0; k0 < 64; k0 += 4)
      w0 = MM::op(Y[(mw * 16 + li) * kLdt + k0 + lk], X[(k0 + lk) * kLdt + nw2 * 16 + li], w0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = mw * 16 + MM::row(lane, j), n = nw2 * 16 + li;
      if (m < kk && n < kk) ow[m * kmax + n] = w0[j];
    }
  }
}

// ------------------------------------------------------------------------
// Strip form of the fused tile kernel, for batches whose walkers ask for one
// column chunk per row strip: one workgroup of 16 waves per (matrix, row
// strip of 64 rows) walks all tiles of its strip as a two-stage pipeline.
// Waves 0-7 (flush waves) apply the pending flush to tile t of T (each wave a
// 16 x 32 block in registers), store it and copy it to LDS; in the same step
// waves 8-15 (panel waves) form the P2 partial and the P1 share of tile t - 1
// from the copy made one step earlier.  Tile copies, the flush's P2 columns
// and the L_g rows are double-buffered in LDS (150 KB at KP = 32), so a step
// ends on one barrier and the halves' MFMA and memory work overlap.  Every
// product has the operands and the order of accumulation of the one-chunk
// tile kernel above, so the two give the same bits.
// ------------------------------------------------------------------------
constexpr int kStripThreads = 1024;

template <int KP, class R>
__global__ __launch_bounds__(kStripThreads) void group_strip_kernel(Batch<TileArgs> B) {
  typedef Mma<R> MM;
  typedef typename MM::acc Acc2[2];
  constexpr int NTR = kStripThreads / 2;             // threads per role
  constexpr int NW = NTR / 64;                       // waves per role
  constexpr int kPre = 64 * KP / NTR;                // per lane: a KP x 64 operand
  constexpr int kpad = KP;
  constexpr int QS = KP / 4;                         // depth steps of the flush
  const int per = gridDim.x >> 3;   // the grid is a multiple of 8
  const int flat = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int spm = B.w[0].tpm;       // row strips per matrix (the largest walker's)
  const int mat = flat / spm;
  if (mat >= B.w[0].nmat) return;
  const TileArgs &a = B.w[mat >> 1];
  const int s = mat & 1;
  const int Ns = a.m.Ns[s];
  const int nt = (Ns + 63) / 64;
  const int rb = flat % spm;
  if (rb >= nt) return;
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const bool fwave = wv < NW;
  const int tr = fwave ? t : t - NTR;                // thread index within the role
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (wv >> 1) & 3, wn = wv & 1;         // flush waves' 16 x 32 block
  const int row0 = rb * 64;
  const int kmax = a.g.kmax;
  const int kk = a.kk, kkp = a.kk_prev;
  const int n = nt;                                  // tiles of the strip
  R *T = tile_matrix<R>(a.m, s);
  const double *P2 = a.g.P2[s];
  const double *ULt = a.m.ULt[s];
  extern __shared__ double lds_raw[];
  R *lds = reinterpret_cast<R *>(lds_raw);
  R *Y = lds;                      // KP x kLdt: U_g over the strip's rows
  R *Xb = Y + KP * kLdt;           // 2 x 64 x kLdt: tile copies
  R *Pb = Xb + 2 * 64 * kLdt;      // 2 x KP x kLdt: the flush's P2 columns
  R *Lb = Pb + 2 * KP * kLdt;      // 2 x KP x kLdt: L_g columns

  Acc2 accA, accB;                 // flush waves: two tiles' blocks of T
  // flush waves: P2 columns of the next tile; panel waves: L_g rows of the
  // next tile
  double ra[kPre];
  auto load_t = [&](int cb, Acc2 &acc) {
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + wm * 16 + MM::row(lane, j), c = cb * 64 + wn * 32 + ni * 16 + li;
        acc[ni][j] = T[(long)min(r, Ns - 1) * Ns + min(c, Ns - 1)];
      }
  };
  auto load_l = [&](int cb) {
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int e = tr + NTR * i;
      const int m = e >> 6, c = cb * 64 + (e & 63);
      ra[i] = ULt[(long)(a.g0 + min(m, kk - 1)) * Ns + min(c, Ns - 1)];
    }
  };
  // the panel waves' first L_g rows go out before the set-up
  const bool fl = a.flush && a.g.nA[0] > 0;
  if (!fwave && kk > 0) load_l(0);
  const int na = fl ? a.g.nA[0] : 0;
  const int kp = (na + 3) & ~3;
  __shared__ int al_s[KP];
  for (int e = t; e < KP; e += kStripThreads)
    al_s[e] = (e < na) ? a.g.alist[e] : (na > 0 ? a.g.alist[na - 1] : 0);
  __syncthreads();
  auto load_p = [&](int cb, double (&pv)[kPre]) {
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
      const int e = tr + NTR * i;
      const int m = e >> 6, c = cb * 64 + (e & 63);
      pv[i] = P2[(long)al_s[min(m, KP - 1)] * Ns + min(c, Ns - 1)];
    }
  };
  if (fwave && fl) load_p(0, ra);   // the first tile's P2 columns, before the set-up

  // accepted rows of U_R, by the first strip
  if (fl && rb == 0) {
    const double *sc = a.g.sc[s];
    double *UR = a.m.UR[s];
    for (int e = t; e < kkp * Ns; e += kStripThreads) {
      const int m = e / Ns, c = e % Ns;
      UR[(long)(a.g0_prev + m) * Ns + c] *= sc[m];
    }
  }
  // U_g over the strip's rows (the next group's panels)
  if (kk > 0) {
    const double *UR = a.m.UR[s];
    for (int e = t; e < KP * 64; e += kStripThreads) {
      const int m = e >> 6, c = e & 63;
      Y[m * kLdt + c] = (m < kk && row0 + c < Ns) ? UR[(long)(a.g0 + m) * Ns + row0 + c] : 0.0;
    }
  }
  // -(P1 Mc) rows of the strip, into the flush waves' registers in the A
  // layout of the flush: qa[q] = Q[wm 16 + li][4 q + lk]
  R qa[QS];
  if (fl) {
    const int ld1 = kpad + 1;
    R *A1 = Xb;                      // 64 x ld1 (aliases the tile copies before the walk)
    R *M1 = A1 + 64 * ld1;           // kpad x ld1
    const double *P1 = a.g.P1[s], *Mc = a.g.Mc[s];
    for (int e = t; e < 64 * kpad; e += kStripThreads) {
      const int r = e / kpad, m = e % kpad;
      A1[r * ld1 + m] =
          (m < na && row0 + r < Ns) ? (R)P1[(long)(row0 + r) * kmax + al_s[m]] : (R)0.0;
    }
    for (int e = t; e < kpad * kpad; e += kStripThreads) {
      const int ma = e / kpad, mb = e % kpad;
      M1[ma * ld1 + mb] = (ma < na && mb < na) ? (R)Mc[al_s[ma] * kmax + al_s[mb]] : (R)0.0;
    }
    __syncthreads();
    constexpr int QT = KP / 16, QV = (QT + 1) / 2;
    const int rq = wv & 3, uh = (wv >> 2) & 1;
    typename MM::acc q[QV];
    if (fwave) {
#pragma unroll
      for (int v = 0; v < QV; ++v) q[v] = MM::zero();
      for (int k0 = 0; k0 < kp; k0 += 4) {
        const R av = A1[(16 * rq + li) * ld1 + k0 + lk];
#pragma unroll
        for (int v = 0; v < QV; ++v) {
          const int u = uh + 2 * v;
          if (u < QT) q[v] = MM::op(av, M1[(k0 + lk) * ld1 + u * 16 + li], q[v]);
        }
      }
    }
    __syncthreads();
    if (fwave) {
#pragma unroll
      for (int v = 0; v < QV; ++v) {
        const int u = uh + 2 * v;
        if (u < QT)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            A1[(16 * rq + MM::row(lane, j)) * ld1 + u * 16 + li] = -q[v][j];
      }
    }
    __syncthreads();
    if (fwave) {
#pragma unroll
      for (int q2 = 0; q2 < QS; ++q2) qa[q2] = A1[(wm * 16 + li) * ld1 + 4 * q2 + lk];
    }
  }
  __syncthreads();   // Y staged; A1 / M1 free
  const int mtk = (kk + 15) >> 4;

  // flush waves: one pipeline step flushes tile st (in `cur`), stores it and
  // copies it to LDS.  The loads of the step before are waited for by the
  // first use of their registers, and only then are this step's issued, so
  // that they have a whole step to arrive.
  auto fwalk = [&](auto flc, auto nxc) {
    constexpr bool FL = decltype(flc)::value, NX = decltype(nxc)::value;
    auto put_p = [&](int cb) {
      R *P = Pb + (cb & 1) * KP * kLdt;
#pragma unroll
      for (int i = 0; i < kPre; ++i) {
        const int e = tr + NTR * i;
        P[(e >> 6) * kLdt + (e & 63)] = (R)ra[i];
      }
    };
    auto fstep = [&](int st, Acc2 &cur, Acc2 &nxt) {
      if (st < n) {
        const int cb = st, col0 = cb * 64;
        if (FL) {
          if (st + 1 < n) put_p(cb + 1);
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 4; ++j) asm volatile("" ::"v"(cur[ni][j]));
          if (st + 2 < n) load_p(cb + 2, ra);
          if (st + 1 < n) load_t(cb + 1, nxt);
          const R *P = Pb + (cb & 1) * KP * kLdt;
#pragma unroll
          for (int q = 0; q < QS; ++q) {
            if (4 * q < kp) {
              const R b0 = P[(4 * q + lk) * kLdt + wn * 32 + li];
              const R b1 = P[(4 * q + lk) * kLdt + wn * 32 + 16 + li];
              cur[0] = MM::op(qa[q], b0, cur[0]);
              cur[1] = MM::op(qa[q], b1, cur[1]);
            }
          }
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int r = row0 + wm * 16 + MM::row(lane, j), c = col0 + wn * 32 + ni * 16 + li;
              if (r < Ns && c < Ns) T[(long)r * Ns + c] = cur[ni][j];
            }
        }
        if (NX) {
          R *X = Xb + (cb & 1) * 64 * kLdt;
#pragma unroll
          for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              X[(wm * 16 + MM::row(lane, j)) * kLdt + wn * 32 + ni * 16 + li] = cur[ni][j];
        }
        if (!FL && st + 1 < n) load_t(cb + 1, nxt);
      }
      __syncthreads();
    };
    load_t(0, accA);
    if (FL) {
      put_p(0);
      if (n > 1) load_p(1, ra);
    }
    __syncthreads();
    for (int st = 0; st <= n; st += 2) {
      fstep(st, accA, accB);
      if (st + 1 <= n) fstep(st + 1, accB, accA);
    }
    __syncthreads();   // the panel waves' epilogue
  };

  // panel waves: one pipeline step forms the P2 partial and the P1 share of
  // tile st - 1 from its copy in LDS; the L_g rows of the next tile arrive in
  // registers
  auto gwalk = [&](auto nxc) {
    constexpr bool NX = decltype(nxc)::value;
    const int gw = wv - NW;
    constexpr int U1 = (4 * (KP / 16) + NW - 1) / NW;
    constexpr int U2 = (4 * (KP / 16) + NW - 1) / NW;
    typename MM::acc p1acc[U1];
    int rt1[U1], mt1[U1];
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int tt = gw + NW * u;
      const bool v = tt < 4 * mtk;
      rt1[u] = v ? tt / mtk : 0;
      mt1[u] = v ? tt % mtk : 0;
      p1acc[u] = MM::zero();
    }
    double *o2 = a.g.P2part[s] + (long)rb * kmax * Ns;
    auto put_l = [&](int cb) {
      R *L = Lb + (cb & 1) * KP * kLdt;
#pragma unroll
      for (int i = 0; i < kPre; ++i) {
        const int e = tr + NTR * i;
        const int m = e >> 6, c = cb * 64 + (e & 63);
        L[m * kLdt + (e & 63)] = (R)(ra[i] * ((m < kk && c < Ns) ? 1.0 : 0.0));
      }
    };
    __syncthreads();
    for (int st = 0; st <= n; ++st) {
      if (NX) {
        if (st < n) put_l(st);
        if (st + 1 < n) load_l(st + 1);
        if (st >= 1) {
          const int cb = st - 1, col0 = cb * 64;
          const R *X = Xb + (cb & 1) * 64 * kLdt;
          const R *L = Lb + (cb & 1) * KP * kLdt;
          // P2 partial of the tile: U_g[:, strip rows] T_tile (kk x 64)
#pragma unroll
          for (int u = 0; u < U2; ++u) {
            const int tt = gw + NW * u;
            if (tt >= 4 * mtk) continue;
            const int mt2 = tt >> 2, ct2 = tt & 3;
            typename MM::acc p2t = MM::zero();
            for (int k0 = 0; k0 < 64; k0 += 4)
              p2t = MM::op(Y[(mt2 * 16 + li) * kLdt + k0 + lk],
                           X[(k0 + lk) * kLdt + ct2 * 16 + li], p2t);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int m = mt2 * 16 + MM::row(lane, j), c = col0 + ct2 * 16 + li;
              if (m < kk && c < Ns) o2[(long)m * Ns + c] = p2t[j];
            }
          }
          // P1 rows of the strip += T_tile L_g[tile columns, :]
#pragma unroll
          for (int u = 0; u < U1; ++u) {
            if (gw + NW * u >= 4 * mtk) continue;
            for (int k0 = 0; k0 < 64; k0 += 4)
              p1acc[u] = MM::op(X[(rt1[u] * 16 + li) * kLdt + k0 + lk],
                                L[(mt1[u] * 16 + li) * kLdt + k0 + lk], p1acc[u]);
          }
        }
      }
      __syncthreads();
    }
    if (!NX) {
      __syncthreads();
      return;
    }
    // P1 partial of the strip (one column chunk), then its W0 partial U_g P1
    double *o1 = a.g.P1part[s];
    R *X = Xb;
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      if (gw + NW * u >= 4 * mtk) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + rt1[u] * 16 + MM::row(lane, j), m1 = mt1[u] * 16 + li;
        if (r < Ns && m1 < kk) o1[(long)r * kmax + m1] = p1acc[u][j];
        X[(rt1[u] * 16 + MM::row(lane, j)) * kLdt + mt1[u] * 16 + li] = p1acc[u][j];
      }
    }
    __syncthreads();   // (the flush waves' last barrier)
    constexpr int UW = (KP / 16 * KP / 16 + NW - 1) / NW;
    double *ow = a.g.W0part[s] + (long)rb * kmax * kmax;
#pragma unroll
    for (int u = 0; u < UW; ++u) {
      const int tt = gw + NW * u;
      if (tt >= mtk * mtk) continue;
      const int mw = tt / mtk, nw2 = tt % mtk;
      typename MM::acc w0 = MM::zero();
      for (int k0 = 0; k0 < 64; k0 += 4)
        w0 = MM::op(Y[(mw * 16 + li) * kLdt + k0 + lk], X[(k0 + lk) * kLdt + nw2 * 16 + li], w0);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = mw * 16 + MM::row(lane, j), n2 = nw2 * 16 + li;
        if (m < kk && n2 < kk) ow[m * kmax + n2] = w0[j];
      }
    }
  };

  if (fwave) {
    if (fl && kk > 0) fwalk(std::true_type{}, std::true_type{});
    else if (kk > 0) fwalk(std::false_type{}, std::true_type{});
    else if (fl) fwalk(std::true_type{}, std::false_type{});
  } else {
    if (kk > 0) gwalk(std::true_type{});
    else if (fl) gwalk(std::false_type{});
  }
}

}  // namespace

// kernel arguments are passed by value: keep every batch within 4 KB
static_assert(sizeof(Batch<LocalArgs>) <= 4096 && sizeof(Batch<ReduceArgs>) <= 4096 &&
                  sizeof(Batch<DecideArgs>) <= 4096 && sizeof(Batch<QArgs>) <= 4096 &&
                  sizeof(Batch<TileArgs>) <= 4096,
              "kernel argument batch above 4 KB");

hipError_t local_step(const SpinMats *m, const LocalBufs *b, const SweepCtx *c, int nw, int i,
                      int nt_max, hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  Batch<LocalArgs> B{};
  for (int w = 0; w < nw; ++w) B.w[w] = LocalArgs{m[w], b[w], c[w], i};
  const int nt2 = nt_max * nt_max, total = nt2 * 2 * nw;
  hipLaunchKernelGGL(local_step_kernel, dim3((total + 7) / 8 * 8), dim3(256), 0, st, B, nt2,
                     total);
  return hipGetLastError();
}

namespace {
int max_tiles(const SpinMats *m, int nw) {
  int ns = 0;
  for (int w = 0; w < nw; ++w) ns = max(ns, max(m[w].Ns[0], m[w].Ns[1]));
  return (ns + 63) / 64;
}

hipError_t launch_reduce(const SpinMats *m, const GroupBufs *g, const SweepCtx *c, int nw,
                         int mode, int g0, const int *kk, int do_panels, int w0_mode,
                         hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  const int ntm = max_tiles(m, nw);
  Batch<ReduceArgs> B{};
  int kkm = 0;
  for (int w = 0; w < nw; ++w) {
    B.w[w] = ReduceArgs{m[w], g[w], g0, kk[w], ntm, do_panels, w0_mode, mode,
                        c[w].key0, c[w].key1, c[w].sweep, c[w].slice_code, c[w].force,
                        c[w].fields + (long)c[w].li * c[w].N, c[w].sweep_dev};
    kkm = max(kkm, kk[w]);
  }
  const int nP = do_panels ? ntm * kRedParts : 0, nW = w0_mode ? kkm : 0;
  hipLaunchKernelGGL(group_reduce_kernel, dim3(nP + nW + 1, 2, nw), dim3(kRedThreads), 0, st, B);
  return hipGetLastError();
}
}  // namespace

hipError_t group_panels(const SpinMats *m, const GroupBufs *g, const SweepCtx *c, int nw,
                        int mode, int g0, const int *kk, hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  // split-K partial panels, then their sums (and the group's uniforms)
  for (int w0 = 0; w0 < nw; w0 += kGemmMaxBatch / 2) {
    GemmBatch b2{}, b1{};
    for (int w = w0; w < min(nw, w0 + kGemmMaxBatch / 2); ++w)
      for (int s = 0; s < 2; ++s) {
        if (kk[w] <= 0) continue;
        const int Ns = m[w].Ns[s];
        GemmDesc d = gemm_desc(m[w].UR[s] + (long)g0 * Ns, Ns, m[w].T[s], Ns, g[w].P2part[s], Ns,
                               kk[w], Ns, Ns);
        d.ksplit = 64;
        d.csplit = (long)g[w].kmax * Ns;
        b2.d[b2.count++] = d;
        GemmDesc e = gemm_desc(m[w].T[s], Ns, m[w].ULt[s] + (long)g0 * Ns, Ns, g[w].P1part[s],
                               g[w].kmax, Ns, kk[w], Ns);
        e.ksplit = 64;
        e.csplit = (long)Ns * g[w].kmax;
        b1.d[b1.count++] = e;
      }
    hipError_t err = gemm(b2, false, false, st);
    if (err != hipSuccess) return err;
    err = gemm(b1, false, true, st);
    if (err != hipSuccess) return err;
  }
  hipError_t err = launch_reduce(m, g, c, nw, mode, g0, kk, 1, 0, st);
  if (err != hipSuccess) return err;
  // W0 = P2 L_g^T, split over column strips, then its partials added
  for (int w0 = 0; w0 < nw; w0 += kGemmMaxBatch / 2) {
    GemmBatch bw{};
    for (int w = w0; w < min(nw, w0 + kGemmMaxBatch / 2); ++w)
      for (int s = 0; s < 2; ++s) {
        if (kk[w] <= 0) continue;
        const int Ns = m[w].Ns[s];
        GemmDesc d = gemm_desc(g[w].P2[s], Ns, m[w].ULt[s] + (long)g0 * Ns, Ns, g[w].W0part[s],
                               g[w].kmax, kk[w], kk[w], Ns);
        d.ksplit = 64;
        d.csplit = (long)g[w].kmax * g[w].kmax;
        bw.d[bw.count++] = d;
      }
    err = gemm(bw, false, true, st);
    if (err != hipSuccess) return err;
  }
  return launch_reduce(m, g, c, nw, kUniNone, g0, kk, 0, 2, st);
}

namespace {
Batch<DecideArgs> decide_batch(const GroupBufs *g, const SweepCtx *c, int nw, int g0,
                               const int *kk, long long block_index) {
  Batch<DecideArgs> B{};
  for (int w = 0; w < nw; ++w) {
    B.w[w].g = g[w];
    B.w[w].c = c[w];
    B.w[w].g0 = g0;
    B.w[w].kk = kk[w];
    B.w[w].block_index = block_index;
  }
  return B;
}
}  // namespace

// The decision kernel is chosen by each walker's own group size, so that a
// walker in a batch of mixed lattice sizes runs the kernel it runs alone (and
// gets the same bits): walkers are split by kernel class into sub-batches.
template <class F>
hipError_t decide_by_class(const Batch<DecideArgs> &B, int nw, const int *kkw, int nclass,
                           int (*cls)(int), F launch) {
  for (int k = 0; k < nclass; ++k) {
    Batch<DecideArgs> S{};
    int n = 0;
    for (int w = 0; w < nw; ++w)
      if (kkw[w] > 0 && cls(kkw[w]) == k) S.w[n++] = B.w[w];
    if (n == 0) continue;
    launch(k, S, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// grid rows of a decision launch: the decisions, and with `panels` one row per
// (spin, column strip, part) of the panel sums of the class's largest walker
int decide_rows(const Batch<DecideArgs> &S, int n, bool panels) {
  if (!panels) return 1;
  int nt = 0;
  for (int w = 0; w < n; ++w)
    nt = max(nt, (max(S.w[w].g.Ns[0], S.w[w].g.Ns[1]) + 63) / 64);
  return 1 + 2 * nt * kRedParts;
}

int delayed_class(int kk) { return kk <= 8 ? 0 : kk <= 16 ? 1 : kk <= 32 ? 2 : kk <= 64 ? 3 : 4; }
int block_class(int kk) { return kk <= 16 ? 0 : 1; }

hipError_t delayed_decide(const GroupBufs *g, const SweepCtx *c, int nw, int g0,
                          const int *kkw, bool panels, hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  const Batch<DecideArgs> B = decide_batch(g, c, nw, g0, kkw, 0);
  // measured at 40x40: k = 32 takes 19.5 us with one wave per spin against
  // 21.6 us with both spins in one wave; k = 64 fits the per-spin layout
  return decide_by_class(B, nw, kkw, 5, delayed_class,
                         [&](int k, const Batch<DecideArgs> &S, int n) {
    const dim3 grid(n, decide_rows(S, n, panels));
    switch (k) {
      case 0: hipLaunchKernelGGL((delayed_decide_wave_kernel<8>), grid, dim3(64), 0, st, S); break;
      case 1: hipLaunchKernelGGL((delayed_decide_wave_kernel<16>), grid, dim3(64), 0, st, S); break;
      case 2: hipLaunchKernelGGL((delayed_decide_spin_kernel<32>), grid, dim3(128), 0, st, S); break;
      case 3: hipLaunchKernelGGL((delayed_decide_spin_kernel<64>), grid, dim3(128), 0, st, S); break;
      default: hipLaunchKernelGGL((delayed_decide_kernel<1024, 16>), grid, dim3(1024), 0, st, S);
    }
  });
}

hipError_t block_decide(const GroupBufs *g, const SweepCtx *c, int nw, int g0, const int *kkw,
                        long long block_index, bool panels, hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  const Batch<DecideArgs> B = decide_batch(g, c, nw, g0, kkw, block_index);
  const size_t lds = sizeof(double) * 2 * 64 * 65;
  // set once, thread-safely (batches on several streams run from several host threads)
  static const hipError_t attr = [lds] {
    hipError_t e = hipFuncSetAttribute((const void *)block_decide_kernel<256>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)block_decide_kernel<128>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }();
  if (attr != hipSuccess) return attr;
  return decide_by_class(B, nw, kkw, 2, block_class,
                         [&](int k, const Batch<DecideArgs> &S, int n) {
    const dim3 grid(n, decide_rows(S, n, panels));
    // kk <= 16: one wave per spin sector, each inverting its own matrices
    if (k == 0) hipLaunchKernelGGL((block_decide_kernel<128>), grid, dim3(128), lds, st, S);
    else hipLaunchKernelGGL((block_decide_kernel<256>), grid, dim3(256), lds, st, S);
  });
}

template <int KP, class R>
hipError_t launch_tile(const Batch<TileArgs> &B, int nw, hipStream_t st) {
  // Y, X and Zb (the set-up's P1 rows and Mc alias X and Zb): at most 66.5 KB
  // (KP = 32, double) so that two workgroups share a CU
  const size_t lds = sizeof(R) * ((size_t)2 * KP + 64) * kLdt;
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)group_tile_kernel<KP, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const int total = 2 * nw * B.w[0].tpm;
  hipLaunchKernelGGL((group_tile_kernel<KP, R>), dim3((total + 7) / 8 * 8), dim3(kTileThreads),
                     lds, st, B);
  return hipGetLastError();
}

template <int KP, class R>
hipError_t launch_strip(const Batch<TileArgs> &B, int nw, hipStream_t st) {
  // Y, two tile copies, two P2-column and two L_g buffers: 150 KB (KP = 32,
  // double), one workgroup per CU
  const size_t lds = sizeof(R) * ((size_t)5 * KP + 128) * kLdt;
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)group_strip_kernel<KP, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const int total = 2 * nw * B.w[0].tpm;
  hipLaunchKernelGGL((group_strip_kernel<KP, R>), dim3((total + 7) / 8 * 8), dim3(kStripThreads),
                     lds, st, B);
  return hipGetLastError();
}

hipError_t group_tile(const SpinMats *m, const GroupBufs *g, int nw, int g0_prev,
                      const int *kk_prev, int g0, const int *kk, bool fp32, hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  Batch<TileArgs> B{};
  int kmax = 0;
  for (int w = 0; w < nw; ++w) {
    TileArgs &a = B.w[w];
    a.m = m[w];
    a.g = g[w];
    a.flush = kk_prev[w] > 0 ? 1 : 0;
    a.g0_prev = g0_prev;
    a.kk_prev = kk_prev[w];
    a.g0 = g0;
    a.kk = kk[w];
    kmax = max(kmax, g[w].kmax);
  }
  const int nt = max_tiles(m, nw);
  int chm = 1;
  for (int w = 0; w < nw; ++w)
    for (int s = 0; s < 2; ++s) chm = max(chm, strip_chunks((m[w].Ns[s] + 63) / 64, g[w].chunks));
  for (int w = 0; w < nw; ++w) {
    B.w[w].nmat = 2 * nw;
    B.w[w].chm = chm;
    B.w[w].tpm = nt * chm;
  }
  // one chunk per strip for every walker, groups of 17-32 sites, float64:
  // the pipelined strip kernel (the same bits as the one-chunk tile kernel)
  if (chm == 1 && !fp32 && kmax > 16 && kmax <= 32) return launch_strip<32, double>(B, nw, st);
  if (fp32) {
    if (kmax <= 16) return launch_tile<16, float>(B, nw, st);
    if (kmax <= 32) return launch_tile<32, float>(B, nw, st);
    if (kmax <= 64) return launch_tile<64, float>(B, nw, st);
    return hipErrorInvalidValue;
  }
  if (kmax <= 16) return launch_tile<16, double>(B, nw, st);
  if (kmax <= 32) return launch_tile<32, double>(B, nw, st);
  if (kmax <= 64) return launch_tile<64, double>(B, nw, st);
  return hipErrorInvalidValue;
}

hipError_t group_reduce(const SpinMats *m, const GroupBufs *g, const SweepCtx *c, int nw,
                        int mode, int g0, const int *kk, hipStream_t st) {
  // W0 and the uniforms only: the panel sums run in the decision launch
  return launch_reduce(m, g, c, nw, mode, g0, kk, 0, 1, st);
}

hipError_t group_flush(const SpinMats *m, const GroupBufs *g, int nw, int g0, const int *kk,
                       hipStream_t st) {
  if (nw < 1 || nw > kMaxBatch) return hipErrorInvalidValue;
  const int nt = max_tiles(m, nw);
  Batch<QArgs> B{};
  int kmax = 0;
  for (int w = 0; w < nw; ++w) {
    B.w[w] = QArgs{m[w], g[w], g0, kk[w]};
    kmax = max(kmax, g[w].kmax);
  }
  const size_t lds = sizeof(double) * 64 * (size_t)(kmax + 1);
  // 66 KB for kmax = 128; set once, thread-safely
  static const hipError_t attr = hipFuncSetAttribute(
      (const void *)group_q_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)(sizeof(double) * 64 * 129));
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(group_q_kernel, dim3(nt, 2, nw), dim3(256), lds, st, B);
  for (int w0 = 0; w0 < nw; w0 += kGemmMaxBatch / 2) {
    GemmBatch b{};
    for (int w = w0; w < min(nw, w0 + kGemmMaxBatch / 2); ++w)
      for (int s = 0; s < 2; ++s) {
        if (kk[w] <= 0) continue;
        const int Ns = m[w].Ns[s];
        GemmDesc d = gemm_desc(g[w].Q[s], g[w].kmax, g[w].P2[s], Ns, m[w].T[s], Ns, Ns, Ns, kk[w],
                               -1.0, 1.0, m[w].T[s], Ns);
        d.Kdev = g[w].nA + 1;   // rank kk, or 0 when nothing was accepted
        b.d[b.count++] = d;
      }
    hipError_t e = gemm(b, false, false, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace pq
