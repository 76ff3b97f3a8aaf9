// Persistent local updates of one slice (Sec. II D): one cooperative launch
// per slice visit, the matrix that the rank-1 upgrades change held in
// registers across all sites, one grid barrier per site.
//
// T-form (the paper's local update, Eqs. (20)-(21)).  T_s (N_s x N_s) is
// cut into pr x pc blocks of at most 64 x 128; one 256-thread workgroup
// holds one block of one spin in registers for the whole slice.  Per site i
// every workgroup forms its block's share of
//   y^T = u_i^T T (columns of its block),  T v_i (rows),  u_i^T T v_i,
// with u_i the row of U_R and v_i = Delta_i (column i of U_L), and writes
// them to a partial buffer (double-buffered by site parity).  After the
// barrier each workgroup sums, in one fixed order, the partials it needs:
// the scalars of both spins (every workgroup takes the same decision,
// r_up r_dn against the same Philox uniform) and, on acceptance, y over its
// columns and x = T v / r over its rows for T <- T - x y^T.
//
// G-form (the O(N^2)-per-site local update on G = 1 - U_R T U_L).  G_s
// (N x N) is cut into row blocks; workgroup w holds rows [w BR, (w+1) BR) of
// both spins.  Per site i the owner of row i publishes it (both spins) and,
// after the barrier, every workgroup takes r_s = 1 + Delta_s (1 - G_s,ii)
// and applies G <- G - (Delta / r) G[:, i] (e_i^T - G[i, :]) to its rows.
//
// Barrier: one epoch flag per workgroup, written once the workgroup's
// shared stores have completed and watched by the others, and a bounded
// wait: a workgroup that has waited more than the spin limit sets an abort
// flag, which every waiting workgroup also watches, so that every wave leaves
// the kernel whatever happens; the host reports the abort as a device
// error.  The launch is cooperative, so all workgroups are resident at once.
#include "engine.hpp"

namespace pq {

namespace {

__device__ __forceinline__ void record(const SweepCtx &c, long long idx, int site, bool acc,
                                       double margin) {
  if (c.log_meta && idx < c.log_cap) {
    c.log_meta[3 * idx + 0] = (int32_t)c.slice_code;
    c.log_meta[3 * idx + 1] = site;
    c.log_meta[3 * idx + 2] = acc ? 1 : 0;
    c.log_margin[idx] = margin;
  }
}

// Data that one workgroup writes and others read within the launch moves
// through agent-scope relaxed atomic stores and loads: such an access is
// coherent across the GPU's L2 caches by itself, so no cache-wide fence
// (L2 write-back or invalidate) is needed around the barrier.
__device__ __forceinline__ void put(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier on a flag array: workgroup w stores the epoch to flags[w]
// once every thread's shared stores have completed (s_waitcnt before the
// workgroup barrier), then thread t watches flags[t], t < gridDim.x, so the
// waits are spread over distinct words instead of one counter.  Bounded:
// past spin_limit polls a waiter sets *abort, which every waiter also
// watches.  All threads call it; returns false when abandoned.
__device__ bool grid_barrier(const GridSync &g, unsigned epoch) {
  __shared__ int s_abort;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    s_abort = 0;
    __hip_atomic_store(g.flags + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  for (unsigned w = threadIdx.x; w < gridDim.x; w += blockDim.x) {
    unsigned spins = 0;
    while (__hip_atomic_load(g.flags + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      if (__hip_atomic_load(g.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        s_abort = 1;
        break;
      }
      if (++spins > g.spin_limit) {
        atomicMax(g.abort, 1u);
        s_abort = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return s_abort == 0;
}

constexpr int kLpThreads = 256;
constexpr int kLpBR = 64, kLpBC = 128, kLpQ = kLpBR / 2;
// at most 256 workgroups: n <= 1024 gives pr <= 16 row blocks, pc <= 8 column blocks
constexpr int kLpMaxPr = 16, kLpMaxPc = 8;

// ------------------------------------------------------------------ T-form
__global__ __launch_bounds__(kLpThreads) void local_t_kernel(LocalPersistArgs a) {
  const int id = blockIdx.x;
  const int s = id < a.P[0] ? 0 : 1;
  const int lid = s ? id - a.P[0] : id;
  const int n = a.m.Ns[s], pr = a.pr[s], pc = a.pc[s];
  const int BR = (n + pr - 1) / pr, BC = (n + pc - 1) / pc;
  const int ra = lid / pc, cb = lid % pc;
  const int row0 = ra * BR, col0 = cb * BC;
  const int nr = max(0, min(BR, n - row0)), nc = max(0, min(BC, n - col0));
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int cl = t & (kLpBC - 1), rp = t >> 7;
  const SweepCtx &C = a.c;
  const int N = C.N;
  double *T = a.m.T[s];
  const double *UR = a.m.UR[s];
  const double *ULt = a.m.ULt[s];

  __shared__ double su[kLpBR], sv[kLpBC];
  __shared__ double yred[2][kLpBC];
  __shared__ double xred[4][kLpQ];
  __shared__ double ys[kLpBC], xs[kLpBR];
  __shared__ double rr[2];

  double tv[kLpQ];
#pragma unroll
  for (int q = 0; q < kLpQ; ++q) {
    const int r = rp + 2 * q;
    tv[q] = (r < nr && cl < nc) ? T[(long)(row0 + r) * n + col0 + cl] : 0.0;
  }
  // this thread's entries of u_i (rows) and v_i (columns), prefetched one
  // site ahead; the fields of a slice change only at the site being decided
  double u_next = 0.0, v_next = 0.0;
  int8_t x_next = 1;
  auto fetch = [&](int i) {
    x_next = C.fields[(long)C.li * N + i];
    u_next = (t < nr) ? UR[(long)i * n + row0 + t] : 0.0;
    v_next = (t < nc) ? ULt[(long)i * n + col0 + t] : 0.0;
  };
  fetch(0);
  unsigned long long n_acc = 0, n_low = 0, n_neg = 0;
  bool any_nan = false;
  bool alive = true;
  for (int i = 0; i < N && alive; ++i) {
    const int par = i & 1;
    const int8_t xi = x_next;
    const double dl = C.dflip[s][xi > 0 ? 0 : 1];
    if (t < kLpBR) su[t] = u_next;
    if (t < kLpBC) sv[t] = dl * v_next;
    __syncthreads();
    if (i + 1 < N) fetch(i + 1);
    // y partial over this thread's rows, x partial per row over the block's columns
    double yp = 0.0;
#pragma unroll
    for (int q = 0; q < kLpQ; ++q) yp += su[(rp + 2 * q) & (kLpBR - 1)] * tv[q];
    yred[rp][cl] = yp;
    const double vc = sv[cl];
#pragma unroll
    for (int q = 0; q < kLpQ; ++q) {
      const double w = wave_sum(tv[q] * vc);
      if (lane == 0) xred[wave][q] = w;
    }
    __syncthreads();
    double *yout = a.ypart[s] + ((long)par * pr + ra) * n;
    double *xout = a.xpart[s] + ((long)par * pc + cb) * n;
    if (t < nc) put(yout + col0 + t, yred[0][t] + yred[1][t]);
    if (wave == 2) {
      // x partial of row r (= rp + 2 q) from the two waves of its parity
      const int r = lane;
      const double xp = (r < nr) ? xred[2 * (r & 1)][r >> 1] + xred[2 * (r & 1) + 1][r >> 1] : 0.0;
      if (r < nr) put(xout + row0 + r, xp);
      const double sp = wave_sum(xp * su[r]);
      if (lane == 0) put(a.spart[s] + par * a.P[s] + lid, sp);
    }
    alive = grid_barrier(a.g, (unsigned)(i + 1));
    if (!alive) break;
    // r_s = 1 + u^T T v for both spins, summed in the same order everywhere
    if (wave < 2) {
      const int ss = wave, P = a.P[ss];
      const double *sp = a.spart[ss] + par * P;
      const double v0 = get(sp + min(lane, P - 1)), v1 = get(sp + min(lane + 64, P - 1));
      double acc = (lane < P ? v0 : 0.0) + (lane + 64 < P ? v1 : 0.0);
      acc = wave_sum(acc);
      if (lane == 0) rr[ss] = 1.0 + acc;
    }
    __syncthreads();
    const double r0 = rr[0], r1 = rr[1];
    const double R = r0 * r1;
    const double absA = fabs(R);
    const double u = C.force ? forced_uniform(C.force[i] != 0)
                             : philox_uniform(C.key0, C.key1, sweep_of(C.sweep, C.sweep_dev),
                                              C.slice_code, (uint64_t)i, kPurposeMH);
    const bool finite = !isnan(absA);
    const bool acc = __builtin_amdgcn_readfirstlane((finite && (u < absA)) ? 1 : 0) != 0;
    if (id == 0 && t == 0) {
      const double margin = absA - u;
      n_acc += acc ? 1 : 0;
      n_low += (fabs(margin) < 1e-12) ? 1 : 0;
      n_neg += (R < 0.0) ? 1 : 0;
      any_nan = any_nan || !finite;
      record(C, C.log_base + i, i, acc, margin);
      if (acc) C.fields[(long)C.li * N + i] = (int8_t)(-xi);
    }
    if (acc) {
      const double rs = s ? r1 : r0;
      // all partials in flight together (clamped in-range addresses), then
      // summed in index order
      if (t < nc) {
        const double *yp2 = a.ypart[s] + (long)par * pr * n + col0 + t;
        double v[kLpMaxPr];
#pragma unroll
        for (int e = 0; e < kLpMaxPr; ++e) v[e] = get(yp2 + (long)min(e, pr - 1) * n);
        double y = 0.0;
#pragma unroll
        for (int e = 0; e < kLpMaxPr; ++e) y += e < pr ? v[e] : 0.0;
        ys[t] = y;
      } else if (t >= kLpBC && t - kLpBC < nr) {
        const int r = t - kLpBC;
        const double *xp2 = a.xpart[s] + (long)par * pc * n + row0 + r;
        double v[kLpMaxPc];
#pragma unroll
        for (int e = 0; e < kLpMaxPc; ++e) v[e] = get(xp2 + (long)min(e, pc - 1) * n);
        double x = 0.0;
#pragma unroll
        for (int e = 0; e < kLpMaxPc; ++e) x += e < pc ? v[e] : 0.0;
        xs[r] = x / rs;
      }
      __syncthreads();
      const double yc = ys[cl];
#pragma unroll
      for (int q = 0; q < kLpQ; ++q) tv[q] -= xs[(rp + 2 * q) & (kLpBR - 1)] * yc;
      // row i of U_R <- (1 + Delta) row i, by the first block column
      if (cb == 0 && t < nr) a.m.UR[s][(long)i * n + row0 + t] *= 1.0 + dl;
    }
  }
  if (!alive) {
    if (t == 0) atomicOr(&C.stats[kStError], (unsigned long long)kErrBarrier);
    return;
  }
#pragma unroll
  for (int q = 0; q < kLpQ; ++q) {
    const int r = rp + 2 * q;
    if (r < nr && cl < nc) T[(long)(row0 + r) * n + col0 + cl] = tv[q];
  }
  if (id == 0 && t == 0) {
    C.stats[kStProposed] += N;
    C.stats[kStFieldUpdates] += N;
    C.stats[kStAccepted] += n_acc;
    C.stats[kStFlips] += n_acc;
    C.stats[kStLowMargin] += n_low;
    C.stats[kStNegative] += n_neg;
    if (any_nan) C.stats[kStError] |= kErrNonFinite;
  }
}

// ------------------------------------------------------------------ G-form
constexpr int kLgThreads = 512;
constexpr int kLgRows = 8;      // rows of each spin per workgroup
constexpr int kLgCols = 4;      // columns per thread: N <= 2048

__global__ __launch_bounds__(kLgThreads) void local_g_kernel(LocalPersistArgs a) {
  const int w = blockIdx.x;
  const int t = threadIdx.x;
  const SweepCtx &C = a.c;
  const int N = C.N, BR = a.grow;
  const int row0 = w * BR;
  const int nr = max(0, min(BR, N - row0));
  __shared__ double pub[2][2048];      // the published row i of both spins
  __shared__ double gcol[2][kLgRows];  // G[r][i] of this workgroup's rows
  __shared__ double gii[2];

  double g[2][kLgRows][kLgCols];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int r = 0; r < kLgRows; ++r)
#pragma unroll
      for (int j = 0; j < kLgCols; ++j) {
        const int c = t + kLgThreads * j;
        g[s][r][j] = (r < nr && c < N) ? a.Gm[s][(long)(row0 + r) * N + c] : 0.0;
      }
  // the owner of row i writes it, both spins, to parity buffer i & 1
  auto publish = [&](int i) {
    const int r = i - row0;
    if (r < 0 || r >= nr) return;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rr = 0; rr < kLgRows; ++rr)
        if (rr == r)
#pragma unroll
          for (int j = 0; j < kLgCols; ++j) {
            const int c = t + kLgThreads * j;
            if (c < N) put(a.grow_buf[s] + (long)(i & 1) * N + c, g[s][rr][j]);
          }
  };
  publish(0);
  unsigned long long n_acc = 0, n_low = 0, n_neg = 0;
  bool any_nan = false;
  bool alive = true;
  for (int i = 0; i < N && alive; ++i) {
    // x_i before the barrier: workgroup 0 flips it only after every
    // workgroup has arrived there
    const int8_t xi = C.fields[(long)C.li * N + i];
    alive = grid_barrier(a.g, (unsigned)(i + 1));
    if (!alive) break;
    const int par = i & 1;
    {
      // the published rows, all loads in flight together
      double v[2][kLgCols];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < kLgCols; ++j)
          v[s][j] = get(a.grow_buf[s] + (long)par * N + min(t + kLgThreads * j, N - 1));
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < kLgCols; ++j)
          if (t + kLgThreads * j < N) pub[s][t + kLgThreads * j] = v[s][j];
    }
    // this workgroup's G[r][i], from the thread holding column i
    {
      const int jt = i / kLgThreads, owner = i % kLgThreads;
      if (t == owner)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int r = 0; r < kLgRows; ++r)
#pragma unroll
            for (int j = 0; j < kLgCols; ++j)
              if (j == jt) gcol[s][r] = g[s][r][j];
    }
    __syncthreads();
    const double d0 = C.dflip[0][xi > 0 ? 0 : 1], d1 = C.dflip[1][xi > 0 ? 0 : 1];
    const double r0 = 1.0 + d0 * (1.0 - pub[0][i]);
    const double r1 = 1.0 + d1 * (1.0 - pub[1][i]);
    const double R = r0 * r1;
    const double absA = fabs(R);
    const double u = C.force ? forced_uniform(C.force[i] != 0)
                             : philox_uniform(C.key0, C.key1, sweep_of(C.sweep, C.sweep_dev),
                                              C.slice_code, (uint64_t)i, kPurposeMH);
    const bool finite = !isnan(absA);
    const bool acc = __builtin_amdgcn_readfirstlane((finite && (u < absA)) ? 1 : 0) != 0;
    if (w == 0 && t == 0) {
      const double margin = absA - u;
      n_acc += acc ? 1 : 0;
      n_low += (fabs(margin) < 1e-12) ? 1 : 0;
      n_neg += (R < 0.0) ? 1 : 0;
      any_nan = any_nan || !finite;
      record(C, C.log_base + i, i, acc, margin);
      if (acc) C.fields[(long)C.li * N + i] = (int8_t)(-xi);
    }
    if (acc) {
      const double f0 = d0 / r0, f1 = d1 / r1;
#pragma unroll
      for (int j = 0; j < kLgCols; ++j) {
        const int c = t + kLgThreads * j;
        const double e0 = (c == i ? 1.0 : 0.0) - pub[0][min(c, N - 1)];
        const double e1 = (c == i ? 1.0 : 0.0) - pub[1][min(c, N - 1)];
#pragma unroll
        for (int r = 0; r < kLgRows; ++r) {
          g[0][r][j] -= f0 * gcol[0][r] * e0;
          g[1][r][j] -= f1 * gcol[1][r] * e1;
        }
      }
      // row i of U_R <- (1 + Delta) row i
      if (w == 0) {
        for (int s = 0; s < 2; ++s) {
          const int n = a.m.Ns[s];
          const double f = 1.0 + (s ? d1 : d0);
          for (int e = t; e < n; e += kLgThreads) a.m.UR[s][(long)i * n + e] *= f;
        }
      }
    }
    if (i + 1 < N) publish(i + 1);
  }
  if (!alive) {
    if (t == 0) atomicOr(&C.stats[kStError], (unsigned long long)kErrBarrier);
    return;
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int r = 0; r < kLgRows; ++r)
#pragma unroll
      for (int j = 0; j < kLgCols; ++j) {
        const int c = t + kLgThreads * j;
        if (r < nr && c < N) a.Gm[s][(long)(row0 + r) * N + c] = g[s][r][j];
      }
  if (w == 0 && t == 0) {
    C.stats[kStProposed] += N;
    C.stats[kStFieldUpdates] += N;
    C.stats[kStAccepted] += n_acc;
    C.stats[kStFlips] += n_acc;
    C.stats[kStLowMargin] += n_low;
    C.stats[kStNegative] += n_neg;
    if (any_nan) C.stats[kStError] |= kErrNonFinite;
  }
}

__global__ void zero_sync_kernel(GridSync g, int n) {
  for (int w = threadIdx.x; w < n; w += blockDim.x) g.flags[w] = 0u;
  if (threadIdx.x == 0) *g.abort = 0u;
}

hipError_t cooperative_ok() {
  static const hipError_t ok = [] {
    int dev = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess && !coop) e = hipErrorNotSupported;
    return e;
  }();
  return ok;
}

}  // namespace

bool local_persist_fits(int n_up, int n_dn, int N, bool gform) {
  if (gform) return N <= kLgThreads * kLgCols && (N + kLgRows - 1) / kLgRows <= 256;
  int wg = 0;
  for (int n : {n_up, n_dn}) {
    const int pr = (n + kLpBR - 1) / kLpBR, pc = (n + kLpBC - 1) / kLpBC;
    wg += pr * pc;
  }
  return wg <= 256;
}

void local_persist_grid(int n, int *pr, int *pc) {
  *pr = (n + kLpBR - 1) / kLpBR;
  *pc = (n + kLpBC - 1) / kLpBC;
}

hipError_t local_persist(const LocalPersistArgs &a0, bool gform, hipStream_t st) {
  hipError_t e = cooperative_ok();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_sync_kernel, dim3(1), dim3(256), 0, st, a0.g, kLocalMaxGroups);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  LocalPersistArgs a = a0;
  void *args[] = {&a};
  if (gform) {
    const int nwg = (a.c.N + a.grow - 1) / a.grow;
    return hipLaunchCooperativeKernel((const void *)local_g_kernel, dim3(nwg), dim3(kLgThreads),
                                      args, 0, st);
  }
  return hipLaunchCooperativeKernel((const void *)local_t_kernel, dim3(a.P[0] + a.P[1]),
                                    dim3(kLpThreads), args, 0, st);
}

}  // namespace pq
