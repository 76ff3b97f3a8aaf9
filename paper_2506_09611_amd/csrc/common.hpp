// Shared device helpers for the PQMC sweep kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mfma.hpp"

namespace pq {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
// published round function: two 64x64->128 products per round, the key
// bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

enum : uint64_t { kPurposeInit = 1, kPurposeMH = 2, kPurposeHB = 3 };

__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t lo0 = kPhiloxM0 * c0, hi0 = __umul64hi(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2, hi1 = __umul64hi(kPhiloxM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// u in [0,1): top 53 bits of word 0 times 2^-53.
__device__ __forceinline__ double philox_uniform(uint64_t k0, uint64_t k1, uint64_t c0,
                                                 uint64_t c1, uint64_t c2, uint64_t c3) {
  return (double)(philox_word0(c0, c1, c2, c3, k0, k1) >> 11) * (1.0 / 9007199254740992.0);
}

// Sweep-wide constants every update kernel needs.
struct SweepCtx {
  uint64_t key0, key1;      // Philox key (seed, walker id)
  uint64_t sweep;           // counter word 0 (unless sweep_dev is set)
  const uint64_t *sweep_dev;  // graph-captured sweeps: counter word 0 read from here
  uint64_t slice_code;      // counter word 1: dir * M + (l - 1)
  int li;                   // slice index l - 1 into the field array
  int N;                    // sites
  int8_t *fields;           // M x N
  double dflip[2][2];       // e^{-2 alpha f_s x} - 1 for [spin][x>0 ? 0 : 1]
  double dremove[2][2];     // e^{-alpha f_s x} - 1 (block force bias)
  double alpha;             // real coupling
  unsigned long long *stats;  // device counters
  int32_t *log_meta;        // 3 ints per decision (or null)
  double *log_margin;
  int32_t *hb_meta;
  double *hb_margin;
  long long log_base;       // index of this slice's first decision in the log
  long long hb_base;        // index of this slice's first heat-bath draw (+ site)
  long long log_cap;
  // Replay (null otherwise): this slice visit's forced outcomes, one per site
  // (nonzero: the site's field flips).  A forced Metropolis test draws
  // u = -0 (accepted for any nonzero finite ratio, and the logged margin
  // |A| - u is |A| itself) or u = +inf (rejected); a forced heat-bath draw
  // proposes the listed field by the same two values.
  const int8_t *force;
};

// Philox counter word 0 of the current sweep: a value baked into the launch,
// or read from device memory when the sweep is a replayed graph
__device__ __forceinline__ uint64_t sweep_of(uint64_t v, const uint64_t *dev) {
  return dev ? *dev : v;
}

// uniform that forces an outcome of "accept iff u < a" for any finite a > 0
__device__ __forceinline__ double forced_uniform(bool take) {
  return take ? -0.0 : __builtin_inf();
}

// stats slots
enum { kStProposed = 0, kStAccepted = 1, kStFlips = 2, kStLowMargin = 3, kStNegative = 4,
       kStFieldUpdates = 5, kStError = 8, kStDrift = 9 };
enum { kErrNonFinite = 1, kErrSingular = 2, kErrBarrier = 4 };

// sum_{i < n} p[i * stride] in index order; loads issued eight at a time so
// the partial-sum chains are not serialised on memory latency.
__device__ __forceinline__ double sum_strided(const double *p, long stride, int n) {
  double s = 0.0;
  for (int b = 0; b < n; b += 8) {
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (b + i < n) ? p[(long)(b + i) * stride] : 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
  }
  return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace pq

#define PQ_HIP_CHECK(expr)                                                        \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) return ::pq::fail_device(_e, #expr, __FILE__, __LINE__); \
  } while (0)
