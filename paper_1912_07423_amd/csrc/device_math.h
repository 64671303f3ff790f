// device_math.h -- counter-based random numbers, the binary64 logarithm of the
// spacing generator, and wavefront (64-lane) primitives for gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

constexpr uint32_t kStreamConn = 1u;
constexpr uint32_t kStreamVinit = 2u;
constexpr uint32_t kStreamPoisson = 3u;
constexpr int kWave = 64;

struct Words4 {
  uint32_t w[4];
};

// Philox4x32-10 (Salmon et al., SC'11): per round, multiply words 0 and 2 by the two
// Philox multipliers, recombine the high halves with words 1 and 3 and the round
// key, keep the low halves; bump the key by the two Weyl constants.
__device__ __forceinline__ Words4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32 x 32 -> 64-bit product gives both halves (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words4 r;
  r.w[0] = c0;
  r.w[1] = c1;
  r.w[2] = c2;
  r.w[3] = c3;
  return r;
}

// -ln(u), u in (0, 1], as a fixed sequence of IEEE binary64 operations: split
// u = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh((m-1)/(m+1)) as
// 2r * sum_{n<=11} z^n/(2n+1), z = r^2, by Horner with fused multiply-adds;
// ln u = fma(e, ln 2, ln m).
__device__ __forceinline__ double neg_log(double u) {
  constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
  constexpr double kLn2 = 0x1.62e42fefa39efp-1;
  int e = 0;
  double m = frexp(u, &e);
  if (m < kSqrtHalf) {
    m = m + m;
    e = e - 1;
  }
  const double r = (m - 1.0) / (m + 1.0);
  const double z = r * r;
  double acc = 1.0 / 23.0;
#pragma unroll
  for (int n = 10; n >= 0; --n) acc = fma(acc, z, 1.0 / (double)(2 * n + 1));
  const double ln_m = (r + r) * acc;
  return -fma((double)e, kLn2, ln_m);
}

// Gap of the spacing generator in 2^-24 fixed point from one 32-bit word.
__device__ __forceinline__ uint64_t spacing_gap(uint32_t word) {
  const double u = (double)((word >> 8) + 1u) * 0x1p-24;
  return (uint64_t)(neg_log(u) * 16777216.0);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const T y = __shfl_up(x, d, kWave);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// 32-bit inclusive scan over the wave by DPP lane shifts (one VALU operation per step
// instead of an LDS permute): shifts by 1, 2, 4 and 8 inside each row of 16 lanes, then
// the last lane of rows 0 and 2 added into rows 1 and 3, then lane 31 into rows 2 and 3.
// Every lane of the wave must be active.
template <>
__device__ __forceinline__ uint32_t wave_inclusive_scan<uint32_t>(uint32_t x) {
  int v = (int)x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false); // row_bcast:15, rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false); // row_bcast:31, rows 2 and 3
  return (uint32_t)v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

// Constants of the LIF update (Sec. IV: current-based LIF), derived once on the host.
struct LifConst {
  float alpha;      // fl32(exp(-dt / tau_m))
  float v_inf;      // fl32(V_rest + V_bg)
  float v_th, v_reset;
  int32_t ref_steps;
  int32_t w_ext_q16;  // Q16 weight of one virtual drive input
};

// One neuron, one step, in binary32 without contraction and in this order: a
// refractory neuron counts down and discards its input; otherwise the Q16 input plus
// k drive inputs (int32, wrapping) is added to V, V leaks towards v_inf by alpha, and
// V >= V_th emits a spike, resets V and starts the refractory count.  Returns the spike.
// Written without branches: the candidate V is computed for every lane and a
// refractory lane keeps its old V (the same values as skipping the computation).
__device__ __forceinline__ bool lif_advance(float &v, int32_t &ref, int32_t input, int32_t k,
                                            const LifConst &c) {
  const bool refractory = ref > 0;
  const uint32_t sum = (uint32_t)input + (uint32_t)k * (uint32_t)c.w_ext_q16;
  const float dv = (float)(int32_t)sum * 0x1p-16f;
  float vv = v + dv;
  const float diff = vv - c.v_inf;
  const float leak = diff * c.alpha;
  vv = c.v_inf + leak;
  const bool spike = !refractory && vv >= c.v_th;
  v = refractory ? v : (spike ? c.v_reset : vv);
  ref = refractory ? ref - 1 : (spike ? c.ref_steps : ref);
  return spike;
}

// Word u (0..3) of a Philox block by selects, never by a dynamic register index.
__device__ __forceinline__ uint32_t word_of(const Words4 &r, uint32_t u) {
  const uint32_t lo = (u & 1u) ? r.w[1] : r.w[0];
  const uint32_t hi = (u & 1u) ? r.w[3] : r.w[2];
  return (u & 2u) ? hi : lo;
}

}  // namespace snn
