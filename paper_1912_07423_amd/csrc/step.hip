// step.hip -- the per-step kernels of the work-queue pipeline (Sec. III-A.1, Fig. 1).
//
//  k_update          Update Neurons for a window of consecutive steps: each lane owns
//                    one neuron and keeps V/ref/traces in registers across the window;
//                    the ballot of each step is both the step's raster word and the
//                    compaction mask of the spike queue (one queue reservation per
//                    workgroup and step).
//  k_deliver_atomic  Receive Spikes, one or more wavefronts per dequeued spike,
//                    aligned 16-byte loads of targets/weights, no-return int32 atomics
//                    into the Q16 input accumulators in global memory.
//  k_deliver_tiled   Receive Spikes, one workgroup per (range of target tiles, emission
//                    step): the workgroup reads the range's slice of every dequeued
//                    spike's sorted row from the 16-bit copy of the targets (weights
//                    per source, per synapse in Q16, or plastic FP32 ones), accumulates
//                    in LDS with int32 atomics and writes the range's input
//                    accumulators with plain stores.  With eager STDP both deliveries
//                    also advance the traces in one extra workgroup.
//  k_stdp_fused      Update Synapses: depression over S_{t-d}'s plastic out-edges and
//                    potentiation over S_t's plastic in-edges (transposed index).
//  k_stdp_ltd, k_lazy  the lazy form: depression, then pending potentiation replayed
//                    at transmission or expiry, with the delivery of the transmitting
//                    rows.
//
// Step bookkeeping lives on the device (Ctl) so that a captured HIP graph replays
// correctly; no kernel waits on another workgroup of its own launch.
#include <algorithm>

#include "device_math.h"
#include "snn_internal.h"

namespace snn {
namespace {

// Ring indices: the window's first step is reduced modulo each ring size once per
// launch; step t0 + w is then reached by one conditional subtraction, which needs
// w < size (the window fits every ring, checked by the host).
__device__ __forceinline__ uint32_t ring_add(uint32_t base, uint32_t w, uint32_t size) {
  const uint32_t x = base + w;
  return x >= size ? x - size : x;
}

// floor-modulo of a possibly negative step
__device__ __forceinline__ uint32_t ring_of(int64_t x, uint32_t size) {
  const int64_t r = x % (int64_t)size;
  return (uint32_t)(r < 0 ? r + size : r);
}

__device__ __forceinline__ uint32_t *qcount(const QueueRef &q, uint32_t slot, uint32_t g) {
  return q.qlen + (size_t)(slot * kQueueGroups + g) * kQlenStride;
}

// Exclusive prefix of the sub-queue lengths of one slot: pre[kQueueGroups] = total.
__device__ __forceinline__ void queue_prefix(const QueueRef &q, uint32_t slot,
                                             uint32_t (&pre)[kQueueGroups + 1]) {
  pre[0] = 0;
#pragma unroll
  for (uint32_t g = 0; g < kQueueGroups; ++g) pre[g + 1] = pre[g] + min(*qcount(q, slot, g), q.group_cap);
}

// The f-th spike (f < pre[kQueueGroups]) of a slot.
__device__ __forceinline__ int32_t queue_entry(const QueueRef &q, uint32_t slot,
                                               const uint32_t (&pre)[kQueueGroups + 1], uint32_t f) {
  uint32_t g = 0;
#pragma unroll
  for (uint32_t k = 1; k < kQueueGroups; ++k) g += f >= pre[k] ? 1u : 0u;
  return q.ids[(size_t)slot * q.stride + g * q.group_cap + (f - pre[g])];
}

__device__ __forceinline__ void add_part(uint64_t *counter, uint32_t part, uint64_t x) {
  if (x) atomicAdd((unsigned long long *)&counter[(part % kCounterParts) * kLineU64], (unsigned long long)x);
}

constexpr int kUpdateWaves = kUpdateBlock / kWave;
constexpr int kPrefetch = 16;  // steps of input in flight (4 quads)
constexpr int kShortQuads = 5;  // windows of 4 or 5 quads take the batched path

// Update Neurons for `steps` (<= 64) consecutive steps.  The LIF arithmetic is
// sequential per neuron; the rest is batched.  Steps are processed in quads aligned
// to absolute time (one Philox block per quad, its word t mod 4 feeding step t); the
// inputs of the next 4 quads are always in flight (a rolling register window, static
// indices only); the ballot of step w is parked in lane w; after the loop one thread
// per step reserves the workgroup's space in its sub-queue with one atomic.
// The drive count k = #{j : tbl[j] <= r} over the thresholds below 2^32 (an entry
// equal to 2^32 cannot be reached by a 32-bit word) is found from a guide table over
// the top 12 bits of r, which holds the count at both ends of each bucket, plus a
// short scan when a threshold falls inside the bucket.
// The drive and the LIF arithmetic run on every lane without branching on the neuron's
// state: a refractory neuron discards its drive inside lif_advance, and a lane past n
// never reports a spike or stores.
// kShort: the launch's windows span 4 or 5 quads (13 to 17 steps) and take the batched
// path; other window lengths are built without it (fewer registers and less code).
template <bool kShort>
__global__ __launch_bounds__(kUpdateBlock) void k_update(UpdateArgs a, uint32_t steps) {
  __shared__ __align__(16) uint32_t tbl[kTableCap];
  __shared__ __align__(16) uint16_t guide[kGuideBuckets];
  __shared__ uint32_t s_base[kUpdateWaves][kWave];
  __shared__ uint32_t s_exp[kUpdateWaves];  // lazy plasticity: expiring rows per wave, then base
  static_assert(kTableCap / 4 <= kUpdateBlock && kGuideBuckets / 8 == 2 * kUpdateBlock,
                "one 16-byte table load per lane, two guide loads");

  const uint64_t t0 = a.ctl->t;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->t_deliver = t0;
  const uint32_t in0 = (uint32_t)(t0 % a.n_inbuf);
  const uint32_t slot0 = (uint32_t)(t0 % a.slots);
  const uint32_t ras0 = (uint32_t)(t0 % a.raster_cap);
  const uint32_t off = (uint32_t)(t0 & 3u);      // position of t0 in its quad
  const uint64_t quad0 = t0 >> 2;
  const uint32_t n_quads = (off + steps + 3) >> 2;
  const uint32_t group = blockIdx.x % kQueueGroups;
  const uint32_t i = blockIdx.x * kUpdateBlock + threadIdx.x;
  const bool active = i < a.n;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t word = i / kWave;
  const bool drive = a.table_len > 1;
  const LifConst lif{a.alpha, a.v_inf, a.v_th, a.v_reset, a.ref_steps, a.w_ext_q16};

  // input of window position p = w + off (w = p - off), zeroed behind the read if the
  // delivery accumulates with atomics
  auto load_input = [&](int32_t p) -> int32_t {
    const int32_t w = p - (int32_t)off;
    if (!active || w < 0 || w >= (int32_t)steps) return 0;
    int32_t *in = a.input + (size_t)ring_add(in0, (uint32_t)w, a.n_inbuf) * a.n + i;
    const int32_t x = *in;
    if (a.zero_input) *in = 0;
    return x;
  };

  // ---- one round trip: drive tables (16-byte loads, issued first so that waiting for
  //      them leaves the later loads in flight), state, first kPrefetch inputs ----
  int4 tv = {0, 0, 0, 0}, gv0 = {0, 0, 0, 0}, gv1 = {0, 0, 0, 0};
  if (drive) {
    if (threadIdx.x < kTableCap / 4) tv = reinterpret_cast<const int4 *>(a.table32)[threadIdx.x];
    gv0 = reinterpret_cast<const int4 *>(a.guide)[threadIdx.x];
    gv1 = reinterpret_cast<const int4 *>(a.guide)[threadIdx.x + kUpdateBlock];
  }
  float v = 0.f, xp = 0.f, xq = 0.f;
  int32_t ref = 0;
  const bool lazy = a.lazy.hist != nullptr;  // one step per launch
  uint64_t hist = 0;
  uint32_t age = 0, plen = 0;
  if (active) {
    v = a.v[i];
    ref = a.ref[i];
    if (a.plastic) {
      xp = a.x_pre[i];
      xq = a.x_post[i];
    }
    if (lazy) {
      hist = a.lazy.hist[i];
      age = a.lazy.age[i];
      plen = a.lazy.plast_len[i];
    }
  }
  int32_t acc[kPrefetch];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) acc[j] = load_input(j);
  if (drive) {
    if (threadIdx.x < kTableCap / 4) reinterpret_cast<int4 *>(tbl)[threadIdx.x] = tv;
    reinterpret_cast<int4 *>(guide)[threadIdx.x] = gv0;
    reinterpret_cast<int4 *>(guide)[threadIdx.x + kUpdateBlock] = gv1;
  }
  __syncthreads();

  uint64_t my_mask = 0;    // lane w: ballot of step w
  uint64_t my_spikes = 0;  // bit w: this neuron spiked at step w
  // One LIF step at window position p (step w = p - off) with drive count k.
  auto lif_step = [&](int32_t p, int32_t x, int32_t k) {
    const int32_t w = p - (int32_t)off;
    const bool spike = lif_advance(v, ref, x, k, lif) && active;
    if (a.plastic) {
      xp = xp * a.beta_plus;
      xq = xq * a.beta_minus;
    }
    const uint64_t mask = __ballot(spike);
    if (lane == (uint32_t)w) my_mask = mask;
    if (spike) my_spikes |= 1ull << w;
  };
  if (kShort && n_quads >= kShortQuads - 1 && n_quads <= kShortQuads) {
    // A window of 4 or 5 quads (a 15-step window): its Philox blocks and all its drive
    // lookups are independent of the membrane, so they are issued side by side first
    // (their latencies overlap), then the LIF steps run.  Shorter and longer windows
    // take the rolling loop below.
    int32_t xs[4 * kShortQuads];
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) xs[j] = acc[j];
#pragma unroll
    for (int j = kPrefetch; j < 4 * kShortQuads; ++j) xs[j] = load_input(j);
    int32_t kd[4 * kShortQuads];
    if (drive) {
      Words4 rnd[kShortQuads];
#pragma unroll
      for (int q = 0; q < kShortQuads; ++q) {
        const uint64_t qa = quad0 + (uint64_t)q;
        rnd[q] = Words4{};
        if ((uint32_t)q < n_quads)  // uniform
          rnd[q] = philox(i, (uint32_t)qa, (uint32_t)(qa >> 32), kStreamPoisson, a.key0, a.key1);
      }
      uint32_t gk[4 * kShortQuads];
#pragma unroll
      for (int j = 0; j < 4 * kShortQuads; ++j)
        gk[j] = (uint32_t)(j >> 2) < n_quads ? guide[rnd[j >> 2].w[j & 3] >> (32 - kGuideBits)] : 0u;
#pragma unroll
      for (int j = 0; j < 4 * kShortQuads; ++j) {
        const uint32_t r = rnd[j >> 2].w[j & 3];
        int32_t k = (int32_t)(gk[j] & 0xFFu);
        const int32_t k_hi = (int32_t)(gk[j] >> 8);
        while (k < k_hi && tbl[k] <= r) ++k;
        kd[j] = k;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4 * kShortQuads; ++j) kd[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < 4 * kShortQuads; ++j) {
      const int32_t w = j - (int32_t)off;
      if (w >= 0 && w < (int32_t)steps) lif_step(j, xs[j], kd[j]);  // uniform
    }
  } else {
  for (uint32_t qq = 0; qq < n_quads; ++qq) {
    Words4 rnd{};
    if (drive)
      rnd = philox(i, (uint32_t)(quad0 + qq), (uint32_t)((quad0 + qq) >> 32), kStreamPoisson, a.key0, a.key1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t w = (int32_t)(4 * qq + u) - (int32_t)off;
      if (w < 0 || w >= (int32_t)steps) continue;  // uniform
      int32_t k = 0;
      if (drive) {
        const uint32_t r = rnd.w[u];
        const uint32_t gk = guide[r >> (32 - kGuideBits)];
        k = (int32_t)(gk & 0xFFu);
        const int32_t k_hi = (int32_t)(gk >> 8);
        while (k < k_hi && tbl[k] <= r) ++k;
      }
      lif_step((int32_t)(4 * qq + u), acc[u], k);
    }
    // roll the input window by one quad and request the quad kPrefetch / 4 ahead
#pragma unroll
    for (int j = 0; j < kPrefetch - 4; ++j) acc[j] = acc[j + 4];
#pragma unroll
    for (int j = kPrefetch - 4; j < kPrefetch; ++j) acc[j] = load_input((int32_t)(4 * (qq + 1)) + j);
  }
  }
  if (active) {
    a.v[i] = v;
    a.ref[i] = ref;
    if (a.plastic) {
      a.x_pre[i] = xp;
      a.x_post[i] = xq;
    }
  }
  // Lazy plasticity: the spike history gains this step's bit; a plastic row whose pending
  // steps [age, t0] fill the whole history expires now, unless it transmits now (its
  // spike of step t0 - d + 1, history bit d - 1), which brings it current anyway.
  bool expiring = false;
  uint64_t emask = 0;
  if (lazy) {
    hist = (hist << 1) | (my_spikes & 1u);
    const uint32_t pending = (uint32_t)t0 - age + 1u;
    const bool transmits = (hist >> (a.lazy.delay - 1u)) & 1u;
    expiring = active && plen > 0 && pending >= kLazyHistory && !transmits;
    if (active) a.lazy.hist[i] = hist;
    emask = __ballot(expiring);
    if (lane == 0) s_exp[wave] = (uint32_t)__popcll(emask);
  }
  // raster rows and queue reservations of the whole window, one lane per step
  if (lane < steps) {
    if (word < a.words) a.raster[(size_t)ring_add(ras0, lane, a.raster_cap) * a.words + word] = my_mask;
    s_base[wave][lane] = (uint32_t)__popcll(my_mask);
  }
  __syncthreads();
  if (lazy && threadIdx.x == kUpdateBlock - 1) {  // not one of the step threads below
    uint32_t total = 0;
    for (int v2 = 0; v2 < kUpdateWaves; ++v2) {
      const uint32_t c = s_exp[v2];
      s_exp[v2] = total;
      total += c;
    }
    const uint32_t base = total ? atomicAdd(qcount(a.lazy.exq, (uint32_t)(t0 & 1u), group), total) : 0u;
    for (int v2 = 0; v2 < kUpdateWaves; ++v2) s_exp[v2] += base;
  }
  if (threadIdx.x < steps) {
    const uint32_t w = threadIdx.x;
    uint32_t total = 0;
    for (int v2 = 0; v2 < kUpdateWaves; ++v2) {
      const uint32_t c = s_base[v2][w];
      s_base[v2][w] = total;
      total += c;
    }
    const uint32_t base = total ? atomicAdd(qcount(a.q, ring_add(slot0, w, a.slots), group), total) : 0u;
    for (int v2 = 0; v2 < kUpdateWaves; ++v2) s_base[v2][w] += base;
  }
  __syncthreads();
  for (uint32_t w = 0; w < steps; ++w) {
    // step w's ballot from lane w (uniform w: two lane reads, no LDS round trip)
    const uint64_t mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(my_mask >> 32), (int)w) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)my_mask, (int)w);
    if (!mask) continue;
    const uint32_t pos = s_base[wave][w] + lanes_below(mask);
    const uint32_t slot = ring_add(slot0, w, a.slots);
    if (((my_spikes >> w) & 1u) && pos < a.q.group_cap)
      a.q.ids[(size_t)slot * a.q.stride + group * a.q.group_cap + pos] = (int32_t)i;
  }
  if (expiring) {
    const uint32_t pos = s_exp[wave] + lanes_below(emask);
    if (pos < a.lazy.exq.group_cap)
      a.lazy.exq.ids[(size_t)(t0 & 1u) * a.lazy.exq.stride + group * a.lazy.exq.group_cap + pos] = (int32_t)i;
  }
}

// Emission step of the w-th queue delivered by a window starting at t0: spikes of step
// e land in input buffer (e + d) mod n_inbuf, to be read by the update of step e + d.
__device__ __forceinline__ int64_t emission_step(const DeliverArgs &a, uint64_t t0, uint32_t w) {
  return (int64_t)t0 + (int64_t)w + (int64_t)a.n_inbuf - (int64_t)a.delay;
}

// The delivery launch that closes a window clears the next window's queue counters and
// advances the step.  Done by one thread at launch start: no workgroup of this launch
// reads the next window's counters or `t` (they read `t_deliver`), and the next
// launches see the writes after the kernel boundary.
__device__ __forceinline__ void close_window(const DeliverArgs &a, uint64_t t0, uint32_t steps) {
  if (a.advance && blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t next = (uint32_t)((t0 + steps) % a.slots);
    for (uint32_t w = 0; w < a.window_max; ++w)
      for (uint32_t g = 0; g < kQueueGroups; ++g) *qcount(a.q, ring_add(next, w, a.slots), g) = 0u;
    a.ctl->t = t0 + steps;
  }
}

// Eager STDP (one step t = t0 per launch): after the step's plasticity pass has read
// the traces, the delivery launch's last workgroup adds the arrivals S_{t-d} to x_pre
// and S_t to x_post, beside the delivery done by the others.  A spike appears once in
// its step's queue, so every trace has one writer.
template <int kThreads>
__device__ void advance_traces(const DeliverArgs &a, uint64_t t0) {
  const uint32_t slot_t = (uint32_t)(t0 % a.slots);
  const bool has_d = t0 >= a.delay;
  const uint32_t slot_d = has_d ? (uint32_t)((t0 - a.delay) % a.slots) : 0u;
  uint32_t pt[kQueueGroups + 1], pd[kQueueGroups + 1] = {};
  queue_prefix(a.q, slot_t, pt);
  if (has_d) queue_prefix(a.q, slot_d, pd);
  for (uint32_t f = threadIdx.x; f < pt[kQueueGroups]; f += kThreads) {
    const int32_t j = queue_entry(a.q, slot_t, pt, f);
    if ((uint32_t)j < a.n) a.x_post[j] = a.x_post[j] + 1.0f;
  }
  for (uint32_t f = threadIdx.x; f < pd[kQueueGroups]; f += kThreads) {
    const int32_t i = queue_entry(a.q, slot_d, pd, f);
    if ((uint32_t)i < a.n) a.x_pre[i] = a.x_pre[i] + 1.0f;
  }
}

// Disjoint parts per queued spike, one wavefront each, so that a launch's wavefronts
// cover the spikes about once: a step of a plastic network has only ~100 spikes, which
// one wavefront each would leave most of the GPU idle and walk each row serially.
__device__ __forceinline__ uint32_t parts_for(uint32_t spikes, uint32_t waves, uint32_t max_parts) {
  const uint32_t p = spikes ? waves / spikes : 1u;
  return p < 1u ? 1u : (p > max_parts ? max_parts : p);
}

constexpr int kAtomicBlock = 256;
constexpr int kAtomicWaves = kAtomicBlock / kWave;
constexpr uint32_t kAtomicMaxParts = 32;

constexpr int kWeightQ16 = 0, kWeightF32 = 1, kWeightSrc = 2;

// kW: weights per synapse in Q16 (kWeightQ16) or FP32 (kWeightF32), or one per source (kWeightSrc)
template <int kW>
__global__ __launch_bounds__(kAtomicBlock) void k_deliver_atomic(DeliverArgs a, uint32_t steps) {
  __shared__ uint32_t s_pre[kWave][kQueueGroups + 1];  // per step: sub-queue prefix
  __shared__ uint32_t s_slot[kWave];
  __shared__ uint32_t s_step[kWave + 1];               // prefix of the per-step totals
  const uint64_t t0 = a.ctl->t_deliver;
  close_window(a, t0, steps);
  const bool trace_wg = a.x_post != nullptr && blockIdx.x + 1 == gridDim.x && gridDim.x > 1;
  if (trace_wg) {
    advance_traces<kAtomicBlock>(a, t0);
    return;
  }
  const uint32_t deliver_grid = a.x_post != nullptr && gridDim.x > 1 ? gridDim.x - 1 : gridDim.x;
  const int64_t e0 = emission_step(a, t0, 0);
  const uint32_t eslot0 = ring_of(e0, a.slots);
  const uint32_t in0 = (uint32_t)(t0 % a.n_inbuf);
  const uint32_t lane = lane_id();
  if (threadIdx.x < kWave) {
    uint32_t pre[kQueueGroups + 1] = {};
    const uint32_t w = threadIdx.x;
    uint32_t slot = 0;
    if (w < steps && e0 + (int64_t)w >= 0) {
      slot = ring_add(eslot0, w, a.slots);
      queue_prefix(a.q, slot, pre);
    }
    s_slot[w] = slot;
#pragma unroll
    for (uint32_t g = 0; g <= kQueueGroups; ++g) s_pre[w][g] = pre[g];
    const uint32_t c = pre[kQueueGroups];
    const uint32_t incl = wave_inclusive_scan(c);
    s_step[w + 1] = incl;
    if (w == 0) s_step[0] = 0;
  }
  __syncthreads();
  const uint32_t total = s_step[kWave];
  const uint32_t gwave = blockIdx.x * kAtomicWaves + threadIdx.x / kWave;
  const uint32_t n_gwaves = deliver_grid * kAtomicWaves;
  uint64_t ev = 0, n_spk = 0;
  const uint32_t parts = parts_for(total, n_gwaves, kAtomicMaxParts);
  for (uint64_t item = gwave; item < (uint64_t)total * parts; item += n_gwaves) {
    const uint32_t f = (uint32_t)(item / parts), part = (uint32_t)(item % parts);
    uint32_t w = 0;  // step of spike f: last w with s_step[w] <= f
    for (uint32_t half = kWave / 2; half > 0; half >>= 1)
      if (s_step[w + half] <= f) w += half;
    uint32_t pre[kQueueGroups + 1];
#pragma unroll
    for (uint32_t g = 0; g <= kQueueGroups; ++g) pre[g] = s_pre[w][g];
    const int32_t src = queue_entry(a.q, s_slot[w], pre, f - s_step[w]);
    if ((uint32_t)src >= a.n) continue;
    int32_t *in = a.input + (size_t)ring_add(in0, w, a.n_inbuf) * a.n;
    const uint64_t rs = a.row_ptr[src], re = a.row_ptr[src + 1];
    const int32_t ws = kW == kWeightSrc ? a.w_src[src] : 0;
    // this part's contiguous share of the row's 16-byte groups
    const uint64_t g_lo = rs >> 2, g_hi = (re + 3) >> 2;
    const uint64_t share = (g_hi - g_lo + parts - 1) / parts;
    const uint64_t p_lo = g_lo + part * share, p_hi = min(g_hi, p_lo + share);
    for (uint64_t g = p_lo + lane; g < p_hi; g += kWave) {
      const int4 c4 = reinterpret_cast<const int4 *>(a.col)[g];
      int32_t wv[4];
      if constexpr (kW == kWeightSrc) {
        wv[0] = wv[1] = wv[2] = wv[3] = ws;
      } else if constexpr (kW == kWeightF32) {
        const float4 f4 = reinterpret_cast<const float4 *>(a.w_f32)[g];
        wv[0] = __float2int_rn(f4.x * 65536.0f);
        wv[1] = __float2int_rn(f4.y * 65536.0f);
        wv[2] = __float2int_rn(f4.z * 65536.0f);
        wv[3] = __float2int_rn(f4.w * 65536.0f);
      } else {
        const int4 w4 = reinterpret_cast<const int4 *>(a.w_q16)[g];
        wv[0] = w4.x;
        wv[1] = w4.y;
        wv[2] = w4.z;
        wv[3] = w4.w;
      }
      const int32_t cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t idx = 4 * g + q;
        if (idx >= rs && idx < re)
          __hip_atomic_fetch_add(in + cv[q], wv[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (part == 0) {
      ev += re - rs;
      ++n_spk;
    }
  }
  if (lane == 0) {
    add_part(a.ctl->events, gwave, ev);
    add_part(a.ctl->spikes, gwave, n_spk);
  }
}

// 16-byte groups per lane per batch (8 targets each; with weights stored per synapse,
// also their 32 bytes of weights).  A wave's share of a step is short (about 14 groups
// per lane on the 1e9-synapse network), so two per batch, with the next two in flight,
// beat three or four: the last, partly filled batch is shorter.  Three or four batches
// in flight instead of two measured no faster: the stream then runs at the rate the
// memory system gives pieces of a few hundred bytes at random addresses.
constexpr int tiled_groups() { return 2; }

// One 16-byte group of the tiled delivery's target stream: 8 consecutive 16-bit
// targets of the flattened sub-rows, the Q16 weights of those 8 synapses (w0: 0-3,
// w1: 4-7; with source weights w0.x is the sub-row's weight), and the mask of the
// elements that lie inside the sub-row.
struct TiledGroup {
  int4 c, w0, w1;
  uint32_t mask;
};

// Sub-rows are streamed as 16-byte aligned groups of 8 synapses of the 16-bit target
// array; the elements of a group outside its sub-row are masked off.  Loads kU groups of
// the flattened group range, 64 apart, from this lane's group `first`; `o` is the lane's
// current sub-row (monotone).  FP32 weights (plastic synapses) are taken to Q16 with the
// atomic delivery's rounding: round(w * 2^16), ties to even.
template <int kU, int kW>
__device__ __forceinline__ void tiled_load(const DeliverArgs &a, const uint64_t *s_lo,
                                           const uint32_t *s_len, const uint32_t *s_pre,
                                           const int32_t *s_w, uint32_t first, uint32_t end,
                                           uint32_t &o, TiledGroup (&gr)[kU]) {
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const uint32_t idx = first + u * kWave;
    gr[u].mask = 0;
    gr[u].w0 = make_int4(0, 0, 0, 0);
    gr[u].w1 = make_int4(0, 0, 0, 0);
    if (idx < end) {
      while (s_pre[o + 1] <= idx) ++o;
      const uint64_t lo = s_lo[o], hi = lo + s_len[o];
      const uint64_t g = (lo >> 3) + (idx - s_pre[o]);
      gr[u].c = reinterpret_cast<const int4 *>(a.col16)[g];
      if constexpr (kW == kWeightSrc) {
        gr[u].w0.x = s_w[o];
      } else if constexpr (kW == kWeightF32) {
        const float4 f0 = reinterpret_cast<const float4 *>(a.w_f32)[2 * g];
        const float4 f1 = reinterpret_cast<const float4 *>(a.w_f32)[2 * g + 1];
        gr[u].w0 = make_int4(__float2int_rn(f0.x * 65536.0f), __float2int_rn(f0.y * 65536.0f),
                             __float2int_rn(f0.z * 65536.0f), __float2int_rn(f0.w * 65536.0f));
        gr[u].w1 = make_int4(__float2int_rn(f1.x * 65536.0f), __float2int_rn(f1.y * 65536.0f),
                             __float2int_rn(f1.z * 65536.0f), __float2int_rn(f1.w * 65536.0f));
      } else {
        gr[u].w0 = reinterpret_cast<const int4 *>(a.w_q16)[2 * g];
        gr[u].w1 = reinterpret_cast<const int4 *>(a.w_q16)[2 * g + 1];
      }
      const uint64_t e0 = g << 3;
      const uint32_t first_q = lo > e0 ? (uint32_t)(lo - e0) : 0u;
      const uint32_t last_q = hi - e0 < 8 ? (uint32_t)(hi - e0) : 8u;
      gr[u].mask = ((1u << last_q) - 1u) & ~((1u << first_q) - 1u);
    }
  }
}

// Adds the masked elements of one group into the range's LDS accumulators.  A range
// spans fewer than 65,536 targets, so a target t of the range is recovered from its low
// 16 bits: t - range_lo = (t16 - range_lo) mod 2^16.
template <int kW>
__device__ __forceinline__ void tiled_accumulate(int32_t *acc, const TiledGroup &g, uint32_t range_lo) {
  const uint32_t words[4] = {(uint32_t)g.c.x, (uint32_t)g.c.y, (uint32_t)g.c.z, (uint32_t)g.c.w};
  const int32_t w[8] = {g.w0.x, g.w0.y, g.w0.z, g.w0.w, g.w1.x, g.w1.y, g.w1.z, g.w1.w};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (g.mask & (1u << k)) {
      const uint32_t t16 = (k & 1) ? words[k >> 1] >> 16 : words[k >> 1];
      atomicAdd(&acc[(t16 - range_lo) & 0xFFFFu], kW == kWeightSrc ? w[0] : w[k]);
    }
  }
}

// Balanced schedule of one window, derived by every workgroup from the step counts
// c_w with the same operations on the same values, so that all derive one schedule.
// Step w is cut into r_w ranges of consecutive base tiles, one workgroup each; range j
// covers tiles [floor(j P / r_w), floor((j + 1) P / r_w)) of the P tiles.  A range's
// work is about c_w P / r_w sub-rows, so the schedule takes
//   r_w(X) = clamp(ceil(c_w P / X), r_min, P),   r_min = ceil(P / kTileGroupMax),
// for (close to) the smallest work bound X at which sum_w r_w(X) fits the grid.  r_min
// keeps every range within kTileGroupMax tiles (the LDS accumulators); the host sizes
// the grid to at least steps * r_min, where an infinite X (every r_w = r_min) fits.
struct TileSchedule {
  uint32_t r[kWave];          // ranges of each step
  uint32_t first[kWave + 1];  // first work unit of each step
};

// r_w at the bound X = 1 / inv_x (inv_x = 0: X infinite) for work = c_w * P.
__device__ __forceinline__ uint32_t ranges_at(float work, float inv_x, uint32_t r_min, uint32_t tiles) {
  const float q = ceilf(work * inv_x);
  return (uint32_t)fminf(fmaxf(q, (float)r_min), (float)tiles);
}

// sum_w r_w at this lane's bound; c is lane w's count (zero past `steps`).
__device__ __forceinline__ uint32_t ranges_needed(uint32_t c, uint32_t steps, float p_f, float inv_x,
                                                  uint32_t r_min, uint32_t tiles) {
  uint32_t sum = 0;
  for (uint32_t w = 0; w < steps; ++w) {
    const float work = (float)(uint32_t)__builtin_amdgcn_readlane((int)c, (int)w) * p_f;
    sum += ranges_at(work, inv_x, r_min, tiles);
  }
  return sum;
}

// Wave 0 (lane w holds c_w, zero past `steps`): the bound by two parallel rounds over
// the 64 lanes, then each step's range count and their prefix.  Round 1 tries
// X_j = X_lb 2^(j/4), X_lb = sum_w c_w P / grid (below it no schedule fits unless ranges
// are clamped to single tiles; round 2 then still finds the bound); round 2 tries 64
// evenly spaced bounds in (X_{j-1}, X_j] for the first feasible X_j, the last being X_j
// itself.  Without a feasible X_j every step takes r_min ranges.
__device__ void make_schedule(uint32_t c, uint32_t steps, uint32_t tiles, uint32_t grid, TileSchedule &sch) {
  const uint32_t lane = lane_id();
  const uint32_t r_min = (tiles + kTileGroupMax - 1) / kTileGroupMax;
  const float p_f = (float)tiles;
  const uint32_t total = wave_sum(c);
  float inv_best = 0.f;
  if (total > 0 && grid > steps * r_min) {
    const float x_lb = (float)total * p_f / (float)grid;
    const float x1 = x_lb * exp2f(0.25f * (float)lane);
    const uint64_t ok1 = __ballot(ranges_needed(c, steps, p_f, 1.0f / x1, r_min, tiles) <= grid);
    if (ok1) {
      const uint32_t j = (uint32_t)__builtin_ctzll(ok1);
      const float hi = x_lb * exp2f(0.25f * (float)j);
      const float lo = j ? x_lb * exp2f(0.25f * (float)(j - 1)) : 0.f;
      const float x2 = lane == kWave - 1 ? hi : lo + (hi - lo) * ((float)(lane + 1) * (1.0f / kWave));
      const float inv2 = 1.0f / x2;
      const uint64_t ok2 = __ballot(ranges_needed(c, steps, p_f, inv2, r_min, tiles) <= grid);
      const uint32_t k = ok2 ? (uint32_t)__builtin_ctzll(ok2) : kWave - 1;  // lane 63 fits: x2 = X_j
      inv_best = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(inv2), (int)k));
    }
  }
  const uint32_t r = lane < steps ? ranges_at((float)c * p_f, inv_best, r_min, tiles) : 0u;
  const uint32_t incl = wave_inclusive_scan(r);
  sch.r[lane] = r;
  sch.first[lane + 1] = incl;
  if (lane == 0) sch.first[0] = 0;
}

constexpr uint32_t kXcds = 8;  // accelerator complex dies, each with its own L2

// Work unit of workgroup b among `units` (<= grid).  Workgroups are dispatched to the
// XCDs round-robin (b on XCD b mod 8); units are numbered so that each XCD takes one
// contiguous run of them.  Neighbouring tiles of a step then share, in one L2, the
// cache lines that straddle their sub-rows and the step's row pointers and tile offsets.
// Units past `units` are idle (returned as >= units).
__device__ __forceinline__ uint32_t xcd_unit(uint32_t b, uint32_t grid, uint32_t units) {
  if (grid % kXcds != 0) return b;
  const uint32_t per = (units + kXcds - 1) / kXcds;  // <= grid / kXcds
  const uint32_t j = b / kXcds;
  return j < per ? (b % kXcds) * per + j : units;
}

// A workgroup owns (a range of consecutive base tiles, one emission step): it
// accumulates that step's deliveries to the range's targets in LDS and then writes the
// range's input accumulators.  Spikes are processed in chunks of kBlock: every thread
// fetches one spike's sub-row bounds (the edges of the spike's sorted row that fall in
// the range), a block scan lays the sub-rows end to end, and each wave streams a
// contiguous share of the flattened 16-byte groups, 64 x tiled_groups() at a time, with
// the next batch's loads issued before the current batch's LDS atomics.
template <int kBlock, int kW>
__global__ __launch_bounds__(kBlock) void k_deliver_tiled(DeliverArgs a, uint32_t steps) {
  extern __shared__ __align__(16) int32_t acc[];
  constexpr int kWaves = kBlock / kWave;
  constexpr int kU = tiled_groups();
  constexpr bool kSrcW = kW == kWeightSrc;
  __shared__ uint64_t s_lo[kBlock];
  __shared__ uint32_t s_len[kBlock];
  __shared__ uint32_t s_pre[kBlock + 1];
  __shared__ int32_t s_w[kSrcW ? kBlock : 1];
  __shared__ unsigned long long s_ev;
  __shared__ uint32_t s_wave[kWaves];
  __shared__ uint32_t s_qpre[kWave][kQueueGroups + 1];
  __shared__ uint32_t s_slot[kWave];
  __shared__ TileSchedule sch;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t t0 = a.ctl->t_deliver;
  close_window(a, t0, steps);
  if (a.x_post != nullptr && blockIdx.x + 1 == gridDim.x) {  // eager STDP: the traces
    advance_traces<kBlock>(a, t0);
    return;
  }
  const uint32_t grid = a.x_post != nullptr ? gridDim.x - 1 : gridDim.x;  // delivering workgroups

  // ---- the window's queue lengths and the balanced schedule (wave 0), while the
  // other waves clear the accumulators ----
  if (wave == 0) {
    uint32_t qp[kQueueGroups + 1] = {};
    uint32_t slot = 0;
    const int64_t e = emission_step(a, t0, lane);
    if (lane < steps && e >= 0) {
      slot = ring_of(e, a.slots);
      queue_prefix(a.q, slot, qp);
    }
    s_slot[lane] = slot;
#pragma unroll
    for (uint32_t g = 0; g <= kQueueGroups; ++g) s_qpre[lane][g] = qp[g];
    make_schedule(qp[kQueueGroups], steps, a.tiles, grid, sch);
  } else {
    const uint32_t acc_n = min(kTileGroupMax, a.tiles) * a.tile_size;
    for (uint32_t j = threadIdx.x - kWave; j < acc_n; j += kBlock - kWave) acc[j] = 0;
  }
  __syncthreads();
  const uint32_t unit = xcd_unit(blockIdx.x, grid, sch.first[steps]);
  if (unit >= sch.first[steps]) return;  // more workgroups than ranges this window
  uint32_t w = 0;
  while (sch.first[w + 1] <= unit) ++w;
  const uint32_t r_w = sch.r[w], jr = unit - sch.first[w];
  const uint32_t tile_a = (uint32_t)((uint64_t)jr * a.tiles / r_w);
  const uint32_t tile_b = (uint32_t)((uint64_t)(jr + 1) * a.tiles / r_w);
  const uint32_t tile_lo = tile_a * a.tile_size;
  const uint32_t tile_n = min(tile_b * a.tile_size, a.n) - tile_lo;

  const uint32_t slot = s_slot[w];
  uint32_t qpre[kQueueGroups + 1];
#pragma unroll
  for (uint32_t g = 0; g <= kQueueGroups; ++g) qpre[g] = s_qpre[w][g];
  const uint32_t cnt = qpre[kQueueGroups];
  uint64_t ev = 0;  // synapses of the sub-rows this thread fetched
  if (threadIdx.x == 0) s_ev = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < cnt; c0 += kBlock) {
    const uint32_t mm = min((uint32_t)kBlock, cnt - c0);
    // (1) sub-row bounds of this chunk's spikes and their 16-byte group counts
    uint32_t len = 0, groups = 0;
    uint64_t lo = 0;
    int32_t ws = 0;
    if (threadIdx.x < mm) {
      const int32_t src = queue_entry(a.q, slot, qpre, c0 + threadIdx.x);
      if ((uint32_t)src < a.n) {
        const size_t row = (size_t)src * (a.tiles + 1);
        uint32_t o0, o1;
        if (a.off16) {
          const uint16_t *to = static_cast<const uint16_t *>(a.tile_off) + row;
          o0 = to[tile_a];
          o1 = to[tile_b];
        } else {
          const uint32_t *to = static_cast<const uint32_t *>(a.tile_off) + row;
          o0 = to[tile_a];
          o1 = to[tile_b];
        }
        lo = a.row_ptr[src] + o0;
        len = o1 - o0;
        groups = len ? (uint32_t)(((lo + len + 7) >> 3) - (lo >> 3)) : 0u;
        if (kSrcW) ws = a.w_src[src];
      }
    }
    ev += len;
    // (2) block-wide exclusive scan of the group counts
    const uint32_t incl = wave_inclusive_scan(groups);
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    if (wave == 0) {
      const uint32_t x = lane < kWaves ? s_wave[lane] : 0u;
      const uint32_t xi = wave_inclusive_scan(x);
      if (lane < kWaves) s_wave[lane] = xi - x;
    }
    __syncthreads();
    const uint32_t pre = s_wave[wave] + incl - groups;
    if (threadIdx.x < mm) {
      s_pre[threadIdx.x] = pre;
      s_lo[threadIdx.x] = lo;
      s_len[threadIdx.x] = len;
      if (kSrcW) s_w[threadIdx.x] = ws;
    }
    if (threadIdx.x == kBlock - 1) s_pre[mm] = pre + groups;
    __syncthreads();
    const uint32_t total = s_pre[mm];
    // (3) this wave's contiguous share of the flattened groups
    const uint32_t share = (total + kWaves - 1) / kWaves;
    const uint32_t beg = min(wave * share, total), end = min(beg + share, total);
    if (beg < end) {
      uint32_t lo_j = 0, hi_j = mm;  // sub-row holding group beg
      while (hi_j - lo_j > 1) {
        const uint32_t mid = (lo_j + hi_j) >> 1;
        if (s_pre[mid] <= beg) lo_j = mid;
        else hi_j = mid;
      }
      uint32_t o = lo_j;
      TiledGroup cur[kU], nxt[kU];
      tiled_load<kU, kW>(a, s_lo, s_len, s_pre, s_w, beg + lane, end, o, cur);
      for (uint32_t b0 = beg; b0 < end; b0 += kWave * kU) {
        const uint32_t nb = b0 + kWave * kU;
#pragma unroll
        for (int u = 0; u < kU; ++u) nxt[u].mask = 0;
        if (nb < end) tiled_load<kU, kW>(a, s_lo, s_len, s_pre, s_w, nb + lane, end, o, nxt);
#pragma unroll
        for (int u = 0; u < kU; ++u) tiled_accumulate<kW>(acc, cur[u], tile_lo);
#pragma unroll
        for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
      }
    }
    __syncthreads();
  }
  ev = wave_sum(ev);
  if (lane == 0 && ev) atomicAdd(&s_ev, (unsigned long long)ev);
  __syncthreads();
  int32_t *out = a.input + (size_t)ring_add((uint32_t)(t0 % a.n_inbuf), w, a.n_inbuf) * a.n + tile_lo;
  if ((reinterpret_cast<uintptr_t>(out) & 15u) == 0) {
    // 16-byte stores over whole quads (acc is 16-byte aligned), the rest one by one
    const uint32_t quads = tile_n / 4;
    for (uint32_t j = threadIdx.x; j < quads; j += kBlock)
      reinterpret_cast<int4 *>(out)[j] = reinterpret_cast<const int4 *>(acc)[j];
    for (uint32_t j = 4 * quads + threadIdx.x; j < tile_n; j += kBlock) out[j] = acc[j];
  } else {
    for (uint32_t j = threadIdx.x; j < tile_n; j += kBlock) out[j] = acc[j];
  }
  if (threadIdx.x == 0) {
    add_part(a.ctl->events, blockIdx.x, s_ev);
    if (tile_a == 0) add_part(a.ctl->spikes, blockIdx.x, cnt);
  }
}

constexpr int kStdpBlock = 256;
constexpr int kStdpWaves = kStdpBlock / kWave;
// at most this many wavefronts share one queued spike's synapses (disjoint parts: still
// one writer per synapse); a step has few spikes, so this is what fills the GPU
constexpr uint32_t kStdpMaxSplit = 64;

__global__ __launch_bounds__(kStdpBlock) void k_stdp_ltd(StdpArgs a) {
  const uint64_t t = a.ctl->t;
  if (t < a.delay) return;
  const uint32_t slot = (uint32_t)((t - a.delay) % a.slots);
  uint32_t pre[kQueueGroups + 1];
  queue_prefix(a.q, slot, pre);
  const uint32_t cnt = pre[kQueueGroups];
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * kStdpWaves + threadIdx.x / kWave;
  const uint32_t n_gwaves = gridDim.x * kStdpWaves;
  const uint32_t split = parts_for(cnt, n_gwaves, kStdpMaxSplit);
  uint64_t touched = 0;
  for (uint64_t item = gwave; item < (uint64_t)cnt * split; item += n_gwaves) {
    const uint32_t s = (uint32_t)(item / split), part = (uint32_t)(item % split);
    const int32_t i = queue_entry(a.q, slot, pre, s);
    if ((uint32_t)i >= a.n) continue;
    if (part == 0 && lane == 0) a.x_pre[i] = a.x_pre[i] + 1.0f;
    const uint64_t lo = a.row_ptr[i] + a.plast_rel[i];
    const uint32_t len = a.plast_len[i];
    const uint32_t chunk = (len + split - 1) / split;
    const uint32_t k0 = part * chunk, k1 = min(len, k0 + chunk);
    for (uint32_t k = k0 + lane; k < k1; k += kWave) {
      const uint64_t e = lo + k;
      const float dw = a.a_minus * a.x_post[a.col[e]];
      float wv = a.w_f32[e] - dw;
      if (wv < 0.0f) wv = 0.0f;
      a.w_f32[e] = wv;
    }
    touched += k1 > k0 ? k1 - k0 : 0;
  }
  if (lane == 0) add_part(a.ctl->touches, gwave, touched);
}

// Depression and potentiation of step t in one pass.  Work items are the rows of
// S_{t-d} (depression over each row's plastic prefix) and the in-edge lists of S_t
// (potentiation), each cut into disjoint parts.  A synapse i -> j with i in S_{t-d}
// and j in S_t takes both updates, depression first: its row part skips it and its
// in-edge part applies both, so every synapse still has one writer.  The traces are
// not written here (the delivery that follows adds the arrivals S_{t-d} to x_pre and
// S_t to x_post): potentiation reads x_pre[i] + 1 for a source i in S_{t-d}, which is
// the value the two-kernel order gives.  Membership of S_t and S_{t-d} is read from
// the raster.
__global__ __launch_bounds__(kStdpBlock) void k_stdp_fused(StdpArgs a) {
  const uint64_t t = a.ctl->t;
  const bool has_d = t >= a.delay;
  const uint32_t slot_d = has_d ? (uint32_t)((t - a.delay) % a.slots) : 0u;
  const uint32_t slot_p = (uint32_t)(t % a.slots);
  uint32_t pd[kQueueGroups + 1] = {}, pp[kQueueGroups + 1];
  if (has_d) queue_prefix(a.q, slot_d, pd);
  queue_prefix(a.q, slot_p, pp);
  const uint32_t cnt_d = pd[kQueueGroups], cnt_p = pp[kQueueGroups];
  const uint64_t *row_p = a.raster + (size_t)(t % a.raster_cap) * a.words;
  const uint64_t *row_d = a.raster + (size_t)(has_d ? (t - a.delay) % a.raster_cap : 0) * a.words;
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * kStdpWaves + threadIdx.x / kWave;
  const uint32_t n_gwaves = gridDim.x * kStdpWaves;
  const uint32_t split = parts_for(cnt_d + cnt_p, n_gwaves, kStdpMaxSplit);
  uint64_t touched = 0;
  for (uint64_t item = gwave; item < (uint64_t)(cnt_d + cnt_p) * split; item += n_gwaves) {
    const uint32_t s = (uint32_t)(item / split), part = (uint32_t)(item % split);
    if (s < cnt_d) {
      const int32_t i = queue_entry(a.q, slot_d, pd, s);
      if ((uint32_t)i >= a.n) continue;
      const uint64_t lo = a.row_ptr[i] + a.plast_rel[i];
      const uint32_t len = a.plast_len[i];
      const uint32_t chunk = (len + split - 1) / split;
      const uint32_t k0 = part * chunk, k1 = min(len, k0 + chunk);
      for (uint32_t k = k0 + lane; k < k1; k += kWave) {
        const uint64_t e = lo + k;
        const int32_t j = a.col[e];
        if ((row_p[(uint32_t)j >> 6] >> ((uint32_t)j & 63u)) & 1u) continue;  // its in-edge part
        const float dw = a.a_minus * a.x_post[j];
        float wv = a.w_f32[e] - dw;
        if (wv < 0.0f) wv = 0.0f;
        a.w_f32[e] = wv;
      }
      touched += k1 > k0 ? k1 - k0 : 0;
    } else {
      const int32_t j = queue_entry(a.q, slot_p, pp, s - cnt_d);
      if ((uint32_t)j >= a.n) continue;
      const uint64_t lo = a.in_ptr[j], len = a.in_ptr[j + 1] - lo;
      const uint64_t chunk = (len + split - 1) / split;
      const uint64_t m0 = lo + part * chunk, m1 = min(lo + len, m0 + chunk);
      const float xq = a.x_post[j];
      for (uint64_t m = m0 + lane; m < m1; m += kWave) {
        const uint32_t e = a.in_edge[m];
        const int32_t i = a.in_src[m];
        float wv = a.w_f32[e];
        float xpi = a.x_pre[i];
        if (has_d && ((row_d[(uint32_t)i >> 6] >> ((uint32_t)i & 63u)) & 1u)) {
          const float dm = a.a_minus * xq;
          wv = wv - dm;
          if (wv < 0.0f) wv = 0.0f;
          xpi = xpi + 1.0f;  // its arrival of step t
        }
        const float dp = a.a_plus * xpi;
        wv = wv + dp;
        if (wv > a.w_max) wv = a.w_max;
        a.w_f32[e] = wv;
      }
      // the synapses taking depression here were counted by their row's part
      touched += m1 > m0 ? m1 - m0 : 0;
    }
  }
  if (lane == 0) add_part(a.ctl->touches, gwave, touched);
}

// ---- lazy plasticity (Sec. III-A.1, "lazy variation of plasticity") ------------------
// A plastic row keeps an age (its first pending step) and its presynaptic trace at that
// step.  Its depression events are applied eagerly (k_stdp_ltd: they come once per
// arrival, over the row's contiguous plastic prefix); its potentiation events, one per
// postsynaptic spike of each target, wait until the row transmits or its oldest pending
// step would leave the targets' 64-step spike histories.  Then one workgroup replays
// them in registers, oldest first, with the same binary32 operations as the eager form.
constexpr int kLazyBlock = 256;
constexpr int kLazyUnroll = 4;  // synapses per thread in flight

struct LazyCounts {
  uint64_t events = 0, spikes = 0, touches = 0;
};

// Row i, pending steps [t_end - L + 1, t_end] (L <= kLazyHistory; the targets' histories
// end at step t_end).  The row's presynaptic trace over those steps is the iterated
// product X(age + m) = X(age) * beta^m, one rounding per step, as the neuron update
// computes it; no arrival lies inside a pending window (an arrival follows the row's own
// transmission, which brings the row current).  With `transmit`, every synapse of the row
// is then delivered with its current weight.  Called by the whole workgroup; s_traj holds
// kLazyHistory floats.
__device__ void lazy_row(const LazyArgs &a, int32_t i, uint32_t L, bool transmit, float *s_traj,
                         LazyCounts &cnt) {
  const uint64_t rs = a.row_ptr[i], re = a.row_ptr[i + 1];
  const uint32_t plen = a.lazy.plast_len[i];
  const uint64_t plo = rs + (plen ? a.plast_rel[i] : 0u), phi = plo + plen;
  if (plen && L) {
    if (threadIdx.x < kWave) {
      float x = a.lazy.x_age[i];
      for (uint32_t q = 1; q < L; ++q)
        if (threadIdx.x >= q) x = x * a.beta_plus;
      if (threadIdx.x < L) s_traj[threadIdx.x] = x;
    }
    __syncthreads();
  }
  const uint64_t win = L >= 64 ? ~0ull : ((1ull << L) - 1ull);
  const uint64_t lo = transmit ? rs : plo, hi = transmit ? re : phi;
  for (uint64_t e0 = lo; e0 < hi; e0 += (uint64_t)kLazyBlock * kLazyUnroll) {
    int32_t j[kLazyUnroll];
    uint64_t bits[kLazyUnroll];
    float w[kLazyUnroll];
#pragma unroll
    for (int u = 0; u < kLazyUnroll; ++u) {
      const uint64_t e = e0 + threadIdx.x + (uint64_t)u * kLazyBlock;
      j[u] = e < hi ? a.col[e] : -1;
    }
#pragma unroll
    for (int u = 0; u < kLazyUnroll; ++u) {
      const uint64_t e = e0 + threadIdx.x + (uint64_t)u * kLazyBlock;
      const bool plastic = e >= plo && e < phi && L;
      bits[u] = plastic && j[u] >= 0 ? a.lazy.hist[j[u]] & win : 0ull;
      w[u] = (j[u] >= 0 && (transmit || bits[u])) ? a.w_f32[e] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kLazyUnroll; ++u) {
      const uint64_t e = e0 + threadIdx.x + (uint64_t)u * kLazyBlock;
      uint64_t b = bits[u];
      if (b) {
        cnt.touches += (uint64_t)__popcll(b);
        float wv = w[u];
        while (b) {  // oldest pending postsynaptic spike first: highest bit
          const uint32_t k = 63u - (uint32_t)__builtin_clzll(b);
          b &= ~(1ull << k);
          const float dw = a.a_plus * s_traj[L - 1u - k];
          float x = wv + dw;
          if (x > a.w_max) x = a.w_max;
          wv = x;
        }
        w[u] = wv;
        a.w_f32[e] = wv;
      }
      if (transmit && j[u] >= 0)
        __hip_atomic_fetch_add(a.input + j[u], __float2int_rn(w[u] * 65536.0f), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (transmit && threadIdx.x == 0) {
    cnt.events += re - rs;
    ++cnt.spikes;
  }
}

// The row's new age t_next and its presynaptic trace there: x_pre (the trace of step
// t_next - 1) decayed once, plus one if the row's spike arrives at t_next.
__device__ __forceinline__ void lazy_rebase(const LazyArgs &a, int32_t i, uint64_t t_next, bool arrives) {
  const float xb = a.x_pre[i] * a.beta_plus;
  a.lazy.x_age[i] = arrives ? xb + 1.0f : xb;
  a.lazy.age[i] = (uint32_t)t_next;
}

__device__ __forceinline__ void lazy_commit(const LazyArgs &a, const LazyCounts &c) {
  const uint32_t part = blockIdx.x * (kLazyBlock / kWave) + threadIdx.x / kWave;
  const uint64_t ev = wave_sum(c.events), sp = wave_sum(c.spikes), to = wave_sum(c.touches);
  if (lane_id() == 0) {
    add_part(a.ctl->events, part, ev);
    add_part(a.ctl->spikes, part, sp);
    add_part(a.ctl->touches, part, to);
  }
}

// Step t (after the update and the depression pass): one workgroup per transmitting row
// (S_{t-d+1}) or expiring row; closes the step.
__global__ __launch_bounds__(kLazyBlock) void k_lazy(LazyArgs a) {
  __shared__ float s_traj[kLazyHistory];
  const uint64_t t = a.ctl->t_deliver;
  const uint32_t cur = (uint32_t)(t % a.slots);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // next step's spike and expiring-row counters start empty; no workgroup of this
    // launch reads them, and the next update sees the writes after the kernel boundary
    const uint32_t next = (uint32_t)((t + 1) % a.slots);
    for (uint32_t g = 0; g < kQueueGroups; ++g) {
      *qcount(a.q, next, g) = 0u;
      *qcount(a.lazy.exq, (uint32_t)((t + 1) & 1u), g) = 0u;
    }
    a.ctl->t = t + 1;
  }
  uint32_t txp[kQueueGroups + 1] = {}, exp[kQueueGroups + 1], pst[kQueueGroups + 1];
  const bool has_tx = t + 1 >= a.delay;
  const uint32_t tx_slot = has_tx ? (uint32_t)((t + 1 - a.delay) % a.slots) : 0u;
  if (has_tx) queue_prefix(a.q, tx_slot, txp);
  queue_prefix(a.lazy.exq, (uint32_t)(t & 1u), exp);
  queue_prefix(a.q, cur, pst);
  // postsynaptic traces of S_t (the depression pass of this step has read them)
  for (uint32_t f = blockIdx.x * kLazyBlock + threadIdx.x; f < pst[kQueueGroups]; f += gridDim.x * kLazyBlock) {
    const int32_t j = queue_entry(a.q, cur, pst, f);
    if ((uint32_t)j < a.n) a.x_post[j] = a.x_post[j] + 1.0f;
  }
  const uint32_t n_tx = txp[kQueueGroups], n_items = n_tx + exp[kQueueGroups];
  LazyCounts c;
  for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const bool tx = item < n_tx;
    const int32_t i = tx ? queue_entry(a.q, tx_slot, txp, item)
                         : queue_entry(a.lazy.exq, (uint32_t)(t & 1u), exp, item - n_tx);
    if ((uint32_t)i >= a.n) continue;
    const bool plastic = a.lazy.plast_len[i] > 0;
    uint32_t L = plastic ? (uint32_t)t - a.lazy.age[i] + 1u : 0u;  // pending steps [age, t]
    if (L > kLazyHistory) {
      if (threadIdx.x == 0) atomicAdd((unsigned long long *)&a.ctl->lazy_overrun, 1ull);
      L = kLazyHistory;
    }
    lazy_row(a, i, L, tx, s_traj, c);
    __syncthreads();  // every thread is done with s_traj and with the row's age
    if (plastic && threadIdx.x == 0) lazy_rebase(a, i, t + 1, tx);
  }
  lazy_commit(a, c);
}

// Every plastic row brought current at the step boundary t (after step t - 1): pending
// steps [age, t - 1] applied, age t, trace rebuilt (the row's spike of step t - d arrives
// at t: history bit d - 1 after the update of step t - 1).
__global__ __launch_bounds__(kLazyBlock) void k_lazy_flush(LazyArgs a, uint64_t t) {
  __shared__ float s_traj[kLazyHistory];
  LazyCounts c;
  for (uint32_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    if (a.lazy.plast_len[i] == 0) continue;
    uint32_t L = (uint32_t)t - a.lazy.age[i];  // pending steps [age, t - 1]
    if (L > kLazyHistory) {
      if (threadIdx.x == 0) atomicAdd((unsigned long long *)&a.ctl->lazy_overrun, 1ull);
      L = kLazyHistory;
    }
    if (L) lazy_row(a, (int32_t)i, L, false, s_traj, c);
    __syncthreads();
    if (threadIdx.x == 0) {
      const bool arrives = t >= a.delay && ((a.lazy.hist[i] >> (a.delay - 1u)) & 1u);
      lazy_rebase(a, (int32_t)i, t, arrives);
    }
  }
  lazy_commit(a, c);
}

// Stages a caller's spike list as one window's queues for a delivery launch (the
// delivery-timing entry points): position p of step w goes to sub-queue
// p mod kQueueGroups at index p / kQueueGroups, as the update kernel's appends would
// lay it out.  Step w's ids are ids[off[w] .. off[w+1]), or, with round_robin, every
// id k with k mod steps = w (position k / steps).  Also sets every (step, sub-queue)
// counter of the window, zeroes the control block (then sets t_deliver) and clears the
// n_input accumulators.  Grid-stride over each part; the parts are disjoint.
__global__ __launch_bounds__(256) void k_stage_window(StageArgs a) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = tid; k < a.n_ids; k += nthreads) {
    uint32_t w, p;
    if (a.round_robin) {
      w = (uint32_t)(k % a.steps);
      p = (uint32_t)(k / a.steps);
    } else {
      w = 0;  // last w with off[w] <= k
      while (w + 1 < a.steps && a.off[w + 1] <= k) ++w;
      p = (uint32_t)(k - a.off[w]);
    }
    a.q.ids[(size_t)w * a.q.stride + (size_t)(p % kQueueGroups) * a.q.group_cap + p / kQueueGroups] = a.ids[k];
  }
  for (uint64_t j = tid; j < (uint64_t)a.steps * kQueueGroups; j += nthreads) {
    const uint32_t w = (uint32_t)(j / kQueueGroups), g = (uint32_t)(j % kQueueGroups);
    const uint32_t c = a.off[w + 1] - a.off[w];
    a.q.qlen[j * kQlenStride] = c > g ? (c - g + kQueueGroups - 1) / kQueueGroups : 0u;
  }
  uint64_t *ctl = reinterpret_cast<uint64_t *>(a.ctl);
  for (uint64_t j = tid; j < sizeof(Ctl) / sizeof(uint64_t); j += nthreads)
    ctl[j] = j == offsetof(Ctl, t_deliver) / sizeof(uint64_t) ? a.t_deliver : 0ull;
  for (uint64_t j = tid; j < a.n_input; j += nthreads) a.input[j] = 0;
}

}  // namespace

// One launch, through hipExtLaunchKernel when timing events are requested.
template <typename... KArgs, typename... Args>
void launch_kernel(void (*kernel)(KArgs...), uint32_t grid, uint32_t block, size_t lds, hipStream_t s,
                   hipEvent_t start, hipEvent_t stop, Args... args) {
  if (start || stop) hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), (uint32_t)lds, s, start, stop, 0u, args...);
  else kernel<<<grid, block, lds, s>>>(args...);
}

hipError_t launch_update(const UpdateArgs &a, uint32_t steps, hipStream_t s, const LaunchEvents &ev) {
  const uint32_t grid = (a.n + kUpdateBlock - 1) / kUpdateBlock;
  // windows of 13 to 17 steps always span 4 or 5 quads, whatever their first step
  if (steps >= 4 * (kShortQuads - 1) - 3 && steps <= 4 * kShortQuads - 3)
    launch_kernel(k_update<true>, grid, kUpdateBlock, 0, s, ev.start, ev.stop, a, steps);
  else
    launch_kernel(k_update<false>, grid, kUpdateBlock, 0, s, ev.start, ev.stop, a, steps);
  return hipGetLastError();
}

hipError_t launch_deliver_atomic(const DeliverArgs &a, uint32_t steps, uint32_t grid, hipStream_t s,
                                 const LaunchEvents &ev) {
  auto k = a.w_f32 ? k_deliver_atomic<kWeightF32> : a.w_src ? k_deliver_atomic<kWeightSrc> : k_deliver_atomic<kWeightQ16>;
  if (a.x_post && grid < 2) grid = 2;  // the last workgroup advances the traces
  launch_kernel(k, grid, kAtomicBlock, 0, s, ev.start, ev.stop, a, steps);
  return hipGetLastError();
}

// Largest dynamic LDS (bytes) a tiled-delivery workgroup of this size may request on the
// current device, after raising the kernel's dynamic-LDS attribute to that limit.
hipError_t prepare_deliver_tiled(uint32_t block, size_t *max_dynamic_lds) {
  int dev = 0, limit = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  const void *fns[3];
  if (block == 256) {
    fns[0] = reinterpret_cast<const void *>(&k_deliver_tiled<256, kWeightQ16>);
    fns[1] = reinterpret_cast<const void *>(&k_deliver_tiled<256, kWeightF32>);
    fns[2] = reinterpret_cast<const void *>(&k_deliver_tiled<256, kWeightSrc>);
  } else if (block == 512) {
    fns[0] = reinterpret_cast<const void *>(&k_deliver_tiled<512, kWeightQ16>);
    fns[1] = reinterpret_cast<const void *>(&k_deliver_tiled<512, kWeightF32>);
    fns[2] = reinterpret_cast<const void *>(&k_deliver_tiled<512, kWeightSrc>);
  } else {
    fns[0] = reinterpret_cast<const void *>(&k_deliver_tiled<1024, kWeightQ16>);
    fns[1] = reinterpret_cast<const void *>(&k_deliver_tiled<1024, kWeightF32>);
    fns[2] = reinterpret_cast<const void *>(&k_deliver_tiled<1024, kWeightSrc>);
  }
  size_t dyn = (size_t)limit;
  for (const void *fn : fns) {
    hipFuncAttributes attr{};
    e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return e;
    dyn = std::min(dyn, (size_t)limit > attr.sharedSizeBytes ? (size_t)limit - attr.sharedSizeBytes : (size_t)0);
  }
  for (const void *fn : fns) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
  }
  *max_dynamic_lds = dyn;
  return hipSuccess;
}

hipError_t launch_deliver_tiled(const DeliverArgs &a, uint32_t steps, uint32_t block,
                                uint32_t grid, hipStream_t s, const LaunchEvents &ev) {
  // the schedule always fits when every step uses maximal ranges
  const uint32_t floor_grid = steps * ((a.tiles + kTileGroupMax - 1) / kTileGroupMax);
  if (grid < floor_grid) grid = floor_grid;
  if (a.x_post) ++grid;  // one more workgroup advances the STDP traces
  const size_t lds = (size_t)min(kTileGroupMax, a.tiles) * a.tile_size * sizeof(int32_t);
  const int kind = a.w_src ? kWeightSrc : a.w_f32 ? kWeightF32 : kWeightQ16;
  auto pick = [kind](auto q16, auto f32, auto src) { return kind == kWeightSrc ? src : kind == kWeightF32 ? f32 : q16; };
  switch (block) {
    case 256:
      launch_kernel(pick(k_deliver_tiled<256, kWeightQ16>, k_deliver_tiled<256, kWeightF32>,
                         k_deliver_tiled<256, kWeightSrc>),
                    grid, 256, lds, s, ev.start, ev.stop, a, steps);
      break;
    case 512:
      launch_kernel(pick(k_deliver_tiled<512, kWeightQ16>, k_deliver_tiled<512, kWeightF32>,
                         k_deliver_tiled<512, kWeightSrc>),
                    grid, 512, lds, s, ev.start, ev.stop, a, steps);
      break;
    default:
      launch_kernel(pick(k_deliver_tiled<1024, kWeightQ16>, k_deliver_tiled<1024, kWeightF32>,
                         k_deliver_tiled<1024, kWeightSrc>),
                    grid, 1024, lds, s, ev.start, ev.stop, a, steps);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_stdp_fused(const StdpArgs &a, uint32_t grid, hipStream_t s, const LaunchEvents &ev) {
  launch_kernel(k_stdp_fused, grid, kStdpBlock, 0, s, ev.start, ev.stop, a);
  return hipGetLastError();
}

hipError_t launch_stdp_ltd(const StdpArgs &a, uint32_t grid, hipStream_t s, const LaunchEvents &ev) {
  launch_kernel(k_stdp_ltd, grid, kStdpBlock, 0, s, ev.start, ev.stop, a);
  return hipGetLastError();
}

hipError_t launch_lazy(const LazyArgs &a, uint32_t grid, hipStream_t s, const LaunchEvents &ev) {
  launch_kernel(k_lazy, grid, kLazyBlock, 0, s, ev.start, ev.stop, a);
  return hipGetLastError();
}

hipError_t launch_lazy_flush(const LazyArgs &a, uint64_t t, uint32_t grid, hipStream_t s) {
  k_lazy_flush<<<grid, kLazyBlock, 0, s>>>(a, t);
  return hipGetLastError();
}

hipError_t launch_stage_window(const StageArgs &a, hipStream_t s) {
  k_stage_window<<<1024, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace snn
