// step.hip -- the per-step kernels of the work-queue pipeline (Sec. III-A.1, Fig. 1).
//
//  k_update          Update Neurons for a window of consecutive steps: each lane owns
//                    one neuron, keeps V/ref/traces in registers across the window,
//                    and appends its spikes to the step's queue with one ballot and
//                    one queue-counter atomic per wavefront; the ballot is also the
//                    step's raster word.
//  k_deliver_atomic  Receive Spikes, one wavefront per dequeued spike, aligned 16-byte
//                    loads of targets/weights, no-return int32 atomics into the Q16
//                    input accumulators in global memory.
//  k_deliver_tiled   Receive Spikes, one workgroup per (target tile, emission step):
//                    the workgroup reads the tile's slice of every dequeued spike's
//                    sorted row, accumulates in LDS with int32 atomics and writes the
//                    tile's input accumulators with plain stores.
//  k_stdp_ltd/ltp    Update Synapses: depression over S_{t-d}'s plastic out-edges,
//                    potentiation over S_t's plastic in-edges (transposed index).
//
// Step bookkeeping lives on the device (Ctl::t) so that a captured HIP graph replays
// correctly: every kernel reads the step, and the last workgroup of the delivery
// kernel that closes a window clears the next window's queue counters and advances t.
#include "device_math.h"
#include "snn_internal.h"

namespace snn {
namespace {

constexpr int kUpdateBlock = 256;

__global__ __launch_bounds__(kUpdateBlock) void k_update(UpdateArgs a, uint32_t steps) {
  __shared__ uint64_t tbl[kTableCap];
  for (uint32_t j = threadIdx.x; j < a.table_len; j += kUpdateBlock) tbl[j] = a.table[j];
  __syncthreads();

  const uint64_t t0 = a.ctl->t;
  const uint32_t i = blockIdx.x * kUpdateBlock + threadIdx.x;
  const bool active = i < a.n;
  const uint32_t lane = lane_id();
  const uint32_t word = i / kWave;
  const bool drive = a.table_len > 1;

  float v = 0.f, xp = 0.f, xq = 0.f;
  int32_t ref = 0;
  if (active) {
    v = a.v[i];
    ref = a.ref[i];
    if (a.plastic) {
      xp = a.x_pre[i];
      xq = a.x_post[i];
    }
  }
  Words4 rnd{};
  for (uint32_t w = 0; w < steps; ++w) {
    const uint64_t t = t0 + w;
    bool spike = false;
    if (active) {
      int32_t *in = a.input + (size_t)(t % a.n_inbuf) * a.n + i;
      const int32_t acc = *in;
      if (a.zero_input) *in = 0;
      if (drive && (w == 0 || (t & 3u) == 0))
        rnd = philox(i, (uint32_t)(t >> 2), (uint32_t)(t >> 34), kStreamPoisson, a.key0, a.key1);
      if (ref > 0) {
        ref -= 1;
      } else {
        int32_t k = 0;
        if (drive) {
          const uint64_t r = rnd.w[t & 3u];
          while (r >= tbl[k]) ++k;
        }
        const uint32_t sum = (uint32_t)acc + (uint32_t)k * (uint32_t)a.w_ext_q16;
        const float dv = (float)(int32_t)sum * 0x1p-16f;
        float vv = v + dv;
        const float diff = vv - a.v_inf;
        const float leak = diff * a.alpha;
        vv = a.v_inf + leak;
        if (vv >= a.v_th) {
          spike = true;
          vv = a.v_reset;
          ref = a.ref_steps;
        }
        v = vv;
      }
      if (a.plastic) {
        xp = xp * a.beta_plus;
        xq = xq * a.beta_minus;
      }
    }
    const uint64_t mask = __ballot(spike);
    const uint32_t slot = (uint32_t)(t % a.slots);
    if (lane == 0 && word < a.words) a.raster[(size_t)(t % a.raster_cap) * a.words + word] = mask;
    if (mask) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&a.qlen[slot], (uint32_t)__popcll(mask));
      base = __shfl(base, 0, kWave);
      const uint32_t pos = base + lanes_below(mask);
      if (spike && pos < a.n) a.queue[(size_t)slot * a.n + pos] = (int32_t)i;
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
}

// Hand-off at the end of the delivery kernel: the last workgroup to finish clears the
// queue counters of the next window and advances the step counter.
__device__ __forceinline__ void finish_window(const DeliverArgs &a, uint64_t t0, uint32_t steps) {
  __shared__ bool last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&a.ctl->done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    if (a.advance) {
      for (uint32_t w = 0; w < a.window_max; ++w) a.qlen[(t0 + steps + w) % a.slots] = 0u;
      a.ctl->t = t0 + steps;
    }
    a.ctl->done = 0u;
    __threadfence();
  }
}

template <bool kPlasticW>
__device__ __forceinline__ int32_t q16_of(const DeliverArgs &a, uint64_t e) {
  if constexpr (kPlasticW) return __float2int_rn(a.w_f32[e] * 65536.0f);
  else return a.w_q16[e];
}

// Emission step of the w-th queue delivered by a window starting at t0: spikes of step
// e land in input buffer (e + d) mod n_inbuf, to be read by the update of step e + d.
__device__ __forceinline__ int64_t emission_step(const DeliverArgs &a, uint64_t t0, uint32_t w) {
  return (int64_t)t0 + (int64_t)w + (int64_t)a.n_inbuf - (int64_t)a.delay;
}

constexpr int kAtomicBlock = 256;

template <bool kPlasticW>
__global__ __launch_bounds__(kAtomicBlock) void k_deliver_atomic(DeliverArgs a, uint32_t steps) {
  const uint64_t t0 = a.ctl->t;
  const uint32_t lane = lane_id();
  uint32_t c = 0;
  if (lane < steps) {
    const int64_t e = emission_step(a, t0, lane);
    if (e >= 0) c = min(a.qlen[(uint64_t)e % a.slots], a.n);
  }
  const uint32_t incl = wave_inclusive_scan(c);
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  const uint32_t gwave = blockIdx.x * (kAtomicBlock / kWave) + threadIdx.x / kWave;
  const uint32_t n_gwaves = gridDim.x * (kAtomicBlock / kWave);
  uint64_t ev = 0;
  for (uint32_t f = gwave; f < total; f += n_gwaves) {
    const uint32_t w = (uint32_t)__popcll(__ballot(incl <= f));
    const uint32_t prev = __shfl(incl, (w + kWave - 1) % kWave, kWave);
    const uint32_t before = w ? prev : 0u;
    const uint64_t e = (uint64_t)emission_step(a, t0, w);
    const uint32_t slot = (uint32_t)(e % a.slots);
    int32_t *in = a.input + (size_t)((t0 + w) % a.n_inbuf) * a.n;
    const int32_t src = a.queue[(size_t)slot * a.n + (f - before)];
    if ((uint32_t)src >= a.n) continue;
    const uint64_t rs = a.row_ptr[src], re = a.row_ptr[src + 1];
    for (uint64_t g = (rs >> 2) + lane; g < ((re + 3) >> 2); g += kWave) {
      const int4 c4 = reinterpret_cast<const int4 *>(a.col)[g];
      int32_t wv[4];
      if constexpr (kPlasticW) {
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
    ev += re - rs;
  }
  if (lane == 0 && ev) atomicAdd((unsigned long long *)&a.ctl->events, (unsigned long long)ev);
  finish_window(a, t0, steps);
}

template <int kBlock>
__global__ __launch_bounds__(kBlock) void k_deliver_tiled(DeliverArgs a) {
  extern __shared__ int32_t acc[];
  constexpr int kWaves = kBlock / kWave;
  const uint64_t t0 = a.ctl->t;
  const uint32_t tile = blockIdx.x % a.tiles;
  const uint32_t w = blockIdx.x / a.tiles;
  const uint32_t steps = gridDim.x / a.tiles;
  const uint32_t tile_lo = tile * a.tile_size;
  const uint32_t tile_n = min(a.tile_size, a.n - tile_lo);
  for (uint32_t j = threadIdx.x; j < tile_n; j += kBlock) acc[j] = 0;
  __syncthreads();

  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const int64_t e_step = emission_step(a, t0, w);
  uint64_t ev = 0;
  if (e_step >= 0) {
    const uint32_t slot = (uint32_t)((uint64_t)e_step % a.slots);
    const uint32_t cnt = min(a.qlen[slot], a.n);
    const int32_t *ids = a.queue + (size_t)slot * a.n;
    for (uint32_t s = wave; s < cnt; s += kWaves) {
      const int32_t src = ids[s];
      if ((uint32_t)src >= a.n) continue;
      const uint64_t base = a.row_ptr[src];
      const uint32_t *to = a.tile_off + (size_t)src * (a.tiles + 1) + tile;
      const uint64_t lo = base + to[0], hi = base + to[1];
      for (uint64_t e = lo + lane; e < hi; e += 4 * kWave) {
        int32_t cv[4], wv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint64_t x = e + (uint64_t)q * kWave;
          cv[q] = x < hi ? a.col[x] : (int32_t)tile_lo;
          wv[q] = x < hi ? a.w_q16[x] : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (wv[q]) atomicAdd(&acc[cv[q] - (int32_t)tile_lo], wv[q]);
      }
      ev += hi - lo;
    }
  }
  __syncthreads();
  int32_t *out = a.input + (size_t)((t0 + w) % a.n_inbuf) * a.n + tile_lo;
  for (uint32_t j = threadIdx.x; j < tile_n; j += kBlock) out[j] = acc[j];
  if (lane == 0 && ev) atomicAdd((unsigned long long *)&a.ctl->events, (unsigned long long)ev);
  finish_window(a, t0, steps);
}

constexpr int kStdpBlock = 256;

__global__ __launch_bounds__(kStdpBlock) void k_stdp_ltd(StdpArgs a) {
  const uint64_t t = a.ctl->t;
  if (t < a.delay) return;
  const uint32_t slot = (uint32_t)((t - a.delay) % a.slots);
  const uint32_t cnt = min(a.qlen[slot], a.n);
  const int32_t *ids = a.queue + (size_t)slot * a.n;
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * (kStdpBlock / kWave) + threadIdx.x / kWave;
  const uint32_t n_gwaves = gridDim.x * (kStdpBlock / kWave);
  uint64_t touched = 0;
  for (uint32_t s = gwave; s < cnt; s += n_gwaves) {
    const int32_t i = ids[s];
    if ((uint32_t)i >= a.n) continue;
    if (lane == 0) a.x_pre[i] = a.x_pre[i] + 1.0f;
    const uint64_t lo = a.row_ptr[i] + a.plast_rel[i];
    const uint32_t len = a.plast_len[i];
    for (uint32_t k = lane; k < len; k += kWave) {
      const uint64_t e = lo + k;
      const float dw = a.a_minus * a.x_post[a.col[e]];
      float wv = a.w_f32[e] - dw;
      if (wv < 0.0f) wv = 0.0f;
      a.w_f32[e] = wv;
    }
    touched += len;
  }
  if (lane == 0 && touched) atomicAdd((unsigned long long *)&a.ctl->touches, (unsigned long long)touched);
}

__global__ __launch_bounds__(kStdpBlock) void k_stdp_ltp(StdpArgs a) {
  const uint64_t t = a.ctl->t;
  const uint32_t slot = (uint32_t)(t % a.slots);
  const uint32_t cnt = min(a.qlen[slot], a.n);
  const int32_t *ids = a.queue + (size_t)slot * a.n;
  const uint32_t lane = lane_id();
  const uint32_t gwave = blockIdx.x * (kStdpBlock / kWave) + threadIdx.x / kWave;
  const uint32_t n_gwaves = gridDim.x * (kStdpBlock / kWave);
  uint64_t touched = 0;
  for (uint32_t s = gwave; s < cnt; s += n_gwaves) {
    const int32_t j = ids[s];
    if ((uint32_t)j >= a.n) continue;
    if (lane == 0) a.x_post[j] = a.x_post[j] + 1.0f;
    const uint64_t lo = a.in_ptr[j], hi = a.in_ptr[j + 1];
    for (uint64_t m = lo + lane; m < hi; m += kWave) {
      const uint32_t e = a.in_edge[m];
      const float dw = a.a_plus * a.x_pre[a.in_src[m]];
      float wv = a.w_f32[e] + dw;
      if (wv > a.w_max) wv = a.w_max;
      a.w_f32[e] = wv;
    }
    touched += hi - lo;
  }
  if (lane == 0 && touched) atomicAdd((unsigned long long *)&a.ctl->touches, (unsigned long long)touched);
}

}  // namespace

hipError_t launch_update(const UpdateArgs &a, uint32_t steps, hipStream_t s) {
  const uint32_t grid = (a.n + kUpdateBlock - 1) / kUpdateBlock;
  k_update<<<grid, kUpdateBlock, 0, s>>>(a, steps);
  return hipGetLastError();
}

hipError_t launch_deliver_atomic(const DeliverArgs &a, uint32_t steps, uint32_t grid,
                                 bool plastic_w, hipStream_t s) {
  if (plastic_w) k_deliver_atomic<true><<<grid, kAtomicBlock, 0, s>>>(a, steps);
  else k_deliver_atomic<false><<<grid, kAtomicBlock, 0, s>>>(a, steps);
  return hipGetLastError();
}

hipError_t launch_deliver_tiled(const DeliverArgs &a, uint32_t steps, uint32_t block,
                                hipStream_t s) {
  const uint32_t grid = a.tiles * steps;
  const size_t lds = (size_t)a.tile_size * sizeof(int32_t);
  switch (block) {
    case 256: k_deliver_tiled<256><<<grid, 256, lds, s>>>(a); break;
    case 512: k_deliver_tiled<512><<<grid, 512, lds, s>>>(a); break;
    default: k_deliver_tiled<1024><<<grid, 1024, lds, s>>>(a); break;
  }
  return hipGetLastError();
}

hipError_t launch_stdp(const StdpArgs &a, uint32_t grid, hipStream_t s) {
  k_stdp_ltd<<<grid, kStdpBlock, 0, s>>>(a);
  k_stdp_ltp<<<grid, kStdpBlock, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace snn
