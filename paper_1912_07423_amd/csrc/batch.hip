// batch.hip -- many independent static networks stepped by one persistent launch.
//
// Every workgroup owns one network for the whole launch and runs the step pipeline of
// Fig. 1 for it step after step, with nothing shared between workgroups:
//   * V and the refractory counters live in registers (kPer neurons per lane);
//   * the delay ring of Q16 input accumulators ([delay][n] int32) lives in LDS, so
//     Receive Spikes is an LDS atomic add per synaptic event and the CSR rows are the
//     only HBM stream;
//   * the step's spike queue is compacted with one ballot per wavefront and one LDS
//     counter reservation per wavefront, into the network's queue buffer;
//   * two workgroup barriers per step separate update, delivery and the next update.
// The launch starts from, and (when `commit` is set) leaves, each network's state in
// the network's own buffers with the same layout the single-network pipeline uses, so
// both pipelines and every reader agree on a network's state between launches.
#include "device_math.h"
#include "snn_internal.h"

namespace snn {
namespace {

template <int kBlock, int kPer>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchNet *nets, const uint32_t *order,
                                                  uint32_t steps, uint32_t flags) {
  extern __shared__ int32_t s_dyn[];  // [delay][n] accumulators, then the drive thresholds
  __shared__ uint32_t s_qn[2];
  __shared__ unsigned long long s_count[2];

  const BatchNet d = nets[order[blockIdx.x]];
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const uint32_t n = d.n, delay = d.delay;
  int32_t *acc = s_dyn;
  uint32_t *tbl = reinterpret_cast<uint32_t *>(s_dyn + (size_t)delay * n);
  const LifConst lif{d.alpha, d.v_inf, d.v_th, d.v_reset, d.ref_steps, d.w_ext_q16};
  const uint64_t t0 = d.ctl->t;

  float v[kPer];
  int32_t ref[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t i = (uint32_t)k * kBlock + tid;
    v[k] = i < n ? d.v[i] : 0.f;
    ref[k] = i < n ? d.ref[i] : 0;
  }
  for (uint32_t j = tid; j < delay * n; j += kBlock) acc[j] = d.input[j];
  for (uint32_t j = tid; j < d.below; j += kBlock) tbl[j] = d.table32[j];
  if (tid < 2) {
    s_qn[tid] = 0;
    s_count[tid] = 0;
  }
  __syncthreads();

  const uint32_t shift = d.lanes_shift;
  const uint32_t lanes = 1u << shift, groups = kBlock >> shift;
  const uint32_t grp = tid >> shift, gl = tid & (lanes - 1u);
  const bool write_raster = (flags & kBatchWriteRaster) != 0;
  uint32_t slot = (uint32_t)(t0 % delay);
  uint32_t ras = (uint32_t)(t0 % d.raster_cap);
  uint64_t events = 0, spikes = 0;

  for (uint32_t s = 0; s < steps; ++s) {
    const uint64_t t = t0 + s;
    int32_t *in = acc + (size_t)slot * n;
    uint32_t *qn = &s_qn[s & 1u];
    // ---- Update Neurons: step t for every neuron of the network ----
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = (uint32_t)k * kBlock + tid;
      bool spike = false;
      if (i < n) {
        int32_t kk = 0;
        if (d.below && ref[k] <= 0) {
          const Words4 r4 = philox(i, (uint32_t)(t >> 2), (uint32_t)(t >> 34), kStreamPoisson, d.key0, d.key1);
          const uint32_t r = word_of(r4, (uint32_t)t & 3u);
          while (kk < (int32_t)d.below && tbl[kk] <= r) ++kk;
        }
        const int32_t x = in[i];
        in[i] = 0;
        spike = lif_advance(v[k], ref[k], x, kk, lif);
      }
      const uint64_t mask = __ballot(spike);
      const uint32_t word = (uint32_t)k * (kBlock / kWave) + wave;
      if (write_raster && lane == 0 && word < d.words) d.raster[(size_t)ras * d.words + word] = mask;
      if (mask) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(qn, (uint32_t)__popcll(mask));
        base = __shfl(base, 0, kWave);
        if (spike) d.queue[base + lanes_below(mask)] = (int32_t)i;
      }
    }
    __syncthreads();
    // ---- Receive Spikes: S_t into the accumulator of arrival step t + delay, which
    //      is slot t mod delay again (read and cleared above) ----
    if (tid == 0) s_qn[(s + 1) & 1u] = 0;
    const uint32_t count = *qn;
    for (uint32_t q = grp; q < count; q += groups) {
      const int32_t src = d.queue[q];
      const uint64_t lo = d.row_ptr[src], hi = d.row_ptr[(uint32_t)src + 1u];
      if (gl == 0) {
        events += hi - lo;
        spikes += 1;
      }
      uint64_t e = lo + gl;
      if (d.w_src) {  // one weight per source: only the targets are streamed
        const int32_t ws = d.w_src[src];
        for (; e + 3u * lanes < hi; e += 4u * lanes) {
          const int32_t c0 = d.col[e], c1 = d.col[e + lanes];
          const int32_t c2 = d.col[e + 2u * lanes], c3 = d.col[e + 3u * lanes];
          atomicAdd(&in[c0], ws);
          atomicAdd(&in[c1], ws);
          atomicAdd(&in[c2], ws);
          atomicAdd(&in[c3], ws);
        }
        for (; e < hi; e += lanes) atomicAdd(&in[d.col[e]], ws);
      } else {
        for (; e + 3u * lanes < hi; e += 4u * lanes) {
          const int32_t c0 = d.col[e], c1 = d.col[e + lanes];
          const int32_t c2 = d.col[e + 2u * lanes], c3 = d.col[e + 3u * lanes];
          const int32_t w0 = d.w_q16[e], w1 = d.w_q16[e + lanes];
          const int32_t w2 = d.w_q16[e + 2u * lanes], w3 = d.w_q16[e + 3u * lanes];
          atomicAdd(&in[c0], w0);
          atomicAdd(&in[c1], w1);
          atomicAdd(&in[c2], w2);
          atomicAdd(&in[c3], w3);
        }
        for (; e < hi; e += lanes) atomicAdd(&in[d.col[e]], d.w_q16[e]);
      }
    }
    __syncthreads();
    slot = slot + 1u == delay ? 0u : slot + 1u;
    ras = ras + 1u == d.raster_cap ? 0u : ras + 1u;
  }

  if (!(flags & kBatchCommit)) return;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t i = (uint32_t)k * kBlock + tid;
    if (i < n) {
      d.v[i] = v[k];
      d.ref[i] = ref[k];
    }
  }
  for (uint32_t j = tid; j < delay * n; j += kBlock) d.input[j] = acc[j];
  events = wave_sum(events);
  spikes = wave_sum(spikes);
  if (lane == 0) {
    if (events) atomicAdd(&s_count[0], (unsigned long long)events);
    if (spikes) atomicAdd(&s_count[1], (unsigned long long)spikes);
  }
  __syncthreads();
  if (tid == 0) {
    d.ctl->events[0] += s_count[0];
    d.ctl->spikes[0] += s_count[1];
    d.ctl->t = t0 + steps;
  }
}

template <int kBlock, int kPer>
hipError_t launch_one(const BatchNet *nets, const uint32_t *order, uint32_t n_nets, uint32_t steps,
                      uint32_t flags, size_t lds, hipStream_t s) {
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<kBlock, kPer>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch<kBlock, kPer>), dim3(n_nets), dim3(kBlock), lds, s, nets, order, steps, flags);
  return hipGetLastError();
}

}  // namespace

bool batch_variant_supported(uint32_t block, uint32_t per) {
  switch (block) {
    case 256: return per == 16 || per == 32 || per == 64 || per == 80;
    case 512: return per == 8 || per == 16 || per == 32 || per == 40;
    case 1024: return per == 4 || per == 8 || per == 16 || per == 20;
    default: return false;
  }
}

uint32_t batch_per_lane(uint32_t block, uint32_t n_max) {
  const uint32_t need = (n_max + block - 1) / block;
  static const uint32_t k256[] = {16, 32, 64, 80}, k512[] = {8, 16, 32, 40}, k1024[] = {4, 8, 16, 20};
  const uint32_t *opts = block == 256 ? k256 : block == 512 ? k512 : k1024;
  for (int j = 0; j < 4; ++j)
    if (opts[j] >= need) return opts[j];
  return 0;
}

hipError_t launch_batch(const BatchNet *nets, const uint32_t *order, uint32_t n_nets, uint32_t steps,
                        uint32_t block, uint32_t per, uint32_t flags, size_t lds, hipStream_t s) {
#define SNN_BATCH_CASE(B, K) \
  if (block == B && per == K) return launch_one<B, K>(nets, order, n_nets, steps, flags, lds, s);
  SNN_BATCH_CASE(256, 16) SNN_BATCH_CASE(256, 32) SNN_BATCH_CASE(256, 64) SNN_BATCH_CASE(256, 80)
  SNN_BATCH_CASE(512, 8) SNN_BATCH_CASE(512, 16) SNN_BATCH_CASE(512, 32) SNN_BATCH_CASE(512, 40)
  SNN_BATCH_CASE(1024, 4) SNN_BATCH_CASE(1024, 8) SNN_BATCH_CASE(1024, 16) SNN_BATCH_CASE(1024, 20)
#undef SNN_BATCH_CASE
  return hipErrorInvalidValue;
}

}  // namespace snn
