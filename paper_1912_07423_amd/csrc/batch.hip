// batch.hip -- many independent static networks stepped by one persistent launch.
//
// Every workgroup owns one network for the whole launch and runs the step pipeline of
// Fig. 1 for it step after step, with nothing shared between workgroups:
//   * V and the refractory counters live in registers (kPer neurons per lane);
//   * the delay ring of Q16 input accumulators ([delay][n] int32) lives in LDS, so
//     Receive Spikes is an LDS atomic add per synaptic event and the CSR rows are the
//     only HBM stream, read as 16-byte groups of 4 targets, several per lane in flight;
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

// 16-byte groups of a row per lane per round: four, except in 1,024-thread workgroups
// (at most 128 registers per lane): two, and one where the drive's code also holds
// registers beside 16 or more neurons per lane (more groups in flight would spill).
// Two groups instead of one in the drive-free 1,024 x 20 shape: 8.87 -> 8.59 us per step
// of the 512-network sweep.
constexpr int groups_in_flight(int block, int per, bool drive) {
  return block == 1024 ? (per >= 16 && drive ? 1 : 2) : 4;
}

// LDS atomic adds of the elements [lo, hi) of one 16-byte group starting at edge e0.
__device__ __forceinline__ void add_group(int32_t *in, const int4 &c, const int4 &w, uint64_t e0, uint64_t lo,
                                          uint64_t hi) {
  const int32_t cv[4] = {c.x, c.y, c.z, c.w}, wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (e0 + q >= lo && e0 + q < hi) atomicAdd(&in[cv[q]], wv[q]);
}

template <int kBlock, int kPer, bool kDrive>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchNet *nets, const uint32_t *order,
                                                  uint32_t steps, uint32_t flags) {
  extern __shared__ int32_t s_dyn[];  // [delay][n] accumulators, then the drive thresholds
  __shared__ uint32_t s_qn[2];
  __shared__ unsigned long long s_count[2];

  constexpr int kGroupsInFlight = groups_in_flight(kBlock, kPer, kDrive);
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
  if (kDrive)
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
        if (kDrive && d.below && ref[k] <= 0) {
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
      // the row as 16-byte groups of 4 targets (the arrays are padded to whole groups),
      // up to kGroupsInFlight groups per lane requested before their adds; elements
      // outside the row are masked
      const uint64_t g_lo = lo >> 2, g_hi = (hi + 3) >> 2;
      const int4 *col4 = reinterpret_cast<const int4 *>(d.col);
      const int4 *w4 = reinterpret_cast<const int4 *>(d.w_q16);
      const int32_t ws = d.w_src ? d.w_src[src] : 0;  // one weight per source: targets only
      for (uint64_t g0 = g_lo + gl; g0 < g_hi; g0 += (uint64_t)kGroupsInFlight * lanes) {
        int4 c[kGroupsInFlight], w[kGroupsInFlight];
#pragma unroll
        for (int u = 0; u < kGroupsInFlight; ++u) {
          const uint64_t g = g0 + (uint64_t)u * lanes;
          c[u] = g < g_hi ? col4[g] : make_int4(0, 0, 0, 0);
          w[u] = make_int4(ws, ws, ws, ws);
          if (!d.w_src && g < g_hi) w[u] = w4[g];
        }
#pragma unroll
        for (int u = 0; u < kGroupsInFlight; ++u) {
          const uint64_t g = g0 + (uint64_t)u * lanes;
          if (g < g_hi) add_group(in, c[u], w[u], 4 * g, lo, hi);
        }
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
  // without a Poisson drive in any member the kernel is built without the drive's code
  // (Philox and the threshold scan), which would otherwise take registers
  auto k = (flags & kBatchDrive) ? k_batch<kBlock, kPer, true> : k_batch<kBlock, kPer, false>;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_nets), dim3(kBlock), lds, s, nets, order, steps, flags);
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
