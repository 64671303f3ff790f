// bptt.hip -- surrogate-gradient BPTT of a recurrent LIF network with sparse input and
// recurrent weights (CSR, FP32) and a dense leaky readout: forward pass and hand-written
// adjoint.
//
// Layouts (batch innermost, so that one wavefront = 64 batch elements of one neuron and
// every gather of a presynaptic value is one coalesced 256-byte row):
//   xt    [T][n_in][64]      input spikes (transposed from the caller's [B][T][n_in])
//   s     [T][H][64]         hidden outputs of every step
//   vck   [T/K][H][64]       membrane potential before each checkpoint segment
//   vseg  [K][H][64]         membranes of one segment, recomputed in the backward pass
//   lamu  [T][O][64]         readout adjoint
//   lamv  [T][H][64]         membrane adjoint of every step (+ zeros [H][64] for step T)
//   xbits [C][T], sbits [H][T]  64-bit batch masks of the binary input and hidden spikes
//                            (8 readable entries after each, and before sbits)
// Weights stay in the caller's CSR order (rows = presynaptic neuron, sorted targets);
// the forward current is a gather over the transposed index (per target, sources in
// ascending order, input projection first), the adjoint's dL/ds a gather over the
// forward rows, and every weight gradient has exactly one owner.
#include <algorithm>

#include "device_math.h"
#include "snn_internal.h"

namespace snn {
namespace {

__device__ __forceinline__ float spike_fn(float z, float slope, bool smooth) {
  if (smooth) {
    const float a = slope * z;
    const float d = 1.0f + fabsf(a);
    return 0.5f + 0.5f * (a / d);
  }
  return z >= 0.0f ? 1.0f : 0.0f;
}

__device__ __forceinline__ float surrogate(float z, float slope, bool smooth) {
  const float d = 1.0f + slope * fabsf(z);
  const float g = 1.0f / (d * d);
  return smooth ? 0.5f * slope * g : g;
}

// x [B][T][C] -> xt [T][C][64]; lanes >= B hold zeros.  A workgroup per (step t, block of
// 64 inputs) reads the 64 batch rows of its block (256 bytes each, coalesced) into LDS and
// writes the block transposed; a wavefront per input c then also writes that input's
// batch mask xbits[c][t] (bit b: x != 0) and sets *flag if some value is neither 0 nor 1
// (k_bits' rule).
__global__ __launch_bounds__(256) void k_transpose_x(const float *x, float *xt, uint64_t *xbits, uint32_t *flag,
                                                     uint32_t B, uint32_t T, uint32_t C) {
  __shared__ float tile[64][65];
  const uint32_t t = blockIdx.y, c0 = blockIdx.x * 64u;
  const uint32_t l = threadIdx.x % 64u, r = threadIdx.x / 64u;
  for (uint32_t b = r; b < 64u; b += 4u)
    tile[b][l] = b < B && c0 + l < C ? x[((uint64_t)b * T + t) * C + c0 + l] : 0.0f;
  __syncthreads();
  for (uint32_t k = r; k < 64u && c0 + k < C; k += 4u) {
    const uint32_t c = c0 + k;
    const float v = tile[l][k];
    xt[((uint64_t)t * C + c) * 64u + l] = v;
    const bool on = l < B && v != 0.0f;
    const uint64_t m = __ballot(on);
    const uint64_t bad = __ballot(on && v != 1.0f);
    if (l == 0) {
      xbits[(size_t)c * T + t] = m;
      if (bad) atomicOr(flag, 1u);
    }
  }
}

// Transposed-order copy of a CSR weight vector: w_t[e] = w[edge[e]].
__global__ void k_gather_t(const float *w, const uint32_t *edge, float *w_t, uint64_t nnz) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) w_t[e] = w[edge[e]];
}

// sum += w[e] * val[src[e] * 64 + b] over [e0, e1), one term at a time in edge order.
// The (wave-uniform) sources and weights of the next kChunk edges are fetched while the
// presynaptic values of the current chunk are in flight, so each chunk costs about one
// memory round trip.
constexpr int kChunk = 16;
__device__ __forceinline__ float ordered_gather_sum(float acc, uint64_t e0, uint64_t e1, const int32_t *src,
                                                    const float *w, const float *val, uint32_t b) {
  uint64_t e = e0;
  int32_t sr[kChunk];
  float wv[kChunk];
  if (e + kChunk <= e1) {
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      sr[u] = src[e + u];
      wv[u] = w[e + u];
    }
  }
  while (e + kChunk <= e1) {
    float xv[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) xv[u] = val[(size_t)sr[u] * 64 + b];
    int32_t sn[kChunk];
    float wn[kChunk];
    const bool more = e + 2 * kChunk <= e1;
    if (more) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        sn[u] = src[e + kChunk + u];
        wn[u] = w[e + kChunk + u];
      }
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) acc = acc + wv[u] * xv[u];
    if (more) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        sr[u] = sn[u];
        wv[u] = wn[u];
      }
    }
    e += kChunk;
  }
  for (; e < e1; ++e) acc = acc + w[e] * val[(size_t)src[e] * 64 + b];
  return acc;
}

// The same ordered sum with two chunks of presynaptic values in flight: the values of
// chunk c + 1 are requested before the terms of chunk c are added, so that a chunk costs
// about half a memory round trip.  For the per-step kernels, where one wavefront per
// neuron is all the parallelism a step has.
__device__ __forceinline__ float ordered_gather_pipe(float acc, uint64_t e0, uint64_t e1, const int32_t *src,
                                                     const float *w, const float *val, uint32_t b) {
  uint64_t e = e0;
  if (e + 2 * kChunk <= e1) {
    int32_t sa[kChunk], sb[kChunk];
    float wa[kChunk], wb[kChunk], xa[kChunk], xb[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      sa[u] = src[e + u];
      wa[u] = w[e + u];
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) xa[u] = val[(size_t)sa[u] * 64 + b];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      sb[u] = src[e + kChunk + u];
      wb[u] = w[e + kChunk + u];
    }
    // invariant: chunk e is in (wa, xa), chunk e + kChunk (whole) has its sources in sb
    while (true) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) xb[u] = val[(size_t)sb[u] * 64 + b];
      const bool more = e + 3 * kChunk <= e1;
      if (more) {
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          sa[u] = src[e + 2 * kChunk + u];
        }
      }
#pragma unroll
      for (int u = 0; u < kChunk; ++u) acc = acc + wa[u] * xa[u];
      e += kChunk;
      // chunk e is in (wb, xb)
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        wa[u] = wb[u];
        xa[u] = xb[u];
      }
      if (!more) break;
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        sb[u] = sa[u];
        wb[u] = w[e + kChunk + u];
      }
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) acc = acc + wa[u] * xa[u];
    e += kChunk;
  }
  for (; e < e1; ++e) acc = acc + w[e] * val[(size_t)src[e] * 64 + b];
  return acc;
}

// The same ordered sum where every presynaptic value is 0 or 1, given as 64-bit batch
// masks: masks[src * stride + col] has bit b set where the value of batch element b is 1.
// A term then adds w[e] where the lane's bit is set and leaves the sum as it is where it
// is clear; that is the sum's own value, since w * 1 = w exactly and, for finite weights,
// adding w * 0 = +-0 leaves a sum that starts from +0 unchanged.  Lanes load the sources,
// weights and masks of 64 edges at once (two chunks, all requested before any term is
// added), and each edge's mask and weight reach the wavefront by lane reads, the mask as
// the lane condition: about two dependent memory round trips per 128 edges.
__device__ __forceinline__ uint64_t lane_read64(uint64_t x, uint32_t u) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)u);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ float ordered_mask_sum(float acc, uint64_t e0, uint64_t e1, const int32_t *src,
                                                  const float *w, const uint64_t *masks, uint64_t stride,
                                                  uint32_t col) {
  const uint32_t l = lane_id();
  for (uint64_t base = e0; base < e1; base += 2u * kWave) {
    // loads from indices clamped to the last edge, issued unconditionally so that they
    // are all in flight together; the masks of lanes past e1 are then cleared
    const uint64_t last = e1 - 1;
    const uint64_t ea = std::min<uint64_t>(base + l, last), eb = std::min<uint64_t>(base + kWave + l, last);
    const uint32_t sa = (uint32_t)src[ea], sb = (uint32_t)src[eb];
    const float wa = w[ea], wb = w[eb];
    uint64_t ma = masks[(uint64_t)sa * stride + col];
    uint64_t mb = masks[(uint64_t)sb * stride + col];
    if (base + l >= e1) ma = 0u;
    if (base + kWave + l >= e1) mb = 0u;
    // edges past e1 carry an empty mask, so whole groups of eight run unconditionally
    const uint32_t na = (uint32_t)std::min<uint64_t>(e1 - base, kWave);
#pragma unroll 8
    for (uint32_t u = 0; u < ((na + 7u) & ~7u); ++u) {
      const float sum = acc + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wa), (int)u));
      acc = __builtin_amdgcn_inverse_ballot_w64(lane_read64(ma, u)) ? sum : acc;
    }
    if (e1 - base > kWave) {
      const uint32_t nb = (uint32_t)std::min<uint64_t>(e1 - base - kWave, kWave);
#pragma unroll 8
      for (uint32_t u = 0; u < ((nb + 7u) & ~7u); ++u) {
        const float sum = acc + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wb), (int)u));
        acc = __builtin_amdgcn_inverse_ballot_w64(lane_read64(mb, u)) ? sum : acc;
      }
    }
  }
  return acc;
}

// The ordered mask sums of kSteps consecutive columns at once (acc[u] for column
// col0 + u), for kernels with parallelism to spare: the edges are wave-uniform, so their
// sources, weights and each source's kSteps masks (contiguous in a row) arrive by scalar
// loads, and a mask serves directly as the lane condition.  A term costs one add and one
// select.  The masks of a group of edges and the sources of the next group are requested
// together.  Rows must hold kSteps - 1 readable entries past the last column used.
constexpr int kMaskSteps = 8;
constexpr int kMaskGroup = 4;
__device__ __forceinline__ void ordered_mask_sum_steps(float (&acc)[kMaskSteps], uint64_t e0, uint64_t e1,
                                                       const int32_t *src, const float *w,
                                                       const uint64_t *masks, uint64_t stride, int64_t col0) {
  uint64_t e = e0;
  if (e + kMaskGroup <= e1) {
    uint32_t c[kMaskGroup];
    float wv[kMaskGroup];
#pragma unroll
    for (int g = 0; g < kMaskGroup; ++g) {
      c[g] = (uint32_t)src[e + g];
      wv[g] = w[e + g];
    }
    while (true) {
      uint64_t mk[kMaskGroup][kMaskSteps];
#pragma unroll
      for (int g = 0; g < kMaskGroup; ++g) {
        const uint64_t *row = masks + (int64_t)((uint64_t)c[g] * stride) + col0;
#pragma unroll
        for (int u = 0; u < kMaskSteps; ++u) mk[g][u] = row[u];
      }
      float wc[kMaskGroup];
#pragma unroll
      for (int g = 0; g < kMaskGroup; ++g) wc[g] = wv[g];
      const bool more = e + 2 * kMaskGroup <= e1;
      if (more) {
#pragma unroll
        for (int g = 0; g < kMaskGroup; ++g) {
          c[g] = (uint32_t)src[e + kMaskGroup + g];
          wv[g] = w[e + kMaskGroup + g];
        }
      }
#pragma unroll
      for (int g = 0; g < kMaskGroup; ++g)
#pragma unroll
        for (int u = 0; u < kMaskSteps; ++u) {
          const float sum = acc[u] + wc[g];
          acc[u] = __builtin_amdgcn_inverse_ballot_w64(mk[g][u]) ? sum : acc[u];
        }
      e += kMaskGroup;
      if (!more) break;
    }
  }
  for (; e < e1; ++e) {
    const uint64_t *row = masks + (int64_t)((uint64_t)(uint32_t)src[e] * stride) + col0;
    const float wv = w[e];
#pragma unroll
    for (int u = 0; u < kMaskSteps; ++u) {
      const float sum = acc[u] + wv;
      acc[u] = __builtin_amdgcn_inverse_ballot_w64(row[u]) ? sum : acc[u];
    }
  }
}

// Input-projection current of every step: iin[t][j][b] = sum over j's input in-edges,
// sources ascending, from 0 -- the first part of the hidden current in its defined order.
// It does not depend on the recurrent state, so all steps run in parallel.  Two kernels,
// of which the flag that k_bits set for the inputs lets one work: with binary inputs
// (flags[0] clear) k_input_current takes the terms from the input masks, a wavefront per
// (block of kMaskSteps steps, j); otherwise k_input_current_values gathers the values,
// a wavefront per (t, j).
__global__ __launch_bounds__(256) void k_input_current(BpttArgs a) {
  if (a.flags[0] != 0) return;
  // wave-uniform index (readfirstlane lets the edge lists be read with scalar loads)
  const uint64_t w = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t n_blocks = (a.T + kMaskSteps - 1) / kMaskSteps;
  if (w >= (uint64_t)n_blocks * a.H) return;
  const uint32_t t0 = (uint32_t)(w / a.H) * kMaskSteps, j = (uint32_t)(w % a.H);
  const uint32_t nt = std::min<uint32_t>(kMaskSteps, a.T - t0);
  const uint32_t b = lane_id();
  float acc[kMaskSteps];
#pragma unroll
  for (int u = 0; u < kMaskSteps; ++u) acc[u] = 0.0f;
  ordered_mask_sum_steps(acc, a.in_t_ptr[j], a.in_t_ptr[j + 1], a.in_t_src, a.w_in_t, a.xbits, a.T, t0);
#pragma unroll
  for (int u = 0; u < kMaskSteps; ++u)
    if ((uint32_t)u < nt) a.iin[((size_t)(t0 + u) * a.H + j) * 64 + b] = acc[u];
}

// (a bounded grid that strides over the (t, j) pairs, so that the launch costs little
// when the flag sends it home)
constexpr uint32_t kValuesGrid = 2048;
__global__ __launch_bounds__(256) void k_input_current_values(BpttArgs a) {
  if (a.flags[0] == 0) return;
  const uint32_t b = lane_id();
  const uint64_t first = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (uint64_t w = first; w < (uint64_t)a.T * a.H; w += (uint64_t)gridDim.x * 4) {
    const uint32_t t = (uint32_t)(w / a.H), j = (uint32_t)(w % a.H);
    const float *xt = a.xt + (size_t)t * a.C * 64;
    a.iin[w * 64 + b] = ordered_gather_sum(0.0f, a.in_t_ptr[j], a.in_t_ptr[j + 1], a.in_t_src, a.w_in_t, xt, b);
  }
}

// One step t of the hidden layer: one wavefront per hidden neuron j, lane = batch.  The
// current continues the input part with j's recurrent in-edges (sources ascending).
// vprev/sprev are step t-1 (nullptr at t = 0).  Writes v_out[j][b] and, if s_out is
// set, s_out[j][b].  In spiking mode the spikes are 0 or 1: the recurrent terms come
// from the masks of step t-1, and the step writes its own masks (sbits[j][t]).
__global__ __launch_bounds__(256) void k_hidden_step(BpttArgs a, uint32_t t, const float *vprev,
                                                     const float *sprev, float *v_out, float *s_out) {
  const uint32_t j = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  if (j >= a.H) return;
  const uint32_t b = lane_id();
  const bool binary = a.smooth == 0;
  float acc = a.iin[((size_t)t * a.H + j) * 64 + b];
  if (sprev) {
    if (binary)
      acc = ordered_mask_sum(acc, a.rec_t_ptr[j], a.rec_t_ptr[j + 1], a.rec_t_src, a.w_rec_t, a.sbits, a.T, t - 1);
    else
      acc = ordered_gather_pipe(acc, a.rec_t_ptr[j], a.rec_t_ptr[j + 1], a.rec_t_src, a.w_rec_t, sprev, b);
  }
  const float vp = vprev ? vprev[(size_t)j * 64 + b] : 0.0f;
  const float sp = sprev ? sprev[(size_t)j * 64 + b] : 0.0f;
  float v = a.beta * vp;
  v = v + acc;
  v = v - a.theta * sp;
  v_out[(size_t)j * 64 + b] = v;
  if (s_out) {
    const float sv = spike_fn(v - a.theta, a.slope, a.smooth != 0);
    s_out[(size_t)j * 64 + b] = sv;
    if (binary) {
      const uint64_t m = __ballot(b < a.B && sv != 0.0f);
      if (b == 0) a.sbits[(size_t)j * a.T + t] = m;
    }
  }
}

// The hidden step in spiking mode with the ELL copy of the recurrent in-edges: the row of
// neuron j sits at j * ell_w, so its sources and weights are requested at once, together
// with iin, the state and the previous step's masks of all H neurons, which the workgroup
// stages in LDS (one memory round trip in all, where the CSR form needs the row bounds,
// then the edges, then the masks).  Each lane then reads its edge's mask from LDS, and the
// terms are added in row order, one add and one select each, as in ordered_mask_sum.
// kChunks = ell_w / 64.  The step writes its masks in both layouts.
template <int kChunks>
__global__ __launch_bounds__(256) void k_hidden_step_ell(BpttArgs a, uint32_t t, const float *vprev,
                                                         const float *sprev, float *v_out, float *s_out) {
  extern __shared__ uint64_t prev_masks[];  // [H]: step t - 1
  const uint32_t j = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  // every wave reaches the barrier; one past the last neuron loads neuron 0's data and
  // stores nothing
  const bool live = j < a.H;
  const uint32_t jl = live ? j : 0u;
  const uint32_t b = lane_id();
  const size_t jb = (size_t)jl * 64 + b;
  float acc = a.iin[(size_t)t * a.H * 64 + jb];
  const float vp = vprev ? vprev[jb] : 0.0f;
  const float sp = sprev ? sprev[jb] : 0.0f;
  int32_t src[kChunks];
  float wt[kChunks];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const size_t x = (size_t)jl * a.ell_w + (uint32_t)c * kWave + b;
    src[c] = a.ell_src[x];
    wt[c] = a.ell_wt[x];
  }
  const uint32_t len = a.ell_len[jl];
  if (sprev) {
    // four loads per thread in flight, from indices clamped into the row
    const uint64_t *row = a.sbits_t + (size_t)(t - 1) * a.H;
    for (uint32_t base = 0; base < a.H; base += 4u * 256u) {
      uint64_t v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = row[std::min<uint32_t>(base + (uint32_t)q * 256u + threadIdx.x, a.H - 1)];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + (uint32_t)q * 256u + threadIdx.x;
        if (i < a.H) prev_masks[i] = v[q];
      }
    }
  }
  __syncthreads();
  if (sprev && live) {
    uint64_t m[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) m[c] = (uint32_t)c * kWave + b < len ? prev_masks[src[c]] : 0u;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const uint32_t n = len > (uint32_t)c * kWave ? std::min<uint32_t>(len - (uint32_t)c * kWave, kWave) : 0u;
#pragma unroll 8
      for (uint32_t u = 0; u < ((n + 7u) & ~7u); ++u) {
        const float sum = acc + __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wt[c]), (int)u));
        acc = __builtin_amdgcn_inverse_ballot_w64(lane_read64(m[c], u)) ? sum : acc;
      }
    }
  }
  if (!live) return;
  float v = a.beta * vp;
  v = v + acc;
  v = v - a.theta * sp;
  v_out[jb] = v;
  if (s_out) {
    const float sv = spike_fn(v - a.theta, a.slope, false);
    s_out[jb] = sv;
    const uint64_t mk = __ballot(b < a.B && sv != 0.0f);
    if (b == 0) {
      a.sbits[(size_t)j * a.T + t] = mk;
      a.sbits_t[(size_t)t * a.H + j] = mk;
    }
  }
}

// Backward recomputation of one checkpoint segment [t0, t0 + len).  The spikes of every
// step are stored, so the currents of all the segment's steps are independent: these
// kernels compute them in parallel, each exactly as k_hidden_step does (input part, then
// the recurrent in-edges over s_{t-1} in ascending source order), into cur[k][j][b].  In
// spiking mode k_seg_current takes the terms from the spike masks the forward pass
// wrote, a wavefront per (block of kMaskSteps steps, j); in smooth mode
// k_seg_current_values gathers the values, a wavefront per (k, j).
__global__ __launch_bounds__(256) void k_seg_current(BpttArgs a, uint32_t t0, uint32_t len, float *cur) {
  const uint64_t w = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t n_blocks = (len + kMaskSteps - 1) / kMaskSteps;
  if (w >= (uint64_t)n_blocks * a.H) return;
  const uint32_t k0 = (uint32_t)(w / a.H) * kMaskSteps, j = (uint32_t)(w % a.H);
  const uint32_t nt = std::min<uint32_t>(kMaskSteps, len - k0);
  const uint32_t b = lane_id();
  float acc[kMaskSteps];
#pragma unroll
  for (int u = 0; u < kMaskSteps; ++u)
    acc[u] = (uint32_t)u < nt ? a.iin[((size_t)(t0 + k0 + u) * a.H + j) * 64 + b] : 0.0f;
  const float first = acc[0];
  // column t - 1 of step t; at t = 0 the masks read (entries before the array's start
  // for j = 0) are not used: that step has no recurrent term
  ordered_mask_sum_steps(acc, a.rec_t_ptr[j], a.rec_t_ptr[j + 1], a.rec_t_src, a.w_rec_t, a.sbits, a.T,
                         (int64_t)(t0 + k0) - 1);
  if (t0 + k0 == 0) acc[0] = first;
#pragma unroll
  for (int u = 0; u < kMaskSteps; ++u)
    if ((uint32_t)u < nt) cur[((size_t)(k0 + u) * a.H + j) * 64 + b] = acc[u];
}

__global__ __launch_bounds__(256) void k_seg_current_values(BpttArgs a, uint32_t t0, uint32_t len, float *cur) {
  const uint64_t w = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= (uint64_t)len * a.H) return;
  const uint32_t k = (uint32_t)(w / a.H), j = (uint32_t)(w % a.H), t = t0 + k;
  const uint32_t b = lane_id();
  float acc = a.iin[((size_t)t * a.H + j) * 64 + b];
  if (t > 0)
    acc = ordered_gather_sum(acc, a.rec_t_ptr[j], a.rec_t_ptr[j + 1], a.rec_t_src, a.w_rec_t,
                             a.s + (size_t)(t - 1) * a.H * 64, b);
  cur[w * 64 + b] = acc;
}

// ... then the membranes of the segment from the checkpoint before it (vprev; nullptr at
// step 0), one lane per (j, b), with k_hidden_step's operations in its order; vseg[k]
// holds the current of step t0 + k on entry and V_{t0+k} on return.
__global__ void k_seg_scan(BpttArgs a, uint32_t t0, uint32_t len, const float *vprev, float *vseg) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;  // j * 64 + b
  if (x >= a.H * 64) return;
  float v = vprev ? vprev[x] : 0.0f;
  for (uint32_t k = 0; k < len; ++k) {
    const uint32_t t = t0 + k;
    const float sp = t ? a.s[(size_t)(t - 1) * a.H * 64 + x] : 0.0f;
    float vn = a.beta * v;
    vn = vn + vseg[(size_t)k * a.H * 64 + x];
    vn = vn - a.theta * sp;
    vseg[(size_t)k * a.H * 64 + x] = vn;
    v = vn;
  }
}

// Readout drive of every step: ro[t][o][b] = sum_i s[t][i][b] w_out[i][o], ascending i;
// the loads of 16 consecutive i are issued before their terms are added in order.
__global__ void k_readout_drive(BpttArgs a, float *ro) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)a.T * a.O * 64) return;
  const uint32_t b = (uint32_t)(idx & 63u);
  const uint64_t to = idx >> 6;
  const uint32_t o = (uint32_t)(to % a.O), t = (uint32_t)(to / a.O);
  const float *st = a.s + (size_t)t * a.H * 64 + b;
  const float *wo = a.w_out + o;
  float acc = 0.0f;
  uint32_t i = 0;
  for (; i + 16 <= a.H; i += 16) {
    float sv[16], wv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      sv[u] = st[(size_t)(i + u) * 64];
      wv[u] = wo[(size_t)(i + u) * a.O];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = acc + sv[u] * wv[u];
  }
  for (; i < a.H; ++i) acc = acc + st[(size_t)i * 64] * wo[(size_t)i * a.O];
  ro[idx] = acc;
}

// Leaky readout and its maximum over time (first step attaining it): block o, lane b.
__global__ void k_readout_scan(BpttArgs a, const float *ro) {
  const uint32_t o = blockIdx.x, b = threadIdx.x;
  if (b >= a.B) return;
  float u = 0.0f, m = 0.0f;
  uint32_t tm = 0;
  auto step = [&](uint32_t t, float r) {
    float ut = a.beta_out * u;
    ut = ut + r;
    u = ut;
    if (t == 0 || ut > m) {
      m = ut;
      tm = t;
    }
  };
  uint32_t t = 0;
  for (; t + 8 <= a.T; t += 8) {  // eight drives requested before the eight steps
    float r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = ro[((size_t)(t + q) * a.O + o) * 64 + b];
#pragma unroll
    for (int q = 0; q < 8; ++q) step(t + q, r[q]);
  }
  for (; t < a.T; ++t) step(t, ro[((size_t)t * a.O + o) * 64 + b]);
  a.m[(size_t)b * a.O + o] = m;
  a.tmax[(size_t)b * a.O + o] = (int32_t)tm;
}

// Softmax cross entropy of the maxima, its gradient dL/dmax = (p - onehot) / B, and the
// mean loss; one block of 64 threads (lane b).
__global__ void k_loss(BpttArgs a, const int32_t *labels, float *loss) {
  __shared__ float s_lb[64];
  const uint32_t b = threadIdx.x;
  if (b < a.B) {
    const float *m = a.m + (size_t)b * a.O;
    float mx = m[0];
    for (uint32_t k = 1; k < a.O; ++k) mx = fmaxf(mx, m[k]);
    float z = 0.0f;
    for (uint32_t k = 0; k < a.O; ++k) z += expf(m[k] - mx);
    const int32_t y = labels[b];
    const bool valid = y >= 0 && (uint32_t)y < a.O;  // an invalid label yields NaN
    s_lb[b] = valid ? mx + logf(z) - m[y] : __int_as_float(0x7fc00000);
    for (uint32_t k = 0; k < a.O; ++k) {
      const float p = expf(m[k] - mx) / z;
      a.dm[(size_t)b * a.O + k] = valid ? (p - ((int32_t)k == y ? 1.0f : 0.0f)) / (float)a.B
                                        : __int_as_float(0x7fc00000);
    }
  }
  __syncthreads();
  if (b == 0) {
    float sum = 0.0f;
    for (uint32_t k = 0; k < a.B; ++k) sum += s_lb[k];
    *loss = sum / (float)a.B;
  }
}

// Readout adjoint: lamu[t][o][b] = g_t + beta_out lamu[t+1], g_t = dm at the max step,
// scaled by the incoming gradient of the loss; block o, lane b (zeros for b >= B).
__global__ void k_lam_u(BpttArgs a, const float *g_loss) {
  const uint32_t o = blockIdx.x, b = threadIdx.x;
  const float scale = g_loss ? *g_loss : 1.0f;
  const float g = b < a.B ? a.dm[(size_t)b * a.O + o] * scale : 0.0f;
  const int32_t tm = b < a.B ? a.tmax[(size_t)b * a.O + o] : -1;
  float nxt = 0.0f;
  for (int32_t t = (int32_t)a.T - 1; t >= 0; --t) {
    nxt = (t == tm ? g : 0.0f) + a.beta_out * nxt;
    a.lamu[((size_t)t * a.O + o) * 64 + b] = nxt;
  }
}

// Readout part of the spike adjoint of every step, the first terms of the sum that
// k_adjoint_step completes: dsr[t][i][b] = sum_o w_out[i][o] lamu[t][o][b], ascending o
// from +0.  It does not depend on the membrane adjoint, so all steps run in parallel (a
// wavefront per (t, i)), ahead of the sequential adjoint steps.
__global__ __launch_bounds__(256) void k_readout_adjoint(BpttArgs a, float *dsr) {
  const uint64_t w = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= (uint64_t)a.T * a.H) return;
  const uint32_t t = (uint32_t)(w / a.H), i = (uint32_t)(w % a.H);
  const uint32_t b = lane_id();
  const float *lu = a.lamu + (size_t)t * a.O * 64 + b;
  // in ascending o, eight loads issued before their terms are added
  float ds = 0.0f;
  uint32_t o = 0;
  for (; o + 8 <= a.O; o += 8) {
    float wv[8], lv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      wv[u] = a.w_out[(size_t)i * a.O + o + u];
      lv[u] = lu[(size_t)(o + u) * 64];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) ds = ds + wv[u] * lv[u];
  }
  for (; o < a.O; ++o) ds = ds + a.w_out[(size_t)i * a.O + o] * lu[(size_t)o * 64];
  dsr[w * 64 + b] = ds;
}

// Membrane adjoint of step t: one wavefront per hidden neuron i, lane = batch.
// lam_next = lamV_{t+1} ([H][64], zeros for step T), v_t = V_t; lam_out = lamV_t holds
// the readout part of the spike adjoint (k_readout_adjoint) on entry and receives
// lamV_t.
__global__ __launch_bounds__(256) void k_adjoint_step(BpttArgs a, uint32_t t, const float *v_t,
                                                      const float *lam_next, float *lam_out) {
  const uint32_t i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  if (i >= a.H) return;
  const uint32_t b = lane_id();
  float ds = lam_out[(size_t)i * 64 + b];  // the readout terms, in ascending o
  // the neuron's own values are requested before the gather, so that they are not a
  // round trip of their own after it (0.08 ms per iteration)
  const float ln = lam_next[(size_t)i * 64 + b];
  const float vt = v_t[(size_t)i * 64 + b];
  ds = ordered_gather_pipe(ds, a.rec_ptr[i], a.rec_ptr[i + 1], a.rec_col, a.w_rec, lam_next, b);
  if (!a.detach_reset) ds = ds - a.theta * ln;
  const float z = vt - a.theta;
  lam_out[(size_t)i * 64 + b] = a.beta * ln + surrogate(z, a.slope, a.smooth != 0) * ds;
}

// Batch masks of a [T][rows][64] trajectory: bits[r][t] bit b = (val[t][r][b] != 0) for
// b < B; flag receives 1 if any of those values is neither 0 nor 1 (the masks then do
// not represent the values and the gradients take the general path).  A wavefront per
// (t, r).
__global__ __launch_bounds__(256) void k_bits(const float *val, uint32_t rows, uint32_t T, uint32_t B,
                                              uint64_t *bits, uint32_t *flag) {
  const uint64_t w = (uint64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (w >= (uint64_t)T * rows) return;
  const uint32_t t = (uint32_t)(w / rows), r = (uint32_t)(w % rows), b = lane_id();
  const float x = val[w * 64 + b];
  const bool on = b < B && x != 0.0f;
  const uint64_t m = __ballot(on);
  const uint64_t bad = __ballot(on && x != 1.0f);
  if (b == 0) {
    bits[(size_t)r * T + t] = m;
    if (bad) atomicOr(flag, 1u);
  }
}

constexpr int kGradBlock = 256;
constexpr uint32_t kGradChunk = 128;  // steps of lamV staged in LDS at a time (32 KB)
constexpr int kMaskAhead = 8;         // mask words in flight per lane

// Gradients of the sparse weights, one owner per synapse: the adjoint of the current
// I_t = W_in^T x_t + W_rec^T s_{t-1} gives
//   g_in[c -> j]  = sum_t sum_b x_t[c][b] lamV_t[j][b]
//   g_rec[i -> j] = sum_t sum_b s_{t-1}[i][b] lamV_t[j][b].
// One workgroup per target j stages lamV_t[j][.] in LDS, kGradChunk steps at a time; each
// lane owns one in-edge of j (input projection first, then recurrent, each in ascending
// source order), kGradBlock edges per pass.  With binary presynaptic values (the masks'
// flag clear) the lane walks the set bits of its source's batch mask of every step and
// adds the matching lamV entries in ascending b, summing each step before adding it to
// the edge's total; otherwise it multiplies the stored values in.  The mask words of the
// next kMaskAhead steps are loaded while the current ones are used.
__global__ __launch_bounds__(kGradBlock) void k_grad_edges(BpttArgs a, const uint64_t *xbits,
                                                           const uint64_t *sbits, const uint32_t *flags) {
  extern __shared__ float lam_s[];  // [kGradChunk][64]
  const uint32_t j = blockIdx.x;
  const uint64_t in0 = a.in_t_ptr[j], rec0 = a.rec_t_ptr[j];
  const uint32_t n_in = (uint32_t)(a.in_t_ptr[j + 1] - in0), n_rec = (uint32_t)(a.rec_t_ptr[j + 1] - rec0);
  const uint32_t deg = n_in + n_rec, T = a.T;
  const bool x_bits = flags[0] == 0, s_bits = !a.smooth && flags[1] == 0;
  for (uint32_t base = 0; base < deg; base += kGradBlock) {
    const uint32_t k = base + threadIdx.x;
    const bool live = k < deg, is_in = k < n_in;
    uint32_t src = 0, edge = 0;
    if (live) {
      src = (uint32_t)(is_in ? a.in_t_src[in0 + k] : a.rec_t_src[rec0 + (k - n_in)]);
      edge = is_in ? a.in_t_edge[in0 + k] : a.rec_t_edge[rec0 + (k - n_in)];
    }
    const bool use_bits = is_in ? x_bits : s_bits;
    // the lane's mask row: the input's step t, or the hidden neuron's step t - 1
    const uint64_t *row = is_in ? xbits + (size_t)src * T : sbits + (size_t)src * T;
    const uint32_t lag = is_in ? 0u : 1u;
    auto mask_at = [&](uint32_t t) -> uint64_t {
      return (live && use_bits && t >= lag && t - lag < T) ? row[t - lag] : 0ull;
    };
    float total = 0.0f;
    for (uint32_t tc = 0; tc < T; tc += kGradChunk) {
      const uint32_t len = min(kGradChunk, T - tc);
      __syncthreads();  // the previous chunk has been read by every lane
      for (uint32_t x = threadIdx.x; x < len * 64; x += kGradBlock)
        lam_s[x] = a.lamv[((size_t)(tc + x / 64) * a.H + j) * 64 + (x & 63u)];
      __syncthreads();
      if (!live) continue;
      if (use_bits) {
        uint64_t cur[kMaskAhead], nxt[kMaskAhead];
#pragma unroll
        for (int q = 0; q < kMaskAhead; ++q) cur[q] = mask_at(tc + q);
        for (uint32_t u0 = 0; u0 < len; u0 += kMaskAhead) {
#pragma unroll
          for (int q = 0; q < kMaskAhead; ++q) nxt[q] = u0 + kMaskAhead + q < len ? mask_at(tc + u0 + kMaskAhead + q) : 0ull;
#pragma unroll
          for (int q = 0; q < kMaskAhead; ++q) {
            if (u0 + q >= len) break;
            uint64_t m = cur[q];
            const float *lt = lam_s + (size_t)(u0 + q) * 64;
            float part = 0.0f;
            while (m) {
              part += lt[__builtin_ctzll(m)];
              m &= m - 1;
            }
            total += part;
          }
#pragma unroll
          for (int q = 0; q < kMaskAhead; ++q) cur[q] = nxt[q];
        }
      } else {
        for (uint32_t u = 0; u < len; ++u) {
          const uint32_t t = tc + u;
          if (t < lag) continue;
          const float *val = is_in ? a.xt + ((size_t)t * a.C + src) * 64 : a.s + ((size_t)(t - 1) * a.H + src) * 64;
          const float *lt = lam_s + (size_t)u * 64;
          float part = 0.0f;
          for (uint32_t b = 0; b < a.B; ++b) part += val[b] * lt[b];
          total += part;
        }
      }
    }
    if (live) (is_in ? a.g_w_in : a.g_w_rec)[edge] = total;
  }
}

// Gradient of the dense readout weights over the whole sequence: one wavefront per
// hidden neuron i and output o; four partial sums keep loads of later steps in flight.
__global__ __launch_bounds__(256) void k_grad_out(BpttArgs a) {
  const uint32_t w = blockIdx.x * 4 + threadIdx.x / kWave;
  if (w >= a.H * a.O) return;
  const uint32_t i = w / a.O, o = w % a.O, b = lane_id();
  const float *sp = a.s + (size_t)i * 64 + b;
  const float *lp = a.lamu + (size_t)o * 64 + b;
  const size_t ss = (size_t)a.H * 64, ls = (size_t)a.O * 64;
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  uint32_t t = 0;
  for (; t + 4 <= a.T; t += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += sp[(t + u) * ss] * lp[(t + u) * ls];
  }
  for (; t < a.T; ++t) acc[0] += sp[t * ss] * lp[t * ls];
  const float sum = wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
  if (b == 0) a.g_w_out[(size_t)i * a.O + o] = sum;
}

__global__ void k_fill(float *p, uint64_t n, float v) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) p[idx] = v;
}

uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

}  // namespace

// ELL-order copy of the recurrent weights: w_ell[x] = w[edge[x]], 0 for padding.
__global__ void k_gather_ell(const float *w, const uint32_t *edge, float *w_ell, uint64_t n) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) w_ell[x] = edge[x] == 0xFFFFFFFFu ? 0.0f : w[edge[x]];
}

static void gather_weights(const BpttArgs &a, hipStream_t s) {
  if (a.ell_w)
    hipLaunchKernelGGL(k_gather_ell, dim3(blocks_for((uint64_t)a.H * a.ell_w, 256)), dim3(256), 0, s, a.w_rec,
                       a.ell_edge, a.ell_wt, (uint64_t)a.H * a.ell_w);
  if (a.nnz_in)
    hipLaunchKernelGGL(k_gather_t, dim3(blocks_for(a.nnz_in, 256)), dim3(256), 0, s, a.w_in, a.in_t_edge,
                       a.w_in_t, a.nnz_in);
  if (a.nnz_rec)
    hipLaunchKernelGGL(k_gather_t, dim3(blocks_for(a.nnz_rec, 256)), dim3(256), 0, s, a.w_rec, a.rec_t_edge,
                       a.w_rec_t, a.nnz_rec);
}

// The forward and backward passes each run as three parts.  The prologue and epilogue
// read or write the caller's arrays (inputs, weights, labels, loss, gradients); the body
// in between touches only the plan's own buffers (its weight copies included), so the
// runtime can capture it once per plan in a HIP graph and replay it on every call.

hipError_t bptt_forward_prologue(const BpttArgs &a, const float *x, hipStream_t s) {
  gather_weights(a, s);
  // flags[0] is set below if some input is neither 0 nor 1; flags[1] only by the backward
  // pass of a smooth-mode plan
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, reinterpret_cast<float *>(a.flags), (uint64_t)2, 0.0f);
  hipLaunchKernelGGL(k_transpose_x, dim3((a.C + 63) / 64, a.T), dim3(256), 0, s, x, a.xt, a.xbits, a.flags, a.B,
                     a.T, a.C);
  const hipError_t e = hipMemcpyAsync(a.w_out_c, a.w_out, (size_t)a.H * a.O * 4, hipMemcpyDeviceToDevice, s);
  return e != hipSuccess ? e : hipGetLastError();
}

// g: the plan's arguments with w_out = w_out_c
hipError_t bptt_forward_body(const BpttArgs &g, hipStream_t s) {
  // the inputs' batch masks and flags[0] come from the prologue's transpose
  hipLaunchKernelGGL(k_input_current, dim3(blocks_for((uint64_t)((g.T + kMaskSteps - 1) / kMaskSteps) * g.H, 4)),
                     dim3(256), 0, s, g);
  hipLaunchKernelGGL(k_input_current_values, dim3(std::min<uint32_t>(blocks_for((uint64_t)g.T * g.H, 4), kValuesGrid)),
                     dim3(256), 0, s, g);
  const dim3 grid(blocks_for(g.H, 4));
  float *vprev = nullptr;
  for (uint32_t t = 0; t < g.T; ++t) {
    // V of the step before each checkpoint segment is kept; the others rotate
    float *v_out = (t % g.K == g.K - 1 || t == g.T - 1) ? g.vck + (size_t)(t / g.K) * g.H * 64
                                                          : g.vtmp + (size_t)(t & 1u) * g.H * 64;
    const float *sprev = t ? g.s + (size_t)(t - 1) * g.H * 64 : nullptr;
    float *s_out = g.s + (size_t)t * g.H * 64;
    if (!g.smooth && g.ell_w) {
      const size_t lds = (size_t)g.H * sizeof(uint64_t);
      switch (g.ell_w / kWave) {
        case 1: hipLaunchKernelGGL(k_hidden_step_ell<1>, grid, dim3(256), lds, s, g, t, vprev, sprev, v_out, s_out); break;
        case 2: hipLaunchKernelGGL(k_hidden_step_ell<2>, grid, dim3(256), lds, s, g, t, vprev, sprev, v_out, s_out); break;
        case 3: hipLaunchKernelGGL(k_hidden_step_ell<3>, grid, dim3(256), lds, s, g, t, vprev, sprev, v_out, s_out); break;
        default: hipLaunchKernelGGL(k_hidden_step_ell<4>, grid, dim3(256), lds, s, g, t, vprev, sprev, v_out, s_out); break;
      }
    } else {
      hipLaunchKernelGGL(k_hidden_step, grid, dim3(256), 0, s, g, t, vprev, sprev, v_out, s_out);
    }
    vprev = v_out;
  }
  hipLaunchKernelGGL(k_readout_drive, dim3(blocks_for((uint64_t)g.T * g.O * 64, 256)), dim3(256), 0, s, g,
                     g.ro);
  hipLaunchKernelGGL(k_readout_scan, dim3(g.O), dim3(64), 0, s, g, g.ro);
  return hipGetLastError();
}

hipError_t bptt_forward_epilogue(const BpttArgs &a, const int32_t *labels, float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, s, a, labels, loss);
  return hipGetLastError();
}

hipError_t bptt_backward_prologue(const BpttArgs &a, const float *g_loss, hipStream_t s) {
  gather_weights(a, s);
  hipError_t e = hipMemcpyAsync(a.w_out_c, a.w_out, (size_t)a.H * a.O * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && a.nnz_rec)
    e = hipMemcpyAsync(a.w_rec_c, a.w_rec, (size_t)a.nnz_rec * 4, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lam_u, dim3(a.O), dim3(64), 0, s, a, g_loss);
  return hipGetLastError();
}

// g: the plan's arguments with w_out = w_out_c and w_rec = w_rec_c
hipError_t bptt_backward_body(const BpttArgs &g, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for((uint64_t)g.H * 64, 256)), dim3(256), 0, s, g.lam_carry,
                     (uint64_t)g.H * 64, 0.0f);
  // batch masks of the hidden trajectory for the sparse-weight gradients: in spiking
  // mode the forward pass wrote them (and flags[1] stayed clear); in smooth mode they are
  // taken here, and flag that the values are not binary
  if (g.smooth)
    hipLaunchKernelGGL(k_bits, dim3(blocks_for((uint64_t)g.T * g.H, 4)), dim3(256), 0, s, g.s, g.H, g.T, g.B,
                       g.sbits, g.flags + 1);
  // the readout part of every step's spike adjoint, into lamv (each adjoint step reads
  // its own entries, then overwrites them with lamV_t)
  hipLaunchKernelGGL(k_readout_adjoint, dim3(blocks_for((uint64_t)g.T * g.H, 4)), dim3(256), 0, s, g, g.lamv);
  const dim3 grid(blocks_for(g.H, 4));
  const uint32_t n_seg = (g.T + g.K - 1) / g.K;
  for (int32_t seg = (int32_t)n_seg - 1; seg >= 0; --seg) {
    const uint32_t t0 = (uint32_t)seg * g.K, len = std::min(g.K, g.T - t0);
    // recompute the segment's membranes from the checkpoint before it and the stored
    // spikes (the forward pass's operations): all its currents at once, then the scan
    const float *vprev = seg ? g.vck + (size_t)(seg - 1) * g.H * 64 : nullptr;
    if (g.smooth)
      hipLaunchKernelGGL(k_seg_current_values, dim3(blocks_for((uint64_t)len * g.H, 4)), dim3(256), 0, s, g, t0,
                         len, g.vseg);
    else
      hipLaunchKernelGGL(k_seg_current, dim3(blocks_for((uint64_t)((len + kMaskSteps - 1) / kMaskSteps) * g.H, 4)),
                         dim3(256), 0, s, g, t0, len, g.vseg);
    hipLaunchKernelGGL(k_seg_scan, dim3(blocks_for((uint64_t)g.H * 64, 256)), dim3(256), 0, s, g, t0, len, vprev,
                       g.vseg);
    for (int32_t k = (int32_t)len - 1; k >= 0; --k) {
      const uint32_t t = t0 + (uint32_t)k;
      const float *lam_next = t + 1 < g.T ? g.lamv + (size_t)(t + 1) * g.H * 64 : g.lam_carry;
      hipLaunchKernelGGL(k_adjoint_step, grid, dim3(256), 0, s, g, t, g.vseg + (size_t)k * g.H * 64, lam_next,
                         g.lamv + (size_t)t * g.H * 64);
    }
  }
  return hipGetLastError();
}

// the gradients, written to the caller's arrays
hipError_t bptt_backward_epilogue(const BpttArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_out, dim3(blocks_for((uint64_t)a.H * a.O, 4)), dim3(256), 0, s, a);
  if (a.nnz_in + a.nnz_rec)
    hipLaunchKernelGGL(k_grad_edges, dim3(a.H), dim3(kGradBlock), (size_t)std::min(kGradChunk, a.T) * 64 * 4, s, a,
                       a.xbits, a.sbits, a.flags);
  return hipGetLastError();
}

}  // namespace snn
