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
//   lamv  [K][H][64]         membrane adjoint of one segment (+ carry [H][64])
// Weights stay in the caller's CSR order (rows = presynaptic neuron, sorted targets);
// the forward current is a gather over the transposed index (per target, sources in
// ascending order, input projection first), the adjoint's dL/ds a gather over the
// forward rows, and every weight gradient has exactly one owner.
#include <rocblas/rocblas.h>

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

// x [B][T][C] -> xt [T][C][64]; lanes >= B hold zeros.
__global__ void k_transpose_x(const float *x, float *xt, uint32_t B, uint32_t T, uint32_t C) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = (uint64_t)T * C * 64;
  if (idx >= total) return;
  const uint32_t b = (uint32_t)(idx & 63u);
  const uint64_t tc = idx >> 6;
  const uint32_t c = (uint32_t)(tc % C), t = (uint32_t)(tc / C);
  xt[idx] = b < B ? x[((uint64_t)b * T + t) * C + c] : 0.0f;
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

// Input-projection current of every step: iin[t][j][b] = sum over j's input in-edges,
// sources ascending, from 0 -- the first part of the hidden current in its defined order.
// It does not depend on the recurrent state, so all steps run in parallel (a wavefront
// per (t, j)).
__global__ __launch_bounds__(256) void k_input_current(BpttArgs a) {
  // wave-uniform index (readfirstlane lets the edge lists be read with scalar loads)
  const uint64_t w = (uint64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= (uint64_t)a.T * a.H) return;
  const uint32_t t = (uint32_t)(w / a.H), j = (uint32_t)(w % a.H);
  const uint32_t b = lane_id();
  const float *xt = a.xt + (size_t)t * a.C * 64;
  a.iin[w * 64 + b] = ordered_gather_sum(0.0f, a.in_t_ptr[j], a.in_t_ptr[j + 1], a.in_t_src, a.w_in_t, xt, b);
}

// One step t of the hidden layer: one wavefront per hidden neuron j, lane = batch.  The
// current continues the input part with j's recurrent in-edges (sources ascending).
// vprev/sprev are step t-1 (nullptr at t = 0).  Writes v_out[j][b] and, if s_out is
// set, s_out[j][b].
__global__ __launch_bounds__(256) void k_hidden_step(BpttArgs a, uint32_t t, const float *vprev,
                                                     const float *sprev, float *v_out, float *s_out) {
  const uint32_t j = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  if (j >= a.H) return;
  const uint32_t b = lane_id();
  float acc = a.iin[((size_t)t * a.H + j) * 64 + b];
  if (sprev) acc = ordered_gather_sum(acc, a.rec_t_ptr[j], a.rec_t_ptr[j + 1], a.rec_t_src, a.w_rec_t, sprev, b);
  const float vp = vprev ? vprev[(size_t)j * 64 + b] : 0.0f;
  const float sp = sprev ? sprev[(size_t)j * 64 + b] : 0.0f;
  float v = a.beta * vp;
  v = v + acc;
  v = v - a.theta * sp;
  v_out[(size_t)j * 64 + b] = v;
  if (s_out) s_out[(size_t)j * 64 + b] = spike_fn(v - a.theta, a.slope, a.smooth != 0);
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
  for (uint32_t t = 0; t < a.T; ++t) {
    float ut = a.beta_out * u;
    ut = ut + ro[((size_t)t * a.O + o) * 64 + b];
    u = ut;
    if (t == 0 || ut > m) {
      m = ut;
      tm = t;
    }
  }
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

// Membrane adjoint of step t: one wavefront per hidden neuron i, lane = batch.
// lam_next = lamV_{t+1} ([H][64], zeros past the end), v_t = V_t, lam_out = lamV_t.
__global__ __launch_bounds__(256) void k_adjoint_step(BpttArgs a, uint32_t t, const float *v_t,
                                                      const float *lam_next, float *lam_out) {
  const uint32_t i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  if (i >= a.H) return;
  const uint32_t b = lane_id();
  const float *lu = a.lamu + (size_t)t * a.O * 64 + b;
  float ds = 0.0f;
  for (uint32_t o = 0; o < a.O; ++o) ds = ds + a.w_out[(size_t)i * a.O + o] * lu[(size_t)o * 64];
  ds = ordered_gather_sum(ds, a.rec_ptr[i], a.rec_ptr[i + 1], a.rec_col, a.w_rec, lam_next, b);
  const float ln = lam_next[(size_t)i * 64 + b];
  if (!a.detach_reset) ds = ds - a.theta * ln;
  const float z = v_t[(size_t)i * 64 + b] - a.theta;
  lam_out[(size_t)i * 64 + b] = a.beta * ln + surrogate(z, a.slope, a.smooth != 0) * ds;
}

// Gradients of the sparse weights are masked dense contractions over (t, b):
//   dW_in[c][j]  = sum_{t,b} x_t[c][b] lamV_t[j][b]
//   dW_rec[i][j] = sum_{t,b} s_{t-1}[i][b] lamV_t[j][b]
// Each checkpoint segment lays its trajectories out as [row][(t, b)] matrices and adds
// its contribution with one FP32 GEMM per projection (rocBLAS, accumulating over the
// segments); the entries on the masks are then gathered into the CSR-ordered gradients.
//
// seg[r][k * 64 + b] = src[t0 + k - shift][r][b] (zero before step 0), k < len, for a
// [T][rows][64] trajectory; row stride kcols.
__global__ void k_seg_rows(const float *src, float *seg, uint32_t rows, uint32_t t0, uint32_t len,
                           uint32_t kcols, uint32_t shift) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)rows * len * 64) return;
  const uint32_t b = (uint32_t)(idx & 63u);
  const uint64_t rk = idx >> 6;
  const uint32_t k = (uint32_t)(rk % len), r = (uint32_t)(rk / len);
  const int64_t t = (int64_t)t0 + k - shift;
  seg[(size_t)r * kcols + (size_t)k * 64 + b] = t >= 0 ? src[((size_t)t * rows + r) * 64 + b] : 0.0f;
}

// g[edge] = dense[src][j] for every in-edge (src -> j) of the transposed index; a
// wavefront per target j.
__global__ __launch_bounds__(256) void k_mask_gather(const uint64_t *t_ptr, const int32_t *t_src,
                                                     const uint32_t *t_edge, const float *dense, uint32_t cols,
                                                     uint32_t n_targets, float *g) {
  const uint32_t j = blockIdx.x * 4 + threadIdx.x / kWave;
  if (j >= n_targets) return;
  for (uint64_t e = t_ptr[j] + lane_id(); e < t_ptr[j + 1]; e += kWave)
    g[t_edge[e]] = dense[(size_t)t_src[e] * cols + j];
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

static void gather_weights(const BpttArgs &a, hipStream_t s) {
  if (a.nnz_in)
    hipLaunchKernelGGL(k_gather_t, dim3(blocks_for(a.nnz_in, 256)), dim3(256), 0, s, a.w_in, a.in_t_edge,
                       a.w_in_t, a.nnz_in);
  if (a.nnz_rec)
    hipLaunchKernelGGL(k_gather_t, dim3(blocks_for(a.nnz_rec, 256)), dim3(256), 0, s, a.w_rec, a.rec_t_edge,
                       a.w_rec_t, a.nnz_rec);
}

hipError_t bptt_forward(const BpttArgs &a, const float *x, const int32_t *labels, float *loss,
                        hipStream_t s) {
  gather_weights(a, s);
  hipLaunchKernelGGL(k_transpose_x, dim3(blocks_for((uint64_t)a.T * a.C * 64, 256)), dim3(256), 0, s, x,
                     a.xt, a.B, a.T, a.C);
  hipLaunchKernelGGL(k_input_current, dim3(blocks_for((uint64_t)a.T * a.H, 4)), dim3(256), 0, s, a);
  const dim3 grid(blocks_for(a.H, 4));
  float *vprev = nullptr;
  for (uint32_t t = 0; t < a.T; ++t) {
    // V of the step before each checkpoint segment is kept; the others rotate
    float *v_out = (t % a.K == a.K - 1 || t == a.T - 1) ? a.vck + (size_t)(t / a.K) * a.H * 64
                                                          : a.vtmp + (size_t)(t & 1u) * a.H * 64;
    const float *sprev = t ? a.s + (size_t)(t - 1) * a.H * 64 : nullptr;
    hipLaunchKernelGGL(k_hidden_step, grid, dim3(256), 0, s, a, t, vprev, sprev, v_out,
                       a.s + (size_t)t * a.H * 64);
    vprev = v_out;
  }
  hipLaunchKernelGGL(k_readout_drive, dim3(blocks_for((uint64_t)a.T * a.O * 64, 256)), dim3(256), 0, s, a,
                     a.ro);
  hipLaunchKernelGGL(k_readout_scan, dim3(a.O), dim3(64), 0, s, a, a.ro);
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, s, a, labels, loss);
  return hipGetLastError();
}

hipError_t bptt_backward(const BpttArgs &a, const float *g_loss, rocblas_handle blas, hipStream_t s) {
  if (rocblas_set_stream(blas, s) != rocblas_status_success) return hipErrorUnknown;
  gather_weights(a, s);
  hipLaunchKernelGGL(k_fill, dim3(blocks_for((uint64_t)a.H * 64, 256)), dim3(256), 0, s, a.lam_carry,
                     (uint64_t)a.H * 64, 0.0f);
  hipLaunchKernelGGL(k_lam_u, dim3(a.O), dim3(64), 0, s, a, g_loss);
  hipLaunchKernelGGL(k_grad_out, dim3(blocks_for((uint64_t)a.H * a.O, 4)), dim3(256), 0, s, a);
  const dim3 grid(blocks_for(a.H, 4));
  const uint32_t n_seg = (a.T + a.K - 1) / a.K;
  for (int32_t g = (int32_t)n_seg - 1; g >= 0; --g) {
    const uint32_t t0 = (uint32_t)g * a.K, len = std::min(a.K, a.T - t0);
    // recompute the segment's membranes from the checkpoint before it and the stored
    // spikes (the same kernel and operations as the forward pass)
    const float *vprev = g ? a.vck + (size_t)(g - 1) * a.H * 64 : nullptr;
    for (uint32_t k = 0; k < len; ++k) {
      const uint32_t t = t0 + k;
      float *v_out = a.vseg + (size_t)k * a.H * 64;
      const float *sprev = t ? a.s + (size_t)(t - 1) * a.H * 64 : nullptr;
      hipLaunchKernelGGL(k_hidden_step, grid, dim3(256), 0, s, a, t, vprev, sprev, v_out, (float *)nullptr);
      vprev = v_out;
    }
    for (int32_t k = (int32_t)len - 1; k >= 0; --k) {
      const float *lam_next = k + 1 < (int32_t)len ? a.lamv + (size_t)(k + 1) * a.H * 64 : a.lam_carry;
      hipLaunchKernelGGL(k_adjoint_step, grid, dim3(256), 0, s, a, t0 + (uint32_t)k,
                         a.vseg + (size_t)k * a.H * 64, lam_next, a.lamv + (size_t)k * a.H * 64);
    }
    // this segment's share of the sparse-weight gradients (two GEMMs over k = (t, b))
    const uint32_t kcols = a.K * 64, kk = len * 64;
    hipLaunchKernelGGL(k_seg_rows, dim3(blocks_for((uint64_t)a.H * len * 64, 256)), dim3(256), 0, s, a.lamv,
                       a.lseg, a.H, 0u, len, kcols, 0u);
    hipLaunchKernelGGL(k_seg_rows, dim3(blocks_for((uint64_t)a.C * len * 64, 256)), dim3(256), 0, s, a.xt,
                       a.xseg, a.C, t0, len, kcols, 0u);
    hipLaunchKernelGGL(k_seg_rows, dim3(blocks_for((uint64_t)a.H * len * 64, 256)), dim3(256), 0, s, a.s,
                       a.sseg, a.H, t0, len, kcols, 1u);
    const float one = 1.0f, beta = (uint32_t)g == n_seg - 1 ? 0.0f : 1.0f;
    rocblas_status bs = rocblas_sgemm(blas, rocblas_operation_transpose, rocblas_operation_none, (int)a.H,
                                      (int)a.C, (int)kk, &one, a.lseg, (int)kcols, a.xseg, (int)kcols, &beta,
                                      a.dw_in, (int)a.H);
    if (bs == rocblas_status_success)
      bs = rocblas_sgemm(blas, rocblas_operation_transpose, rocblas_operation_none, (int)a.H, (int)a.H,
                         (int)kk, &one, a.lseg, (int)kcols, a.sseg, (int)kcols, &beta, a.dw_rec, (int)a.H);
    if (bs != rocblas_status_success) return hipErrorUnknown;
    // lamV of the segment's first step is the next (earlier) segment's lamV_{t+1}
    (void)hipMemcpyAsync(a.lam_carry, a.lamv, (size_t)a.H * 64 * 4, hipMemcpyDeviceToDevice, s);
  }
  if (a.nnz_in)
    hipLaunchKernelGGL(k_mask_gather, grid, dim3(256), 0, s, a.in_t_ptr, a.in_t_src, a.in_t_edge, a.dw_in, a.H,
                       a.H, a.g_w_in);
  if (a.nnz_rec)
    hipLaunchKernelGGL(k_mask_gather, grid, dim3(256), 0, s, a.rec_t_ptr, a.rec_t_src, a.rec_t_edge, a.dw_rec,
                       a.H, a.H, a.g_w_rec);
  return hipGetLastError();
}

}  // namespace snn
