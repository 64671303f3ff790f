// runtime.cpp -- host runtime behind the C ABI of include/snn.h: validation, derived
// constants, device allocation, on-device network construction, the window schedule
// of the step pipeline, HIP graph replay, profiling and state/raster readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "snn_internal.h"

namespace {

thread_local std::string g_error;

struct Failure {
  snn_status code;
  std::string msg;
};

[[noreturn]] void fail(snn_status code, const std::string &msg) { throw Failure{code, msg}; }

void check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(SNN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void refuse_member(const snn_network *net) {
  if (net->owner) fail(SNN_E_STATE, "this network belongs to a batch: advance it with snn_batch_run");
}

template <typename F>
snn_status guarded(F &&f) {
  try {
    f();
    return SNN_OK;
  } catch (const Failure &x) {
    g_error = x.msg;
    return x.code;
  } catch (const std::bad_alloc &) {
    g_error = "host allocation failed";
    return SNN_E_OOM;
  } catch (const std::exception &x) {
    g_error = x.what();
    return SNN_E_INVALID;
  }
}

// ---- device memory --------------------------------------------------------------
// Without an allocator callback, device memory comes from the library's own cache
// (Sec. IV: memory is allocated only when necessary, with hysteresis, so back-to-back
// experiments pay for allocation once).  A freed block is kept per device; a request is
// served by the smallest kept block that is at least as large and at most twice as
// large (plus 1 MiB), else by hipMalloc.  When hipMalloc fails, the device's kept blocks
// are returned to HIP and the request is tried once more.  Blocks are handed back only
// after their network's stream has drained (every caller frees after a stream sync), so
// no work can still touch a reused block.
struct PoolBlock {
  int device;
  void *p;
  size_t bytes;
};
std::mutex g_pool_mutex;
std::vector<PoolBlock> g_pool;  // kept blocks
struct PoolStats {
  uint64_t hits = 0, misses = 0;
};
std::map<int, PoolStats> g_pool_stats;

// Returns the kept blocks of `device` (every device if negative) to HIP.
void pool_release(int device) {
  std::vector<PoolBlock> drop;
  {
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    std::vector<PoolBlock> keep;
    for (const PoolBlock &b : g_pool) (device < 0 || b.device == device ? drop : keep).push_back(b);
    g_pool.swap(keep);
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return;
  for (const PoolBlock &b : drop) {
    if (b.device != cur) (void)hipSetDevice(b.device);
    (void)hipFree(b.p);
    if (b.device != cur) (void)hipSetDevice(cur);
  }
}

// Serves `bytes` on `device`; *got receives the size of the block handed out (a kept
// block may be up to twice the request plus 1 MiB), which the caller records and hands
// back to pool_free, so a reused block keeps its true size.
void *pool_alloc(int device, size_t bytes, size_t *got) {
  *got = bytes;
  {
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    size_t best = g_pool.size();
    for (size_t k = 0; k < g_pool.size(); ++k) {
      const PoolBlock &b = g_pool[k];
      if (b.device != device || b.bytes < bytes || b.bytes > 2 * bytes + (1u << 20)) continue;
      if (best == g_pool.size() || b.bytes < g_pool[best].bytes) best = k;
    }
    if (best != g_pool.size()) {
      void *p = g_pool[best].p;
      *got = g_pool[best].bytes;
      g_pool.erase(g_pool.begin() + (std::ptrdiff_t)best);
      ++g_pool_stats[device].hits;
      return p;
    }
    ++g_pool_stats[device].misses;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) == hipSuccess) return p;
  (void)hipGetLastError();
  pool_release(device);
  if (hipMalloc(&p, bytes) == hipSuccess) return p;
  (void)hipGetLastError();
  return nullptr;
}

// Keeps a block for reuse; `bytes` is its true size (as pool_alloc reported it).
void pool_free(int device, void *p, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  g_pool.push_back({device, p, bytes});
}

void *dev_alloc(snn_network *net, size_t bytes) {
  if (bytes == 0) bytes = 16;
  bytes = (bytes + 255) & ~(size_t)255;
  void *p = nullptr;
  if (net->has_alloc) {
    p = net->alloc.alloc(bytes, (void *)net->stream, net->alloc.ctx);
    if (!p) fail(SNN_E_OOM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    size_t got = bytes;
    p = pool_alloc(net->device, bytes, &got);
    if (!p) fail(SNN_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    bytes = got;  // a reused block may be larger than the request: record what is held
  }
  net->allocs.push_back({p, bytes});
  net->device_bytes += bytes;
  return p;
}

template <typename T>
T *dev_array(snn_network *net, size_t count) {
  return static_cast<T *>(dev_alloc(net, count * sizeof(T)));
}

void release(snn_network *net) {
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  if (net->graph) (void)hipGraphExecDestroy(net->graph);
  for (auto &a : net->allocs) {
    if (net->has_alloc) net->alloc.free(a.p, a.bytes, (void *)net->stream, net->alloc.ctx);
    else pool_free(net->device, a.p, a.bytes);
  }
  net->allocs.clear();
  std::vector<hipEvent_t> pend;
  for (auto &r : net->prof_pending) {
    pend.push_back(r.a);
    pend.push_back(r.b);
  }
  std::sort(pend.begin(), pend.end());
  pend.erase(std::unique(pend.begin(), pend.end()), pend.end());
  for (hipEvent_t e : pend) (void)hipEventDestroy(e);
  net->prof_pending.clear();
  for (hipEvent_t e : net->event_pool) (void)hipEventDestroy(e);
  net->event_pool.clear();
  if (net->own_stream && net->stream) (void)hipStreamDestroy(net->stream);
}

// ---- definitions of the derived constants -----------------------------------------
int32_t q16(double w_mV, const char *what) {
  const double s = std::nearbyint(w_mV * 65536.0);
  if (!(s > -2147483648.0 && s < 2147483647.0)) fail(SNN_E_INVALID, std::string(what) + " out of Q16 range");
  return (int32_t)s;
}

// Inverse-CDF thresholds of Binomial(n, p): tbl[j] = floor(CDF(j) 2^32) until the
// first index past the mean whose probability is below 2^-40 (or n), which gets 2^32.
// pmf(0) = q^n by n multiplications; pmf(j) = pmf(j-1) (n-j+1) / j (p/q).
uint32_t binomial_thresholds(uint32_t n, double p, uint64_t *tbl, uint32_t cap) {
  const uint64_t kOne = 1ull << 32;
  if (n == 0 || p <= 0.0) {
    tbl[0] = kOne;
    return 1;
  }
  if (p >= 1.0) {
    if (n + 1 > cap) return 0;
    std::fill(tbl, tbl + n, 0ull);
    tbl[n] = kOne;
    return n + 1;
  }
  const double q = 1.0 - p, ratio = p / q, mean = (double)n * p;
  double pmf = 1.0;
  for (uint32_t j = 0; j < n; ++j) pmf *= q;
  if (!(pmf > 0.0)) return 0;
  double cdf = pmf;
  for (uint32_t j = 0;; ++j) {
    if (j + 1 > cap) return 0;
    if (j == n || ((double)j > mean && pmf < 0x1p-40)) {
      tbl[j] = kOne;
      return j + 1;
    }
    const double scaled = cdf * 4294967296.0;
    tbl[j] = scaled >= 4294967296.0 ? kOne : (uint64_t)scaled;
    pmf *= (double)(n - j);  // (n - (j+1) + 1)
    pmf /= (double)(j + 1);
    pmf *= ratio;
    cdf += pmf;
  }
}

void validate_and_derive(snn_network *net) {
  const snn_params &p = net->prm;
  if (!(p.dt_ms > 0.0)) fail(SNN_E_INVALID, "dt_ms must be > 0");
  if (p.delay_steps < 1) fail(SNN_E_INVALID, "delay_steps must be >= 1");
  if (p.synapse_weights > 1) fail(SNN_E_INVALID, "synapse_weights must be 0 (auto) or 1 (per synapse)");
  if (p.plasticity > SNN_PLASTICITY_LAZY) fail(SNN_E_INVALID, "plasticity must be SNN_PLASTICITY_EAGER or _LAZY");
  if (!(p.tau_m_ms > 0.0)) fail(SNN_E_INVALID, "tau_m_ms must be > 0");
  if (!(p.t_ref_ms >= 0.0)) fail(SNN_E_INVALID, "t_ref_ms must be >= 0");
  if (net->pops.empty()) fail(SNN_E_INVALID, "no populations");
  uint64_t n = 0;
  net->pop_off.assign(1, 0u);
  for (const auto &pop : net->pops) {
    if (pop.size == 0) fail(SNN_E_INVALID, "empty population");
    n += pop.size;
    if (n >= (1ull << 31)) fail(SNN_E_INVALID, "too many neurons (>= 2^31)");
    net->pop_off.push_back((uint32_t)n);
  }
  net->n = (uint32_t)n;
  const uint32_t n_pops = (uint32_t)net->pops.size();
  bool plastic = false;
  for (size_t q = 0; q < net->proj.size(); ++q) {
    const snn_projection &pj = net->proj[q];
    const uint32_t span = pj.to_span ? pj.to_span : 1u;
    if (pj.from >= n_pops || pj.to >= n_pops || span > n_pops - pj.to)
      fail(SNN_E_INVALID, "projection " + std::to_string(q) + ": bad population index");
    for (size_t r = 0; r < q; ++r) {
      const snn_projection &o = net->proj[r];
      const uint32_t os = o.to_span ? o.to_span : 1u;
      if (o.from == pj.from && o.to < pj.to + span && pj.to < o.to + os)
        fail(SNN_E_INVALID, "projections " + std::to_string(r) + " and " + std::to_string(q) +
                                " overlap (same source, overlapping targets)");
    }
    (void)q16(pj.w_mV, "weight");
    const uint64_t tsize = (uint64_t)net->pop_off[pj.to + span] - net->pop_off[pj.to];
    const bool self_in = pj.from >= pj.to && pj.from < pj.to + span;
    const uint64_t cand = tsize - (self_in ? 1u : 0u);
    if (pj.kind == SNN_PROJ_ER) {
      if (!(pj.p >= 0.0 && pj.p <= 1.0)) fail(SNN_E_INVALID, "ER probability outside [0, 1]");
    } else if (pj.kind == SNN_PROJ_FIXED_OUT) {
      if (pj.k > cand) fail(SNN_E_INVALID, "out-degree exceeds the number of candidate targets");
      const uint64_t spare = cand - pj.k;
      if (((uint64_t)pj.k + 1) * (2 * spare + 1) > (1ull << 35))
        fail(SNN_E_INVALID, "out-degree x target range too large for exact 64-bit spacing");
    } else {
      fail(SNN_E_INVALID, "unknown projection kind");
    }
    if (pj.plastic) {
      plastic = true;
      for (size_t r = 0; r < net->proj.size(); ++r)
        if (r != q && net->proj[r].plastic && net->proj[r].from == pj.from)
          fail(SNN_E_INVALID, "at most one plastic projection per source population");
    }
  }
  net->plastic = plastic;
  net->lazy = plastic && p.plasticity == SNN_PLASTICITY_LAZY;
  if (net->lazy && p.delay_steps > snn::kLazyHistory)
    fail(SNN_E_INVALID, "lazy plasticity needs delay_steps <= " + std::to_string(snn::kLazyHistory));
  net->delay = p.delay_steps;
  net->alpha = (float)std::exp(-p.dt_ms / p.tau_m_ms);
  net->v_inf = (float)(p.v_rest_mV + p.v_bg_mV);
  net->v_th = (float)p.v_th_mV;
  net->v_reset = (float)p.v_reset_mV;
  const double rs = std::nearbyint(p.t_ref_ms / p.dt_ms);
  if (rs > 1e9) fail(SNN_E_INVALID, "refractory period too long");
  net->ref_steps = (int32_t)rs;
  net->w_ext_q16 = q16(p.w_ext_mV, "w_ext");
  if (plastic) {
    if (!(p.tau_plus_ms > 0.0 && p.tau_minus_ms > 0.0)) fail(SNN_E_INVALID, "STDP time constants must be > 0");
    if (!(p.w_max_mV >= 0.0)) fail(SNN_E_INVALID, "w_max must be >= 0");
    net->beta_plus = (float)std::exp(-p.dt_ms / p.tau_plus_ms);
    net->beta_minus = (float)std::exp(-p.dt_ms / p.tau_minus_ms);
    net->a_plus = (float)p.a_plus;
    net->a_minus = (float)p.a_minus;
    net->w_max = (float)p.w_max_mV;
  }
  const double p_ext = (p.rate_ext_hz * p.dt_ms) / 1000.0;
  if (p.n_ext > 0 && !(p_ext >= 0.0 && p_ext <= 1.0)) fail(SNN_E_INVALID, "drive rate x dt outside [0, 1]");
  net->table_len = binomial_thresholds(p.n_ext, p_ext, net->table, snn::kTableCap);
  if (net->table_len == 0) fail(SNN_E_INVALID, "drive distribution needs more than 256 table entries");
  net->key0 = (uint32_t)p.seed;
  net->key1 = (uint32_t)(p.seed >> 32);
}

// ---- schedule: window, FIFO sizes, delivery variant --------------------------------
void choose_schedule(snn_network *net) {
  const snn_params &p = net->prm;
  if (net->plastic) {
    // Synapses change every step and delivery must see Syn_{t+1}: deliver S_{t-d+1}
    // at step t into a single accumulator (the paper's schedule).
    net->window = 1;
    net->n_inbuf = 1;
    // lazy plasticity delivers inside its own kernel (the atomic kernel serves only
    // delivery timing); eager plasticity takes either delivery, one step per launch
    if (net->lazy && p.delivery == SNN_DELIVERY_TILED)
      fail(SNN_E_INVALID, "lazy plasticity delivers inside its own kernel; tiled delivery needs eager plasticity");
    net->delivery = net->lazy ? SNN_DELIVERY_ATOMIC : p.delivery;
  } else {
    // Static weights: a spike of step e may be delivered any time between the updates
    // of e and e + d; one accumulator per pending arrival step lets a window of up to
    // d updates run in one launch, followed by one delivery launch for its queues.
    net->n_inbuf = net->delay;
    net->window = p.window ? std::min(p.window, net->delay) : net->delay;
    net->window = std::min(net->window, 64u);  // one ballot per lane of the update wave
    net->delivery = p.delivery;
  }
  net->raster_cap = p.raster_steps ? p.raster_steps : 1024u;
  // eager STDP reads the spike bits of step t - d from the raster ring
  if (net->plastic) net->raster_cap = std::max(net->raster_cap, net->delay + 1);
  net->window = std::min(net->window, net->raster_cap);  // kernels step rings by one wrap
  net->slots = std::max(net->delay + 2, 2 * net->window);
  net->words = (net->n + 63) / 64;
}

void choose_delivery(snn_network *net) {
  if (net->delivery == SNN_DELIVERY_AUTO) {
    const double deg = net->n ? (double)net->nnz / net->n : 0.0;
    net->delivery = (net->n >= 16384 && deg >= 64.0) ? SNN_DELIVERY_TILED : SNN_DELIVERY_ATOMIC;
  }
  if (net->delivery == SNN_DELIVERY_TILED) {
    const uint32_t b = net->prm.block;
    if (b != 0 && b != 256 && b != 512 && b != 1024) fail(SNN_E_INVALID, "block must be 256, 512 or 1024");
    net->block = b ? b : 1024;
    // A workgroup accumulates a range of up to kTileGroupMax base tiles in LDS.  The
    // largest base tile is set by the workgroup LDS limit (160 KB on gfx950, less the
    // kernel's static arrays); the default base tile is kDefaultTile targets, so that a
    // range holds up to 18,432 targets (the fastest range size of the launch-shape sweep
    // on the 1e9-synapse network, with 1,024-thread workgroups and one per CU).  Small
    // base tiles let the schedule size ranges in steps of 1/32 of that.
    size_t lds_dyn = 0;
    check(snn::prepare_deliver_tiled(net->block, &lds_dyn), "tiled delivery LDS limit");
    // a range's accumulators fit the LDS, and the delivery reads 16-bit targets, which
    // identify a target only inside a range of fewer than 65,536 targets
    const uint64_t range_cap = std::min<uint64_t>(lds_dyn / 4, 65535);
    constexpr uint32_t kDefaultTile = 576;
    const uint32_t tile_cap = (uint32_t)(range_cap / snn::kTileGroupMax);
    const uint32_t min_tiles = net->n <= range_cap ? 1u : (net->n + tile_cap - 1) / tile_cap;
    uint32_t tiles = net->prm.tiles ? net->prm.tiles : (net->n + kDefaultTile - 1) / kDefaultTile;
    tiles = std::max(std::min(tiles, std::max(1u, net->n / 16u)), min_tiles);
    // a multiple of 4 targets, so that ranges start on 16-byte boundaries of a row of
    // accumulators (the range flush then stores 16 bytes at a time)
    net->tile_size = ((net->n + tiles - 1) / tiles + 3) & ~3u;
    net->tiles = (net->n + net->tile_size - 1) / net->tile_size;
    if ((uint64_t)std::min(net->tiles, snn::kTileGroupMax) * net->tile_size > range_cap)
      fail(SNN_E_INVALID, "tile range too large for LDS or for 16-bit targets");
    // one 1,024-thread workgroup per CU (the kernel's registers allow one resident)
    net->grid = net->prm.grid ? net->prm.grid : net->cu_count * (net->block == 1024 ? 1u : 2u);
  } else if (net->delivery == SNN_DELIVERY_ATOMIC) {
    net->tiles = 1;
    net->tile_size = net->n;
  } else {
    fail(SNN_E_INVALID, "unknown delivery variant");
  }
}

// ---- construction ----------------------------------------------------------------
hipEvent_t new_event() {
  hipEvent_t e;
  // timing markers only: no system-scope fence when the event is recorded, so that a
  // marker between two launches costs as little as possible
  check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
  return e;
}

// Indexes of the tiled delivery: the tile boundaries of every row (uint16 when no row can
// reach 65,536 synapses, else uint32) and the 16-bit copy of the targets it streams.
void alloc_tile_offsets(snn_network *net) {
  const uint64_t count = ((net->nnz + 7) & ~7ull) + 8;  // whole 16-byte groups, one spare
  if (!net->col16) net->col16 = dev_array<uint16_t>(net, count);
  net->tile_off16 = net->row_len_bound < 65536;
  const size_t entries = (size_t)net->n * (net->tiles + 1);
  if (net->tile_off16) net->tile_off = dev_array<uint16_t>(net, entries);
  else net->tile_off = dev_array<uint32_t>(net, entries);
  check(snn::launch_tile_index(net->row_ptr, net->col, net->n, net->nnz, count, net->tiles, net->tile_size,
                               net->col16, net->tile_off, net->tile_off16, net->stream),
        "tile index");
}

void build(snn_network *net) {
  validate_and_derive(net);
  choose_schedule(net);
  hipStream_t s = net->stream;
  const uint32_t n = net->n, n_pops = (uint32_t)net->pops.size();

  // projections grouped by source population, sorted by first target population
  std::vector<snn::GenProj> gp;
  std::vector<uint32_t> pop_proj(n_pops + 1, 0);
  for (uint32_t a = 0; a < n_pops; ++a) {
    std::vector<const snn_projection *> mine;
    for (const auto &pj : net->proj)
      if (pj.from == a) mine.push_back(&pj);
    std::sort(mine.begin(), mine.end(), [](auto *x, auto *y) { return x->to < y->to; });
    pop_proj[a] = (uint32_t)gp.size();
    for (const snn_projection *pj : mine) {
      const uint32_t span = pj->to_span ? pj->to_span : 1u;
      snn::GenProj g{};
      g.kind = pj->kind;
      g.k = pj->k;
      g.first_pop = pj->to;
      g.off = net->pop_off[pj->to];
      g.size = net->pop_off[pj->to + span] - g.off;
      g.self_in = (a >= pj->to && a < pj->to + span) ? 1u : 0u;
      g.plastic = pj->plastic ? 1u : 0u;
      g.w_q16 = q16(pj->w_mV, "weight");
      g.w_f32 = (float)pj->w_mV;
      g.thr = pj->p >= 1.0 ? (1ull << 32) : (uint64_t)(pj->p * 4294967296.0);
      g.spare = pj->kind == SNN_PROJ_FIXED_OUT ? (uint64_t)(g.size - g.self_in - pj->k) : 0;
      gp.push_back(g);
    }
  }
  pop_proj[n_pops] = (uint32_t)gp.size();
  // longest possible row: a source's fixed out-degrees plus the sizes of the target
  // ranges of its ER projections
  net->row_len_bound = 0;
  for (uint32_t a = 0; a < n_pops; ++a) {
    uint64_t b = 0;
    for (uint32_t q = pop_proj[a]; q < pop_proj[a + 1]; ++q)
      b += gp[q].kind == SNN_PROJ_FIXED_OUT ? gp[q].k : gp[q].size;
    net->row_len_bound = std::max(net->row_len_bound, b);
  }

  snn::GenProj *d_proj = dev_array<snn::GenProj>(net, std::max<size_t>(gp.size(), 1));
  uint32_t *d_pop_off = dev_array<uint32_t>(net, n_pops + 1);
  uint32_t *d_pop_proj = dev_array<uint32_t>(net, n_pops + 1);
  if (!gp.empty())
    check(hipMemcpyAsync(d_proj, gp.data(), gp.size() * sizeof(snn::GenProj), hipMemcpyHostToDevice, s), "copy projections");
  check(hipMemcpyAsync(d_pop_off, net->pop_off.data(), (n_pops + 1) * 4, hipMemcpyHostToDevice, s), "copy offsets");
  check(hipMemcpyAsync(d_pop_proj, pop_proj.data(), (n_pops + 1) * 4, hipMemcpyHostToDevice, s), "copy ranges");
  snn::GenArgs g{d_proj, d_pop_off, d_pop_proj, n_pops, n, net->key0, net->key1};

  // row lengths -> row pointers -> rows
  uint32_t *len = dev_array<uint32_t>(net, n);
  if (net->plastic) {
    net->plast_rel = dev_array<uint32_t>(net, n);
    net->plast_len = dev_array<uint32_t>(net, n);
  }
  // setup timing: HIP events on the build stream around the generation phases
  hipEvent_t ev[6];
  for (hipEvent_t &e : ev) e = new_event();
  struct EventGuard {
    hipEvent_t *e;
    ~EventGuard() {
      for (int k = 0; k < 6; ++k) (void)hipEventDestroy(e[k]);
    }
  } ev_guard{ev};
  check(hipEventRecord(ev[0], s), "hipEventRecord");
  check(snn::launch_row_lengths(g, len, net->plast_rel, net->plast_len, s), "row lengths");
  net->row_ptr = dev_array<uint64_t>(net, (size_t)n + 1);
  uint64_t *scan_tmp = dev_array<uint64_t>(net, snn::scan_scratch_elems(n));
  check(snn::launch_scan_u32_to_u64(len, net->row_ptr, n, scan_tmp, s), "row scan");
  check(hipEventRecord(ev[1], s), "hipEventRecord");
  check(hipMemcpyAsync(&net->nnz, net->row_ptr + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s), "read nnz");
  check(hipStreamSynchronize(s), "sync after row scan");
  if (net->plastic && net->nnz >= (1ull << 32)) fail(SNN_E_INVALID, "plastic networks are limited to 2^32 synapses");
  net->nnz_alloc = ((net->nnz + 3) & ~3ull) + 4;  // 16-byte groups of the atomic delivery
  net->col = dev_array<int32_t>(net, net->nnz_alloc);
  // the fill writes every synapse: only the padding past the last one is cleared here
  const size_t pad_bytes = (net->nnz_alloc - net->nnz) * 4;
  check(hipMemsetAsync(net->col + net->nnz, 0, pad_bytes, s), "clear col padding");
  // Table I layout: when every projection from a source population carries the same
  // weight, a synapse stores only its target and the weight is the source's
  bool src_uniform = !net->plastic && net->prm.synapse_weights == 0;
  std::vector<int32_t> pop_w(n_pops, 0);
  for (uint32_t a = 0; a < n_pops && src_uniform; ++a) {
    bool seen = false;
    for (uint32_t q = pop_proj[a]; q < pop_proj[a + 1]; ++q) {
      if (seen && gp[q].w_q16 != pop_w[a]) src_uniform = false;
      pop_w[a] = gp[q].w_q16;
      seen = true;
    }
  }
  if (net->plastic) {
    net->w_f32 = dev_array<float>(net, net->nnz_alloc);
    check(hipMemsetAsync(net->w_f32 + net->nnz, 0, pad_bytes, s), "clear w padding");
  } else if (src_uniform) {
    net->w_src_host.assign(n, 0);
    for (uint32_t a = 0; a < n_pops; ++a)
      std::fill(net->w_src_host.begin() + net->pop_off[a], net->w_src_host.begin() + net->pop_off[a + 1], pop_w[a]);
    net->w_src = dev_array<int32_t>(net, n);
    check(hipMemcpyAsync(net->w_src, net->w_src_host.data(), (size_t)n * 4, hipMemcpyHostToDevice, s),
          "copy source weights");
  } else {
    net->w_q16 = dev_array<int32_t>(net, net->nnz_alloc);
    check(hipMemsetAsync(net->w_q16 + net->nnz, 0, pad_bytes, s), "clear w padding");
  }
  uint32_t max_fixed_k = 0;
  bool all_fixed = true;
  for (const snn::GenProj &q : gp) {
    if (q.kind == SNN_PROJ_FIXED_OUT) max_fixed_k = std::max(max_fixed_k, q.k);
    else all_fixed = false;
  }
  check(hipEventRecord(ev[2], s), "hipEventRecord");
  check(snn::launch_fill_rows(g, max_fixed_k, all_fixed, net->row_ptr, net->col, net->w_q16, net->w_f32, s),
        "fill rows");
  check(hipEventRecord(ev[3], s), "hipEventRecord");
  check(hipEventRecord(ev[4], s), "hipEventRecord");

  if (net->plastic) {
    // plastic in-edges grouped by target: counting sort by target
    uint32_t *cnt = dev_array<uint32_t>(net, n);
    check(hipMemsetAsync(cnt, 0, (size_t)n * 4, s), "clear in-degree");
    check(snn::launch_count_in_edges(net->row_ptr, net->col, net->plast_rel, net->plast_len, n, cnt, s), "count in-edges");
    net->in_ptr = dev_array<uint64_t>(net, (size_t)n + 1);
    check(snn::launch_scan_u32_to_u64(cnt, net->in_ptr, n, scan_tmp, s), "in-edge scan");
    uint64_t n_in = 0;
    check(hipMemcpyAsync(&n_in, net->in_ptr + n, 8, hipMemcpyDeviceToHost, s), "read plastic count");
    check(hipStreamSynchronize(s), "sync");
    net->in_src = dev_array<int32_t>(net, std::max<uint64_t>(n_in, 1));
    net->in_edge = dev_array<uint32_t>(net, std::max<uint64_t>(n_in, 1));
    uint64_t *cursor = dev_array<uint64_t>(net, n);
    check(hipMemcpyAsync(cursor, net->in_ptr, (size_t)n * 8, hipMemcpyDeviceToDevice, s), "cursor");
    check(snn::launch_fill_in_edges(net->row_ptr, net->col, net->plast_rel, net->plast_len, n, cursor,
                                    net->in_src, net->in_edge, s), "fill in-edges");
  }

  choose_delivery(net);
  if (net->delivery == SNN_DELIVERY_TILED) alloc_tile_offsets(net);
  check(hipEventRecord(ev[5], s), "hipEventRecord");

  // neuron state, FIFO, raster, control block
  net->v = dev_array<float>(net, n);
  net->ref = dev_array<int32_t>(net, n);
  net->input = dev_array<int32_t>(net, (size_t)net->n_inbuf * n);
  net->x_pre = dev_array<float>(net, n);
  net->x_post = dev_array<float>(net, n);
  // spike queues: kQueueGroups sub-queues per slot, sub-queue g collecting the spikes
  // of update workgroups b with b % kQueueGroups == g
  const uint32_t upd_blocks = (n + snn::kUpdateBlock - 1) / snn::kUpdateBlock;
  net->group_cap = ((upd_blocks + snn::kQueueGroups - 1) / snn::kQueueGroups) * snn::kUpdateBlock;
  net->queue_stride = snn::kQueueGroups * net->group_cap;
  net->queue = dev_array<int32_t>(net, (size_t)net->slots * net->queue_stride);
  net->qlen = dev_array<uint32_t>(net, (size_t)net->slots * snn::kQueueGroups * snn::kQlenStride);
  net->raster = dev_array<uint64_t>(net, (size_t)net->raster_cap * net->words);
  net->d_table32 = dev_array<uint32_t>(net, snn::kTableCap);
  net->d_guide = dev_array<uint16_t>(net, snn::kGuideBuckets);
  net->ctl = dev_array<snn::Ctl>(net, 1);
  check(hipMemsetAsync(net->input, 0, (size_t)net->n_inbuf * n * 4, s), "clear input");
  check(hipMemsetAsync(net->x_pre, 0, (size_t)n * 4, s), "clear traces");
  check(hipMemsetAsync(net->x_post, 0, (size_t)n * 4, s), "clear traces");
  check(hipMemsetAsync(net->qlen, 0, (size_t)net->slots * snn::kQueueGroups * snn::kQlenStride * 4, s),
        "clear queues");
  check(hipMemsetAsync(net->raster, 0, (size_t)net->raster_cap * net->words * 8, s), "clear raster");
  check(hipMemsetAsync(net->ctl, 0, sizeof(snn::Ctl), s), "clear control");
  if (net->lazy) {
    // Rows start with nothing pending and ages spread over the history, so that as many
    // rows expire at every step: row i's first pending step is -(i mod 64), before which
    // no event exists (empty histories, zero traces).
    net->hist = dev_array<uint64_t>(net, n);
    net->age = dev_array<uint32_t>(net, n);
    net->x_age = dev_array<float>(net, n);
    net->exq = dev_array<int32_t>(net, 2 * (size_t)net->queue_stride);
    net->exq_len = dev_array<uint32_t>(net, 2 * (size_t)snn::kQueueGroups * snn::kQlenStride);
    check(hipMemsetAsync(net->hist, 0, (size_t)n * 8, s), "clear spike history");
    check(hipMemsetAsync(net->x_age, 0, (size_t)n * 4, s), "clear traces at age");
    check(hipMemsetAsync(net->exq_len, 0, 2 * (size_t)snn::kQueueGroups * snn::kQlenStride * 4, s),
          "clear expiring rows");
    std::vector<uint32_t> age0(n);
    for (uint32_t i = 0; i < n; ++i) age0[i] = 0u - (i % snn::kLazyHistory);
    check(hipMemcpyAsync(net->age, age0.data(), (size_t)n * 4, hipMemcpyHostToDevice, s), "row ages");
    check(hipStreamSynchronize(s), "sync");
  }
  // the drive table as the kernels search it: thresholds below 2^32 as 32-bit words, and
  // a guide table giving #{j : tbl[j] <= r} at both ends of each bucket of r's top bits
  {
    std::vector<uint32_t> t32(snn::kTableCap, 0u);
    uint32_t below = 0;
    while (below < net->table_len && net->table[below] < (1ull << 32)) {
      t32[below] = (uint32_t)net->table[below];
      ++below;
    }
    std::vector<uint16_t> guide(snn::kGuideBuckets);
    const uint32_t shift = 32 - snn::kGuideBits;
    for (uint32_t b = 0; b < snn::kGuideBuckets; ++b) {
      const uint64_t r_lo = (uint64_t)b << shift, r_hi = r_lo + ((1ull << shift) - 1);
      uint32_t lo = 0, hi = 0;
      for (uint32_t j = 0; j < below; ++j) {
        lo += t32[j] <= r_lo ? 1u : 0u;
        hi += t32[j] <= r_hi ? 1u : 0u;
      }
      guide[b] = (uint16_t)(lo | (hi << 8));
    }
    check(hipMemcpyAsync(net->d_table32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, s), "copy table");
    check(hipMemcpyAsync(net->d_guide, guide.data(), guide.size() * 2, hipMemcpyHostToDevice, s), "copy guide");
    check(hipStreamSynchronize(s), "sync tables");
  }
  const float lo = (float)net->prm.v0_lo_mV;
  const float span = (float)(net->prm.v0_hi_mV - net->prm.v0_lo_mV);
  check(snn::launch_init_neurons(net->v, net->ref, n, net->key0, net->key1, lo, span, s), "init neurons");
  check(hipStreamSynchronize(s), "sync after build");
  check(hipEventElapsedTime(&net->gen_rows_ms, ev[0], ev[1]), "hipEventElapsedTime");
  check(hipEventElapsedTime(&net->gen_fill_ms, ev[2], ev[3]), "hipEventElapsedTime");
  check(hipEventElapsedTime(&net->index_ms, ev[4], ev[5]), "hipEventElapsedTime");
}

// ---- the step pipeline --------------------------------------------------------------
snn::QueueRef queue_ref(snn_network *net) {
  return snn::QueueRef{net->queue, net->qlen, net->queue_stride, net->group_cap};
}

snn::LazyRef lazy_ref(snn_network *net) {
  snn::LazyRef r{};
  r.hist = net->hist;
  r.age = net->age;
  r.x_age = net->x_age;
  r.plast_len = net->plast_len;
  r.exq = snn::QueueRef{net->exq, net->exq_len, net->queue_stride, net->group_cap};
  r.delay = net->delay;
  return r;
}

snn::UpdateArgs update_args(snn_network *net) {
  snn::UpdateArgs a{};
  a.v = net->v;
  a.ref = net->ref;
  a.input = net->input;
  a.x_pre = net->x_pre;
  a.x_post = net->x_post;
  a.q = queue_ref(net);
  a.raster = net->raster;
  a.table32 = net->d_table32;
  a.guide = net->d_guide;
  a.ctl = net->ctl;
  a.n = net->n;
  a.slots = net->slots;
  a.n_inbuf = net->n_inbuf;
  a.raster_cap = net->raster_cap;
  a.words = net->words;
  a.table_len = net->table_len;
  a.key0 = net->key0;
  a.key1 = net->key1;
  a.alpha = net->alpha;
  a.v_inf = net->v_inf;
  a.v_th = net->v_th;
  a.v_reset = net->v_reset;
  a.beta_plus = net->beta_plus;
  a.beta_minus = net->beta_minus;
  a.ref_steps = net->ref_steps;
  a.w_ext_q16 = net->w_ext_q16;
  // the tiled delivery overwrites every accumulator it owns; the atomic one adds
  a.zero_input = net->delivery == SNN_DELIVERY_ATOMIC ? 1u : 0u;
  a.plastic = net->plastic ? 1u : 0u;
  if (net->lazy) a.lazy = lazy_ref(net);
  return a;
}

snn::DeliverArgs deliver_args(snn_network *net) {
  snn::DeliverArgs a{};
  a.row_ptr = net->row_ptr;
  a.col = net->col;
  a.w_q16 = net->w_q16;
  a.w_f32 = net->w_f32;
  a.w_src = net->w_src;
  a.q = queue_ref(net);
  a.input = net->input;
  a.col16 = net->col16;
  a.tile_off = net->tile_off;
  a.ctl = net->ctl;
  a.n = net->n;
  a.slots = net->slots;
  a.n_inbuf = net->n_inbuf;
  a.delay = net->delay;
  a.window_max = net->window;
  a.tiles = net->tiles;
  a.tile_size = net->tile_size;
  a.off16 = net->tile_off16 ? 1u : 0u;
  a.advance = 1;
  return a;
}

snn::StdpArgs stdp_args(snn_network *net) {
  snn::StdpArgs a{};
  a.row_ptr = net->row_ptr;
  a.col = net->col;
  a.w_f32 = net->w_f32;
  a.plast_rel = net->plast_rel;
  a.plast_len = net->plast_len;
  a.in_ptr = net->in_ptr;
  a.in_src = net->in_src;
  a.in_edge = net->in_edge;
  a.x_pre = net->x_pre;
  a.x_post = net->x_post;
  a.q = queue_ref(net);
  a.ctl = net->ctl;
  a.raster = net->raster;
  a.raster_cap = net->raster_cap;
  a.words = net->words;
  a.n = net->n;
  a.slots = net->slots;
  a.delay = net->delay;
  a.a_plus = net->a_plus;
  a.a_minus = net->a_minus;
  a.w_max = net->w_max;
  return a;
}

snn::LazyArgs lazy_args(snn_network *net) {
  snn::LazyArgs a{};
  a.row_ptr = net->row_ptr;
  a.col = net->col;
  a.w_f32 = net->w_f32;
  a.plast_rel = net->plast_rel;
  a.x_pre = net->x_pre;
  a.x_post = net->x_post;
  a.q = queue_ref(net);
  a.input = net->input;
  a.lazy = lazy_ref(net);
  a.ctl = net->ctl;
  a.n = net->n;
  a.slots = net->slots;
  a.delay = net->delay;
  a.a_plus = net->a_plus;
  a.w_max = net->w_max;
  a.beta_plus = net->beta_plus;
  return a;
}

uint32_t atomic_grid(const snn_network *net) { return net->cu_count * 8; }
uint32_t lazy_grid(const snn_network *net) { return net->cu_count * 4; }

// Lazy plasticity: brings every plastic row current at the step boundary (weights and
// the touch count then equal the eager form's), without changing what the simulation
// computes next.  Ordered on the network's stream.
void lazy_flush(snn_network *net) {
  if (!net->lazy) return;
  check(snn::launch_lazy_flush(lazy_args(net), net->t_host, lazy_grid(net), net->stream), "lazy flush");
}

hipError_t launch_delivery(snn_network *net, const snn::DeliverArgs &d, uint32_t steps,
                           const snn::LaunchEvents &ev = {}) {
  if (net->delivery == SNN_DELIVERY_TILED)
    return snn::launch_deliver_tiled(d, steps, net->block, net->grid, net->stream, ev);
  return snn::launch_deliver_atomic(d, steps, atomic_grid(net), net->stream, ev);
}

hipEvent_t pooled_event(snn_network *net) {
  if (net->event_pool.empty()) return new_event();
  hipEvent_t e = net->event_pool.back();
  net->event_pool.pop_back();
  return e;
}

// With profiling on, every launch gets its own pair of events, stamped by the dispatch
// itself with its begin and end (hipExtLaunchKernel): no marker packet is placed between
// launches, so the durations are the kernels' own and the stream runs as without them.
template <typename F>
void timed(snn_network *net, int kind, F &&launch) {
  if (!net->profiling) {
    check(launch(snn::LaunchEvents{}), "kernel launch");
    return;
  }
  snn::LaunchEvents ev;
  ev.start = pooled_event(net);
  ev.stop = pooled_event(net);
  check(launch(ev), "kernel launch");
  net->prof_pending.push_back(snn_network::ProfRecord{kind, ev.start, ev.stop});
}

void resolve_profile(snn_network *net) {
  auto &v = net->prof_pending;
  if (v.empty()) return;
  check(hipStreamSynchronize(net->stream), "sync");
  std::vector<hipEvent_t> done;
  for (auto &r : v) {
    float ms = 0.f;
    check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    if (r.kind == 0) {
      net->prof.update_ms += ms;
      net->prof.update_launches++;
    } else if (r.kind == 1) {
      net->prof.deliver_ms += ms;
      net->prof.deliver_launches++;
    } else {
      net->prof.stdp_ms += ms;
      net->prof.stdp_launches++;
    }
    done.push_back(r.a);
    done.push_back(r.b);
  }
  std::sort(done.begin(), done.end());
  done.erase(std::unique(done.begin(), done.end()), done.end());
  net->event_pool.insert(net->event_pool.end(), done.begin(), done.end());
  v.clear();
}

// One window of `steps` consecutive steps: update -> [STDP] -> delivery.
void issue_window(snn_network *net, uint32_t steps) {
  const snn::UpdateArgs u = update_args(net);
  timed(net, 0, [&](const snn::LaunchEvents &ev) { return snn::launch_update(u, steps, net->stream, ev); });
  if (net->lazy) {
    // depression over the arriving rows, then one launch for the transmitting rows
    // (pending potentiation, delivery) and the expiring rows
    const snn::StdpArgs sa = stdp_args(net);
    timed(net, 2, [&](const snn::LaunchEvents &ev) { return snn::launch_stdp_ltd(sa, net->cu_count * 4, net->stream, ev); });
    const snn::LazyArgs la = lazy_args(net);
    timed(net, 1, [&](const snn::LaunchEvents &ev) { return snn::launch_lazy(la, lazy_grid(net), net->stream, ev); });
    net->t_host += steps;
    return;
  }
  snn::DeliverArgs d = deliver_args(net);
  if (net->plastic) {
    // depression and potentiation in one pass; the delivery then adds the arrivals to
    // x_pre and S_t to x_post
    const snn::StdpArgs sa = stdp_args(net);
    timed(net, 2, [&](const snn::LaunchEvents &ev) { return snn::launch_stdp_fused(sa, net->cu_count * 4, net->stream, ev); });
    d.x_pre = net->x_pre;
    d.x_post = net->x_post;
  }
  timed(net, 1, [&](const snn::LaunchEvents &ev) { return launch_delivery(net, d, steps, ev); });
  net->t_host += steps;
}

void ensure_graph(snn_network *net) {
  if (net->graph) return;
  const uint32_t windows = std::max(1u, (64u + net->window - 1) / net->window);
  const uint32_t steps = windows * net->window;
  hipGraph_t g = nullptr;
  check(hipStreamBeginCapture(net->stream, hipStreamCaptureModeRelaxed), "begin capture");
  const uint64_t saved = net->t_host;
  try {
    for (uint32_t k = 0; k < windows; ++k) issue_window(net, net->window);
  } catch (...) {
    (void)hipStreamEndCapture(net->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    net->t_host = saved;
    throw;
  }
  net->t_host = saved;
  check(hipStreamEndCapture(net->stream, &g), "end capture");
  const hipError_t e = hipGraphInstantiate(&net->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  check(e, "graph instantiate");
  net->graph_steps = steps;
}

void run(snn_network *net, uint64_t n_steps) {
  while (n_steps > 0) {
    if (!net->profiling && n_steps >= 64 && net->stream) {
      ensure_graph(net);
      if (n_steps >= net->graph_steps) {
        check(hipGraphLaunch(net->graph, net->stream), "graph launch");
        net->t_host += net->graph_steps;
        n_steps -= net->graph_steps;
        continue;
      }
    }
    const uint32_t steps = (uint32_t)std::min<uint64_t>(n_steps, net->window);
    issue_window(net, steps);
    n_steps -= steps;
  }
}

void sync(snn_network *net) {
  check(hipStreamSynchronize(net->stream), "stream sync");
}

struct CtlTotals {
  uint64_t t, events, spikes, touches, lazy_overrun;
};

CtlTotals sum_ctl(const snn::Ctl &c) {
  CtlTotals r{c.t, 0, 0, 0, c.lazy_overrun};
  for (uint32_t p = 0; p < snn::kCounterParts; ++p) {
    r.events += c.events[p * snn::kLineU64];
    r.spikes += c.spikes[p * snn::kLineU64];
    r.touches += c.touches[p * snn::kLineU64];
  }
  return r;
}

CtlTotals read_ctl(snn_network *net) {
  std::vector<snn::Ctl> c(1);
  check(hipMemcpyAsync(c.data(), net->ctl, sizeof(snn::Ctl), hipMemcpyDeviceToHost, net->stream), "read control");
  sync(net);
  return sum_ctl(c[0]);
}

void raster_range_check(snn_network *net, uint64_t t0, uint64_t t1) {
  if (t1 < t0) fail(SNN_E_INVALID, "t_end < t_begin");
  if (t1 > net->t_host) fail(SNN_E_INVALID, "raster range beyond the simulated steps");
  if (net->t_host - t0 > net->raster_cap) fail(SNN_E_INVALID, "raster range no longer held by the ring");
}

void copy_raster_rows(snn_network *net, uint64_t t0, uint64_t t1, uint64_t *out) {
  const size_t row = (size_t)net->words * 8;
  for (uint64_t t = t0; t < t1;) {
    const uint64_t r = t % net->raster_cap;
    const uint64_t run = std::min<uint64_t>(t1 - t, net->raster_cap - r);
    check(hipMemcpyAsync(out + (t - t0) * net->words, net->raster + r * net->words, run * row,
                         hipMemcpyDeviceToHost, net->stream), "raster copy");
    t += run;
  }
  sync(net);
}




// ---- delivery reconfiguration, timing and autotuning --------------------------------
void dev_free(snn_network *net, void *p) {
  for (size_t k = 0; k < net->allocs.size(); ++k)
    if (net->allocs[k].p == p) {
      if (net->has_alloc) net->alloc.free(p, net->allocs[k].bytes, (void *)net->stream, net->alloc.ctx);
      else pool_free(net->device, p, net->allocs[k].bytes);
      net->device_bytes -= net->allocs[k].bytes;
      net->allocs.erase(net->allocs.begin() + (std::ptrdiff_t)k);
      return;
    }
}

// A new delivery variant / tiling / launch shape, taking effect at the next window (the
// input ring holds exactly the pending arrivals at every window boundary, whichever
// variant filled it).  The new configuration is resolved and its tile index built before
// anything of the old one is released; if any of that fails (an impossible block or
// tiling, device memory, a launch), every field and buffer of the old configuration is
// restored, so the network keeps running as before.
void set_delivery(snn_network *net, uint32_t delivery, uint32_t tiles, uint32_t block, uint32_t grid) {
  if (net->lazy) fail(SNN_E_STATE, "lazy plasticity delivers inside its own kernel; there is no variant to choose");
  if (delivery > SNN_DELIVERY_TILED) fail(SNN_E_INVALID, "unknown delivery variant");
  check(hipStreamSynchronize(net->stream), "sync");
  struct Saved {
    uint32_t p_delivery, p_tiles, p_block, p_grid, delivery, block, tiles, tile_size, grid;
    void *tile_off;
    uint16_t *col16;
    bool tile_off16;
  };
  const Saved old{net->prm.delivery, net->prm.tiles, net->prm.block, net->prm.grid, net->delivery,
                  net->block,        net->tiles,     net->tile_size, net->grid,     net->tile_off,
                  net->col16,        net->tile_off16};
  try {
    net->prm.delivery = delivery;
    net->prm.tiles = tiles;
    net->prm.block = block;
    net->prm.grid = grid;
    net->delivery = delivery;
    choose_delivery(net);
    if (net->delivery == SNN_DELIVERY_TILED) {
      net->tile_off = nullptr;  // a fresh index; the old one stays valid until this succeeds
      alloc_tile_offsets(net);  // reuses col16 when it exists (it does not depend on the tiling)
      check(hipStreamSynchronize(net->stream), "sync after tile offsets");
    } else {
      net->tile_off = nullptr;
    }
  } catch (...) {
    (void)hipStreamSynchronize(net->stream);  // no index launch may still write a block freed here
    if (net->tile_off && net->tile_off != old.tile_off) dev_free(net, net->tile_off);
    if (net->col16 && net->col16 != old.col16) dev_free(net, net->col16);
    net->prm.delivery = old.p_delivery;
    net->prm.tiles = old.p_tiles;
    net->prm.block = old.p_block;
    net->prm.grid = old.p_grid;
    net->delivery = old.delivery;
    net->block = old.block;
    net->tiles = old.tiles;
    net->tile_size = old.tile_size;
    net->grid = old.grid;
    net->tile_off = old.tile_off;
    net->col16 = old.col16;
    net->tile_off16 = old.tile_off16;
    throw;
  }
  if (old.tile_off) dev_free(net, old.tile_off);
  if (net->col16 && net->delivery != SNN_DELIVERY_TILED) {
    dev_free(net, net->col16);
    net->col16 = nullptr;
  }
  if (net->graph) {
    (void)hipGraphExecDestroy(net->graph);
    net->graph = nullptr;
  }
}

// Mean time (ms) of one delivery launch over one window whose step w dequeues
// per_step[w], with scratch queues, accumulators and control block (the network's own
// state is untouched); *events = synaptic events of one launch.
double time_delivery(snn_network *net, const std::vector<std::vector<uint32_t>> &per_step, uint32_t reps,
                     uint64_t *events) {
  const uint32_t steps = (uint32_t)per_step.size();
  if (steps == 0 || steps > net->window) fail(SNN_E_INVALID, "steps exceeds the network's window");
  if (reps == 0) reps = 1;
  hipStream_t s = net->stream;
  // queue slots 0..steps-1, laid out as the update kernel appends: position p of a step
  // goes to sub-queue p mod kQueueGroups at index p / kQueueGroups
  std::vector<int32_t> queue((size_t)steps * net->queue_stride, 0);
  std::vector<uint32_t> qlen((size_t)net->slots * snn::kQueueGroups * snn::kQlenStride, 0u);
  for (uint32_t w = 0; w < steps; ++w) {
    if (per_step[w].size() > net->n) fail(SNN_E_INVALID, "more ids in a step than neurons");
    for (size_t p = 0; p < per_step[w].size(); ++p) {
      const uint32_t id = per_step[w][p];
      if (id >= net->n) fail(SNN_E_INVALID, "id out of range");
      const uint32_t g = (uint32_t)(p % snn::kQueueGroups), pos = (uint32_t)(p / snn::kQueueGroups);
      queue[(size_t)w * net->queue_stride + (size_t)g * net->group_cap + pos] = (int32_t)id;
      qlen[((size_t)w * snn::kQueueGroups + g) * snn::kQlenStride]++;
    }
  }
  std::vector<snn_network::Alloc> mark(net->allocs);
  const uint64_t bytes_before = net->device_bytes;
  double ms_out = 0.0;
  try {
    int32_t *d_queue = dev_array<int32_t>(net, (size_t)net->slots * net->queue_stride);
    uint32_t *d_qlen = dev_array<uint32_t>(net, qlen.size());
    int32_t *input = dev_array<int32_t>(net, (size_t)net->n_inbuf * net->n);
    snn::Ctl *ctl = dev_array<snn::Ctl>(net, 1);
    check(hipMemcpyAsync(d_queue, queue.data(), queue.size() * 4, hipMemcpyHostToDevice, s), "queue");
    check(hipMemcpyAsync(d_qlen, qlen.data(), qlen.size() * 4, hipMemcpyHostToDevice, s), "queue lengths");
    check(hipMemsetAsync(input, 0, (size_t)net->n_inbuf * net->n * 4, s), "clear");
    // slots 0..steps-1 are the queues delivered by a window starting at t0 when
    // t0 + n_inbuf - delay = 0 (mod slots)
    std::vector<snn::Ctl> c0(1);
    std::memset(c0.data(), 0, sizeof(snn::Ctl));
    c0[0].t_deliver = (uint64_t)net->delay - net->n_inbuf;
    check(hipMemcpyAsync(ctl, c0.data(), sizeof(snn::Ctl), hipMemcpyHostToDevice, s), "ctl");
    check(hipStreamSynchronize(s), "sync");
    snn::DeliverArgs d = deliver_args(net);
    d.q = snn::QueueRef{d_queue, d_qlen, net->queue_stride, net->group_cap};
    d.input = input;
    d.ctl = ctl;
    d.advance = 0;
    check(launch_delivery(net, d, steps), "warm-up delivery");
    // each launch stamped with its own begin and end (no marker packets between them)
    std::vector<snn::LaunchEvents> evs(reps);
    for (auto &e : evs) {
      e.start = pooled_event(net);
      e.stop = pooled_event(net);
    }
    for (uint32_t r = 0; r < reps; ++r) check(launch_delivery(net, d, steps, evs[r]), "delivery");
    check(hipStreamSynchronize(s), "sync");
    float ms = 0.f;
    for (auto &e : evs) {
      float one = 0.f;
      check(hipEventElapsedTime(&one, e.start, e.stop), "elapsed");
      ms += one;
      net->event_pool.push_back(e.start);
      net->event_pool.push_back(e.stop);
    }
    std::vector<snn::Ctl> c1(1);
    check(hipMemcpy(c1.data(), ctl, sizeof(snn::Ctl), hipMemcpyDeviceToHost), "ctl");
    ms_out = ms / reps;
    if (events) *events = sum_ctl(c1[0]).events / (reps + 1);
  } catch (...) {
    (void)hipStreamSynchronize(s);  // no launch may still use the scratch handed back below
    for (size_t k = mark.size(); k < net->allocs.size(); ++k) {
      if (net->has_alloc) net->alloc.free(net->allocs[k].p, net->allocs[k].bytes, (void *)s, net->alloc.ctx);
      else pool_free(net->device, net->allocs[k].p, net->allocs[k].bytes);
    }
    net->allocs.resize(mark.size());
    net->device_bytes = bytes_before;
    throw;
  }
  for (size_t k = mark.size(); k < net->allocs.size(); ++k) {
    if (net->has_alloc) net->alloc.free(net->allocs[k].p, net->allocs[k].bytes, (void *)s, net->alloc.ctx);
    else pool_free(net->device, net->allocs[k].p, net->allocs[k].bytes);
  }
  net->allocs.resize(mark.size());
  net->device_bytes = bytes_before;
  return ms_out;
}

// ---- delivery timing in a fixed device array (no allocation) ------------------------
// Scratch of snn_time_delivery_static: one window's staged queues and counters, the
// control block and the input accumulators the delivery writes.  Each GPU holds its
// own copy for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns for that device.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
struct StaticScratch {
  unsigned char *ptr = nullptr;            // device address of `scratch` on this device
  hipEvent_t start = nullptr, stop = nullptr;  // timing events, created with it
};
std::mutex g_static_mu;
StaticScratch g_static[kMaxDevices];

// Set-up on the first call on `device`, with that device current: the array's device
// address and the two timing events.  Later calls only read the table.
StaticScratch static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) fail(SNN_E_INVALID, "device id beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticScratch &s = g_static[device];
  if (s.ptr) return s;
  int cur = -1;
  check(hipGetDevice(&cur), "hipGetDevice");
  if (cur != device) check(hipSetDevice(device), "hipSetDevice");
  void *p = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    check(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch set-up");
  }
  s.start = a;
  s.stop = b;
  s.ptr = static_cast<unsigned char *>(p);
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// snn_time_delivery with every device buffer in the static scratch: the ids are checked
// on the host, copied into the scratch as they are, and laid out as the window's queues
// by k_stage_window; then one untimed and `reps` timed launches of the network's
// delivery kernel, the mean taken from the first timed launch's begin to the last one's
// end.
double time_delivery_static(snn_network *net, const uint32_t *ids, uint32_t n_ids, const uint32_t *step_counts,
                            uint32_t steps, uint32_t reps, uint64_t *events) {
  if (steps == 0 || steps > net->window) fail(SNN_E_INVALID, "steps exceeds the network's window");
  if (reps == 0) reps = 1;
  snn::StageArgs st{};
  st.steps = steps;
  st.n_ids = n_ids;
  st.round_robin = step_counts ? 0u : 1u;
  uint64_t k = 0;
  for (uint32_t w = 0; w < steps; ++w) {
    const uint64_t c = step_counts ? step_counts[w] : (n_ids > w ? (n_ids - w + steps - 1) / steps : 0u);
    if (c > net->n) fail(SNN_E_INVALID, "more ids in a step than neurons");
    st.off[w] = (uint32_t)k;
    k += c;
    if (k > n_ids) fail(SNN_E_INVALID, "step counts exceed the ids");
  }
  if (k != n_ids) fail(SNN_E_INVALID, "step counts do not sum to n_ids");
  st.off[steps] = (uint32_t)k;
  for (uint32_t j = 0; j < n_ids; ++j)
    if (ids[j] >= net->n) fail(SNN_E_INVALID, "id out of range");
  const size_t o_qlen = align256(sizeof(snn::Ctl));
  const size_t o_queue = o_qlen + align256((size_t)steps * snn::kQueueGroups * snn::kQlenStride * 4);
  const size_t o_input = o_queue + align256((size_t)steps * net->queue_stride * 4);
  const size_t o_ids = o_input + align256((size_t)net->n_inbuf * net->n * 4);
  const size_t need = o_ids + align256((size_t)n_ids * 4);
  if (need > kStaticScratchBytes)
    fail(SNN_E_INVALID, "this window needs " + std::to_string(need) + " bytes of device scratch; the static scratch holds " +
                            std::to_string(kStaticScratchBytes));
  const StaticScratch sc = static_scratch(net->device);
  hipStream_t s = net->stream;
  snn::Ctl *ctl = reinterpret_cast<snn::Ctl *>(sc.ptr);
  st.q = snn::QueueRef{reinterpret_cast<int32_t *>(sc.ptr + o_queue), reinterpret_cast<uint32_t *>(sc.ptr + o_qlen),
                       net->queue_stride, net->group_cap};
  st.ctl = ctl;
  st.input = reinterpret_cast<int32_t *>(sc.ptr + o_input);
  st.n_input = (uint64_t)net->n_inbuf * net->n;
  st.ids = reinterpret_cast<const int32_t *>(sc.ptr + o_ids);
  // slots 0..steps-1 are the queues delivered by a window starting at t0 when
  // t0 + n_inbuf - delay = 0 (mod slots)
  st.t_deliver = (uint64_t)net->delay - net->n_inbuf;
  if (n_ids)
    check(hipMemcpyAsync(sc.ptr + o_ids, ids, (size_t)n_ids * 4, hipMemcpyHostToDevice, s), "ids");
  check(snn::launch_stage_window(st, s), "stage window");
  snn::DeliverArgs d = deliver_args(net);
  d.q = st.q;
  d.input = st.input;
  d.ctl = ctl;
  d.advance = 0;
  check(launch_delivery(net, d, steps), "warm-up delivery");
  for (uint32_t r = 0; r < reps; ++r) {
    snn::LaunchEvents ev;
    if (r == 0) ev.start = sc.start;
    if (r + 1 == reps) ev.stop = sc.stop;
    check(launch_delivery(net, d, steps, ev), "delivery");
  }
  uint64_t parts[snn::kCounterParts];
  check(hipMemcpy2DAsync(parts, sizeof(uint64_t), ctl->events, snn::kLineU64 * sizeof(uint64_t), sizeof(uint64_t),
                         snn::kCounterParts, hipMemcpyDeviceToHost, s),
        "event counters");
  check(hipStreamSynchronize(s), "sync");
  float ms = 0.f;
  check(hipEventElapsedTime(&ms, sc.start, sc.stop), "elapsed");
  uint64_t total = 0;
  for (uint64_t x : parts) total += x;
  if (events) *events = total / (reps + 1);
  return (double)ms / reps;
}

// Times every candidate delivery configuration on the spikes of the latest window (read
// from the raster ring) and keeps the fastest.
snn_delivery_tuning autotune_delivery(snn_network *net, uint32_t reps) {
  if (net->lazy) fail(SNN_E_STATE, "lazy plasticity delivers inside its own kernel; there is no variant to tune");
  const uint32_t W = net->window;
  if (net->t_host < W) fail(SNN_E_STATE, "run at least one window before autotuning the delivery");
  if (net->raster_cap < W) fail(SNN_E_STATE, "the raster ring holds less than one window");
  sync(net);
  std::vector<uint64_t> rows((size_t)W * net->words);
  raster_range_check(net, net->t_host - W, net->t_host);
  copy_raster_rows(net, net->t_host - W, net->t_host, rows.data());
  std::vector<std::vector<uint32_t>> per_step(W);
  for (uint32_t w = 0; w < W; ++w)
    for (uint32_t k = 0; k < net->words; ++k) {
      uint64_t m = rows[(size_t)w * net->words + k];
      while (m) {
        const uint32_t b = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        per_step[w].push_back(k * 64 + b);
      }
    }
  struct Cand {
    uint32_t delivery, tiles, block, grid;
  };
  std::vector<Cand> cands;
  cands.push_back({SNN_DELIVERY_ATOMIC, 0, 0, 0});
  if (net->n >= 1024) {
    for (uint32_t tile : {384u, 576u, 768u})
      for (uint32_t block : {512u, 1024u})
        for (uint32_t grid : {net->cu_count, 2 * net->cu_count, 3 * net->cu_count})
          cands.push_back({SNN_DELIVERY_TILED, std::max(1u, (net->n + tile - 1) / tile), block, grid});
  }
  const Cand keep{net->delivery, net->prm.tiles, net->prm.block, net->prm.grid};
  snn_delivery_tuning best{};
  best.ms_per_launch = 1e300;
  for (const Cand &c : cands) {
    try {
      set_delivery(net, c.delivery, c.tiles, c.block, c.grid);
    } catch (const Failure &) {
      continue;  // e.g. a tile larger than the LDS allows
    }
    uint64_t ev = 0;
    const double ms = time_delivery(net, per_step, reps, &ev);
    if (ms < best.ms_per_launch) {
      best.ms_per_launch = ms;
      best.delivery = net->delivery;
      best.tiles = net->tiles;
      best.block = net->block;
      best.grid = net->grid;
      best.events_per_launch = ev;
    }
  }
  if (best.ms_per_launch == 1e300) {
    set_delivery(net, keep.delivery, keep.tiles, keep.block, keep.grid);
    fail(SNN_E_STATE, "no delivery configuration could be timed");
  }
  set_delivery(net, best.delivery, best.tiles, best.block, best.grid);
  return best;
}

// ---- batched form ----------------------------------------------------------------
}  // namespace

struct snn_batch {
  std::vector<snn_network *> nets;
  snn_network pool;                  // holds the batch's own allocations and stream
  std::vector<snn::BatchNet> desc;
  std::vector<double> degree;        // mean out-degree of each member
  std::vector<uint32_t> order;       // workgroup -> member, heaviest first
  snn::BatchNet *d_desc = nullptr;
  uint32_t *d_order = nullptr;
  uint32_t n_max = 0;
  size_t lds_need = 0;               // dynamic LDS of the largest member
  uint32_t lds_limit = 0;
  snn_batch_tuning tuning{};
  std::vector<std::pair<uint32_t, hipGraphExec_t>> graphs;  // by steps per launch
};

namespace {

uint32_t lanes_shift_for(double degree, uint32_t degree_div) {
  const double want = degree / (double)std::max(1u, degree_div);
  uint32_t sh = 0;
  while (sh < 6 && (double)(1u << sh) < want) ++sh;
  return sh;
}

void batch_clear_graphs(snn_batch *b) {
  for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

void batch_apply_tuning(snn_batch *b, const snn_batch_tuning &t) {
  if (t.block != 256 && t.block != 512 && t.block != 1024) fail(SNN_E_INVALID, "block must be 256, 512 or 1024");
  if (t.degree_div != 1 && t.degree_div != 2 && t.degree_div != 4 && t.degree_div != 8 && t.degree_div != 16)
    fail(SNN_E_INVALID, "degree_div must be 1, 2, 4, 8 or 16");
  const uint32_t per = snn::batch_per_lane(t.block, b->n_max);
  if (per == 0) fail(SNN_E_INVALID, "largest network does not fit a workgroup of this size");
  for (size_t k = 0; k < b->desc.size(); ++k) b->desc[k].lanes_shift = lanes_shift_for(b->degree[k], t.degree_div);
  check(hipMemcpyAsync(b->d_desc, b->desc.data(), b->desc.size() * sizeof(snn::BatchNet), hipMemcpyHostToDevice,
                       b->pool.stream), "copy batch descriptors");
  check(hipStreamSynchronize(b->pool.stream), "sync");
  b->tuning = t;
  b->tuning.per_lane = per;
  b->tuning.pad_ = 0;
  batch_clear_graphs(b);
}

void batch_launch(snn_batch *b, uint32_t steps, uint32_t flags) {
  for (const snn::BatchNet &d : b->desc)
    if (d.below) flags |= snn::kBatchDrive;
  check(snn::launch_batch(b->d_desc, b->d_order, (uint32_t)b->nets.size(), steps, b->tuning.block,
                          b->tuning.per_lane, flags, b->lds_need, b->pool.stream), "batch launch");
}

hipGraphExec_t batch_graph(snn_batch *b, uint32_t steps) {
  for (auto &g : b->graphs)
    if (g.first == steps) return g.second;
  hipGraph_t g = nullptr;
  hipStream_t s = b->pool.stream;
  check(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "begin capture");
  try {
    batch_launch(b, steps, snn::kBatchCommit | snn::kBatchWriteRaster);
  } catch (...) {
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  check(hipStreamEndCapture(s, &g), "end capture");
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  check(e, "graph instantiate");
  if (b->graphs.size() >= 8) batch_clear_graphs(b);
  b->graphs.push_back({steps, ex});
  return ex;
}

// Each launch advances every member by `chunk` steps; one kernel node per launch,
// replayed from a graph captured once per chunk length.
void batch_run(snn_batch *b, uint64_t n_steps) {
  constexpr uint32_t kMaxChunk = 1u << 14;
  while (n_steps > 0) {
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(n_steps, kMaxChunk);
    check(hipGraphLaunch(batch_graph(b, chunk), b->pool.stream), "graph launch");
    for (snn_network *m : b->nets) m->t_host += chunk;
    n_steps -= chunk;
  }
}

void batch_destroy(snn_batch *b) {
  if (b->pool.stream) (void)hipStreamSynchronize(b->pool.stream);
  batch_clear_graphs(b);
  for (snn_network *m : b->nets) {
    m->owner = nullptr;
    m->own_stream = false;  // the stream belongs to the pool
    release(m);
    delete m;
  }
  b->nets.clear();
  release(&b->pool);
}

void build_batch(snn_batch *b, const snn_batch_member *members, uint32_t n_nets, uint32_t raster_steps) {
  hipStream_t s = b->pool.stream;
  int lds_max = 0;
  check(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->pool.device),
        "LDS limit");
  b->lds_limit = (uint32_t)std::max(0, lds_max - 64);  // the kernel's static LDS
  for (uint32_t k = 0; k < n_nets; ++k) {
    const snn_batch_member &mb = members[k];
    if (!mb.params || (!mb.pops && mb.n_pops) || (!mb.proj && mb.n_proj))
      fail(SNN_E_INVALID, "member " + std::to_string(k) + ": null argument");
    snn_network *m = new snn_network();
    b->nets.push_back(m);
    m->owner = b;
    m->prm = *mb.params;
    m->prm.raster_steps = raster_steps;
    m->prm.window = 0;
    m->prm.delivery = SNN_DELIVERY_ATOMIC;
    m->prm.tiles = m->prm.block = m->prm.grid = 0;
    m->pops.assign(mb.pops, mb.pops + mb.n_pops);
    m->proj.assign(mb.proj, mb.proj + mb.n_proj);
    m->alloc = b->pool.alloc;
    m->has_alloc = b->pool.has_alloc;
    m->device = b->pool.device;
    m->cu_count = b->pool.cu_count;
    m->stream = s;
    try {
      build(m);
    } catch (const Failure &f) {
      fail(f.code, "member " + std::to_string(k) + ": " + f.msg);
    }
    if (m->plastic) fail(SNN_E_INVALID, "member " + std::to_string(k) + ": the batched form needs static weights");
    if (m->n_inbuf != m->delay) fail(SNN_E_INVALID, "member " + std::to_string(k) + ": unexpected input ring");
    uint32_t below = 0;
    while (below < m->table_len && m->table[below] < (1ull << 32)) ++below;
    const size_t lds = ((size_t)m->delay * m->n + below) * 4;
    if (m->n > 20480 || lds > b->lds_limit)
      fail(SNN_E_INVALID, "member " + std::to_string(k) + " does not fit one workgroup (n = " + std::to_string(m->n) +
                              ", delay ring + drive table = " + std::to_string(lds) + " bytes of LDS, limit " +
                              std::to_string(b->lds_limit) + ")");
    b->lds_need = std::max(b->lds_need, (lds + 15) & ~(size_t)15);
    b->n_max = std::max(b->n_max, m->n);
    snn::BatchNet d{};
    d.row_ptr = m->row_ptr;
    d.col = m->col;
    d.w_q16 = m->w_q16;
    d.w_src = m->w_src;
    d.v = m->v;
    d.ref = m->ref;
    d.input = m->input;
    d.queue = m->queue;
    d.raster = m->raster;
    d.table32 = m->d_table32;
    d.ctl = m->ctl;
    d.n = m->n;
    d.words = m->words;
    d.delay = m->delay;
    d.raster_cap = m->raster_cap;
    d.below = below;
    d.key0 = m->key0;
    d.key1 = m->key1;
    d.alpha = m->alpha;
    d.v_inf = m->v_inf;
    d.v_th = m->v_th;
    d.v_reset = m->v_reset;
    d.ref_steps = m->ref_steps;
    d.w_ext_q16 = m->w_ext_q16;
    b->desc.push_back(d);
    b->degree.push_back(m->n ? (double)m->nnz / m->n : 0.0);
  }
  // heaviest networks first: the first workgroups start first and get a CU each
  std::vector<double> work(n_nets);
  for (uint32_t k = 0; k < n_nets; ++k) work[k] = (double)b->nets[k]->nnz + 8.0 * b->nets[k]->n;
  b->order.resize(n_nets);
  std::iota(b->order.begin(), b->order.end(), 0u);
  std::stable_sort(b->order.begin(), b->order.end(), [&](uint32_t x, uint32_t y) { return work[x] > work[y]; });
  b->d_desc = dev_array<snn::BatchNet>(&b->pool, std::max<size_t>(1, n_nets));
  b->d_order = dev_array<uint32_t>(&b->pool, std::max<size_t>(1, n_nets));
  check(hipMemcpyAsync(b->d_order, b->order.data(), n_nets * 4, hipMemcpyHostToDevice, s), "copy order");
  snn_batch_tuning t{};
  t.degree_div = 4;
  t.block = 256;
  for (uint32_t blk : {512u, 1024u, 256u})
    if (snn::batch_per_lane(blk, b->n_max)) {
      t.block = blk;
      break;
    }
  batch_apply_tuning(b, t);
}

snn_batch_tuning batch_autotune(snn_batch *b, uint32_t trial_steps) {
  if (trial_steps == 0) fail(SNN_E_INVALID, "trial_steps must be positive");
  hipStream_t s = b->pool.stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  check(hipEventCreate(&e0), "event");
  check(hipEventCreate(&e1), "event");
  snn_batch_tuning best{};
  double best_ms = 1e300;
  try {
    for (uint32_t blk : {256u, 512u, 1024u}) {
      if (!snn::batch_per_lane(blk, b->n_max)) continue;
      for (uint32_t div : {1u, 2u, 4u, 8u, 16u}) {
        snn_batch_tuning t{};
        t.block = blk;
        t.degree_div = div;
        batch_apply_tuning(b, t);
        batch_launch(b, trial_steps, 0u);  // warm-up
        check(hipEventRecord(e0, s), "event record");
        batch_launch(b, trial_steps, 0u);
        check(hipEventRecord(e1, s), "event record");
        check(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (ms < best_ms) {
          best_ms = ms;
          best = b->tuning;
        }
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  batch_apply_tuning(b, best);
  b->tuning.ms_per_step = best_ms / trial_steps;
  return b->tuning;
}


// ---- surrogate-gradient BPTT plan ------------------------------------------------
}  // namespace

struct snn_bptt {
  snn_bptt_desc desc{};
  snn_network pool;          // holds the plan's allocations and default stream
  snn::BpttArgs args{};
  uint64_t forwards = 0;     // forward passes run (the backward uses the latest)
  hipGraphExec_t g_fwd = nullptr, g_bwd = nullptr;  // captured bodies of the two passes
};

namespace {

// Transposed index of a CSR matrix with `rows` rows and `cols` columns: for each
// column, its (row, edge) pairs in ascending row order (a counting sort over rows).
void transpose_csr(const uint64_t *ptr, const int32_t *col, uint32_t rows, uint32_t cols,
                   std::vector<uint64_t> &t_ptr, std::vector<int32_t> &t_src, std::vector<uint32_t> &t_edge) {
  const uint64_t nnz = ptr[rows];
  t_ptr.assign((size_t)cols + 1, 0);
  for (uint64_t e = 0; e < nnz; ++e) t_ptr[(size_t)col[e] + 1]++;
  for (uint32_t c = 0; c < cols; ++c) t_ptr[c + 1] += t_ptr[c];
  std::vector<uint64_t> fill(t_ptr.begin(), t_ptr.end() - 1);
  t_src.assign(nnz ? nnz : 1, 0);
  t_edge.assign(nnz ? nnz : 1, 0);
  for (uint32_t r = 0; r < rows; ++r)
    for (uint64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
      const uint64_t at = fill[(size_t)col[e]]++;
      t_src[at] = (int32_t)r;
      t_edge[at] = (uint32_t)e;
    }
}

void check_csr(const uint64_t *ptr, const int32_t *col, uint32_t rows, uint32_t cols, uint64_t nnz,
               const char *what) {
  if (!ptr || (!col && nnz)) fail(SNN_E_INVALID, std::string(what) + ": null CSR array");
  if (ptr[0] != 0 || ptr[rows] != nnz) fail(SNN_E_INVALID, std::string(what) + ": row pointers do not span nnz");
  if (nnz >= (1ull << 32)) fail(SNN_E_INVALID, std::string(what) + ": more than 2^32 - 1 synapses");
  for (uint32_t r = 0; r < rows; ++r) {
    if (ptr[r + 1] < ptr[r]) fail(SNN_E_INVALID, std::string(what) + ": decreasing row pointers");
    for (uint64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
      if (col[e] < 0 || (uint32_t)col[e] >= cols) fail(SNN_E_INVALID, std::string(what) + ": target out of range");
      if (e > ptr[r] && col[e] <= col[e - 1]) fail(SNN_E_INVALID, std::string(what) + ": row not strictly ascending");
    }
  }
}

template <typename T>
T *upload(snn_network *pool, const std::vector<T> &v) {
  T *d = dev_array<T>(pool, std::max<size_t>(1, v.size()));
  if (!v.empty())
    check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, pool->stream), "upload");
  return d;
}

void build_bptt(snn_bptt *p, const uint64_t *in_ptr, const int32_t *in_col, const uint64_t *rec_ptr,
                const int32_t *rec_col) {
  const snn_bptt_desc &d = p->desc;
  if (d.batch < 1 || d.batch > 64) fail(SNN_E_INVALID, "batch must be 1..64");
  if (d.steps < 1 || d.n_in < 1 || d.n_hidden < 1 || d.n_out < 1) fail(SNN_E_INVALID, "empty dimension");
  if (d.steps > 65535) fail(SNN_E_INVALID, "at most 65,535 steps");
  if (d.checkpoint < 1 || d.checkpoint > 32) fail(SNN_E_INVALID, "checkpoint interval must be 1..32");
  if (d.n_out > 1024) fail(SNN_E_INVALID, "at most 1024 readouts");
  if (!(d.slope > 0.f) || !(d.beta >= 0.f) || !(d.beta_out >= 0.f)) fail(SNN_E_INVALID, "invalid constants");
  const uint64_t nnz_in = in_ptr ? in_ptr[d.n_in] : 0, nnz_rec = rec_ptr ? rec_ptr[d.n_hidden] : 0;
  check_csr(in_ptr, in_col, d.n_in, d.n_hidden, nnz_in, "input weights");
  check_csr(rec_ptr, rec_col, d.n_hidden, d.n_hidden, nnz_rec, "recurrent weights");
  std::vector<uint64_t> it_ptr, rt_ptr;
  std::vector<int32_t> it_src, rt_src;
  std::vector<uint32_t> it_edge, rt_edge;
  transpose_csr(in_ptr, in_col, d.n_in, d.n_hidden, it_ptr, it_src, it_edge);
  transpose_csr(rec_ptr, rec_col, d.n_hidden, d.n_hidden, rt_ptr, rt_src, rt_edge);
  snn::BpttArgs &a = p->args;
  snn_network *pool = &p->pool;
  a.B = d.batch;
  a.T = d.steps;
  a.C = d.n_in;
  a.H = d.n_hidden;
  a.O = d.n_out;
  a.K = d.checkpoint;
  a.beta = d.beta;
  a.beta_out = d.beta_out;
  a.theta = d.theta;
  a.slope = d.slope;
  a.smooth = d.smooth ? 1u : 0u;
  a.detach_reset = d.smooth ? 0u : 1u;
  a.nnz_in = nnz_in;
  a.nnz_rec = nnz_rec;
  a.in_t_ptr = upload(pool, it_ptr);
  a.in_t_src = upload(pool, it_src);
  a.in_t_edge = upload(pool, it_edge);
  a.rec_t_ptr = upload(pool, rt_ptr);
  a.rec_t_src = upload(pool, rt_src);
  a.rec_t_edge = upload(pool, rt_edge);
  a.rec_ptr = upload(pool, std::vector<uint64_t>(rec_ptr, rec_ptr + d.n_hidden + 1));
  a.rec_col = upload(pool, std::vector<int32_t>(rec_col, rec_col + nnz_rec));
  const size_t HB = (size_t)a.H * 64, n_seg = (a.T + a.K - 1) / a.K;
  // 8 readable entries past the end, and for the spike masks 8 before the start: the
  // forward's input currents and the backward's segment currents read 8 steps of masks
  // per load, the latter from step t - 1 (whose values at t = 0 are not used)
  a.xbits = dev_array<uint64_t>(pool, (size_t)a.C * a.T + 8);
  a.sbits = dev_array<uint64_t>(pool, (size_t)a.H * a.T + 16) + 8;
  a.sbits_t = dev_array<uint64_t>(pool, (size_t)a.T * a.H);
  // ELL copy of the recurrent in-edges for the hidden steps (rows padded to a multiple of
  // 64, at most 256 wide, and at most 8,192 neurons, whose masks a workgroup stages)
  uint64_t max_deg = 0;
  for (uint32_t j = 0; j < a.H; ++j) max_deg = std::max<uint64_t>(max_deg, rt_ptr[j + 1] - rt_ptr[j]);
  a.ell_w = 0;
  if (nnz_rec && max_deg <= snn::kEllMaxWidth && a.H <= snn::kEllMaxNeurons) {
    const uint32_t wd = (uint32_t)((max_deg + 63) / 64 * 64);
    std::vector<int32_t> es((size_t)a.H * wd, 0);
    std::vector<uint32_t> ee((size_t)a.H * wd, 0xFFFFFFFFu), el(a.H);
    for (uint32_t j = 0; j < a.H; ++j) {
      el[j] = (uint32_t)(rt_ptr[j + 1] - rt_ptr[j]);
      for (uint64_t e = rt_ptr[j]; e < rt_ptr[j + 1]; ++e) {
        es[(size_t)j * wd + (e - rt_ptr[j])] = rt_src[e];
        ee[(size_t)j * wd + (e - rt_ptr[j])] = rt_edge[e];
      }
    }
    a.ell_w = wd;
    a.ell_src = upload(pool, es);
    a.ell_edge = upload(pool, ee);
    a.ell_len = upload(pool, el);
    a.ell_wt = dev_array<float>(pool, es.size());
  }
  a.flags = dev_array<uint32_t>(pool, 2);
  a.w_in_t = dev_array<float>(pool, std::max<uint64_t>(1, nnz_in));
  a.w_rec_t = dev_array<float>(pool, std::max<uint64_t>(1, nnz_rec));
  a.w_rec_c = dev_array<float>(pool, std::max<uint64_t>(1, nnz_rec));
  a.w_out_c = dev_array<float>(pool, (size_t)a.H * a.O);
  a.xt = dev_array<float>(pool, (size_t)a.T * a.C * 64);
  a.iin = dev_array<float>(pool, (size_t)a.T * HB);
  a.s = dev_array<float>(pool, (size_t)a.T * HB);
  a.vck = dev_array<float>(pool, n_seg * HB);
  a.vtmp = dev_array<float>(pool, 2 * HB);
  a.vseg = dev_array<float>(pool, (size_t)a.K * HB);
  a.ro = dev_array<float>(pool, (size_t)a.T * a.O * 64);
  a.lamu = dev_array<float>(pool, (size_t)a.T * a.O * 64);
  a.lamv = dev_array<float>(pool, (size_t)a.T * HB);
  a.lam_carry = dev_array<float>(pool, HB);
  a.m = dev_array<float>(pool, (size_t)a.B * a.O);
  a.dm = dev_array<float>(pool, (size_t)a.B * a.O);
  a.tmax = dev_array<int32_t>(pool, (size_t)a.B * a.O);
  check(hipStreamSynchronize(pool->stream), "sync after plan");
}

// Runs a pass's body: from its HIP graph (captured on the first call, on the call's
// stream), or launched kernel by kernel when the plan is eager.
template <typename F>
void bptt_body(snn_bptt *p, hipGraphExec_t &exec, hipStream_t s, F &&body) {
  if (p->desc.eager) {
    check(body(s), "bptt launch");
    return;
  }
  if (!exec) {
    hipGraph_t g = nullptr;
    check(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "begin capture");
    const hipError_t e = body(s);
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      check(e != hipSuccess ? e : e2, "bptt capture");
    }
    const hipError_t e3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check(e3, "bptt graph instantiate");
  }
  check(hipGraphLaunch(exec, s), "bptt graph launch");
}

void bptt_release_graphs(snn_bptt *p) {
  if (p->g_fwd) (void)hipGraphExecDestroy(p->g_fwd);
  if (p->g_bwd) (void)hipGraphExecDestroy(p->g_bwd);
  p->g_fwd = p->g_bwd = nullptr;
}

}  // namespace

extern "C" {

snn_status snn_build_network(const snn_params *prm, const snn_population *pops, uint32_t n_pops,
                             const snn_projection *proj, uint32_t n_proj, const snn_allocator *alloc,
                             void *stream, snn_network **out) {
  return guarded([&] {
    if (!prm || !out || (!pops && n_pops) || (!proj && n_proj)) fail(SNN_E_INVALID, "null argument");
    *out = nullptr;
    snn_network *net = new snn_network();
    try {
      net->prm = *prm;
      net->pops.assign(pops, pops + n_pops);
      net->proj.assign(proj, proj + n_proj);
      if (alloc && alloc->alloc && alloc->free) {
        net->alloc = *alloc;
        net->has_alloc = true;
      }
      check(hipGetDevice(&net->device), "hipGetDevice");
      hipDeviceProp_t props;
      check(hipGetDeviceProperties(&props, net->device), "hipGetDeviceProperties");
      net->cu_count = (uint32_t)std::max(1, props.multiProcessorCount);
      if (stream) {
        net->stream = (hipStream_t)stream;
      } else {
        check(hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking), "hipStreamCreate");
        net->own_stream = true;
      }
      const auto t0 = std::chrono::steady_clock::now();
      build(net);
      net->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    } catch (...) {
      release(net);
      delete net;
      throw;
    }
    *out = net;
  });
}

snn_status snn_spacing_gaps(const uint32_t *words, uint64_t n, uint32_t *gaps, void *stream) {
  return guarded([&] {
    if (n && (!words || !gaps)) fail(SNN_E_INVALID, "null argument");
    check(snn::launch_spacing_gaps(words, n, gaps, (hipStream_t)stream), "spacing gaps launch");
  });
}

snn_status snn_step(snn_network *net) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    refuse_member(net);
    issue_window(net, 1);
  });
}

snn_status snn_run(snn_network *net, uint32_t n_steps) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    refuse_member(net);
    run(net, n_steps);
  });
}

snn_status snn_memory_cache_stats(int device, uint64_t *bytes, uint64_t *blocks, uint64_t *hits,
                                  uint64_t *misses) {
  return guarded([&] {
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    uint64_t b = 0, n = 0;
    for (const PoolBlock &k : g_pool)
      if (k.device == device) {
        b += k.bytes;
        ++n;
      }
    const PoolStats st = g_pool_stats.count(device) ? g_pool_stats[device] : PoolStats{};
    if (bytes) *bytes = b;
    if (blocks) *blocks = n;
    if (hits) *hits = st.hits;
    if (misses) *misses = st.misses;
  });
}

snn_status snn_memory_cache_release(int device) {
  return guarded([&] { pool_release(device); });
}

snn_status snn_sync(snn_network *net) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    sync(net);
  });
}

snn_status snn_get_raster_bits(snn_network *net, uint64_t t_begin, uint64_t t_end, uint64_t *words) {
  return guarded([&] {
    if (!net || (!words && t_end > t_begin)) fail(SNN_E_INVALID, "null argument");
    raster_range_check(net, t_begin, t_end);
    copy_raster_rows(net, t_begin, t_end, words);
  });
}

snn_status snn_get_raster(snn_network *net, uint64_t t_begin, uint64_t t_end, uint32_t *steps,
                          uint32_t *ids, uint64_t capacity, uint64_t *n_spikes) {
  return guarded([&] {
    if (!net || !n_spikes) fail(SNN_E_INVALID, "null argument");
    raster_range_check(net, t_begin, t_end);
    std::vector<uint64_t> rows((size_t)(t_end - t_begin) * net->words);
    copy_raster_rows(net, t_begin, t_end, rows.data());
    uint64_t count = 0;
    for (uint64_t w : rows) count += (uint64_t)__builtin_popcountll(w);
    *n_spikes = count;
    if (count > capacity) fail(SNN_E_OVERFLOW, "raster holds " + std::to_string(count) + " spikes");
    if (count && (!steps || !ids)) fail(SNN_E_INVALID, "null output arrays");
    uint64_t k = 0;
    for (uint64_t t = t_begin; t < t_end; ++t)
      for (uint32_t w = 0; w < net->words; ++w) {
        uint64_t bits = rows[(t - t_begin) * net->words + w];
        while (bits) {
          const int b = __builtin_ctzll(bits);
          bits &= bits - 1;
          steps[k] = (uint32_t)t;
          ids[k] = w * 64u + (uint32_t)b;
          ++k;
        }
      }
  });
}

snn_status snn_get_info(snn_network *net, snn_info *info) {
  return guarded([&] {
    if (!net || !info) fail(SNN_E_INVALID, "null argument");
    lazy_flush(net);  // pending potentiation counted as touches
    const CtlTotals c = read_ctl(net);
    if (c.lazy_overrun) fail(SNN_E_STATE, "lazy plasticity: a row had more pending steps than the spike history holds");
    snn_info r{};
    r.n = net->n;
    r.delay = net->delay;
    r.queue_slots = net->slots;
    r.queue_groups = snn::kQueueGroups;
    r.queue_stride = net->queue_stride;
    r.input_buffers = net->n_inbuf;
    r.window = net->window;
    r.delivery = net->delivery;
    r.tiles = net->tiles;
    r.plastic = net->plastic ? 1u : 0u;
    r.raster_steps = net->raster_cap;
    r.source_weights = net->w_src ? 1u : 0u;
    r.raster_words = net->words;
    r.table_len = net->table_len;
    r.nnz = net->nnz;
    r.t = c.t;
    r.events = c.events;
    r.spikes = c.spikes;
    r.touches = c.touches;
    r.device_bytes = net->device_bytes;
    r.build_ms = net->build_ms;
    r.gen_rows_ms = net->gen_rows_ms;
    r.gen_fill_ms = net->gen_fill_ms;
    r.index_ms = net->index_ms;
    r.tile_offset_bytes = net->tile_off ? (net->tile_off16 ? 2u : 4u) : 0u;
    r.target_bytes = net->delivery == SNN_DELIVERY_TILED ? 2u : 4u;
    r.plasticity = net->lazy ? SNN_PLASTICITY_LAZY : SNN_PLASTICITY_EAGER;
    if (c.t != net->t_host) fail(SNN_E_STATE, "device step counter disagrees with the host");
    *info = r;
  });
}

snn_status snn_get_state(snn_network *net, const snn_state *st) {
  return guarded([&] {
    if (!net || !st) fail(SNN_E_INVALID, "null argument");
    lazy_flush(net);  // weights as the eager form holds them
    hipStream_t s = net->stream;
    const size_t n = net->n;
    auto d2h = [&](void *dst, const void *src, size_t bytes) {
      if (dst) check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), "state copy");
    };
    d2h(st->v, net->v, n * 4);
    d2h(st->ref, net->ref, n * 4);
    d2h(st->input, net->input, (size_t)net->n_inbuf * n * 4);
    d2h(st->x_pre, net->x_pre, n * 4);
    d2h(st->x_post, net->x_post, n * 4);
    d2h(st->queue, net->queue, (size_t)net->slots * net->queue_stride * 4);
    if (st->queue_len)
      check(hipMemcpy2DAsync(st->queue_len, 4, net->qlen, snn::kQlenStride * 4, 4,
                             (size_t)net->slots * snn::kQueueGroups, hipMemcpyDeviceToHost, s),
            "queue counters");
    if (st->w_f32) {
      if (!net->plastic) fail(SNN_E_INVALID, "w_f32 requested from a static network");
      d2h(st->w_f32, net->w_f32, net->nnz * 4);
    }
    sync(net);
  });
}

snn_status snn_set_state(snn_network *net, const snn_state *st) {
  return guarded([&] {
    if (!net || !st) fail(SNN_E_INVALID, "null argument");
    // lazy plasticity: pending potentiation is applied with the traces it was due under;
    // the rows' traces at age are rebuilt from the new x_pre afterwards
    lazy_flush(net);
    hipStream_t s = net->stream;
    const size_t n = net->n;
    auto h2d = [&](void *dst, const void *src, size_t bytes) {
      if (src) check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "state copy");
    };
    h2d(net->v, st->v, n * 4);
    h2d(net->ref, st->ref, n * 4);
    h2d(net->input, st->input, (size_t)net->n_inbuf * n * 4);
    h2d(net->x_pre, st->x_pre, n * 4);
    h2d(net->x_post, st->x_post, n * 4);
    h2d(net->queue, st->queue, (size_t)net->slots * net->queue_stride * 4);
    if (st->queue_len)
      check(hipMemcpy2DAsync(net->qlen, snn::kQlenStride * 4, st->queue_len, 4, 4,
                             (size_t)net->slots * snn::kQueueGroups, hipMemcpyHostToDevice, s),
            "queue counters");
    if (st->w_f32) {
      if (!net->plastic) fail(SNN_E_INVALID, "w_f32 given to a static network");
      h2d(net->w_f32, st->w_f32, net->nnz * 4);
    }
    lazy_flush(net);
    sync(net);
  });
}

snn_status snn_get_row(snn_network *net, uint32_t i, int32_t *col, int32_t *w_q16, float *w_f32,
                       uint64_t cap, uint64_t *len) {
  return guarded([&] {
    if (!net || !len) fail(SNN_E_INVALID, "null argument");
    if (i >= net->n) fail(SNN_E_INVALID, "neuron id out of range");
    uint64_t rp[2];
    check(hipMemcpyAsync(rp, net->row_ptr + i, 16, hipMemcpyDeviceToHost, net->stream), "row ptr");
    sync(net);
    *len = rp[1] - rp[0];
    if (*len > cap) fail(SNN_E_OVERFLOW, "row longer than cap");
    if (*len == 0) return;
    if (col) check(hipMemcpyAsync(col, net->col + rp[0], *len * 4, hipMemcpyDeviceToHost, net->stream), "row");
    if (w_q16) {
      if (net->w_src) std::fill(w_q16, w_q16 + *len, net->w_src_host[i]);
      else if (!net->w_q16) fail(SNN_E_INVALID, "network has FP32 weights");
      else check(hipMemcpyAsync(w_q16, net->w_q16 + rp[0], *len * 4, hipMemcpyDeviceToHost, net->stream), "row");
    }
    if (w_f32) {
      if (!net->w_f32) fail(SNN_E_INVALID, "network has Q16 weights");
      lazy_flush(net);
      check(hipMemcpyAsync(w_f32, net->w_f32 + rp[0], *len * 4, hipMemcpyDeviceToHost, net->stream), "row");
    }
    sync(net);
  });
}

snn_status snn_get_synapses(snn_network *net, uint64_t *row_ptr, int32_t *col, int32_t *w_q16,
                            float *w_f32) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    hipStream_t s = net->stream;
    if (row_ptr) check(hipMemcpyAsync(row_ptr, net->row_ptr, ((size_t)net->n + 1) * 8, hipMemcpyDeviceToHost, s), "copy");
    if (col) check(hipMemcpyAsync(col, net->col, net->nnz * 4, hipMemcpyDeviceToHost, s), "copy");
    if (w_q16) {
      if (net->w_src) {
        std::vector<uint64_t> rp((size_t)net->n + 1);
        check(hipMemcpyAsync(rp.data(), net->row_ptr, rp.size() * 8, hipMemcpyDeviceToHost, s), "copy");
        sync(net);
        for (uint32_t i = 0; i < net->n; ++i) std::fill(w_q16 + rp[i], w_q16 + rp[i + 1], net->w_src_host[i]);
      } else if (!net->w_q16) {
        fail(SNN_E_INVALID, "network has FP32 weights");
      } else {
        check(hipMemcpyAsync(w_q16, net->w_q16, net->nnz * 4, hipMemcpyDeviceToHost, s), "copy");
      }
    }
    if (w_f32) {
      if (!net->w_f32) fail(SNN_E_INVALID, "network has Q16 weights");
      lazy_flush(net);
      check(hipMemcpyAsync(w_f32, net->w_f32, net->nnz * 4, hipMemcpyDeviceToHost, s), "copy");
    }
    sync(net);
  });
}

snn_status snn_get_drive_table(snn_network *net, uint64_t *table, uint32_t cap) {
  return guarded([&] {
    if (!net || !table) fail(SNN_E_INVALID, "null argument");
    if (cap < net->table_len) fail(SNN_E_OVERFLOW, "table longer than cap");
    std::memcpy(table, net->table, net->table_len * 8);
  });
}

snn_status snn_set_profiling(snn_network *net, int32_t on) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    net->profiling = on != 0;
  });
}

snn_status snn_get_profile(snn_network *net, snn_profile *prof) {
  return guarded([&] {
    if (!net || !prof) fail(SNN_E_INVALID, "null argument");
    resolve_profile(net);
    *prof = net->prof;
  });
}

snn_status snn_reset_profile(snn_network *net) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    resolve_profile(net);
    net->prof = snn_profile{};
  });
}

snn_status snn_time_delivery(snn_network *net, const uint32_t *ids_host, uint32_t n_ids,
                             const uint32_t *step_counts, uint32_t steps, uint32_t reps,
                             double *avg_ms, uint64_t *events) {
  return guarded([&] {
    if (!net || (!ids_host && n_ids) || !avg_ms) fail(SNN_E_INVALID, "null argument");
    refuse_member(net);
    if (steps == 0) steps = net->window;
    if (steps > net->window) fail(SNN_E_INVALID, "steps exceeds the network's window");
    std::vector<std::vector<uint32_t>> per_step(steps);
    if (step_counts) {
      uint64_t k = 0;
      for (uint32_t w = 0; w < steps; ++w) {
        if (k + step_counts[w] > n_ids) fail(SNN_E_INVALID, "step counts exceed the ids");
        per_step[w].assign(ids_host + k, ids_host + k + step_counts[w]);
        k += step_counts[w];
      }
      if (k != n_ids) fail(SNN_E_INVALID, "step counts do not sum to n_ids");
    } else {
      for (uint32_t k = 0; k < n_ids; ++k) per_step[k % steps].push_back(ids_host[k]);
    }
    uint64_t ev = 0;
    *avg_ms = time_delivery(net, per_step, reps, &ev);
    if (events) *events = ev;
  });
}

snn_status snn_time_delivery_static(snn_network *net, const uint32_t *ids_host, uint32_t n_ids,
                                    const uint32_t *step_counts, uint32_t steps, uint32_t reps,
                                    double *avg_ms, uint64_t *events) {
  return guarded([&] {
    if (!net || (!ids_host && n_ids) || !avg_ms) fail(SNN_E_INVALID, "null argument");
    refuse_member(net);
    if (steps == 0) steps = net->window;
    *avg_ms = time_delivery_static(net, ids_host, n_ids, step_counts, steps, reps, events);
  });
}

snn_status snn_set_delivery(snn_network *net, uint32_t delivery, uint32_t tiles, uint32_t block, uint32_t grid) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    refuse_member(net);
    set_delivery(net, delivery, tiles, block, grid);
  });
}

snn_status snn_autotune_delivery(snn_network *net, uint32_t reps, snn_delivery_tuning *chosen) {
  return guarded([&] {
    if (!net) fail(SNN_E_INVALID, "null network");
    refuse_member(net);
    const snn_delivery_tuning t = autotune_delivery(net, reps);
    if (chosen) *chosen = t;
  });
}

void snn_destroy(snn_network *net) {
  if (!net || net->owner) return;
  try {
    resolve_profile(net);
  } catch (...) {
  }
  release(net);
  delete net;
}

const char *snn_last_error(const snn_network *) { return g_error.c_str(); }

snn_status snn_build_batch(const snn_batch_member *nets, uint32_t n_nets, uint32_t raster_steps,
                           const snn_allocator *alloc, void *stream, snn_batch **out) {
  return guarded([&] {
    if (!out || (!nets && n_nets)) fail(SNN_E_INVALID, "null argument");
    *out = nullptr;
    if (n_nets == 0) fail(SNN_E_INVALID, "a batch needs at least one network");
    snn_batch *b = new snn_batch();
    try {
      if (alloc && alloc->alloc && alloc->free) {
        b->pool.alloc = *alloc;
        b->pool.has_alloc = true;
      }
      check(hipGetDevice(&b->pool.device), "hipGetDevice");
      hipDeviceProp_t props;
      check(hipGetDeviceProperties(&props, b->pool.device), "hipGetDeviceProperties");
      b->pool.cu_count = (uint32_t)std::max(1, props.multiProcessorCount);
      if (stream) {
        b->pool.stream = (hipStream_t)stream;
      } else {
        check(hipStreamCreateWithFlags(&b->pool.stream, hipStreamNonBlocking), "hipStreamCreate");
        b->pool.own_stream = true;
      }
      build_batch(b, nets, n_nets, raster_steps);
    } catch (...) {
      batch_destroy(b);
      delete b;
      throw;
    }
    *out = b;
  });
}

snn_status snn_batch_run(snn_batch *b, uint32_t n_steps) {
  return guarded([&] {
    if (!b) fail(SNN_E_INVALID, "null batch");
    batch_run(b, n_steps);
  });
}

snn_status snn_batch_sync(snn_batch *b) {
  return guarded([&] {
    if (!b) fail(SNN_E_INVALID, "null batch");
    check(hipStreamSynchronize(b->pool.stream), "stream sync");
  });
}

snn_status snn_batch_network(snn_batch *b, uint32_t k, snn_network **net) {
  return guarded([&] {
    if (!b || !net) fail(SNN_E_INVALID, "null argument");
    if (k >= b->nets.size()) fail(SNN_E_INVALID, "member index out of range");
    *net = b->nets[k];
  });
}

snn_status snn_batch_autotune(snn_batch *b, uint32_t trial_steps, snn_batch_tuning *chosen) {
  return guarded([&] {
    if (!b) fail(SNN_E_INVALID, "null batch");
    const snn_batch_tuning t = batch_autotune(b, trial_steps);
    if (chosen) *chosen = t;
  });
}

snn_status snn_batch_set_tuning(snn_batch *b, const snn_batch_tuning *tuning) {
  return guarded([&] {
    if (!b || !tuning) fail(SNN_E_INVALID, "null argument");
    check(hipStreamSynchronize(b->pool.stream), "stream sync");
    batch_apply_tuning(b, *tuning);
  });
}

snn_status snn_batch_get_tuning(snn_batch *b, snn_batch_tuning *tuning) {
  return guarded([&] {
    if (!b || !tuning) fail(SNN_E_INVALID, "null argument");
    *tuning = b->tuning;
  });
}

void snn_batch_destroy(snn_batch *b) {
  if (!b) return;
  batch_destroy(b);
  delete b;
}

snn_status snn_bptt_create(const snn_bptt_desc *desc, const uint64_t *in_row_ptr, const int32_t *in_col,
                           const uint64_t *rec_row_ptr, const int32_t *rec_col, const snn_allocator *alloc,
                           void *stream, snn_bptt **out) {
  return guarded([&] {
    if (!desc || !out || !in_row_ptr || !rec_row_ptr) fail(SNN_E_INVALID, "null argument");
    *out = nullptr;
    snn_bptt *p = new snn_bptt();
    try {
      p->desc = *desc;
      if (alloc && alloc->alloc && alloc->free) {
        p->pool.alloc = *alloc;
        p->pool.has_alloc = true;
      }
      check(hipGetDevice(&p->pool.device), "hipGetDevice");
      if (stream) {
        p->pool.stream = (hipStream_t)stream;
      } else {
        check(hipStreamCreateWithFlags(&p->pool.stream, hipStreamNonBlocking), "hipStreamCreate");
        p->pool.own_stream = true;
      }
      build_bptt(p, in_row_ptr, in_col, rec_row_ptr, rec_col);
    } catch (...) {
      release(&p->pool);
      delete p;
      throw;
    }
    *out = p;
  });
}

snn_status snn_bptt_forward(snn_bptt *p, const float *x, const float *w_in, const float *w_rec,
                            const float *w_out, const int32_t *labels, float *loss, void *stream) {
  return guarded([&] {
    if (!p || !x || !w_out || !labels || !loss || (!w_in && p->args.nnz_in) || (!w_rec && p->args.nnz_rec))
      fail(SNN_E_INVALID, "null argument");
    snn::BpttArgs a = p->args;
    a.w_in = w_in;
    a.w_rec = w_rec;
    a.w_out = w_out;
    hipStream_t s = stream ? (hipStream_t)stream : p->pool.stream;
    check(snn::bptt_forward_prologue(a, x, s), "bptt forward");
    snn::BpttArgs g = p->args;  // the body reads the plan's buffers only
    g.w_out = g.w_out_c;
    bptt_body(p, p->g_fwd, s, [&](hipStream_t st) { return snn::bptt_forward_body(g, st); });
    check(snn::bptt_forward_epilogue(a, labels, loss, s), "bptt forward");
    p->forwards++;
  });
}

snn_status snn_bptt_backward(snn_bptt *p, const float *w_in, const float *w_rec, const float *w_out,
                             const float *g_loss, float *g_w_in, float *g_w_rec, float *g_w_out,
                             void *stream) {
  return guarded([&] {
    if (!p || !w_out || !g_w_out || (!w_in && p->args.nnz_in) || (!w_rec && p->args.nnz_rec) ||
        (!g_w_in && p->args.nnz_in) || (!g_w_rec && p->args.nnz_rec))
      fail(SNN_E_INVALID, "null argument");
    if (p->forwards == 0) fail(SNN_E_STATE, "backward before any forward pass");
    snn::BpttArgs a = p->args;
    a.w_in = w_in;
    a.w_rec = w_rec;
    a.w_out = w_out;
    a.g_w_in = g_w_in;
    a.g_w_rec = g_w_rec;
    a.g_w_out = g_w_out;
    hipStream_t s = stream ? (hipStream_t)stream : p->pool.stream;
    check(snn::bptt_backward_prologue(a, g_loss, s), "bptt backward");
    snn::BpttArgs g = p->args;
    g.w_out = g.w_out_c;
    g.w_rec = g.w_rec_c;
    bptt_body(p, p->g_bwd, s, [&](hipStream_t st) { return snn::bptt_backward_body(g, st); });
    check(snn::bptt_backward_epilogue(a, s), "bptt backward");
  });
}

snn_status snn_bptt_get_trace(snn_bptt *p, float *spikes, float *v_checkpoints, float *readout_max,
                              int32_t *readout_argmax, void *stream) {
  return guarded([&] {
    if (!p) fail(SNN_E_INVALID, "null plan");
    const snn::BpttArgs &a = p->args;
    hipStream_t s = stream ? (hipStream_t)stream : p->pool.stream;
    const size_t HB = (size_t)a.H * 64, n_seg = (a.T + a.K - 1) / a.K;
    if (spikes) check(hipMemcpyAsync(spikes, a.s, (size_t)a.T * HB * 4, hipMemcpyDeviceToHost, s), "copy");
    if (v_checkpoints) check(hipMemcpyAsync(v_checkpoints, a.vck, n_seg * HB * 4, hipMemcpyDeviceToHost, s), "copy");
    if (readout_max) check(hipMemcpyAsync(readout_max, a.m, (size_t)a.B * a.O * 4, hipMemcpyDeviceToHost, s), "copy");
    if (readout_argmax)
      check(hipMemcpyAsync(readout_argmax, a.tmax, (size_t)a.B * a.O * 4, hipMemcpyDeviceToHost, s), "copy");
    check(hipStreamSynchronize(s), "sync");
  });
}

void snn_bptt_destroy(snn_bptt *p) {
  if (!p) return;
  if (p->pool.stream) (void)hipStreamSynchronize(p->pool.stream);
  bptt_release_graphs(p);
  release(&p->pool);
  delete p;
}

}  // extern "C"
