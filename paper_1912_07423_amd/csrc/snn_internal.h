// snn_internal.h -- library-private types shared by the host runtime and kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/snn.h"

namespace snn {

constexpr uint32_t kTableCap = 256;

// Many workgroups update the same counters at the same moment; same-line atomics
// from a burst of workgroups serialise, so every shared counter gets its own
// 256-byte line and the hot ones are split into independent parts.
constexpr uint32_t kQlenStride = 64;    // uint32 per counter line
constexpr uint32_t kLineU64 = 32;       // uint64 per 256-byte line
constexpr uint32_t kQueueGroups = 8;    // sub-queues of a step's spike queue
constexpr uint32_t kCounterParts = 64;  // partial sums of the event/spike/touch counters
constexpr uint32_t kUpdateBlock = 256;  // neurons per update workgroup
constexpr uint32_t kGuideBits = 12;     // drive guide table: buckets on the top bits of r
constexpr uint32_t kGuideBuckets = 1u << kGuideBits;

// Device-resident control block.  `t` is the first step of the next update launch;
// the update launch copies it to `t_deliver` and the delivery launch that closes the
// window advances `t`, so every kernel finds its step on the device and a captured
// HIP graph replays correctly.
struct Ctl {
  uint64_t t;
  uint64_t t_deliver;
  uint64_t lazy_overrun;  // rows found with more pending steps than the history holds
  uint64_t pad[kLineU64 - 3];
  uint64_t events[kCounterParts * kLineU64];   // part p at [p * kLineU64]
  uint64_t spikes[kCounterParts * kLineU64];
  uint64_t touches[kCounterParts * kLineU64];
};

// A step's spike queue is kQueueGroups sub-queues of group_cap entries each; update
// workgroup b appends to sub-queue b % kQueueGroups.  Counter of (slot, group) at
// qlen[(slot * kQueueGroups + group) * kQlenStride].
struct QueueRef {
  int32_t *ids;       // [slots][stride]
  uint32_t *qlen;
  uint32_t stride;    // kQueueGroups * group_cap
  uint32_t group_cap;
};

// One projection as the device generators see it (per source population, sorted by
// first target population).
struct GenProj {
  uint32_t kind;     // SNN_PROJ_*
  uint32_t k;        // out-degree (fixed)
  uint32_t first_pop;  // first target population (stream id of the fixed generator)
  uint32_t off;      // first target id
  uint32_t size;     // number of target ids
  uint32_t self_in;  // sources of this projection lie inside the target range
  uint32_t plastic;
  int32_t w_q16;
  float w_f32;
  uint32_t pad;
  uint64_t thr;      // ER: edge iff word < thr
  uint64_t spare;    // fixed: candidates - k
};

struct GenArgs {
  const GenProj *proj;      // [n_proj] sorted by (source population, first target)
  const uint32_t *pop_off;  // [n_pops + 1]
  const uint32_t *pop_proj; // [n_pops + 1] projection range of each source population
  uint32_t n_pops, n;
  uint32_t key0, key1;
};

// Lazy plasticity (Sec. III-A.1, Table I "bitmasks", "ages", "expirations").  Row i's
// potentiation events of the steps [age_i, t] are pending: they wait in the targets'
// spike histories and are applied when the row transmits or, at the latest, when the
// oldest pending step is about to leave the kLazyHistory-step history.
constexpr uint32_t kLazyHistory = 64;  // steps of spike history per neuron (one uint64)
struct LazyRef {
  uint64_t *hist;         // [n] bit k: the neuron spiked at step t - k (t the last update)
  uint32_t *age;          // [n] first pending step of the row, mod 2^32
  float *x_age;           // [n] the row's presynaptic trace at its age step
  const uint32_t *plast_len;  // [n] plastic synapses of each row (0: no age kept)
  QueueRef exq;           // 2 slots: the expiring rows of step t in slot t mod 2, laid out
                          // as a spike queue (kQueueGroups sub-queues)
  uint32_t delay;
};

struct UpdateArgs {
  float *v;
  int32_t *ref;
  int32_t *input;     // [n_inbuf][n]
  float *x_pre, *x_post;
  QueueRef q;
  uint64_t *raster;   // [raster_cap][words]
  const uint32_t *table32;  // drive thresholds below 2^32
  const uint16_t *guide;    // [kGuideBuckets]: count at the bucket's low end | high end << 8
  Ctl *ctl;
  uint32_t n, slots, n_inbuf, raster_cap, words, table_len;
  uint32_t key0, key1;
  float alpha, v_inf, v_th, v_reset, beta_plus, beta_minus;
  int32_t ref_steps, w_ext_q16;
  uint32_t zero_input, plastic;
  // lazy plasticity (one step per launch): spike history, ages and the expiring-row
  // queue, all null otherwise
  LazyRef lazy;
};

struct DeliverArgs {
  const uint64_t *row_ptr;
  const int32_t *col;
  const int32_t *w_q16;   // static networks with a weight per synapse
  const float *w_f32;     // plastic networks
  const int32_t *w_src;   // static networks with one weight per source population:
                          // Q16 weight of every synapse of source i (no w_q16)
  QueueRef q;
  int32_t *input;
  const uint16_t *col16;  // tiled delivery: low 16 bits of every target, [nnz] padded to
                          // whole 16-byte groups
  const void *tile_off;   // [n][tiles + 1] tile boundaries of each row, relative to the
                          // row's start: uint16 when off16, else uint32
  Ctl *ctl;
  uint32_t n, slots, n_inbuf, delay, window_max;
  uint32_t tiles, tile_size;
  uint32_t off16;
  uint32_t advance;       // this launch closes the window: advance the step counter
  float *x_pre, *x_post;  // eager STDP: here x_pre += 1 for S_{t-d}, x_post += 1 for S_t (else null)
};

// The lazy plasticity kernel of one step t: rows of S_{t-d+1} transmit (pending
// potentiation applied, then delivered with the current weights), expiring rows are
// brought current, and the postsynaptic traces of S_t are incremented.
struct LazyArgs {
  const uint64_t *row_ptr;
  const int32_t *col;
  float *w_f32;
  const uint32_t *plast_rel;
  float *x_pre, *x_post;
  QueueRef q;
  int32_t *input;
  LazyRef lazy;
  Ctl *ctl;
  uint32_t n, slots, delay;
  float a_plus, w_max, beta_plus;
};

struct StdpArgs {
  const uint64_t *row_ptr;
  const int32_t *col;
  float *w_f32;
  const uint32_t *plast_rel, *plast_len;
  const uint64_t *in_ptr;
  const int32_t *in_src;
  const uint32_t *in_edge;
  float *x_pre, *x_post;
  QueueRef q;
  Ctl *ctl;
  const uint64_t *raster;  // [raster_cap][words] spike bits (the fused pass tests S_t, S_{t-d})
  uint32_t raster_cap, words;
  uint32_t n, slots, delay;
  float a_plus, a_minus, w_max;
};

// One network of a batch as the persistent batch kernel sees it: pointers into the
// network's own buffers (state layout identical to the single-network pipeline) and
// its derived constants.
struct BatchNet {
  const uint64_t *row_ptr;
  const int32_t *col, *w_q16;
  const int32_t *w_src;      // one weight per source neuron (then w_q16 is null)
  float *v;
  int32_t *ref;
  int32_t *input;            // [delay][n] Q16 accumulators, slot t mod delay
  int32_t *queue;            // >= n spike ids
  uint64_t *raster;          // [raster_cap][words]
  const uint32_t *table32;   // drive thresholds below 2^32
  Ctl *ctl;
  uint32_t n, words, delay, raster_cap;
  uint32_t below;            // number of drive thresholds below 2^32 (0: no drive)
  uint32_t lanes_shift;      // log2 of the lanes that share one spike's row
  uint32_t key0, key1;
  float alpha, v_inf, v_th, v_reset;
  int32_t ref_steps, w_ext_q16;
};
constexpr uint32_t kBatchCommit = 1u;       // write state, counters and t back
constexpr uint32_t kBatchWriteRaster = 2u;  // write the raster rows
constexpr uint32_t kBatchDrive = 4u;        // some member has a Poisson drive
bool batch_variant_supported(uint32_t block, uint32_t per);
uint32_t batch_per_lane(uint32_t block, uint32_t n_max);  // 0: n_max too large for block
hipError_t launch_batch(const BatchNet *nets, const uint32_t *order, uint32_t n_nets, uint32_t steps,
                        uint32_t block, uint32_t per, uint32_t flags, size_t lds, hipStream_t s);

// Surrogate-gradient BPTT plan as its kernels see it (bptt.hip).  Batch <= 64: lane b
// of a wavefront is batch element b; sizes are B batch, T steps, C inputs, H hidden,
// O readouts, K steps per checkpoint segment (<= 32).
// Limits of the ELL form of the hidden steps: rows of at most 256 in-edges (four lane
// loads), and at most 8,192 hidden neurons (their 64 KiB of spike masks in LDS).
constexpr uint32_t kEllMaxWidth = 256;
constexpr uint32_t kEllMaxNeurons = 8192;
struct BpttArgs {
  uint32_t B, T, C, H, O, K;
  float beta, beta_out, theta, slope;
  uint32_t smooth, detach_reset;
  uint64_t nnz_in, nnz_rec;
  const uint64_t *in_t_ptr;    // W_in transposed: in-edges of each hidden neuron,
  const int32_t *in_t_src;     //   sources ascending, with their CSR edge index
  const uint32_t *in_t_edge;
  const uint64_t *rec_t_ptr;   // W_rec transposed, likewise
  const int32_t *rec_t_src;
  const uint32_t *rec_t_edge;
  const uint64_t *rec_ptr;     // W_rec forward rows
  const int32_t *rec_col;
  const float *w_in, *w_rec, *w_out;  // caller's weights: CSR order, CSR order, [H][O]
  float *g_w_in, *g_w_rec, *g_w_out;
  float *w_in_t, *w_rec_t;     // weights gathered into transposed (per-target) order
  float *w_out_c, *w_rec_c;    // the plan's copies of w_out and of w_rec in CSR order
  float *iin;                  // [T][H][64] input-projection current of every step
  uint64_t *xbits, *sbits;     // batch masks of the input and hidden spikes: [C][T], [H][T]
  uint64_t *sbits_t;           // the hidden spike masks again, step-major: [T][H]
  uint32_t ell_w;              // width of the ELL copy of W_rec's in-edges (0: none)
  const int32_t *ell_src;      // [H][ell_w] sources, ascending, then 0-padding
  const uint32_t *ell_edge;    // [H][ell_w] CSR edge index (padding: 0xFFFFFFFF)
  const uint32_t *ell_len;     // [H] in-degree
  float *ell_wt;               // [H][ell_w] weights gathered into that order (padding: 0)
  uint32_t *flags;             // [2]: a value of x / s is neither 0 nor 1 (masks not used)
  float *xt, *s, *vck, *vtmp, *vseg, *ro, *lamu, *lamv, *lam_carry, *m, *dm;
  int32_t *tmax;
};
// Forward and backward passes in three parts each: prologue and epilogue touch the
// caller's arrays, the body only the plan's buffers (capturable once per plan).  The body
// takes the plan's arguments with w_out (and, backward, w_rec) pointing at the plan's
// copies w_out_c / w_rec_c, which the prologue fills.
hipError_t bptt_forward_prologue(const BpttArgs &a, const float *x, hipStream_t s);
hipError_t bptt_forward_body(const BpttArgs &g, hipStream_t s);
hipError_t bptt_forward_epilogue(const BpttArgs &a, const int32_t *labels, float *loss, hipStream_t s);
hipError_t bptt_backward_prologue(const BpttArgs &a, const float *g_loss, hipStream_t s);
hipError_t bptt_backward_body(const BpttArgs &g, hipStream_t s);
hipError_t bptt_backward_epilogue(const BpttArgs &a, hipStream_t s);

// Optional timing events of one launch.  When set, the kernel is launched with
// hipExtLaunchKernel, which stamps `start` and `stop` with the dispatch's own begin and
// end (no marker packet is placed between launches); launches that span two kernels
// stamp the first one's begin and the last one's end.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool on() const { return start != nullptr || stop != nullptr; }
};

// kernel launchers (step.hip / generate.hip)
hipError_t launch_update(const UpdateArgs &a, uint32_t steps, hipStream_t s, const LaunchEvents &ev = {});
hipError_t launch_deliver_atomic(const DeliverArgs &a, uint32_t steps, uint32_t grid,
                                 hipStream_t s, const LaunchEvents &ev = {});
hipError_t launch_deliver_tiled(const DeliverArgs &a, uint32_t steps, uint32_t block,
                                uint32_t grid, hipStream_t s, const LaunchEvents &ev = {});
constexpr uint32_t kTileGroupMax = 32;  // base tiles one tiled-delivery workgroup may own
hipError_t prepare_deliver_tiled(uint32_t block, size_t *max_dynamic_lds);
hipError_t launch_stdp_ltd(const StdpArgs &a, uint32_t grid, hipStream_t s, const LaunchEvents &ev = {});
hipError_t launch_stdp_fused(const StdpArgs &a, uint32_t grid, hipStream_t s, const LaunchEvents &ev = {});
hipError_t launch_lazy(const LazyArgs &a, uint32_t grid, hipStream_t s, const LaunchEvents &ev = {});
// Brings every plastic row current at step boundary t (pending potentiation applied,
// age t, trace at age rebuilt from x_pre and the arrivals of step t).
hipError_t launch_lazy_flush(const LazyArgs &a, uint64_t t, uint32_t grid, hipStream_t s);
// One window's queues staged from a caller's spike list (k_stage_window): step w's
// ids are ids[off[w] .. off[w+1]), or dealt round-robin over the steps when
// round_robin is set (off then still holds each step's count as a prefix).
struct StageArgs {
  QueueRef q;             // `steps` slots
  Ctl *ctl;
  int32_t *input;         // n_input accumulators, cleared
  const int32_t *ids;
  uint64_t n_input;
  uint64_t t_deliver;
  uint32_t n_ids, steps, round_robin;
  uint32_t off[65];       // steps <= 64
};
hipError_t launch_stage_window(const StageArgs &a, hipStream_t s);
hipError_t launch_row_lengths(const GenArgs &g, uint32_t *len, uint32_t *plast_rel,
                              uint32_t *plast_len, hipStream_t s);
// all_fixed: every projection is fixed out-degree (no ER rows), which allows one
// workgroup per row for long rows.
hipError_t launch_fill_rows(const GenArgs &g, uint32_t max_fixed_k, bool all_fixed, const uint64_t *row_ptr,
                            int32_t *col, int32_t *w_q16, float *w_f32, hipStream_t s);
hipError_t launch_spacing_gaps(const uint32_t *words, uint64_t n, uint32_t *gaps, hipStream_t s);
hipError_t launch_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint32_t n,
                                  uint64_t *block_sums, hipStream_t s);
size_t scan_scratch_elems(uint32_t n);
hipError_t launch_count_in_edges(const uint64_t *row_ptr, const int32_t *col,
                                 const uint32_t *plast_rel, const uint32_t *plast_len,
                                 uint32_t n, uint32_t *count, hipStream_t s);
hipError_t launch_fill_in_edges(const uint64_t *row_ptr, const int32_t *col,
                                const uint32_t *plast_rel, const uint32_t *plast_len,
                                uint32_t n, uint64_t *cursor, int32_t *in_src,
                                uint32_t *in_edge, hipStream_t s);
hipError_t launch_tile_index(const uint64_t *row_ptr, const int32_t *col, uint32_t n, uint64_t nnz,
                             uint64_t count, uint32_t tiles, uint32_t tile_size, uint16_t *col16,
                             void *tile_off, bool off16, hipStream_t s);
hipError_t launch_init_neurons(float *v, int32_t *ref, uint32_t n, uint32_t key0, uint32_t key1,
                               float lo, float span, hipStream_t s);

}  // namespace snn

// The network object behind the opaque handle.
struct snn_network {
  // description
  std::vector<snn_population> pops;
  std::vector<snn_projection> proj;
  std::vector<uint32_t> pop_off;
  snn_params prm;
  // setup timing (host wall time of the build; device time of its generation phases)
  double build_ms = 0;
  float gen_rows_ms = 0, gen_fill_ms = 0, index_ms = 0;
  uint32_t key0 = 0, key1 = 0;

  // sizes and schedule
  uint32_t n = 0, delay = 1, slots = 2, n_inbuf = 1, window = 1;
  uint32_t delivery = SNN_DELIVERY_ATOMIC, tiles = 1, tile_size = 1, block = 512, grid = 512;
  uint32_t raster_cap = 1024, words = 1;
  bool plastic = false;
  bool lazy = false;  // plastic, with SNN_PLASTICITY_LAZY
  uint64_t nnz = 0, nnz_alloc = 0;

  // derived constants
  float alpha = 0, v_inf = 0, v_th = 0, v_reset = 0;
  float beta_plus = 0, beta_minus = 0, a_plus = 0, a_minus = 0, w_max = 0;
  int32_t ref_steps = 0, w_ext_q16 = 0;
  uint64_t table[snn::kTableCap] = {};
  uint32_t table_len = 0;

  // device memory
  uint64_t *row_ptr = nullptr;
  int32_t *col = nullptr, *w_q16 = nullptr;
  float *w_f32 = nullptr;
  int32_t *w_src = nullptr;             // per-source weights (Table I layout)
  std::vector<int32_t> w_src_host;
  uint32_t *plast_rel = nullptr, *plast_len = nullptr;
  uint64_t *in_ptr = nullptr;
  int32_t *in_src = nullptr;
  uint32_t *in_edge = nullptr;
  void *tile_off = nullptr;
  uint16_t *col16 = nullptr;   // low 16 bits of every target (tiled delivery)
  bool tile_off16 = false;    // tile boundaries stored as uint16 (every row < 65,536 synapses)
  uint64_t row_len_bound = 0; // upper bound on a row's length, from the projections
  float *v = nullptr, *x_pre = nullptr, *x_post = nullptr;
  int32_t *ref = nullptr, *input = nullptr, *queue = nullptr;
  uint32_t *qlen = nullptr;
  uint32_t queue_stride = 0, group_cap = 0;  // entries per queue slot / per sub-queue
  uint64_t *raster = nullptr;
  uint32_t *d_table32 = nullptr;
  uint16_t *d_guide = nullptr;
  snn::Ctl *ctl = nullptr;
  // lazy plasticity: per-neuron spike history, row ages and traces at age, expiring rows
  uint64_t *hist = nullptr;
  uint32_t *age = nullptr;
  float *x_age = nullptr;
  int32_t *exq = nullptr;
  uint32_t *exq_len = nullptr;

  // bookkeeping
  struct Alloc {
    void *p;
    size_t bytes;
  };
  std::vector<Alloc> allocs;
  snn_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  uint32_t cu_count = 256;
  uint64_t t_host = 0;  // steps issued (mirror of the device counter)
  snn_batch *owner = nullptr;  // set for the members of a batch
  uint64_t device_bytes = 0;

  // graph of a fixed chunk of windows
  hipGraphExec_t graph = nullptr;
  uint32_t graph_steps = 0;

  // profiling: hipEvent pairs around launches, resolved at the next readout
  struct ProfRecord {
    int kind;  // 0 update, 1 deliver, 2 stdp
    hipEvent_t a, b;
  };
  bool profiling = false;
  snn_profile prof{};
  std::vector<ProfRecord> prof_pending;
  std::vector<hipEvent_t> event_pool;
};
