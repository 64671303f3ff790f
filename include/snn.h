/*
 * snn.h -- C ABI of the MI355X clock-driven spiking-network simulator.
 *
 * The library simulates the work-queue pipeline of Bautembach et al., "Faster and
 * Simpler SNN Simulation with Work Queues" (IJCNN 2020), Sec. III-A, Fig. 1: per step,
 * Update Neurons emits a queue of spikes S_t; a FIFO of per-step queues delays them by
 * d >= 1 steps (Sec. III-A.1, "non-instantaneous connections"); Receive Spikes
 * delivers each dequeued spike over its neuron's out-edges; optionally Update
 * Synapses applies STDP driven by S_{t-d} (pre) and S_t (post).  The network is built
 * on the device from a seed (Init stage; adjacency generation of Sec. III-A.2, Fig. 2).
 *
 * Conventions
 *  - Every call returns snn_status: SNN_OK (0) or a negative error code.  No C++
 *    exception crosses this interface.  snn_last_error(net) returns a message for
 *    the last failing call on the calling thread (storage owned by the library, valid
 *    until the next call on that thread).
 *  - snn_network is opaque; the library owns it and every device buffer it holds.
 *    The caller owns every host array passed in or out.  Host arrays are read or
 *    written before the call returns.
 *  - Device work is issued on the stream given at build time (a hipStream_t passed as
 *    void*; NULL makes the library create its own stream).  snn_step/snn_run are
 *    asynchronous; every call that returns host data synchronises that stream first.
 *  - Neuron ids are global: population k holds ids [off_k, off_k + size_k) with
 *    populations laid out in the order given.
 *  - Units: ms, mV, Hz.  Synaptic input is accumulated as int32 fixed point in units
 *    of 2^-16 mV ("Q16"), so the order in which spikes are delivered cannot change a
 *    result.
 *  - Not thread-safe per network: calls on one network must not overlap.
 */
#ifndef SNN_H
#define SNN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t snn_status;
#define SNN_OK 0
#define SNN_E_INVALID (-1)  /* bad argument or parameter combination */
#define SNN_E_OOM (-2)      /* device or host allocation failed */
#define SNN_E_HIP (-3)      /* a HIP runtime call or kernel launch failed */
#define SNN_E_OVERFLOW (-4) /* caller buffer too small; the required size is returned */
#define SNN_E_STATE (-5)    /* call not valid in the network's current state */

#define SNN_PROJ_ER 0u        /* each ordered pair (i, j), j != i, independently w.p. p */
#define SNN_PROJ_FIXED_OUT 1u /* every source has exactly k distinct targets (Fig. 2) */

#define SNN_DELIVERY_AUTO 0u   /* tiled for networks of >= 16,384 neurons and a mean
                                  out-degree >= 64, else atomic */
#define SNN_DELIVERY_ATOMIC 1u /* wavefront(s) per spike, int32 atomics in global memory */
#define SNN_DELIVERY_TILED 2u  /* per (target tile, step) workgroup, int32 atomics in LDS;
                                  static and eagerly plastic networks (not lazy ones) */

/* Update Synapses with STDP (Sec. III-A.1).  Both forms give the same weights, traces
 * and spikes at every step. */
#define SNN_PLASTICITY_EAGER 0u /* each step: depression over the arriving spikes' rows,
                                   potentiation over the spiking neurons' in-edges */
#define SNN_PLASTICITY_LAZY 1u  /* the paper's lazy variation: a row's potentiation events
                                   wait in a per-neuron spike history (64 steps) and are
                                   applied in registers when the row transmits or its
                                   oldest pending step is about to leave the history
                                   ("expiring neurons", a queue produced by Update
                                   Neurons); per-neuron ages record what is pending.
                                   Needs delay_steps <= 64. */

typedef struct {
    uint32_t size;       /* neurons in the population (>= 1) */
    uint32_t excitatory; /* informational */
} snn_population;

typedef struct {
    uint32_t from;    /* source population */
    uint32_t to;      /* first target population */
    uint32_t kind;    /* SNN_PROJ_ER or SNN_PROJ_FIXED_OUT */
    uint32_t k;       /* out-degree (SNN_PROJ_FIXED_OUT) */
    double p;         /* connection probability (SNN_PROJ_ER) */
    double w_mV;      /* initial synaptic weight, |w| < 2^15 mV */
    uint32_t plastic; /* STDP on this projection (at most one per source population) */
    uint32_t to_span; /* targets are populations [to, to + to_span); 0 means 1 */
} snn_projection;

typedef struct {
    double dt_ms;          /* time step (> 0) */
    uint32_t delay_steps;  /* synaptic delay d >= 1 in steps (Sec. III-A.1) */
    uint32_t n_ext;        /* virtual Poisson inputs per neuron (0: no drive) */
    double tau_m_ms;       /* membrane time constant */
    double v_rest_mV;      /* resting potential */
    double v_bg_mV;        /* constant background drive added to the rest potential */
    double v_th_mV;        /* threshold (spike when V >= V_th) */
    double v_reset_mV;     /* reset potential */
    double t_ref_ms;       /* absolute refractory period */
    double v0_lo_mV;       /* initial V uniform in [v0_lo, v0_hi) */
    double v0_hi_mV;
    double rate_ext_hz;    /* rate of each virtual input */
    double w_ext_mV;       /* weight of each virtual input */
    double tau_plus_ms;    /* STDP potentiation trace time constant */
    double tau_minus_ms;   /* STDP depression trace time constant */
    double a_plus;         /* potentiation step per unit trace (mV) */
    double a_minus;        /* depression step per unit trace (mV) */
    double w_max_mV;       /* plastic weights are clipped to [0, w_max] */
    uint64_t seed;         /* key of every counter-based random stream */
    uint32_t raster_steps; /* spike-raster ring capacity in steps (0: 1024; at least delay + 1 for
                              plastic networks, whose plasticity pass reads step t - delay) */
    uint32_t window;       /* max steps per update launch (0: auto, <= delay) */
    uint32_t delivery;     /* SNN_DELIVERY_* */
    uint32_t tiles;        /* target tiles of the tiled delivery (0: auto) */
    uint32_t block;        /* workgroup size of the tiled delivery: 256, 512, 1024 (0: auto) */
    uint32_t grid;         /* workgroups of the tiled delivery (0: auto) */
    uint32_t synapse_weights; /* 0: auto -- when every projection from a source population
                                 has the same weight, store only the 4-byte target per
                                 synapse and one weight per source (Table I layout);
                                 1: a Q16 weight per synapse as well (8 bytes per synapse) */
    uint32_t plasticity;   /* SNN_PLASTICITY_*: how STDP weights are kept current */
} snn_params;

/* Optional device-memory provider (e.g. a framework's caching allocator).  alloc
 * returns NULL on failure; memory must be usable on the build stream. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, size_t bytes, void *stream, void *ctx);
    void *ctx;
} snn_allocator;

typedef struct snn_network snn_network;

typedef struct {
    uint32_t n;             /* neurons */
    uint32_t delay;         /* d */
    uint32_t queue_slots;   /* spike queues held by the FIFO ring */
    uint32_t input_buffers; /* Q16 input accumulators, one per pending arrival step */
    uint32_t window;        /* steps advanced per update launch */
    uint32_t delivery;      /* SNN_DELIVERY_ATOMIC or SNN_DELIVERY_TILED */
    uint32_t tiles;         /* target tiles (tiled delivery) */
    uint32_t plastic;       /* 1 if any projection is plastic (FP32 weights) */
    uint32_t raster_steps;  /* raster ring capacity */
    uint32_t raster_words;  /* uint64 words per raster row = ceil(n / 64) */
    uint32_t table_len;     /* entries of the drive's inverse-CDF table */
    uint32_t queue_groups;  /* sub-queues per spike queue */
    uint32_t queue_stride;  /* entries per queue slot (queue_groups equal sub-queues) */
    uint32_t source_weights; /* 1: one weight per source neuron, 4 bytes per synapse */
    uint64_t nnz;           /* synapses */
    uint64_t t;             /* steps simulated */
    uint64_t events;        /* synaptic events delivered (sum of out-degrees of delivered spikes) */
    uint64_t spikes;        /* spikes dequeued and delivered */
    uint64_t touches;       /* plastic synapse updates */
    uint64_t device_bytes;  /* device memory held */
    double build_ms;        /* host wall time of snn_build_network (allocation included) */
    float gen_rows_ms;      /* device time of the row-length pass and its scan */
    float gen_fill_ms;      /* device time of the synapse fill */
    float index_ms;         /* device time of the delivery indexes (in-edge index with STDP,
                               tile offsets of the tiled delivery; stream time between two
                               events, host allocation gaps included) */
    uint32_t tile_offset_bytes; /* bytes per stored tile boundary of the tiled delivery: 2
                                   (every row below 65,536 synapses) or 4; 0 without tiles */
    uint32_t target_bytes;  /* bytes per target the delivery reads: 2 for the tiled delivery
                               (a 16-bit copy of the targets, held beside the 4-byte
                               array), 4 for the atomic delivery */
    uint32_t plasticity;    /* SNN_PLASTICITY_* of a plastic network */
} snn_info;

/* Host views for reading or writing the dynamic state; NULL members are skipped.
 * Sizes: v, ref, x_pre, x_post: n; input: input_buffers * n (buffer b holds the
 * Q16 input of the steps u with u mod input_buffers == b); queue: queue_slots *
 * queue_stride (slot s holds queue_groups sub-queues of queue_stride / queue_groups
 * entries); queue_len: queue_slots * queue_groups sub-queue lengths; w_f32: nnz
 * (plastic networks only). */
typedef struct {
    float *v;
    int32_t *ref;
    int32_t *input;
    float *x_pre;
    float *x_post;
    int32_t *queue;
    uint32_t *queue_len;
    float *w_f32;
} snn_state;

/* Accumulated device time of each kernel kind while profiling is on (hipEvents
 * around every launch on the network's stream). */
typedef struct {
    double update_ms, deliver_ms, stdp_ms;
    uint64_t update_launches, deliver_launches, stdp_launches;
} snn_profile;

/* Build a network: validate, allocate, generate the synapses on the device from the
 * seed, initialise neurons (Init stage of Sec. III-A.1).  pops/proj are read only.
 * Errors: SNN_E_INVALID (parameters), SNN_E_OOM, SNN_E_HIP.  On success *out owns
 * all device memory; release it with snn_destroy. */
snn_status snn_build_network(const snn_params *prm, const snn_population *pops, uint32_t n_pops,
                             const snn_projection *proj, uint32_t n_proj,
                             const snn_allocator *alloc, void *stream, snn_network **out);

/* Step (b) of the generator of Fig. 2 (Sec. III-A.2) as the fixed out-degree fill
 * evaluates it: gaps[k] = floor(-ln(u) 2^24) with u = ((words[k] >> 8) + 1) 2^-24 and
 * -ln the library's fixed binary64 logarithm (2 atanh series after reduction to
 * [sqrt(1/2), sqrt(2)), the same for every caller).  words and gaps are device
 * pointers to n uint32 each (4-byte aligned; not overlapping), owned by the caller;
 * the kernel is queued on `stream` (NULL: the default stream) and the call returns
 * without waiting.  SNN_E_INVALID for NULL pointers with n > 0, SNN_E_HIP if the
 * launch fails.  Exists so that the fill's gap evaluation can be checked on every one
 * of its 2^24 inputs. */
snn_status snn_spacing_gaps(const uint32_t *words, uint64_t n, uint32_t *gaps, void *stream);

/* Advance one step t -> t+1 (Fig. 1: update neurons, FIFO, [update synapses],
 * receive spikes).  Asynchronous. */
snn_status snn_step(snn_network *net);

/* Advance n_steps steps: the loop of repeated step() calls that drives a network in
 * the paper's interface (Sec. III-B, the listing that ends in `while (true)
 * net.step()`), each step being the Fig. 1 pipeline.  Launches are grouped into windows
 * of up to `window` steps and replayed from a captured HIP graph where possible.  The
 * result is identical to n_steps calls of snn_step.  Asynchronous.  SNN_E_STATE for a
 * batch member; SNN_E_HIP if a launch fails. */
snn_status snn_run(snn_network *net, uint32_t n_steps);

/* Download of timestamped spikes (Sec. III-B: the simulators compared there let the
 * user download the spikes of a run with their time stamps): the spikes of steps
 * [t_begin, t_end) as (step, id) pairs sorted by step, then by id, written to the
 * caller's host arrays steps[] and ids[] (capacity entries each).  *n_spikes always
 * receives the number of spikes in the range.  Synchronises the network's stream.
 * Errors: SNN_E_INVALID if t_end < t_begin, if the range reaches past the simulated
 * steps or is no longer held by the raster ring (raster_steps most recent steps), or if
 * an output array is NULL while the range holds spikes; SNN_E_OVERFLOW if capacity is
 * below the count (nothing is written; call again with *n_spikes entries). */
snn_status snn_get_raster(snn_network *net, uint64_t t_begin, uint64_t t_end, uint32_t *steps,
                          uint32_t *ids, uint64_t capacity, uint64_t *n_spikes);

/* Raw raster rows: words[(t - t_begin) * raster_words + i / 64] bit (i % 64) is set iff
 * neuron i spiked at step t.  words holds (t_end - t_begin) * raster_words uint64. */
snn_status snn_get_raster_bits(snn_network *net, uint64_t t_begin, uint64_t t_end,
                               uint64_t *words);

snn_status snn_get_info(snn_network *net, snn_info *info);
snn_status snn_get_state(snn_network *net, const snn_state *state);
snn_status snn_set_state(snn_network *net, const snn_state *state);

/* Synapses of one source neuron: its sorted targets and weights (Q16 for static
 * networks, FP32 for plastic ones; either pointer may be NULL).  SNN_E_OVERFLOW with
 * *len = row length if cap is too small. */
snn_status snn_get_row(snn_network *net, uint32_t i, int32_t *col, int32_t *w_q16, float *w_f32,
                       uint64_t cap, uint64_t *len);

/* The whole CSR: row_ptr[n+1], col[nnz] and the weights (either may be NULL). */
snn_status snn_get_synapses(snn_network *net, uint64_t *row_ptr, int32_t *col, int32_t *w_q16,
                            float *w_f32);

/* The drive's inverse-CDF table (table_len entries, 2^32 marks the last). */
snn_status snn_get_drive_table(snn_network *net, uint64_t *table, uint32_t cap);

snn_status snn_set_profiling(snn_network *net, int32_t on);
snn_status snn_get_profile(snn_network *net, snn_profile *prof);
snn_status snn_reset_profile(snn_network *net);
snn_status snn_sync(snn_network *net);

/* Deliver a caller-given spike list with the network's delivery kernel as one window of
 * `steps` emission steps (0: the network's window) into scratch accumulators, `reps`
 * times; returns the mean kernel time in ms (HIP events) and the events of one launch.
 * With step_counts == NULL the ids are spread round-robin over the steps; otherwise
 * step w dequeues the next step_counts[w] ids (the counts sum to n_ids).  The network's
 * own state is left unchanged.  Used to measure the delivery kernel alone at a chosen
 * load. */
snn_status snn_time_delivery(snn_network *net, const uint32_t *ids_host, uint32_t n_ids,
                             const uint32_t *step_counts, uint32_t steps, uint32_t reps,
                             double *avg_ms, uint64_t *events);

/* snn_time_delivery for callers that cannot allocate device memory (code that must not
 * call hipMalloc: tight measurement or serving loops, harnesses that forbid it).  Same
 * arguments, checks and results, except that the mean time runs from the first timed
 * launch's begin to the last one's end (back-to-back launches).  Every device buffer
 * (the staged queues and counters, the control block, the input accumulators and the
 * copied ids) lives in one fixed 64 MiB device array that each GPU holds for the life of
 * the process; the call allocates no device memory (its first call on a GPU looks the
 * array up and creates two timing events).  SNN_E_INVALID if the window needs more than
 * 64 MiB: 49,408 + steps * (2,048 + 4 * queue_stride) + 4 * input_buffers * n +
 * 4 * n_ids bytes, each part rounded up to 256.  Every call on a GPU shares its array and
 * clears what it uses first; calls that overlap on one GPU (other threads or streams)
 * race and must not be made.  Synchronises the network's stream, so it cannot be
 * captured into a graph. */
snn_status snn_time_delivery_static(snn_network *net, const uint32_t *ids_host, uint32_t n_ids,
                                    const uint32_t *step_counts, uint32_t steps, uint32_t reps,
                                    double *avg_ms, uint64_t *events);

/* Switch a network's delivery variant (SNN_DELIVERY_*; AUTO picks by size and
 * degree), its base tiles, workgroup size and grid (0 = auto), from the next step on.
 * Rebuilds the tile boundaries; the simulation state is unchanged.  SNN_E_INVALID for
 * an impossible configuration; SNN_E_STATE for a network with lazy plasticity, which
 * delivers inside its own kernel. */
snn_status snn_set_delivery(snn_network *net, uint32_t delivery, uint32_t tiles, uint32_t block,
                            uint32_t grid);

typedef struct {
    uint32_t delivery, tiles, block, grid;  /* the configuration kept */
    double ms_per_launch;                   /* its mean delivery time on the sample */
    uint64_t events_per_launch;             /* synaptic events of the sample */
} snn_delivery_tuning;

/* Time the atomic variant and the tiled one over base tiles of about 384, 576 and
 * 768 targets (ranges of up to 32) x 512/1024-thread workgroups x 1, 2 and 3
 * workgroups per CU (the tiled ones for networks of at least 1,024 neurons), each on
 * the spikes of the network's latest window (taken from its raster), `reps` launches
 * each, on scratch queues and accumulators; keep the fastest and return it.  The
 * simulation state (weights and traces included) is unchanged.  SNN_E_STATE if fewer
 * than `window` steps have run, or for a network with lazy plasticity. */
snn_status snn_autotune_delivery(snn_network *net, uint32_t reps, snn_delivery_tuning *chosen);

void snn_destroy(snn_network *net);
/* Message of the last failing call on the calling thread (thread-local storage owned by
 * the library, valid until the next call on that thread).  `net` may be NULL: the
 * message does not depend on it. */
const char *snn_last_error(const snn_network *net);

/* ---- Device-memory cache (Sec. IV: allocate only when necessary, with hysteresis) ---
 *
 * Networks, batches and BPTT plans built without an allocator callback take device
 * memory from the library's cache.  Destroying them keeps their blocks.  A later
 * request on the same device is served by the smallest kept block that is at least as
 * large and at most twice as large (plus 1 MiB); otherwise it is served by hipMalloc.
 * So back-to-back experiments pay for allocation once.  When hipMalloc fails, the
 * device's kept blocks are released and the request is retried once.  Blocks are kept
 * only after their stream has drained.
 *
 * snn_memory_cache_stats: bytes and blocks kept on `device`, and the requests served
 * from the cache (hits) and by hipMalloc (misses) since the process started; NULL
 * outputs are skipped.  snn_memory_cache_release: return the kept blocks of `device`
 * (every device if negative) to HIP.  Neither call touches memory that is in use. */
snn_status snn_memory_cache_stats(int device, uint64_t *bytes, uint64_t *blocks, uint64_t *hits,
                                  uint64_t *misses);
snn_status snn_memory_cache_release(int device);

/* ---- Batched form: many independent static networks, one persistent launch -------
 *
 * Parameter sweeps and seed studies run hundreds of small networks of uneven size.
 * One at a time they leave most of the GPU idle, so a batch steps all of them in one
 * persistent kernel (captured in a HIP graph and replayed): each workgroup owns one
 * network for the whole launch and runs its step pipeline (update, spike queue, delay
 * ring, delivery) with the delay ring of Q16 accumulators in LDS.  Every network has
 * exactly the semantics of snn_build_network + snn_run with the same parameters
 * (same synapses, same spikes, same state). */
typedef struct snn_batch snn_batch;

typedef struct {
    const snn_params *params;      /* raster_steps, window, delivery, tiles, block and
                                      grid are ignored (the batch sets them) */
    const snn_population *pops;
    const snn_projection *proj;
    uint32_t n_pops, n_proj;
} snn_batch_member;

/* Launch shape of the batch kernel, chosen by snn_batch_autotune or set by hand. */
typedef struct {
    uint32_t block;        /* workgroup size: 256, 512 or 1024 */
    uint32_t per_lane;     /* neurons per lane (output; derived from block and the largest network) */
    uint32_t degree_div;   /* lanes per spike = the power of two >= mean out-degree / degree_div,
                              clamped to [1, 64]: 1, 2, 4, 8 or 16 */
    uint32_t pad_;
    double ms_per_step;    /* output of snn_batch_autotune: measured time of the chosen shape */
} snn_batch_tuning;

/* Build every member (validated and generated exactly as snn_build_network does) and
 * the batch around them.  Members must be static (no plastic projection) and each
 * must fit one workgroup: n <= 20,480 neurons (held in registers) and
 * (delay * n + drive thresholds) * 4 bytes of delay ring within the workgroup LDS
 * limit (160 KB on MI355X).  raster_steps is each member's raster ring.  Errors as
 * snn_build_network; SNN_E_INVALID names the member that does not fit. */
snn_status snn_build_batch(const snn_batch_member *nets, uint32_t n_nets, uint32_t raster_steps,
                           const snn_allocator *alloc, void *stream, snn_batch **out);

/* Advance every network of the batch by n_steps steps (asynchronous). */
snn_status snn_batch_run(snn_batch *b, uint32_t n_steps);
snn_status snn_batch_sync(snn_batch *b);

/* Member k as a network handle owned by the batch: every reader (snn_get_info,
 * snn_get_raster*, snn_get_state, snn_get_row, snn_get_synapses, ...) and
 * snn_set_state work on it; snn_step, snn_run and snn_time_delivery return
 * SNN_E_STATE, and snn_destroy ignores it. */
snn_status snn_batch_network(snn_batch *b, uint32_t k, snn_network **net);

/* Time each candidate launch shape (block 256/512/1024 x degree_div 1..16) over
 * trial_steps steps from the current state without changing it (nothing is written
 * back and no raster row is written), keep the fastest and return it. */
snn_status snn_batch_autotune(snn_batch *b, uint32_t trial_steps, snn_batch_tuning *chosen);
snn_status snn_batch_set_tuning(snn_batch *b, const snn_batch_tuning *tuning);
snn_status snn_batch_get_tuning(snn_batch *b, snn_batch_tuning *tuning);

void snn_batch_destroy(snn_batch *b);

/* ---- Surrogate-gradient BPTT of a recurrent LIF network --------------------------
 *
 * Training needs gradients through spikes, which are discontinuous (Sec. I); this form
 * replaces the spike's derivative by a fast-sigmoid surrogate.  Model, per batch
 * element, steps t = 0 .. steps-1, with V, s, U zero before step 0:
 *   I_t = W_in^T x_t + W_rec^T s_{t-1}            (sparse CSR weights, FP32)
 *   V_t = beta V_{t-1} + I_t - theta s_{t-1}      (reset by subtraction)
 *   s_t = H(V_t - theta)                          (smooth = 0; H(0) = 1)
 *       = 1/2 + 1/2 a/(1+|a|), a = slope (V_t - theta)   (smooth = 1)
 *   U_t = beta_out U_{t-1} + W_out^T s_t          (dense [n_hidden][n_out] readout)
 *   loss = mean_b cross-entropy(max_t U_t[b], label_b)
 * The backward pass is the adjoint recurrence of this model with
 * d s/d V = 1/(1 + slope |V - theta|)^2 and the reset term detached (smooth = 0), or
 * the exact derivative with the reset term (smooth = 1, for finite-difference checks).
 * The forward keeps every step's s and the membrane state at the end of every
 * `checkpoint` steps; the backward recomputes each segment's membranes from its
 * checkpoint.  The current into neuron j sums its in-edges in ascending source order,
 * input projection first, one term at a time; the readout sums ascending; the maximum
 * over time is taken at its first step. */
typedef struct snn_bptt snn_bptt;

typedef struct {
    uint32_t batch;        /* 1..64 */
    uint32_t steps, n_in, n_hidden, n_out;  /* steps 1..65,535; n_out 1..1,024 */
    uint32_t checkpoint;   /* steps per checkpoint segment, 1..32 */
    float beta, beta_out, theta, slope;
    uint32_t smooth;       /* 0: spiking forward, surrogate backward; 1: smooth forward */
    uint32_t eager;        /* 0: replay the per-step kernels of each pass from a HIP graph
                              captured at the plan's first call; 1: launch them one by one
                              (same kernels, same results) */
} snn_bptt_desc;

/* A plan for one network structure: host CSR arrays (rows = presynaptic neuron, targets
 * strictly ascending) of the input (n_in rows, targets < n_hidden) and recurrent
 * (n_hidden rows) weights.  The plan owns its device workspace; weights are passed to
 * each call.  SNN_E_INVALID for invalid sizes or CSR arrays. */
snn_status snn_bptt_create(const snn_bptt_desc *desc, const uint64_t *in_row_ptr, const int32_t *in_col,
                           const uint64_t *rec_row_ptr, const int32_t *rec_col,
                           const snn_allocator *alloc, void *stream, snn_bptt **out);

/* Forward pass on device arrays: x [batch][steps][n_in] (0/1), w_in [nnz_in] and
 * w_rec [nnz_rec] in CSR order, w_out [n_hidden][n_out], labels [batch] int32 in
 * [0, n_out); writes the mean loss to *loss (device).  Asynchronous on `stream`
 * (NULL: the plan's stream).  The plan keeps the trajectory for the next backward. */
snn_status snn_bptt_forward(snn_bptt *p, const float *x, const float *w_in, const float *w_rec,
                            const float *w_out, const int32_t *labels, float *loss, void *stream);

/* Backward pass of the latest forward pass (same weights): writes dloss/dw_in [nnz_in],
 * dloss/dw_rec [nnz_rec] and dloss/dw_out [n_hidden][n_out] (device), each scaled by
 * *g_loss (device scalar; NULL = 1).  SNN_E_STATE before any forward pass. */
snn_status snn_bptt_backward(snn_bptt *p, const float *w_in, const float *w_rec, const float *w_out,
                             const float *g_loss, float *g_w_in, float *g_w_rec, float *g_w_out,
                             void *stream);

/* Host copies of the latest forward pass (any pointer may be NULL): spikes
 * [steps][n_hidden][64] (batch innermost, lanes >= batch unused), membrane checkpoints
 * [ceil(steps/checkpoint)][n_hidden][64], readout maxima and their steps
 * [batch][n_out].  Synchronises the stream. */
snn_status snn_bptt_get_trace(snn_bptt *p, float *spikes, float *v_checkpoints, float *readout_max,
                              int32_t *readout_argmax, void *stream);

void snn_bptt_destroy(snn_bptt *p);

#ifdef __cplusplus
}
#endif
#endif
