/*
 * oracle.h -- plain, single-threaded CPU reference of the clock-driven work-queue
 * SNN simulation of Bautembach et al., "Faster and Simpler SNN Simulation with Work
 * Queues" (IJCNN 2020), Sec. III-A.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU library:
 * its Philox, logarithm, generators, Poisson table, LIF update, FIFO, delivery and
 * STDP are written here, from the definitions, a second time.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math: IEEE binary32/64,
 * round-to-nearest-even, denormals kept).  Every function is deterministic.
 *
 * Parity status of each function (what pins it, see tests/test_oracle_*.py):
 *   orc_philox4x32_10   pinned: published known-answer vectors of Philox4x32-10.
 *   orc_neg_log         pinned: libm log() to 2 ulp on random and edge arguments.
 *   orc_spacing_core    pinned: the worked example of Fig. 2 (steps (a)-(g)).
 *   orc_gen_row         pinned: sortedness/uniqueness/range/self-loop, ER edge-count
 *                       and in-degree statistics, p=0 / p=1 closed forms,
 *                       fixed-degree endpoint/position statistics.
 *   orc_binom_table     pinned: scipy.stats.binom.cdf.
 *   orc_create/orc_run  pinned: closed-form LIF trajectory under constant drive,
 *                       closed-form tonic firing period with refractoriness, dense
 *                       brute-force propagation (int64 mat-vec) incl. delays, the
 *                       ping-pong model of Listing 1, FIFO delay invariants, exact
 *                       event counts, closed-form pair STDP and all-pairs STDP sums.
 *   V0 initialisation   pinned: every value in [lo, hi] (binary32 rounding of
 *                       lo + span u can give hi itself), Kolmogorov-Smirnov test against
 *                       U(lo, hi), mean and variance within 5 standard errors over
 *                       1e5 neurons for several seeds and ranges, independence of the
 *                       network size and of other seeds; planted mistakes (span = hi,
 *                       the unshifted word) fail it.
 *   plastic delivery    pinned: FP32 weights at exact Q16 ties (x.5 2^-16 mV, both
 *                       signs) deliver the round-half-even value; truncation, floor,
 *                       half-up and half-away each fail it.
 */
#ifndef SNN_ORACLE_H
#define SNN_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox stream identifiers (counter word 3). */
#define ORC_STREAM_CONN 1u
#define ORC_STREAM_VINIT 2u
#define ORC_STREAM_POISSON 3u

#define ORC_PROJ_ER 0u        /* Erdos-Renyi: each ordered pair (i,j), j != i, with prob. p */
#define ORC_PROJ_FIXED_OUT 1u /* fixed out-degree k, targets uniform without replacement */

typedef struct {
    uint32_t size;
    uint32_t excitatory; /* informational; weights come from projections */
} orc_pop;

typedef struct {
    uint32_t from, to;  /* source population; first target population */
    uint32_t kind;      /* ORC_PROJ_ER or ORC_PROJ_FIXED_OUT */
    uint32_t k;         /* out-degree for ORC_PROJ_FIXED_OUT */
    double p;           /* connection probability for ORC_PROJ_ER */
    double w_mV;        /* synaptic weight (mV) */
    uint32_t plastic;   /* STDP on this projection */
    uint32_t to_span;   /* targets: populations [to, to + to_span) (0 means 1) */
} orc_proj;

typedef struct {
    double dt_ms;
    uint32_t delay_steps; /* D >= 1 */
    uint32_t n_ext;       /* virtual Poisson inputs per neuron (0 = no drive) */
    double tau_m_ms, v_rest_mV, v_bg_mV, v_th_mV, v_reset_mV, t_ref_ms;
    double v0_lo_mV, v0_hi_mV;
    double rate_ext_hz, w_ext_mV;
    double tau_plus_ms, tau_minus_ms, a_plus, a_minus, w_max_mV;
    uint64_t seed;
} orc_params;

typedef struct orc_net orc_net;

/* A read/write view of the oracle's state (pointers owned by the oracle). */
typedef struct {
    uint32_t n, delay, n_slots, raster_cap, raster_words, plastic, table_len, pad_;
    uint64_t nnz, t, events, touches;
    float *v, *x_pre, *x_post, *w_f32;
    int32_t *ref, *input, *col, *w_q16;
    uint64_t *row_ptr, *raster, *table;
    uint32_t *queue_len;  /* [n_slots] */
    int32_t *queue;       /* [n_slots][n] */
    /* derived constants */
    float alpha, v_inf, v_th, v_reset, beta_plus, beta_minus, a_plus, a_minus, w_max;
    int32_t ref_steps, w_ext_q16;
} orc_view;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_neg_log(double u);
/* Fig. 2 pipeline on n+1 given uniforms u[0..n] in (0,1]: S[0..n+1] (fixed point, 2^-24)
 * and x[0..n-1] = n sorted distinct integers in [0, n + spare). */
void orc_spacing_core(const double *u, uint32_t n, uint64_t spare, uint64_t *S, int64_t *x);
/* Binomial(n, p) inverse-CDF thresholds; returns the table length (<= cap) or 0. */
uint32_t orc_binom_table(uint32_t n, double p, uint64_t *tbl, uint32_t cap);

/* Generate the sorted out-row of neuron i without building the network.  Returns the
 * row length, or -1 if cap is too small / parameters invalid. */
int64_t orc_gen_row(const orc_params *prm, const orc_pop *pops, uint32_t n_pops,
                    const orc_proj *proj, uint32_t n_proj, uint32_t i, int32_t *col,
                    int32_t *w_q16, float *w_f32, int64_t cap);

orc_net *orc_create(const orc_params *prm, const orc_pop *pops, uint32_t n_pops,
                    const orc_proj *proj, uint32_t n_proj, uint32_t raster_cap,
                    char *err, size_t err_len);
void orc_destroy(orc_net *net);
void orc_view_get(orc_net *net, orc_view *view);
void orc_run(orc_net *net, uint32_t n_steps);

/* Stage functions on plain arrays, used to check single transitions of a large
 * network from a snapshot without simulating it end to end. */
/* One neuron update of step t for neurons [0, n): reads input[], writes v, ref,
 * input (zeroed), and the raster word row; returns the number of spikes. */
uint32_t orc_update_range(const orc_net *constants_from, uint64_t t, uint32_t n, float *v,
                          int32_t *ref, int32_t *input, uint64_t *raster_row);
/* Deliver the given spike list into input[] (int32, wrapping) using rows generated on
 * the fly; returns the number of synaptic events. */
uint64_t orc_deliver_generated(const orc_params *prm, const orc_pop *pops, uint32_t n_pops,
                               const orc_proj *proj, uint32_t n_proj, const uint32_t *spikes,
                               uint32_t n_spikes, int32_t *input);
/* A constants-only network (no synapses) for orc_update_range. */
orc_net *orc_create_neurons_only(const orc_params *prm, const orc_pop *pops,
                                 uint32_t n_pops, char *err, size_t err_len);

#ifdef __cplusplus
}
#endif
#endif
