/*
 * simulate.c -- oracle: one clock-driven step of the work-queue pipeline (Fig. 1,
 * Sec. III-A.1), written plainly: Update Neurons -> FIFO -> [Update Synapses] ->
 * Receive Spikes.  Test infrastructure only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "internal.h"

/* Number of virtual Poisson inputs that fire for neuron i at step t: inverse CDF of
 * the binomial table applied to word (t mod 4) of stream POISSON, block
 * (i, t/4, t/2^34). */
static int32_t drive_count(const orc_net *c, uint32_t i, uint64_t t) {
    if (c->table_len <= 1) return 0;
    uint32_t ctr[4] = {i, (uint32_t)(t >> 2), (uint32_t)(t >> 34), ORC_STREAM_POISSON}, r[4];
    orc_philox4x32_10(ctr, c->key, r);
    uint64_t word = r[t & 3];
    int32_t k = 0;
    while (word >= c->table[k]) ++k;
    return k;
}

/* Update Neurons (N_t -> N'_{t+1}, emitting S_t): leaky integrate-and-fire with the
 * input added before the exact exponential leak; refractory neurons hold V_reset
 * and discard input.  binary32, in exactly this operation order. */
static uint32_t update_neurons(const orc_net *c, uint64_t t, uint32_t n, float *v, int32_t *ref,
                               int32_t *input, float *x_pre, float *x_post,
                               uint64_t *raster_row, int32_t *queue) {
    uint32_t n_spikes = 0;
    if (raster_row) memset(raster_row, 0, sizeof(uint64_t) * ((n + 63) / 64));
    for (uint32_t i = 0; i < n; ++i) {
        if (ref[i] > 0) {
            ref[i] = ref[i] - 1;
            input[i] = 0;
        } else {
            int32_t k = drive_count(c, i, t);
            uint32_t sum = (uint32_t)input[i] + (uint32_t)k * (uint32_t)c->w_ext_q16;
            int32_t in = (int32_t)sum;
            input[i] = 0;
            float dv = (float)in * 0x1p-16f;
            float vv = v[i] + dv;
            float diff = vv - c->v_inf;
            float leak = diff * c->alpha;
            vv = c->v_inf + leak;
            if (vv >= c->v_th) {
                if (raster_row) raster_row[i >> 6] |= (uint64_t)1 << (i & 63);
                if (queue) queue[n_spikes] = (int32_t)i;
                ++n_spikes;
                vv = c->v_reset;
                ref[i] = c->ref_steps;
            }
            v[i] = vv;
        }
        if (c->plastic) {
            x_pre[i] = x_pre[i] * c->beta_plus;
            x_post[i] = x_post[i] * c->beta_minus;
        }
    }
    return n_spikes;
}

uint32_t orc_update_range(const orc_net *c, uint64_t t, uint32_t n, float *v, int32_t *ref,
                          int32_t *input, uint64_t *raster_row) {
    orc_net tmp = *c;
    tmp.plastic = 0;
    return update_neurons(&tmp, t, n, v, ref, input, NULL, NULL, raster_row, NULL);
}

static int32_t edge_weight_q16(const orc_net *c, uint64_t e) {
    if (c->w_q16) return c->w_q16[e];
    return (int32_t)nearbyintf(c->w_f32[e] * 65536.0f);
}

/* Update Synapses (Syn_t -> Syn_{t+1}), additive pair-based STDP with all-to-all
 * traces: presynaptic events are the arrivals S_{t-d}, postsynaptic events S_t.
 * Depression of each arriving neuron's plastic out-edges by A- x_post(target) first
 * (x_post not yet incremented for this step), then potentiation of each spiking
 * neuron's plastic in-edges by A+ x_pre(source) (x_pre including this step's
 * arrivals); weights clipped to [0, w_max]. */
static void update_synapses(orc_net *c, const int32_t *pre, uint32_t n_pre, const int32_t *post,
                            uint32_t n_post) {
    for (uint32_t s = 0; s < n_pre; ++s) c->x_pre[pre[s]] = c->x_pre[pre[s]] + 1.0f;
    for (uint32_t s = 0; s < n_pre; ++s) {
        uint32_t i = (uint32_t)pre[s];
        for (uint32_t k = 0; k < c->plast_len[i]; ++k) {
            uint64_t e = c->plast_lo[i] + k;
            float dw = c->a_minus * c->x_post[c->col[e]];
            float w = c->w_f32[e] - dw;
            if (w < 0.0f) w = 0.0f;
            c->w_f32[e] = w;
            ++c->touches;
        }
    }
    for (uint32_t s = 0; s < n_post; ++s) c->x_post[post[s]] = c->x_post[post[s]] + 1.0f;
    for (uint32_t s = 0; s < n_post; ++s) {
        uint32_t j = (uint32_t)post[s];
        for (uint64_t m = c->in_ptr[j]; m < c->in_ptr[j + 1]; ++m) {
            uint64_t e = c->in_edge[m];
            float dw = c->a_plus * c->x_pre[c->in_src[m]];
            float w = c->w_f32[e] + dw;
            if (w > c->w_max) w = c->w_max;
            c->w_f32[e] = w;
            ++c->touches;
        }
    }
}

/* Receive Spikes: every spike of the dequeued queue adds its synapses' Q16 weights to
 * the recipients' input accumulators (two's-complement wrap-around). */
static void receive_spikes(orc_net *c, const int32_t *spikes, uint32_t n_spikes) {
    for (uint32_t s = 0; s < n_spikes; ++s) {
        uint32_t i = (uint32_t)spikes[s];
        for (uint64_t e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) {
            uint32_t sum = (uint32_t)c->input[c->col[e]] + (uint32_t)edge_weight_q16(c, e);
            c->input[c->col[e]] = (int32_t)sum;
        }
        c->events += c->row_ptr[i + 1] - c->row_ptr[i];
    }
}

/* One pipeline iteration t -> t+1.  The FIFO holds d+1 queues: slot t mod (d+1)
 * receives S_t; S_{t-d+1} is delivered (its spikes are integrated by the update of
 * step t+1, i.e. d steps after emission); S_{t-d} feeds plasticity. */
static void step(orc_net *c) {
    uint64_t t = c->t;
    uint32_t n = c->n, slots = c->n_slots, d = c->delay;
    uint32_t cur = (uint32_t)(t % slots);
    uint64_t *row = c->raster + (size_t)(t % c->raster_cap) * c->raster_words;
    int32_t *q_cur = c->queue + (size_t)cur * n;
    c->queue_len[cur] = update_neurons(c, t, n, c->v, c->ref, c->input, c->x_pre, c->x_post,
                                       row, q_cur);
    if (c->plastic) {
        const int32_t *pre = NULL;
        uint32_t n_pre = 0;
        if (t >= d) {
            uint32_t s = (uint32_t)((t - d) % slots);
            pre = c->queue + (size_t)s * n;
            n_pre = c->queue_len[s];
        }
        update_synapses(c, pre, n_pre, q_cur, c->queue_len[cur]);
    }
    if (t + 1 >= d) {
        uint32_t s = (uint32_t)((t + 1 - d) % slots);
        receive_spikes(c, c->queue + (size_t)s * n, c->queue_len[s]);
    }
    c->t = t + 1;
}

void orc_run(orc_net *c, uint32_t n_steps) {
    for (uint32_t k = 0; k < n_steps; ++k) step(c);
}

void orc_view_get(orc_net *c, orc_view *w) {
    memset(w, 0, sizeof(*w));
    w->n = c->n;
    w->delay = c->delay;
    w->n_slots = c->n_slots;
    w->raster_cap = c->raster_cap;
    w->raster_words = c->raster_words;
    w->plastic = (uint32_t)c->plastic;
    w->table_len = c->table_len;
    w->nnz = c->nnz;
    w->t = c->t;
    w->events = c->events;
    w->touches = c->touches;
    w->v = c->v; w->x_pre = c->x_pre; w->x_post = c->x_post; w->w_f32 = c->w_f32;
    w->ref = c->ref; w->input = c->input; w->col = c->col; w->w_q16 = c->w_q16;
    w->row_ptr = c->row_ptr; w->raster = c->raster; w->table = c->table;
    w->queue_len = c->queue_len; w->queue = c->queue;
    w->alpha = c->alpha; w->v_inf = c->v_inf; w->v_th = c->v_th; w->v_reset = c->v_reset;
    w->beta_plus = c->beta_plus; w->beta_minus = c->beta_minus;
    w->a_plus = c->a_plus; w->a_minus = c->a_minus; w->w_max = c->w_max;
    w->ref_steps = c->ref_steps; w->w_ext_q16 = c->w_ext_q16;
}

uint64_t orc_deliver_generated(const orc_params *prm, const orc_pop *pops, uint32_t n_pops,
                               const orc_proj *proj, uint32_t n_proj, const uint32_t *spikes,
                               uint32_t n_spikes, int32_t *input) {
    orc_net c;
    char err[128];
    if (orc_validate_and_derive(&c, prm, pops, n_pops, proj, n_proj, 1, err, sizeof err)) {
        orc_free_fields(&c);
        return (uint64_t)-1;
    }
    uint64_t events = 0;
    int64_t cap = 1 << 16;
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * cap);
    int32_t *wq = (int32_t *)malloc(sizeof(int32_t) * cap);
    float *wf = (float *)malloc(sizeof(float) * cap);
    for (uint32_t s = 0; s < n_spikes; ++s) {
        int64_t len = orc_row_into(&c, spikes[s], col, wq, wf, NULL, NULL, cap);
        if (len > cap) {
            cap = len;
            col = (int32_t *)realloc(col, sizeof(int32_t) * cap);
            wq = (int32_t *)realloc(wq, sizeof(int32_t) * cap);
            wf = (float *)realloc(wf, sizeof(float) * cap);
            len = orc_row_into(&c, spikes[s], col, wq, wf, NULL, NULL, cap);
        }
        for (int64_t e = 0; e < len; ++e) {
            int32_t w = c.plastic ? (int32_t)nearbyintf(wf[e] * 65536.0f) : wq[e];
            input[col[e]] = (int32_t)((uint32_t)input[col[e]] + (uint32_t)w);
        }
        events += (uint64_t)len;
    }
    free(col); free(wq); free(wf);
    orc_free_fields(&c);
    return events;
}
