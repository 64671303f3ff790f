/*
 * network.c -- oracle: parameter validation, derived constants and network
 * construction (the "Init" stage of Sec. III-A.1; adjacency of Sec. III-A.2).
 * Test infrastructure only.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "internal.h"

static int fail(char *err, size_t err_len, const char *msg) {
    if (err && err_len) snprintf(err, err_len, "%s", msg);
    return -1;
}

static void key_of(uint64_t seed, uint32_t key[2]) {
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
}

/* Q16 fixed point (units of 2^-16 mV), rounded half to even in binary64. */
static int to_q16(double w_mV, int32_t *out) {
    double s = nearbyint(w_mV * 65536.0);
    if (!(s > -2147483648.0 && s < 2147483647.0)) return -1;
    *out = (int32_t)s;
    return 0;
}

int orc_validate_and_derive(orc_net *c, const orc_params *prm, const orc_pop *pops,
                            uint32_t n_pops, const orc_proj *proj, uint32_t n_proj,
                            int need_synapses, char *err, size_t err_len) {
    memset(c, 0, sizeof(*c));
    c->prm = *prm;
    if (!(prm->dt_ms > 0.0)) return fail(err, err_len, "dt_ms must be > 0");
    if (prm->delay_steps < 1) return fail(err, err_len, "delay_steps must be >= 1");
    if (!(prm->tau_m_ms > 0.0)) return fail(err, err_len, "tau_m_ms must be > 0");
    if (!(prm->t_ref_ms >= 0.0)) return fail(err, err_len, "t_ref_ms must be >= 0");
    if (n_pops == 0) return fail(err, err_len, "no populations");
    uint64_t n = 0;
    for (uint32_t a = 0; a < n_pops; ++a) {
        if (pops[a].size == 0) return fail(err, err_len, "empty population");
        n += pops[a].size;
    }
    if (n >= ((uint64_t)1 << 31)) return fail(err, err_len, "too many neurons");
    c->n = (uint32_t)n;
    c->n_pops = n_pops;
    c->n_proj = need_synapses ? n_proj : 0;
    c->pops = (orc_pop *)malloc(sizeof(orc_pop) * n_pops);
    c->pop_off = (uint32_t *)malloc(sizeof(uint32_t) * (n_pops + 1));
    c->proj = (orc_proj *)malloc(sizeof(orc_proj) * (n_proj ? n_proj : 1));
    memcpy(c->pops, pops, sizeof(orc_pop) * n_pops);
    c->pop_off[0] = 0;
    for (uint32_t a = 0; a < n_pops; ++a) c->pop_off[a + 1] = c->pop_off[a] + pops[a].size;
    if (need_synapses && n_proj) memcpy(c->proj, proj, sizeof(orc_proj) * n_proj);
    key_of(prm->seed, c->key);

    int plastic = 0;
    for (uint32_t q = 0; q < c->n_proj; ++q) {
        const orc_proj *pj = &proj[q];
        uint32_t span = pj->to_span ? pj->to_span : 1u;
        if (pj->from >= n_pops || pj->to >= n_pops || span > n_pops - pj->to)
            return fail(err, err_len, "bad population index");
        for (uint32_t r = 0; r < q; ++r) {
            uint32_t rs = proj[r].to_span ? proj[r].to_span : 1u;
            if (proj[r].from == pj->from && proj[r].to < pj->to + span && pj->to < proj[r].to + rs)
                return fail(err, err_len, "overlapping projections from one population");
        }
        int32_t wq;
        if (to_q16(pj->w_mV, &wq)) return fail(err, err_len, "weight out of Q16 range");
        uint64_t tsize = (uint64_t)c->pop_off[pj->to + span] - c->pop_off[pj->to];
        int self_in = pj->from >= pj->to && pj->from < pj->to + span;
        uint64_t cand = tsize - (self_in ? 1u : 0u);
        if (pj->kind == ORC_PROJ_ER) {
            if (!(pj->p >= 0.0 && pj->p <= 1.0)) return fail(err, err_len, "p outside [0,1]");
        } else if (pj->kind == ORC_PROJ_FIXED_OUT) {
            if (pj->k > cand) return fail(err, err_len, "out-degree exceeds candidates");
            uint64_t spare = cand - pj->k;
            if (((uint64_t)pj->k + 1) * (2 * spare + 1) > ((uint64_t)1 << 35))
                return fail(err, err_len, "out-degree x population too large");
        } else {
            return fail(err, err_len, "unknown projection kind");
        }
        if (pj->plastic) {
            plastic = 1;
            for (uint32_t r = 0; r < n_proj; ++r)
                if (r != q && proj[r].plastic && proj[r].from == pj->from)
                    return fail(err, err_len, "two plastic projections from one population");
        }
    }
    c->plastic = plastic;
    c->delay = prm->delay_steps;
    c->n_slots = prm->delay_steps + 1;

    /* derived constants of the LIF neuron: exact exponential decay per step */
    c->alpha = (float)exp(-prm->dt_ms / prm->tau_m_ms);
    c->v_inf = (float)(prm->v_rest_mV + prm->v_bg_mV);
    c->v_th = (float)prm->v_th_mV;
    c->v_reset = (float)prm->v_reset_mV;
    double rs = nearbyint(prm->t_ref_ms / prm->dt_ms);
    if (rs > 1e9) return fail(err, err_len, "refractory period too long");
    c->ref_steps = (int32_t)rs;
    if (to_q16(prm->w_ext_mV, &c->w_ext_q16)) return fail(err, err_len, "w_ext out of range");
    if (plastic) {
        if (!(prm->tau_plus_ms > 0.0 && prm->tau_minus_ms > 0.0))
            return fail(err, err_len, "STDP time constants must be > 0");
        if (!(prm->w_max_mV >= 0.0)) return fail(err, err_len, "w_max must be >= 0");
        c->beta_plus = (float)exp(-prm->dt_ms / prm->tau_plus_ms);
        c->beta_minus = (float)exp(-prm->dt_ms / prm->tau_minus_ms);
        c->a_plus = (float)prm->a_plus;
        c->a_minus = (float)prm->a_minus;
        c->w_max = (float)prm->w_max_mV;
    }
    /* virtual Poisson drive: Binomial(n_ext, rate * dt) inputs per step */
    double p_ext = (prm->rate_ext_hz * prm->dt_ms) / 1000.0;
    if (prm->n_ext > 0 && !(p_ext >= 0.0 && p_ext <= 1.0)) return fail(err, err_len, "bad drive rate");
    c->table_len = orc_binom_table(prm->n_ext, p_ext, c->table, ORC_TABLE_CAP);
    if (c->table_len == 0) return fail(err, err_len, "drive table does not fit");
    return 0;
}

/* Out-row of neuron i: the edges of every projection leaving i's population, in
 * ascending order of target population, each sorted by target id (rows sorted for
 * locality, Sec. III-A.2).  Writes nothing past cap; returns the row length. */
int64_t orc_row_into(const orc_net *c, uint32_t i, int32_t *col, int32_t *w_q16,
                     float *w_f32, uint64_t *plast_lo_rel, uint32_t *plast_len, int64_t cap) {
    uint32_t a = 0;
    while (!(i >= c->pop_off[a] && i < c->pop_off[a + 1])) ++a;
    if (plast_lo_rel) *plast_lo_rel = 0;
    if (plast_len) *plast_len = 0;
    int64_t len = 0;
    for (uint32_t b = 0; b < c->n_pops; ++b) {
        const orc_proj *pj = NULL;
        for (uint32_t q = 0; q < c->n_proj; ++q)
            if (c->proj[q].from == a && c->proj[q].to == b) pj = &c->proj[q];
        if (!pj) continue;
        uint32_t span = pj->to_span ? pj->to_span : 1u;
        int32_t wq = 0;
        to_q16(pj->w_mV, &wq);
        float wf = (float)pj->w_mV;
        uint32_t off = c->pop_off[b], size = c->pop_off[b + span] - off;
        int self_in = (a >= b && a < b + span);
        int64_t start = len;
        if (pj->kind == ORC_PROJ_ER) {
            /* edge i->j iff the j-th word of stream CONN, block (i, j/4, 0) is below
             * floor(p * 2^32): one Bernoulli(p) trial per ordered pair */
            uint64_t thr = pj->p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)(pj->p * 4294967296.0);
            uint32_t blk[4] = {0, 0, 0, 0};
            uint32_t cur = 0xFFFFFFFFu;
            for (uint32_t j = off; j < off + size; ++j) {
                if (j == i) continue;
                if ((j >> 2) != cur) {
                    uint32_t ctr[4] = {i, j >> 2, 0u, ORC_STREAM_CONN};
                    orc_philox4x32_10(ctr, c->key, blk);
                    cur = j >> 2;
                }
                if ((uint64_t)blk[j & 3] < thr) {
                    if (len < cap) {
                        col[len] = (int32_t)j;
                        if (w_q16) w_q16[len] = wq;
                        if (w_f32) w_f32[len] = wf;
                    }
                    ++len;
                }
            }
        } else if (!col && !w_q16 && !w_f32) {
            len += pj->k; /* length only: every row of the projection has k edges */
        } else {
            /* fixed out-degree: Fig. 2 generator over the candidate targets of the
             * target range (self excluded), gap k drawn from word k of stream CONN,
             * block (i, k/4, 1 + b) with b the first target population */
            uint32_t k_out = pj->k;
            uint64_t cand = size - (self_in ? 1u : 0u);
            uint64_t spare = cand - k_out;
            double *u = (double *)malloc(sizeof(double) * (k_out + 1));
            uint64_t *S = (uint64_t *)malloc(sizeof(uint64_t) * (k_out + 2));
            int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (k_out + 1));
            uint32_t blk[4];
            for (uint32_t k = 0; k <= k_out; ++k) {
                if ((k & 3) == 0) {
                    uint32_t ctr[4] = {i, k >> 2, 1u + b, ORC_STREAM_CONN};
                    orc_philox4x32_10(ctr, c->key, blk);
                }
                u[k] = (double)((blk[k & 3] >> 8) + 1u) * 0x1p-24;
            }
            orc_spacing_core(u, k_out, spare, S, x);
            for (uint32_t k = 0; k < k_out; ++k) {
                int64_t local = x[k];
                if (self_in && local >= (int64_t)(i - off)) local += 1;
                if (len < cap) {
                    col[len] = (int32_t)(off + local);
                    if (w_q16) w_q16[len] = wq;
                    if (w_f32) w_f32[len] = wf;
                }
                ++len;
            }
            free(u);
            free(S);
            free(x);
        }
        if (pj->plastic) {
            if (plast_lo_rel) *plast_lo_rel = (uint64_t)start;
            if (plast_len) *plast_len = (uint32_t)(len - start);
        }
    }
    return len;
}

void orc_free_fields(orc_net *c) {
    free(c->pops); free(c->proj); free(c->pop_off);
    free(c->row_ptr); free(c->col); free(c->w_q16); free(c->w_f32);
    free(c->plast_lo); free(c->plast_len);
    free(c->in_ptr); free(c->in_src); free(c->in_edge);
    free(c->v); free(c->x_pre); free(c->x_post); free(c->ref); free(c->input);
    free(c->queue); free(c->queue_len); free(c->raster);
}

int64_t orc_gen_row(const orc_params *prm, const orc_pop *pops, uint32_t n_pops,
                    const orc_proj *proj, uint32_t n_proj, uint32_t i, int32_t *col,
                    int32_t *w_q16, float *w_f32, int64_t cap) {
    orc_net c;
    char err[128];
    if (orc_validate_and_derive(&c, prm, pops, n_pops, proj, n_proj, 1, err, sizeof err)) {
        orc_free_fields(&c);
        return -1;
    }
    int64_t len = -1;
    if (i < c.n) len = orc_row_into(&c, i, col, w_q16, w_f32, NULL, NULL, cap);
    orc_free_fields(&c);
    if (len > cap) return -1;
    return len;
}

/* Initial membrane potential: V = lo + (hi - lo) * u in binary32, u = (r >> 8) 2^-24
 * from word 0 of stream VINIT, block (i, 0, 0). */
static void init_neurons(orc_net *c) {
    float lo = (float)c->prm.v0_lo_mV;
    float span = (float)(c->prm.v0_hi_mV - c->prm.v0_lo_mV);
    for (uint32_t i = 0; i < c->n; ++i) {
        uint32_t ctr[4] = {i, 0u, 0u, ORC_STREAM_VINIT}, r[4];
        orc_philox4x32_10(ctr, c->key, r);
        float u = (float)(r[0] >> 8) * 0x1p-24f;
        float prod = span * u;
        c->v[i] = lo + prod;
        c->ref[i] = 0;
        c->input[i] = 0;
    }
}

static int alloc_state(orc_net *c, uint32_t raster_cap) {
    c->v = (float *)calloc(c->n, sizeof(float));
    c->ref = (int32_t *)calloc(c->n, sizeof(int32_t));
    c->input = (int32_t *)calloc(c->n, sizeof(int32_t));
    c->x_pre = (float *)calloc(c->n, sizeof(float));
    c->x_post = (float *)calloc(c->n, sizeof(float));
    c->queue = (int32_t *)calloc((size_t)c->n_slots * c->n, sizeof(int32_t));
    c->queue_len = (uint32_t *)calloc(c->n_slots, sizeof(uint32_t));
    c->raster_cap = raster_cap ? raster_cap : 1;
    c->raster_words = (c->n + 63) / 64;
    c->raster = (uint64_t *)calloc((size_t)c->raster_cap * c->raster_words, sizeof(uint64_t));
    return (c->v && c->ref && c->input && c->x_pre && c->x_post && c->queue && c->queue_len &&
            c->raster) ? 0 : -1;
}

orc_net *orc_create_neurons_only(const orc_params *prm, const orc_pop *pops,
                                 uint32_t n_pops, char *err, size_t err_len) {
    orc_net *c = (orc_net *)malloc(sizeof(orc_net));
    if (orc_validate_and_derive(c, prm, pops, n_pops, NULL, 0, 0, err, err_len) ||
        alloc_state(c, 1)) {
        orc_free_fields(c);
        free(c);
        return NULL;
    }
    init_neurons(c);
    return c;
}

orc_net *orc_create(const orc_params *prm, const orc_pop *pops, uint32_t n_pops,
                    const orc_proj *proj, uint32_t n_proj, uint32_t raster_cap,
                    char *err, size_t err_len) {
    orc_net *c = (orc_net *)malloc(sizeof(orc_net));
    if (orc_validate_and_derive(c, prm, pops, n_pops, proj, n_proj, 1, err, err_len)) {
        orc_free_fields(c);
        free(c);
        return NULL;
    }
    uint32_t n = c->n;
    c->row_ptr = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    c->plast_lo = (uint64_t *)calloc(n, sizeof(uint64_t));
    c->plast_len = (uint32_t *)calloc(n, sizeof(uint32_t));
    /* pass 1: row lengths, then their prefix sum.  Rows are independent, so the row
     * loops of both passes may run on several host threads (OpenMP) without changing
     * a single result. */
    c->row_ptr[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (uint32_t i = 0; i < n; ++i)
        c->row_ptr[i + 1] = (uint64_t)orc_row_into(c, i, NULL, NULL, NULL, NULL, NULL, 0);
    for (uint32_t i = 0; i < n; ++i) c->row_ptr[i + 1] += c->row_ptr[i];
    c->nnz = c->row_ptr[n];
    size_t alloc_nnz = c->nnz ? c->nnz : 1;
    c->col = (int32_t *)malloc(sizeof(int32_t) * alloc_nnz);
    if (c->plastic) c->w_f32 = (float *)malloc(sizeof(float) * alloc_nnz);
    else c->w_q16 = (int32_t *)malloc(sizeof(int32_t) * alloc_nnz);
    if (!c->col || (!c->w_f32 && !c->w_q16)) {
        fail(err, err_len, "out of host memory");
        orc_free_fields(c);
        free(c);
        return NULL;
    }
    /* pass 2: fill */
#pragma omp parallel for schedule(dynamic, 64)
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t b = c->row_ptr[i];
        int64_t len = (int64_t)(c->row_ptr[i + 1] - b);
        uint64_t plo = 0;
        orc_row_into(c, i, c->col + b, c->w_q16 ? c->w_q16 + b : NULL,
                     c->w_f32 ? c->w_f32 + b : NULL, &plo, &c->plast_len[i], len);
        c->plast_lo[i] = b + plo;
    }
    /* plastic in-edges grouped by target (the transposed index used for potentiation) */
    if (c->plastic) {
        c->in_ptr = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t k = 0; k < c->plast_len[i]; ++k)
                c->in_ptr[c->col[c->plast_lo[i] + k] + 1]++;
        for (uint32_t j = 0; j < n; ++j) c->in_ptr[j + 1] += c->in_ptr[j];
        uint64_t m = c->in_ptr[n];
        c->in_src = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
        c->in_edge = (uint64_t *)malloc(sizeof(uint64_t) * (m ? m : 1));
        uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * n);
        for (uint32_t j = 0; j < n; ++j) fill[j] = c->in_ptr[j];
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t k = 0; k < c->plast_len[i]; ++k) {
                uint64_t e = c->plast_lo[i] + k;
                uint64_t slot = fill[c->col[e]]++;
                c->in_src[slot] = (int32_t)i;
                c->in_edge[slot] = e;
            }
        free(fill);
    }
    if (alloc_state(c, raster_cap)) {
        fail(err, err_len, "out of host memory");
        orc_free_fields(c);
        free(c);
        return NULL;
    }
    init_neurons(c);
    return c;
}

void orc_destroy(orc_net *c) {
    if (!c) return;
    orc_free_fields(c);
    free(c);
}
