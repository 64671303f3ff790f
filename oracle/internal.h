/* internal.h -- oracle-private declarations (test infrastructure only). */
#ifndef SNN_ORACLE_INTERNAL_H
#define SNN_ORACLE_INTERNAL_H
#include "oracle.h"

#define ORC_TABLE_CAP 256u

struct orc_net {
    orc_params prm;
    uint32_t n_pops, n_proj;
    orc_pop *pops;
    orc_proj *proj;
    uint32_t *pop_off; /* [n_pops + 1] */
    uint32_t key[2];

    uint32_t n, delay, n_slots;
    int plastic;
    uint64_t nnz;
    uint64_t *row_ptr; /* [n + 1] */
    int32_t *col;      /* [nnz] */
    int32_t *w_q16;    /* [nnz] static networks */
    float *w_f32;      /* [nnz] plastic networks */
    uint64_t *plast_lo;  /* [n] first plastic edge of each row */
    uint32_t *plast_len; /* [n] number of plastic edges of each row */
    uint64_t *in_ptr;    /* [n + 1] plastic in-edges grouped by target */
    int32_t *in_src;     /* [n_plastic] */
    uint64_t *in_edge;   /* [n_plastic] */

    float *v, *x_pre, *x_post;
    int32_t *ref, *input;
    int32_t *queue;     /* [n_slots][n] */
    uint32_t *queue_len;
    uint64_t *raster;   /* [raster_cap][raster_words] */
    uint32_t raster_cap, raster_words;
    uint64_t t, events, touches;

    /* derived constants of the LIF / drive / STDP definitions */
    float alpha, v_inf, v_th, v_reset, beta_plus, beta_minus, a_plus, a_minus, w_max;
    int32_t ref_steps, w_ext_q16;
    uint64_t table[ORC_TABLE_CAP];
    uint32_t table_len;
};

int orc_validate_and_derive(orc_net *c, const orc_params *prm, const orc_pop *pops,
                            uint32_t n_pops, const orc_proj *proj, uint32_t n_proj,
                            int need_synapses, char *err, size_t err_len);
int64_t orc_row_into(const orc_net *c, uint32_t i, int32_t *col, int32_t *w_q16,
                     float *w_f32, uint64_t *plast_lo_rel, uint32_t *plast_len, int64_t cap);
void orc_free_fields(orc_net *c);
#endif
