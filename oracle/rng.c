/*
 * rng.c -- oracle: counter-based random numbers and the exponential-spacing
 * generator of sorted distinct integers (test infrastructure only).
 */
#include <math.h>
#include <stdint.h>
#include "internal.h"

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications by the published
 * constants, a cross-wise xor with the round key, and a Weyl increment of the key
 * after each round. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* -ln(u) for u in (0, 1], in binary64, by a fixed sequence of IEEE operations so that
 * any faithful reimplementation returns the same bits:
 *   u = m * 2^e with m in [sqrt(1/2), sqrt(2));
 *   ln m = 2 atanh(r), r = (m-1)/(m+1), summed as 2r * sum_{n=0..11} r^(2n)/(2n+1)
 *   by Horner's rule in z = r*r with fused multiply-adds;  ln u = e*ln2 + ln m (fma). */
double orc_neg_log(double u) {
    const double sqrt_half = 0x1.6a09e667f3bcdp-1; /* nearest binary64 to sqrt(1/2) */
    const double ln2 = 0x1.62e42fefa39efp-1;       /* nearest binary64 to ln 2 */
    int e = 0;
    double m = frexp(u, &e); /* m in [0.5, 1) */
    if (m < sqrt_half) {
        m = m * 2.0;
        e = e - 1;
    }
    double r = (m - 1.0) / (m + 1.0);
    double z = r * r;
    double acc = 1.0 / 23.0;
    for (int n = 10; n >= 0; --n) acc = fma(acc, z, 1.0 / (double)(2 * n + 1));
    double ln_m = (2.0 * r) * acc;
    double ln_u = fma((double)e, ln2, ln_m);
    return -ln_u;
}

/* The generator of Fig. 2 (Sec. III-A.2): n sorted, distinct integers in [0, n+spare).
 * (a) n+1 uniforms in (0,1]  (b) exponential gaps -ln u  (c) exclusive running sum,
 * whose last entry S[n+1] is the total  (d) normalise by the total  (e) scale by the
 * number of spare slots and round  (f)-(g) add 0..n-1 so the values become distinct.
 * The gaps are truncated to fixed point (2^-24) before the sum, which makes (c)-(e)
 * exact integer arithmetic; rounding in (e) is half-up:
 *   x[k] = floor((2 S[k+1] spare + S[n+1]) / (2 S[n+1])) + k. */
void orc_spacing_core(const double *u, uint32_t n, uint64_t spare, uint64_t *S, int64_t *x) {
    S[0] = 0;
    for (uint32_t k = 0; k <= n; ++k) {
        double gap = orc_neg_log(u[k]);
        uint64_t g = (uint64_t)(gap * 16777216.0);
        S[k + 1] = S[k] + g;
    }
    uint64_t total = S[n + 1];
    for (uint32_t k = 0; k < n; ++k) {
        uint64_t scaled = 0;
        if (total != 0) scaled = (2u * S[k + 1] * spare + total) / (2u * total);
        x[k] = (int64_t)scaled + (int64_t)k;
    }
}

/* Inverse-CDF thresholds of Binomial(n, p) for the virtual Poisson drive: the number
 * of virtual inputs that fire in one step is k = min{ j : r < tbl[j] } for a uniform
 * 32-bit word r.  tbl[j] = floor(CDF(j) * 2^32) for j < J and tbl[J] = 2^32, where J
 * is the first index past the mean whose probability is below 2^-40 (or n).  The
 * probabilities come from the recurrence pmf(j) = pmf(j-1) * (n-j+1) / j * (p/q),
 * pmf(0) = q^n by n successive multiplications, in binary64 in exactly this order. */
uint32_t orc_binom_table(uint32_t n, double p, uint64_t *tbl, uint32_t cap) {
    const uint64_t one = (uint64_t)1 << 32;
    if (cap == 0) return 0;
    if (n == 0 || p <= 0.0) {
        tbl[0] = one;
        return 1;
    }
    if (p >= 1.0) {
        if (n + 1 > cap) return 0;
        for (uint32_t j = 0; j < n; ++j) tbl[j] = 0;
        tbl[n] = one;
        return n + 1;
    }
    double q = 1.0 - p;
    double ratio = p / q;
    double pmf = 1.0;
    for (uint32_t j = 0; j < n; ++j) pmf = pmf * q;
    if (!(pmf > 0.0)) return 0;
    double cdf = pmf;
    double mean = (double)n * p;
    uint32_t j = 0;
    for (;;) {
        if (j + 1 > cap) return 0;
        if (j == n || ((double)j > mean && pmf < 0x1p-40)) {
            tbl[j] = one;
            return j + 1;
        }
        double scaled = cdf * 4294967296.0;
        tbl[j] = scaled >= 4294967296.0 ? one : (uint64_t)scaled;
        j = j + 1;
        pmf = pmf * (double)(n - j + 1);
        pmf = pmf / (double)j;
        pmf = pmf * ratio;
        cdf = cdf + pmf;
    }
}
