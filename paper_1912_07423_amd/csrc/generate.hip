// generate.hip -- on-device network construction (the Init stage of Sec. III-A.1).
//
// Rows are built one wavefront per source neuron ("one warp per job", Sec. III-A.2):
//  * ER projections: one Bernoulli(p) trial per ordered pair, as an integer compare of
//    a Philox word against floor(p 2^32); a count pass sizes the rows, a fill pass
//    regenerates the same words and compacts the hits in ascending target order.
//  * fixed out-degree projections: the exponential-spacing generator of Fig. 2 with
//    the gaps truncated to 2^-24 fixed point, so the prefix sum, normalisation,
//    scaling, rounding and the +k step are exact integer arithmetic.  Each gap is
//    estimated from a 256-entry table and a short series; the few whose estimate lies
//    too close to an integer evaluate the defined binary64 logarithm instead.
#include <algorithm>

#include "device_math.h"
#include "snn_internal.h"

namespace snn {
namespace {

constexpr int kGenBlock = 256;
constexpr int kGenWavesPerBlock = kGenBlock / kWave;

__device__ __forceinline__ uint32_t population_of(const GenArgs &g, uint32_t i) {
  uint32_t a = 0;
  while (i >= g.pop_off[a + 1]) ++a;
  return a;
}

// Edge count of neuron i in an ER projection (whole wave participates).
__device__ uint32_t er_count(const GenArgs &g, const GenProj &pj, uint32_t i) {
  const uint32_t b_lo = pj.off >> 2, b_hi = (pj.off + pj.size - 1) >> 2;
  uint32_t count = 0;
  for (uint32_t b = b_lo + lane_id(); b <= b_hi; b += kWave) {
    const Words4 r = philox(i, b, 0u, kStreamConn, g.key0, g.key1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t j = 4u * b + q;
      count += (j >= pj.off && j < pj.off + pj.size && j != i && (uint64_t)r.w[q] < pj.thr) ? 1u : 0u;
    }
  }
  return wave_sum(count);
}

__global__ __launch_bounds__(kGenBlock) void k_row_lengths(GenArgs g, uint32_t *len,
                                                           uint32_t *plast_rel,
                                                           uint32_t *plast_len) {
  const uint32_t wave = blockIdx.x * kGenWavesPerBlock + threadIdx.x / kWave;
  const uint32_t n_waves = gridDim.x * kGenWavesPerBlock;
  for (uint32_t i = wave; i < g.n; i += n_waves) {
    const uint32_t a = population_of(g, i);
    uint32_t total = 0, prel = 0, plen = 0;
    for (uint32_t q = g.pop_proj[a]; q < g.pop_proj[a + 1]; ++q) {
      const GenProj pj = g.proj[q];
      const uint32_t c = pj.kind == SNN_PROJ_ER ? er_count(g, pj, i) : pj.k;
      if (pj.plastic) {
        prel = total;
        plen = c;
      }
      total += c;
    }
    if (lane_id() == 0) {
      len[i] = total;
      if (plast_rel) {
        plast_rel[i] = prel;
        plast_len[i] = plen;
      }
    }
  }
}

// Writes the ER edges of neuron i from position pos on; returns the end position.
__device__ uint64_t er_fill(const GenArgs &g, const GenProj &pj, uint32_t i, uint64_t pos,
                            int32_t *col, int32_t *w_q16, float *w_f32) {
  const uint32_t b_lo = pj.off >> 2, b_hi = (pj.off + pj.size - 1) >> 2;
  const uint32_t n_iter = (b_hi - b_lo) / kWave + 1;
  for (uint32_t it = 0; it < n_iter; ++it) {
    const uint32_t b = b_lo + it * kWave + lane_id();
    uint32_t hits = 0;
    if (b <= b_hi) {
      const Words4 r = philox(i, b, 0u, kStreamConn, g.key0, g.key1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t j = 4u * b + q;
        if (j >= pj.off && j < pj.off + pj.size && j != i && (uint64_t)r.w[q] < pj.thr) hits |= 1u << q;
      }
    }
    const uint32_t cnt = __popc(hits);
    const uint32_t incl = wave_inclusive_scan(cnt);
    uint64_t p = pos + (incl - cnt);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (hits & (1u << q)) {
        col[p] = (int32_t)(4u * b + q);
        if (w_q16) w_q16[p] = pj.w_q16;
        if (w_f32) w_f32[p] = pj.w_f32;
        ++p;
      }
    }
    pos += __shfl(incl, kWave - 1, kWave);
  }
  return pos;
}

// floor(num / den) for den > 0 and num + 2 den < 2^64, given inv = 1 / den in binary64:
// the estimate num * inv is within one of the quotient while the quotient is below 2^51,
// and is corrected to the exact integer quotient.  Far cheaper on the GPU than a 64-bit
// integer division.
__device__ __forceinline__ uint64_t div_floor_u64(uint64_t num, uint64_t den, double inv) {
  uint64_t q = (uint64_t)((double)num * inv);
  while (q * den > num) --q;
  while ((q + 1) * den <= num) ++q;
  return q;
}

// 64-bit inclusive scan over the wave by DPP lane shifts applied to both halves (the
// same shifts as the 32-bit scan: 1, 2, 4, 8 inside rows of 16 lanes, then rows 0 and 2
// into rows 1 and 3, then lane 31 into rows 2 and 3); every lane must be active.
template <int kCtrl, int kRows, bool kZeroOutside>
__device__ __forceinline__ uint64_t add_dpp_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, kCtrl, kRows, 0xf, kZeroOutside);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), kCtrl, kRows, 0xf, kZeroOutside);
  return v + (((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t x) {
  x = add_dpp_u64<0x111, 0xf, true>(x);   // row_shr:1
  x = add_dpp_u64<0x112, 0xf, true>(x);   // row_shr:2
  x = add_dpp_u64<0x114, 0xf, true>(x);   // row_shr:4
  x = add_dpp_u64<0x118, 0xf, true>(x);   // row_shr:8
  x = add_dpp_u64<0x142, 0xa, false>(x);  // row_bcast:15, rows 1 and 3
  x = add_dpp_u64<0x143, 0xc, false>(x);  // row_bcast:31, rows 2 and 3
  return x;
}

__device__ __forceinline__ uint64_t last_lane_u64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, kWave - 1);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), kWave - 1);
  return ((uint64_t)hi << 32) | lo;
}

// ---- the gaps of Fig. 2, step (b) ----
// The gap of a 32-bit word is floor(-ln(u) 2^24) with u = ((word >> 8) + 1) 2^-24 and
// -ln the fixed binary64 sequence neg_log, about 40 binary64 operations with a
// correctly rounded division among them.  The fill estimates it instead (Tang's table
// method): j = (word >> 8) + 1 = 2^e m with m in [1, 2), i = the kGapBits bits of m after
// its leading one, c_i = 1 + (i + 1/2) 2^-kGapBits, F_i = 1/c_i rounded,
// L_i = neg_log(F_i); then r = m F_i - 1 (|r| <= 2^-(kGapBits+1) up to rounding),
// ln(1 + r) by its Taylor series to r^8, and -ln u = (24 - e) ln 2 - L_i - ln(1 + r).
// Over all 2^24 values of j the estimate, in units of 2^-24, lies within 6e-8 of the
// defined value, so it has the same floor unless its fractional part is within 2^-16 of
// an integer; that happens for 528 of the 2^24 values, and those lanes evaluate neg_log.
// The 16 entries fill the 64 LDS banks once, so a wave's table reads do not conflict
// (a 256-entry table with a 4-term series issues fewer instructions but was slower).
constexpr int kGapBits = 4;
constexpr int kGapTable = 1 << kGapBits;
constexpr int kGapTerms = 8;
constexpr double kGapMargin = 0x1p-16;

// Entry i = {F_i 2^-31, L_i}, written by the calling workgroup; ends with a barrier.
__device__ void load_gap_table(double2 *tbl) {
  for (uint32_t i = threadIdx.x; i < (uint32_t)kGapTable; i += blockDim.x) {
    const double f = 1.0 / (1.0 + ((double)i + 0.5) / (double)kGapTable);
    tbl[i] = make_double2(f * 0x1p-31, neg_log(f));
  }
  __syncthreads();
}

// The table entry of a word: its index, with j = (word >> 8) + 1 normalised to
// jn = m 2^31 and lz = 31 - e.
__device__ __forceinline__ uint32_t gap_index(uint32_t word, uint32_t &jn, uint32_t &lz) {
  const uint32_t j = (word >> 8) + 1u;
  lz = (uint32_t)__builtin_clz(j);  // 7 ... 31
  jn = j << lz;
  return (jn >> (31 - kGapBits)) & (uint32_t)(kGapTable - 1);
}

// The estimate's floor in `gap` from the word's table entry t; false if the estimate is
// too close to an integer.  Branch-free, so that a lane's four estimates overlap.
__device__ __forceinline__ bool gap_estimate(uint32_t jn, uint32_t lz, double2 t, uint32_t &gap) {
  constexpr double kLn2 = 0x1.62e42fefa39efp-1;
  const double r = fma((double)jn, t.x, -1.0);
  // ln(1 + r) = r + r^2 (-1/2 + r (1/3 + r (-1/4 + ...))), coefficients (-1)^(k+1) / k
  double q = ((kGapTerms & 1) ? 1.0 : -1.0) / (double)kGapTerms;
#pragma unroll
  for (int k = kGapTerms - 1; k >= 2; --k) q = fma(r, q, ((k & 1) ? 1.0 : -1.0) / (double)k);
  const double ln1p = fma(r * r, q, r);
  // lz - 7 = 24 - e
  const double y = (fma((double)(int32_t)(lz - 7u), kLn2, -t.y) - ln1p) * 16777216.0;
  const double fr = y - floor(y);
  gap = (uint32_t)fmax(y, 0.0);
  return fr >= kGapMargin && fr <= 1.0 - kGapMargin;
}

__device__ __forceinline__ uint32_t gap_of(uint32_t word, const double2 *tbl) {
  uint32_t jn, lz, gap;
  const double2 t = tbl[gap_index(word, jn, lz)];
  if (!gap_estimate(jn, lz, t, gap)) gap = (uint32_t)spacing_gap(word);
  return gap;
}

// The four gaps of one Philox block; gaps past `last` (k > last) are 0.  The four table
// entries are read before any estimate, so the LDS reads are in flight together.
__device__ __forceinline__ void gaps4(const Words4 &r, uint32_t k0, uint32_t last, const double2 *tbl,
                                      uint32_t g[4]) {
  uint32_t jn[4], lz[4];
  double2 t[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = tbl[gap_index(r.w[q], jn[q], lz[q])];
  bool ok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) ok[q] = gap_estimate(jn[q], lz[q], t[q], g[q]);
  if (!(ok[0] && ok[1] && ok[2] && ok[3])) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (!ok[q]) g[q] = (uint32_t)spacing_gap(r.w[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) g[q] = k0 + q <= last ? g[q] : 0u;
}

// Gaps of one fixed out-degree row kept in LDS between the two passes (the first pass of
// Sec. III-A.2 runs in shared memory): the first 4 x cache_blocks gaps of a row are
// stored as uint32 (a gap is below 2^29: -ln(2^-24) 2^24 < 2.8e8) and read back by the
// second pass; gaps past the cache are regenerated.  The cache is sized at launch to the
// longest fixed out-degree row, at most kGapCacheMax gaps per wavefront: the most that
// lets two workgroups, each with its log table, share one CU's 160 KiB.
constexpr uint32_t kGapCacheMax =
    (uint32_t)((160u * 1024u / 2u - kGapTable * sizeof(double2)) / (kGenWavesPerBlock * sizeof(uint4))) * 4u;
static_assert(kGapCacheMax == 5104, "gap cache of 1,276 blocks of four per wavefront");

// Pass 1 over the blocks [lo, hi) of a fixed out-degree row: the wavefront's total of
// their gaps; the first cache_blocks of them go to `cache` (indexed from lo).  Each block
// of four gaps is written and read back by the same lane, so no barrier.
__device__ uint64_t fixed_pass1(const GenArgs &g, const GenProj &pj, uint32_t i, uint32_t lo,
                                uint32_t hi, uint4 *cache, uint32_t cache_blocks, const double2 *tbl) {
  const uint32_t stream_word2 = 1u + pj.first_pop;
  uint64_t part = 0;
  for (uint32_t b = lo + lane_id(); b < hi; b += kWave) {
    const Words4 r = philox(i, b, stream_word2, kStreamConn, g.key0, g.key1);
    uint32_t gq[4];
    gaps4(r, 4u * b, pj.k, tbl, gq);
    part += (uint64_t)(gq[0] + gq[1] + gq[2] + gq[3]);
    if (b - lo < cache_blocks) cache[b - lo] = make_uint4(gq[0], gq[1], gq[2], gq[3]);
  }
  return wave_sum(part);
}

// Pass 2 over the blocks [lo, hi): running sum S_{k+1} from `carry` (the gaps of the
// blocks before lo), round-half-up of S_{k+1} * spare / total, + k; writes the targets.
__device__ void fixed_pass2(const GenArgs &g, const GenProj &pj, uint32_t i, uint64_t pos,
                            uint32_t lo, uint32_t hi, uint64_t carry, uint64_t total, int32_t *col,
                            int32_t *w_q16, float *w_f32, const uint4 *cache, uint32_t cache_blocks,
                            const double2 *tbl) {
  const uint32_t k_out = pj.k;
  const uint32_t stream_word2 = 1u + pj.first_pop;
  const uint32_t n_iter = (hi - lo + kWave - 1) / kWave;
  const uint64_t two_total = 2u * total;
  const double inv_two_total = total != 0 ? 1.0 / (double)two_total : 0.0;
  const double inv_total = total != 0 ? 1.0 / (double)total : 0.0;
  const double half_total_d = 0.5 * (double)total, spare_d = (double)pj.spare;
  const uint32_t self_local = pj.self_in ? (i - pj.off) : 0xFFFFFFFFu;
  for (uint32_t it = 0; it < n_iter; ++it) {
    const uint32_t b = lo + it * kWave + lane_id();
    uint32_t gap[4] = {0, 0, 0, 0};
    if (b < hi) {
      if (b - lo < cache_blocks) {
        const uint4 c = cache[b - lo];
        gap[0] = c.x;
        gap[1] = c.y;
        gap[2] = c.z;
        gap[3] = c.w;
      } else {
        const Words4 r = philox(i, b, stream_word2, kStreamConn, g.key0, g.key1);
        gaps4(r, 4u * b, k_out, tbl, gap);
      }
    }
    // four gaps are below 2^31 together
    const uint32_t lane_total = gap[0] + gap[1] + gap[2] + gap[3];
    const uint64_t incl = wave_scan_u64(lane_total);
    const uint64_t s0 = carry + (incl - lane_total);
    const double s0_d = (double)s0;
    // q_k = floor(S_{k+1} spare / total + 1/2) <= spare < 2^32 from binary64: the
    // roundings below (s0, s0 + in_lane, total, the fma, 1 / total, the product) add up
    // to a relative error under 7 2^-53 < 2^-50, i.e. under 2^-18 absolute, so the floor
    // of the estimate is exact unless it lies that close to an integer; then the exact
    // integer quotient.  The four estimates come first and the rare exact quotients
    // after them, so that the four chains overlap.  (total = 0 only if every gap is 0;
    // then q_k = 0.)
    uint32_t in_lane[4], qk[4] = {0, 0, 0, 0};
    bool sure[4] = {true, true, true, true};
    in_lane[0] = gap[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) in_lane[q] = in_lane[q - 1] + gap[q];  // S_{k+1} = s0 + in_lane
    if (total != 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double est = fma(s0_d + (double)in_lane[q], spare_d, half_total_d) * inv_total;
        const double fl = floor(est), fr = est - fl;
        qk[q] = (uint32_t)fl;
        sure[q] = fr >= 0x1p-18 && fr <= 1.0 - 0x1p-18;
      }
      if (!(sure[0] && sure[1] && sure[2] && sure[3])) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (!sure[q])
            qk[q] = (uint32_t)div_floor_u64(2u * (s0 + in_lane[q]) * pj.spare + total, two_total, inv_two_total);
      }
    }
    int32_t tgt[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t x = qk[q] + 4u * b + q;
      if (x >= self_local) x += 1;
      tgt[q] = (int32_t)(pj.off + x);
    }
    // a whole block of four targets goes out as one 16-byte store when the row starts
    // on a 16-byte boundary; the row's last, partial block element by element
    const uint64_t p0 = pos + 4u * b;
    if (b < hi) {
      if ((pos & 3u) == 0 && 4u * b + 3u < k_out) {
        *reinterpret_cast<int4 *>(col + p0) = make_int4(tgt[0], tgt[1], tgt[2], tgt[3]);
        if (w_q16) *reinterpret_cast<int4 *>(w_q16 + p0) = make_int4(pj.w_q16, pj.w_q16, pj.w_q16, pj.w_q16);
        if (w_f32) *reinterpret_cast<float4 *>(w_f32 + p0) = make_float4(pj.w_f32, pj.w_f32, pj.w_f32, pj.w_f32);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (4u * b + q < k_out) {
            col[p0 + q] = tgt[q];
            if (w_q16) w_q16[p0 + q] = pj.w_q16;
            if (w_f32) w_f32[p0 + q] = pj.w_f32;
          }
        }
      }
    }
    carry += last_lane_u64(incl);
  }
}


// One fixed out-degree row by one wavefront.
__device__ void fixed_fill(const GenArgs &g, const GenProj &pj, uint32_t i, uint64_t pos,
                           int32_t *col, int32_t *w_q16, float *w_f32, uint4 *cache,
                           uint32_t cache_blocks, const double2 *tbl) {
  if (pj.k == 0) return;
  const uint32_t n_blocks = (pj.k + 1 + 3) / 4;  // gaps 0..k
  const uint64_t total = fixed_pass1(g, pj, i, 0, n_blocks, cache, cache_blocks, tbl);
  fixed_pass2(g, pj, i, pos, 0, n_blocks, 0, total, col, w_q16, w_f32, cache, cache_blocks, tbl);
}

__global__ __launch_bounds__(kGenBlock) void k_fill_rows(GenArgs g, const uint64_t *row_ptr,
                                                         int32_t *col, int32_t *w_q16,
                                                         float *w_f32, uint32_t cache_blocks) {
  extern __shared__ uint4 gap_cache[];  // [kGenWavesPerBlock][cache_blocks]
  __shared__ double2 tbl[kGapTable];
  load_gap_table(tbl);
  uint4 *cache = gap_cache + (threadIdx.x / kWave) * cache_blocks;
  const uint32_t wave = blockIdx.x * kGenWavesPerBlock + threadIdx.x / kWave;
  const uint32_t n_waves = gridDim.x * kGenWavesPerBlock;
  for (uint32_t i = wave; i < g.n; i += n_waves) {
    const uint32_t a = population_of(g, i);
    uint64_t pos = row_ptr[i];
    for (uint32_t q = g.pop_proj[a]; q < g.pop_proj[a + 1]; ++q) {
      const GenProj pj = g.proj[q];
      if (pj.kind == SNN_PROJ_ER) {
        pos = er_fill(g, pj, i, pos, col, w_q16, w_f32);
      } else {
        fixed_fill(g, pj, i, pos, col, w_q16, w_f32, cache, cache_blocks, tbl);
        pos += pj.k;
      }
    }
  }
}

// Networks whose projections are all fixed out-degree, with rows of at least
// kTeamMinK targets: one workgroup per row, each wavefront taking a contiguous quarter of
// the row's blocks.  Pass 1 gives each wavefront the total of its quarter; one barrier
// combines the four into the row's total and each wavefront's carry-in; pass 2 then runs
// on the quarters independently.  A wavefront caches only its quarter's gaps, so four
// times as many workgroups fit a CU (at K = 5,000: 20 KiB instead of 80 KiB each), and
// rows of up to 4 x kTeamCacheMax blocks are generated once.  Shorter rows stay one per
// wavefront: there the per-row latency and set-up, paid four times, outweigh the
// occupancy (rows of 1,000 and 2,000 targets filled 20-35% slower by workgroups).
constexpr uint32_t kTeamMinK = 4096;
constexpr uint32_t kTeamCacheMax =
    (uint32_t)((160u * 1024u / 2u - kGapTable * sizeof(double2) - 2u * kGenWavesPerBlock * sizeof(uint64_t)) /
               (kGenWavesPerBlock * sizeof(uint4)));
static_assert(kTeamCacheMax == 1275, "1,275 blocks of four gaps per wavefront");

__global__ __launch_bounds__(kGenBlock) void k_fill_fixed_rows(GenArgs g, const uint64_t *row_ptr,
                                                               int32_t *col, int32_t *w_q16,
                                                               float *w_f32, uint32_t cache_blocks) {
  extern __shared__ uint4 gap_cache[];  // [kGenWavesPerBlock][cache_blocks]
  __shared__ double2 tbl[kGapTable];
  __shared__ uint64_t sums[2][kGenWavesPerBlock];  // alternate per row segment
  load_gap_table(tbl);
  const uint32_t w = threadIdx.x / kWave;
  uint4 *cache = gap_cache + w * cache_blocks;
  uint32_t seg = 0;
  for (uint32_t i = blockIdx.x; i < g.n; i += gridDim.x) {
    const uint32_t a = population_of(g, i);
    uint64_t pos = row_ptr[i];
    for (uint32_t q = g.pop_proj[a]; q < g.pop_proj[a + 1]; ++q) {
      const GenProj pj = g.proj[q];
      if (pj.k == 0) continue;
      const uint32_t n_blocks = (pj.k + 1 + 3) / 4;  // gaps 0..k
      const uint32_t per = (n_blocks + kGenWavesPerBlock - 1) / kGenWavesPerBlock;
      const uint32_t lo = min(w * per, n_blocks), hi = min(lo + per, n_blocks);
      const uint64_t mine = fixed_pass1(g, pj, i, lo, hi, cache, cache_blocks, tbl);
      // The slot written here was last read before the previous segment's barrier.
      uint64_t *s = sums[seg & 1u];
      if (lane_id() == 0) s[w] = mine;
      __syncthreads();
      uint64_t total = 0, before = 0;
#pragma unroll
      for (uint32_t v = 0; v < (uint32_t)kGenWavesPerBlock; ++v) {
        total += s[v];
        if (v < w) before += s[v];
      }
      fixed_pass2(g, pj, i, pos, lo, hi, before, total, col, w_q16, w_f32, cache, cache_blocks, tbl);
      pos += pj.k;
      ++seg;
    }
  }
}

// The gaps of caller-given words, by the fill's own evaluation.
__global__ __launch_bounds__(kGenBlock) void k_spacing_gaps(const uint32_t *words, uint64_t n,
                                                            uint32_t *gaps) {
  __shared__ double2 tbl[kGapTable];
  load_gap_table(tbl);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    gaps[k] = gap_of(words[k], tbl);
  }
}

// ---- exclusive scan of uint32 lengths into uint64 offsets (out has n + 1 entries) ----
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(const uint32_t *in, uint64_t *out,
                                                            uint32_t n, uint64_t *block_sums) {
  __shared__ uint64_t wave_tot[kScanBlock / kWave];
  const uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x;
  const uint64_t x = idx < n ? in[idx] : 0u;
  const uint64_t incl = wave_inclusive_scan(x);
  const uint32_t w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wave_tot[w] = incl;
  __syncthreads();
  if (w == 0) {
    const uint64_t t = lane_id() < kScanBlock / kWave ? wave_tot[lane_id()] : 0u;
    const uint64_t ti = wave_inclusive_scan(t);
    if (lane_id() < kScanBlock / kWave) wave_tot[lane_id()] = ti - t;
    if (lane_id() == kScanBlock / kWave - 1) block_sums[blockIdx.x] = ti;
  }
  __syncthreads();
  if (idx < n) out[idx] = wave_tot[w] + incl - x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(uint64_t *block_sums, uint32_t n_blocks,
                                                          uint64_t *out, uint32_t n) {
  __shared__ uint64_t wave_tot[kScanBlock / kWave];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n_blocks; base += kScanBlock) {
    const uint32_t idx = base + threadIdx.x;
    const uint64_t x = idx < n_blocks ? block_sums[idx] : 0u;
    const uint64_t incl = wave_inclusive_scan(x);
    const uint32_t w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wave_tot[w] = incl;
    __syncthreads();
    if (w == 0) {
      const uint64_t t = lane_id() < kScanBlock / kWave ? wave_tot[lane_id()] : 0u;
      const uint64_t ti = wave_inclusive_scan(t);
      if (lane_id() < kScanBlock / kWave) wave_tot[lane_id()] = ti - t;
    }
    __syncthreads();
    const uint64_t excl = carry + wave_tot[w] + incl - x;
    if (idx < n_blocks) block_sums[idx] = excl;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry = excl + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(uint64_t *out, uint32_t n,
                                                         const uint64_t *block_sums) {
  const uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x;
  if (idx < n) out[idx] += block_sums[blockIdx.x];
}

// ---- transposed index of plastic edges (in-edges grouped by target) ----
__global__ __launch_bounds__(kGenBlock) void k_count_in(const uint64_t *row_ptr, const int32_t *col,
                                                        const uint32_t *plast_rel,
                                                        const uint32_t *plast_len, uint32_t n,
                                                        uint32_t *count) {
  const uint32_t wave = blockIdx.x * kGenWavesPerBlock + threadIdx.x / kWave;
  const uint32_t n_waves = gridDim.x * kGenWavesPerBlock;
  for (uint32_t i = wave; i < n; i += n_waves) {
    const uint64_t lo = row_ptr[i] + plast_rel[i];
    for (uint32_t k = lane_id(); k < plast_len[i]; k += kWave) atomicAdd(&count[col[lo + k]], 1u);
  }
}

__global__ __launch_bounds__(kGenBlock) void k_fill_in(const uint64_t *row_ptr, const int32_t *col,
                                                       const uint32_t *plast_rel,
                                                       const uint32_t *plast_len, uint32_t n,
                                                       uint64_t *cursor, int32_t *in_src,
                                                       uint32_t *in_edge) {
  const uint32_t wave = blockIdx.x * kGenWavesPerBlock + threadIdx.x / kWave;
  const uint32_t n_waves = gridDim.x * kGenWavesPerBlock;
  for (uint32_t i = wave; i < n; i += n_waves) {
    const uint64_t lo = row_ptr[i] + plast_rel[i];
    for (uint32_t k = lane_id(); k < plast_len[i]; k += kWave) {
      const uint64_t e = lo + k;
      const uint64_t slot = atomicAdd((unsigned long long *)&cursor[col[e]], 1ull);
      in_src[slot] = (int32_t)i;
      in_edge[slot] = (uint32_t)e;
    }
  }
}

// ---- indexes of the tiled delivery: tile boundaries and 16-bit targets ----
// Tile of target t, floor(t / tile_size): a binary64 estimate from the reciprocal (relative
// error ~2^-52, so within one of the quotient for any 32-bit t), corrected exactly in
// integers.
__device__ __forceinline__ uint32_t tile_of(uint32_t t, uint32_t tile_size, double inv) {
  uint32_t q = (uint32_t)((double)t * inv);
  if ((uint64_t)q * tile_size > t) --q;
  else if ((uint64_t)(q + 1) * tile_size <= t) ++q;
  return q;
}

// One wave per (sorted) row, streaming the row's targets once:
//  * col16[e] = col[e] mod 2^16, the tiled delivery's 2-byte target stream (a range spans
//    fewer than 65,536 targets, so the low 16 bits identify a target inside it);
//  * entry p of the row's tile boundaries is the offset, from the row's start, of the
//    first target >= p * tile_size (entry `tiles` is the row length).  Targets are
//    sorted, so element e is that boundary for every p in (tile(e - 1), tile(e)]; the
//    entries past the last element's tile get the row length.  Stored as uint16 when
//    every row is shorter than 65,536 synapses.
// The padding of col16 past nnz (up to `count`) is cleared by the first thread.  A lane
// takes groups of four consecutive targets: one 16-byte load and one 8-byte col16 store
// each where the row starts on a 16-byte boundary, element by element otherwise.
constexpr int kIndexGroups = 2;  // groups of four per lane in flight
__global__ __launch_bounds__(kGenBlock) void k_tile_index(const uint64_t *row_ptr, const int32_t *col,
                                                          uint32_t n, uint64_t nnz, uint64_t count,
                                                          uint32_t tiles, uint32_t tile_size, double inv,
                                                          uint16_t *col16, void *tile_off, bool off16) {
  const uint32_t lane = lane_id();
  const uint32_t wave = blockIdx.x * kGenWavesPerBlock + threadIdx.x / kWave;
  const uint32_t n_waves = gridDim.x * kGenWavesPerBlock;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (uint64_t e = nnz; e < count; ++e) col16[e] = 0;
  auto put = [&](uint64_t at, uint32_t rel) {
    if (off16) static_cast<uint16_t *>(tile_off)[at] = (uint16_t)rel;
    else static_cast<uint32_t *>(tile_off)[at] = rel;
  };
  for (uint32_t i = wave; i < n; i += n_waves) {
    const uint64_t lo = row_ptr[i], hi = row_ptr[i + 1];
    const uint64_t out = (uint64_t)i * (tiles + 1);
    const bool aligned = (lo & 3u) == 0;
    int32_t carry = -1;  // tile of the element before this group (-1 at the row's start)
    for (uint64_t base = lo; base < hi; base += (uint64_t)kWave * 4u * kIndexGroups) {
      int32_t t[kIndexGroups][4];
#pragma unroll
      for (int gi = 0; gi < kIndexGroups; ++gi) {
        const uint64_t e0 = base + ((uint64_t)gi * kWave + lane) * 4u;
        if (aligned && e0 + 4u <= hi) {
          const int4 v = *reinterpret_cast<const int4 *>(col + e0);
          t[gi][0] = v.x;
          t[gi][1] = v.y;
          t[gi][2] = v.z;
          t[gi][3] = v.w;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) t[gi][j] = e0 + j < hi ? col[e0 + j] : 0;
        }
      }
#pragma unroll
      for (int gi = 0; gi < kIndexGroups; ++gi) {
        const uint64_t e0 = base + ((uint64_t)gi * kWave + lane) * 4u;
        int32_t tl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          tl[j] = e0 + j < hi ? (int32_t)tile_of((uint32_t)t[gi][j], tile_size, inv) : (int32_t)tiles;
        const int32_t up = __shfl_up(tl[3], 1, kWave);
        int32_t prev = lane == 0 ? carry : up;
        if (aligned && e0 + 4u <= hi) {
          *reinterpret_cast<uint2 *>(col16 + e0) =
              make_uint2(((uint32_t)t[gi][0] & 0xFFFFu) | ((uint32_t)t[gi][1] << 16),
                         ((uint32_t)t[gi][2] & 0xFFFFu) | ((uint32_t)t[gi][3] << 16));
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (e0 + j < hi) col16[e0 + j] = (uint16_t)(uint32_t)t[gi][j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (e0 + j < hi) {
            for (int32_t p = prev + 1; p <= tl[j]; ++p) put(out + (uint32_t)p, (uint32_t)(e0 + j - lo));
            prev = tl[j];
          }
        }
        carry = __shfl(tl[3], kWave - 1, kWave);
      }
    }
    // entries past the last element's tile: the row length
    int32_t last = -1;
    if (hi > lo) last = (int32_t)tile_of((uint32_t)col[hi - 1], tile_size, inv);
    for (uint32_t p = (uint32_t)(last + 1) + lane; p <= tiles; p += kWave) put(out + p, (uint32_t)(hi - lo));
  }
}

// V = lo + span * u, u = (word0 >> 8) 2^-24 of stream VINIT at block (i, 0, 0).
__global__ __launch_bounds__(kGenBlock) void k_init_neurons(float *v, int32_t *ref, uint32_t n,
                                                            uint32_t key0, uint32_t key1, float lo,
                                                            float span) {
  const uint32_t i = blockIdx.x * kGenBlock + threadIdx.x;
  if (i >= n) return;
  const Words4 r = philox(i, 0u, 0u, kStreamVinit, key0, key1);
  const float u = (float)(r.w[0] >> 8) * 0x1p-24f;
  const float prod = span * u;
  v[i] = lo + prod;
  ref[i] = 0;
}


uint32_t row_grid(uint32_t n) {
  const uint32_t blocks = (n + kGenWavesPerBlock - 1) / kGenWavesPerBlock;
  return blocks < 8192u ? (blocks ? blocks : 1u) : 8192u;
}

}  // namespace

hipError_t launch_row_lengths(const GenArgs &g, uint32_t *len, uint32_t *plast_rel,
                              uint32_t *plast_len, hipStream_t s) {
  k_row_lengths<<<row_grid(g.n), kGenBlock, 0, s>>>(g, len, plast_rel, plast_len);
  return hipGetLastError();
}

hipError_t launch_fill_rows(const GenArgs &g, uint32_t max_fixed_k, bool all_fixed, const uint64_t *row_ptr,
                            int32_t *col, int32_t *w_q16, float *w_f32, hipStream_t s) {
  int dev = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  const bool team = all_fixed && max_fixed_k >= kTeamMinK;
  const uint32_t blocks = max_fixed_k ? (max_fixed_k + 1 + 3) / 4 : 0u;  // of the longest row
  uint32_t cache_blocks = team ? std::min((blocks + kGenWavesPerBlock - 1) / kGenWavesPerBlock, kTeamCacheMax)
                               : std::min(blocks, kGapCacheMax / 4);
  cache_blocks = std::min<uint32_t>(cache_blocks, (uint32_t)lds_max / (kGenWavesPerBlock * sizeof(uint4)));
  const size_t lds = (size_t)kGenWavesPerBlock * cache_blocks * sizeof(uint4);
  const void *fn = team ? reinterpret_cast<const void *>(&k_fill_fixed_rows)
                        : reinterpret_cast<const void *>(&k_fill_rows);
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (team)
    k_fill_fixed_rows<<<std::min(g.n ? g.n : 1u, 8192u), kGenBlock, lds, s>>>(g, row_ptr, col, w_q16, w_f32,
                                                                              cache_blocks);
  else
    k_fill_rows<<<row_grid(g.n), kGenBlock, lds, s>>>(g, row_ptr, col, w_q16, w_f32, cache_blocks);
  return hipGetLastError();
}

hipError_t launch_spacing_gaps(const uint32_t *words, uint64_t n, uint32_t *gaps, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + kGenBlock - 1) / kGenBlock;
  k_spacing_gaps<<<(uint32_t)std::min<uint64_t>(blocks, 8192u), kGenBlock, 0, s>>>(words, n, gaps);
  return hipGetLastError();
}

hipError_t launch_tile_index(const uint64_t *row_ptr, const int32_t *col, uint32_t n, uint64_t nnz,
                             uint64_t count, uint32_t tiles, uint32_t tile_size, uint16_t *col16,
                             void *tile_off, bool off16, hipStream_t s) {
  if (count < nnz || tile_size == 0 || tiles == 0 || (uint64_t)tiles * tile_size < n) return hipErrorInvalidValue;
  k_tile_index<<<row_grid(n), kGenBlock, 0, s>>>(row_ptr, col, n, nnz, count, tiles, tile_size,
                                                 1.0 / (double)tile_size, col16, tile_off, off16);
  return hipGetLastError();
}

size_t scan_scratch_elems(uint32_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint32_t n,
                                  uint64_t *block_sums, hipStream_t s) {
  const uint32_t blocks = (n + kScanBlock - 1) / kScanBlock;
  if (blocks == 0) {
    k_scan_sums<<<1, kScanBlock, 0, s>>>(block_sums, 0, out, n);
    return hipGetLastError();
  }
  k_scan_blocks<<<blocks, kScanBlock, 0, s>>>(in, out, n, block_sums);
  k_scan_sums<<<1, kScanBlock, 0, s>>>(block_sums, blocks, out, n);
  k_scan_add<<<blocks, kScanBlock, 0, s>>>(out, n, block_sums);
  return hipGetLastError();
}

hipError_t launch_count_in_edges(const uint64_t *row_ptr, const int32_t *col,
                                 const uint32_t *plast_rel, const uint32_t *plast_len,
                                 uint32_t n, uint32_t *count, hipStream_t s) {
  k_count_in<<<row_grid(n), kGenBlock, 0, s>>>(row_ptr, col, plast_rel, plast_len, n, count);
  return hipGetLastError();
}

hipError_t launch_fill_in_edges(const uint64_t *row_ptr, const int32_t *col,
                                const uint32_t *plast_rel, const uint32_t *plast_len,
                                uint32_t n, uint64_t *cursor, int32_t *in_src,
                                uint32_t *in_edge, hipStream_t s) {
  k_fill_in<<<row_grid(n), kGenBlock, 0, s>>>(row_ptr, col, plast_rel, plast_len, n, cursor,
                                               in_src, in_edge);
  return hipGetLastError();
}


hipError_t launch_init_neurons(float *v, int32_t *ref, uint32_t n, uint32_t key0, uint32_t key1,
                               float lo, float span, hipStream_t s) {
  k_init_neurons<<<(n + kGenBlock - 1) / kGenBlock, kGenBlock, 0, s>>>(v, ref, n, key0, key1, lo,
                                                                     span);
  return hipGetLastError();
}


}  // namespace snn
