/*
 * Seeded synthetic column generators.
 *
 * This module only produces input columns. It holds none of the relational
 * arithmetic (no predicate, join or aggregation): both the CPU checker and the
 * GPU library consume the arrays it writes, so their agreement never depends
 * on the generator, only reproducibility does.
 *
 * Random source: element i of stream (seed, stream_id) is the (i+1)-th output
 * of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) started from a state
 * derived from (seed, stream_id). Because that output is a pure function of
 * the counter, columns are generated in parallel and stay identical for any
 * thread count.
 *
 * Bounded integers use Lemire's multiply-shift mapping (ACM TOMS 2019) on the
 * full 64-bit draw, x * range >> 64, without the rejection step: the bias is
 * below range / 2^64 (< 1e-12 for every range used here).
 *
 * Zipf(s) keys are drawn with Walker's alias method, built with Vose's
 * linear-time construction (IEEE TSE 1991).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DG_GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t dg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t dg_base(uint64_t seed, uint64_t stream) {
  return dg_mix64(seed * DG_GAMMA + dg_mix64(stream + 0x632BE59BD9B4E019ull));
}

static inline uint64_t dg_at(uint64_t base, uint64_t i) { return dg_mix64(base + (i + 1) * DG_GAMMA); }

static inline uint64_t dg_bounded(uint64_t x, uint64_t range) {
  return (uint64_t)(((unsigned __int128)x * range) >> 64);
}

uint64_t dg_draw_u64(uint64_t seed, uint64_t stream, uint64_t i) { return dg_at(dg_base(seed, stream), i); }

/* Uniform double in [0, 1) from the top 53 bits. */
double dg_draw_unit(uint64_t seed, uint64_t stream, uint64_t i) {
  return (double)(dg_at(dg_base(seed, stream), i) >> 11) * (1.0 / 9007199254740992.0);
}

void dg_uniform_i64(int64_t* out, int64_t n, int64_t lo, int64_t hi, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
  const uint64_t range = (uint64_t)hi - (uint64_t)lo + 1u; /* 0 means the full 2^64 range */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint64_t x = dg_at(b, (uint64_t)i);
    out[i] = (int64_t)((uint64_t)lo + (range ? dg_bounded(x, range) : x));
  }
}

void dg_uniform_i32(int32_t* out, int64_t n, int64_t lo, int64_t hi, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
  const uint64_t range = (uint64_t)(hi - lo) + 1u;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)(lo + (int64_t)dg_bounded(dg_at(b, (uint64_t)i), range));
}

void dg_uniform_i8(int8_t* out, int64_t n, int64_t lo, int64_t hi, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
  const uint64_t range = (uint64_t)(hi - lo) + 1u;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (int8_t)(lo + (int64_t)dg_bounded(dg_at(b, (uint64_t)i), range));
}

void dg_unit_f64(double* out, int64_t n, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (double)(dg_at(b, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
}

/* out[0..m) = a uniformly random permutation of base, base+1, ..., base+m-1
 * (Durstenfeld's in-place Fisher-Yates, drawing j uniform in [0, i]). */
void dg_permutation_i32(int32_t* out, int64_t m, int64_t base, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
  for (int64_t i = 0; i < m; ++i) out[i] = (int32_t)(base + i);
  for (int64_t i = m - 1; i > 0; --i) {
    int64_t j = (int64_t)dg_bounded(dg_at(b, (uint64_t)i), (uint64_t)i + 1u);
    int32_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

/* out[i] = k - 1 + offset where rank k in 1..m has probability proportional to k^-s.
 * s = 0 gives a uniform draw. Returns 0, or -1 when memory runs out. */
int dg_zipf_i32(int32_t* out, int64_t n, int64_t m, double s, int64_t offset, uint64_t seed, uint64_t stream) {
  if (m <= 0) return n == 0 ? 0 : -1;
  double* prob = (double*)malloc(sizeof(double) * (size_t)m);
  int32_t* alias = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int32_t* work = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  if (!prob || !alias || !work) {
    free(prob); free(alias); free(work);
    return -1;
  }
  double total = 0.0;
  for (int64_t k = 0; k < m; ++k) {
    prob[k] = pow((double)(k + 1), -s);
    total += prob[k];
  }
  /* Vose: scale to mean 1, split into small (<1) and large (>=1) worklists
   * kept at the two ends of one array. */
  int64_t ns = 0, nl = 0;
  for (int64_t k = 0; k < m; ++k) {
    prob[k] = prob[k] * (double)m / total;
    alias[k] = (int32_t)k;
    if (prob[k] < 1.0) work[ns++] = (int32_t)k;
    else work[m - 1 - nl++] = (int32_t)k;
  }
  while (ns > 0 && nl > 0) {
    int32_t sm = work[--ns];
    int32_t lg = work[m - nl];
    alias[sm] = lg;
    prob[lg] = (prob[lg] + prob[sm]) - 1.0;
    if (prob[lg] < 1.0) {
      --nl;
      work[ns++] = lg;
    }
  }
  while (nl > 0) prob[work[m - nl--]] = 1.0;
  while (ns > 0) prob[work[--ns]] = 1.0;
  free(work);
  const uint64_t b_col = dg_base(seed, stream);
  const uint64_t b_coin = dg_base(seed, stream ^ 0x5A5A5A5A00000000ull);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = (int64_t)dg_bounded(dg_at(b_col, (uint64_t)i), (uint64_t)m);
    double u = (double)(dg_at(b_coin, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    int64_t r = u < prob[k] ? k : (int64_t)alias[k];
    out[i] = (int32_t)(r + offset);
  }
  free(prob);
  free(alias);
  return 0;
}

/* Sample without replacement is not needed: the planner's row sample draws
 * indices with replacement, uniform in [0, n). */
void dg_sample_index_i64(int64_t* out, int64_t k, int64_t n, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
  for (int64_t i = 0; i < k; ++i) out[i] = n > 0 ? (int64_t)dg_bounded(dg_at(b, (uint64_t)i), (uint64_t)n) : 0;
}

/* Column correlated with a key column: out[i] = clamp(lo + (key[i]-kmin) * span / kspan + noise, lo, hi),
 * noise uniform in [-jitter, jitter]. Used to give the planner's training runs
 * columns that move with the key. */
void dg_correlated_i32(int32_t* out, const int32_t* key, int64_t n, int64_t kmin, int64_t kmax, int64_t lo, int64_t hi,
                       int64_t jitter, uint64_t seed, uint64_t stream) {
  const uint64_t b = dg_base(seed, stream);
  const double kspan = (double)(kmax - kmin) + 1.0;
  const double span = (double)(hi - lo) + 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t v = lo + (int64_t)(((double)key[i] - (double)kmin) * span / kspan);
    int64_t j = jitter > 0 ? (int64_t)dg_bounded(dg_at(b, (uint64_t)i), (uint64_t)(2 * jitter + 1)) - jitter : 0;
    v += j;
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    out[i] = (int32_t)v;
  }
}
