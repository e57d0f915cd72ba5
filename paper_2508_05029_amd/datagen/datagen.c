/*
 * Seeded, counter-based generators for synthetic columnar tables.
 *
 * These routines only draw input values (uniform integers, sequences, keyed
 * permutations, Zipf ranks, log-uniform sizes, exponential gaps). They hold
 * none of the query arithmetic: no predicate, product, hash, join or
 * aggregation. Both the CPU oracle and the GPU path consume their output.
 *
 * Every value is a pure function of (seed, stream, index), so the result does
 * not depend on the number of threads that fill an array.
 *
 *   mix64      SplitMix64 finaliser (Steele, Lea, Flood 2014; constants as in
 *              the published SplitMix64 reference).
 *   draw       the SplitMix64 output for counter i of a keyed stream.
 *   bounded    Lemire's multiply-shift with rejection (Lemire 2019), made
 *              counter based: a rejected draw is re-mixed, never re-counted.
 *   perm       a keyed 4-round Feistel bijection on [0, 2^2h) with
 *              cycle-walking down to [0, n) (Black and Rogaway 2002).
 *   zipf       inverse CDF over double partial sums of k^-s.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Key of stream `stream` under `seed`. */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed) ^ (stream * 0xD1B54A32D192ED03ULL + 0x8CB92BA72F3D8DD7ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GOLDEN); }

/* Unbiased integer in [0, range) from one counter draw; range == 0 means 2^64. */
static inline uint64_t bounded(uint64_t x, uint64_t range) {
  if (range == 0) return x;
  unsigned __int128 m = (unsigned __int128)x * range;
  uint64_t l = (uint64_t)m;
  if (l < range) {
    uint64_t t = (0 - range) % range;
    while (l < t) {
      x = mix64(x ^ 0xA0761D6478BD642FULL);
      m = (unsigned __int128)x * range;
      l = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

static inline double unit_double(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* ---- column fillers ---------------------------------------------------- */

void tg_uniform_i64(int64_t* dst, int64_t n, uint64_t seed, uint64_t stream, int64_t lo, int64_t hi,
                    int64_t first) {
  uint64_t key = stream_key(seed, stream);
  uint64_t range = (uint64_t)hi - (uint64_t)lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++)
    dst[i] = (int64_t)((uint64_t)lo + bounded(draw(key, (uint64_t)(first + i)), range));
}

void tg_uniform_i32(int32_t* dst, int64_t n, uint64_t seed, uint64_t stream, int64_t lo, int64_t hi,
                    int64_t first) {
  uint64_t key = stream_key(seed, stream);
  uint64_t range = (uint64_t)hi - (uint64_t)lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++)
    dst[i] = (int32_t)((uint64_t)lo + bounded(draw(key, (uint64_t)(first + i)), range));
}

void tg_uniform_u8(uint8_t* dst, int64_t n, uint64_t seed, uint64_t stream, int64_t lo, int64_t hi,
                   int64_t first) {
  uint64_t key = stream_key(seed, stream);
  uint64_t range = (uint64_t)hi - (uint64_t)lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++)
    dst[i] = (uint8_t)((uint64_t)lo + bounded(draw(key, (uint64_t)(first + i)), range));
}

void tg_sequence_i64(int64_t* dst, int64_t n, int64_t start) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) dst[i] = start + i;
}

/* ---- keyed permutation of [0, n) --------------------------------------- */

typedef struct {
  int h;          /* half width in bits */
  uint64_t mask;  /* (1 << h) - 1 */
  uint64_t k[4];  /* round keys */
  uint64_t n;
} feistel;

static void feistel_init(feistel* f, uint64_t n, uint64_t seed, uint64_t stream) {
  int bits = 2;
  while (bits < 64 && (1ULL << bits) < n) bits++;
  if (bits & 1) bits++;
  f->h = bits / 2;
  f->mask = (f->h >= 64) ? ~0ULL : ((1ULL << f->h) - 1);
  uint64_t key = stream_key(seed, stream);
  for (int r = 0; r < 4; r++) f->k[r] = draw(key, (uint64_t)r);
  f->n = n;
}

static inline uint64_t feistel_once(const feistel* f, uint64_t x) {
  uint64_t l = (x >> f->h) & f->mask, r = x & f->mask;
  for (int i = 0; i < 4; i++) {
    uint64_t t = l ^ (mix64(r ^ f->k[i]) & f->mask);
    l = r;
    r = t;
  }
  return (l << f->h) | r;
}

static inline uint64_t feistel_perm(const feistel* f, uint64_t i) {
  uint64_t x = feistel_once(f, i);
  while (x >= f->n) x = feistel_once(f, x); /* cycle-walk stays inside [0, n) */
  return x;
}

/* dst[i] = offset + pi(first + i), pi a keyed bijection of [0, n). */
void tg_permutation_i64(int64_t* dst, int64_t count, int64_t n, uint64_t seed, uint64_t stream,
                        int64_t first, int64_t offset) {
  feistel f;
  feistel_init(&f, (uint64_t)n, seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; i++) dst[i] = offset + (int64_t)feistel_perm(&f, (uint64_t)(first + i));
}

/* ---- Zipf ranks --------------------------------------------------------- */

/* cdf[k] = (sum_{j=1}^{k+1} j^-s) / (sum_{j=1}^{G} j^-s), cdf[G-1] forced to 1. */
void tg_zipf_cdf(double* cdf, int64_t G, double s) {
  double acc = 0.0;
  for (int64_t k = 0; k < G; k++) {
    acc += pow((double)(k + 1), -s);
    cdf[k] = acc;
  }
  for (int64_t k = 0; k < G; k++) cdf[k] /= acc;
  cdf[G - 1] = 1.0;
}

/* dst[i] = rank - 1 for a Zipf(s) draw over ranks 1..G (0 is the most frequent). */
void tg_zipf_i64(int64_t* dst, int64_t n, const double* cdf, int64_t G, uint64_t seed, uint64_t stream,
                 int64_t first) {
  uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double u = unit_double(draw(key, (uint64_t)(first + i)));
    int64_t lo = 0, hi = G - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    dst[i] = lo;
  }
}

/* ---- scalar draws for sizes and arrivals -------------------------------- */

/* floor(10^(a + (b - a) * U)) clamped to [lo, hi]. */
void tg_log_uniform_i64(int64_t* dst, int64_t n, double a, double b, int64_t lo, int64_t hi,
                        uint64_t seed, uint64_t stream) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < n; i++) {
    double u = unit_double(draw(key, (uint64_t)i));
    double v = floor(pow(10.0, a + (b - a) * u));
    int64_t x = (int64_t)v;
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    dst[i] = x;
  }
}

/* floor(base * 2^(e * U)) clamped to [lo, hi]. */
void tg_log2_uniform_i64(int64_t* dst, int64_t n, double base, double e, int64_t lo, int64_t hi,
                         uint64_t seed, uint64_t stream) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < n; i++) {
    double u = unit_double(draw(key, (uint64_t)i));
    int64_t x = (int64_t)floor(base * pow(2.0, e * u));
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    dst[i] = x;
  }
}

/* Exponential gaps with rate lambda: -ln(1 - U) / lambda. */
void tg_exponential_f64(double* dst, int64_t n, double lambda, uint64_t seed, uint64_t stream) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < n; i++) dst[i] = -log1p(-unit_double(draw(key, (uint64_t)i))) / lambda;
}

/* Uniform doubles in [0, 1). */
void tg_unit_f64(double* dst, int64_t n, uint64_t seed, uint64_t stream) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < n; i++) dst[i] = unit_double(draw(key, (uint64_t)i));
}
