/*
 * Seeded synthetic inputs for sparse Tucker workloads.
 *
 * This file holds only random-number generation and the sampling recipes of
 * the synthetic tensors (coordinates, values, initial factors, the draws of a
 * planted completion model).  It contains none of the decomposition's
 * arithmetic.
 * Both the FP64 checker and the GPU library consume the bytes written here,
 * so the two sides always see identical inputs.
 *
 * Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used in counter mode: draw i of stream s
 * under seed q is mix64(key(q, s) + (i + 1) * GAMMA), where mix64 is the
 * SplitMix64 output function.  Every draw depends only on (q, s, i), so any
 * thread count produces the same bytes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed * GAMMA + 0x632BE59BD9B4E019ULL) ^ (stream * 0xD1B54A32D192ED03ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

/* 53-bit uniform in [0, 1). */
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Standard normal from counters 2i and 2i+1 (Box-Muller, cosine branch). */
static inline double normal_at(uint64_t key, uint64_t i) {
  double u1 = 1.0 - u01(draw(key, 2 * i));     /* (0, 1] */
  double u2 = u01(draw(key, 2 * i + 1));
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

void synth_u01(uint64_t seed, uint64_t stream, int64_t n, double* out) {
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = u01(draw(k, (uint64_t)i));
}

void synth_normal(uint64_t seed, uint64_t stream, int64_t n, double* out) {
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = normal_at(k, (uint64_t)i);
}

/* lognormal(0, 1) rounded to float. */
void synth_lognormal_f32(uint64_t seed, uint64_t stream, int64_t n, float* out) {
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (float)exp(normal_at(k, (uint64_t)i));
}

/* uniform(0, 1) drawn in FP64 and rounded to float. */
void synth_uniform_f32(uint64_t seed, uint64_t stream, int64_t n, float* out) {
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (float)u01(draw(k, (uint64_t)i));
}

/* Fisher-Yates shuffle of [0, L): for j = L-1 down to 1 swap perm[j] with
 * perm[floor(u_j * (j+1))], u_j the j-th draw of the stream. */
void synth_perm(uint64_t seed, uint64_t stream, int64_t L, int32_t* perm) {
  uint64_t k = stream_key(seed, stream);
  for (int64_t i = 0; i < L; ++i) perm[i] = (int32_t)i;
  for (int64_t j = L - 1; j >= 1; --j) {
    int64_t r = (int64_t)(u01(draw(k, (uint64_t)j)) * (double)(j + 1));
    if (r > j) r = j;
    int32_t t = perm[j]; perm[j] = perm[r]; perm[r] = t;
  }
}

/* Coordinates uniform over [0, L): floor(u * L). */
void synth_uniform_idx(uint64_t seed, uint64_t stream, int64_t L, int64_t n, int32_t* out) {
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t v = (int64_t)(u01(draw(k, (uint64_t)i)) * (double)L);
    out[i] = (int32_t)(v < L ? v : L - 1);
  }
}

/* Zipf(s) over ranks 1..L, P(k) = k^-s / H_{L,s}, sampled by inverse CDF:
 * the FP64 prefix table c[k] = sum_{j<=k} j^-s is built in index order, a
 * uniform u is scaled by c[L] and located by binary search (first k with
 * c[k] > u * c[L]).  The rank k maps to coordinate perm[k-1]. */
void synth_zipf_idx(uint64_t seed, uint64_t stream, double s, int64_t L,
                    const int32_t* perm, int64_t n, int32_t* out) {
  double* c = (double*)malloc(sizeof(double) * (size_t)L);
  double acc = 0.0;
  for (int64_t j = 0; j < L; ++j) { acc += pow((double)(j + 1), -s); c[j] = acc; }
  const double total = c[L - 1];
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double x = u01(draw(k, (uint64_t)i)) * total;
    int64_t lo = 0, hi = L - 1;            /* first j with c[j] > x */
    while (lo < hi) {
      int64_t mid = lo + ((hi - lo) >> 1);
      if (c[mid] > x) hi = mid; else lo = mid + 1;
    }
    out[i] = perm[lo];
  }
  free(c);
}

/* The same Zipf draws, faster, in ranges of the counter.
 *
 * synth_zipf_table writes the prefix table c (built exactly as above).
 * synth_zipf_guide writes, for the 2^g buckets of the 53-bit uniform u,
 * guide[b] = first j with c[j] > fl(b 2^-g * total) (L - 1 if none), for
 * b = 0 .. 2^g.  A draw u in bucket b has fl(u * total) between the products
 * of its bucket's two ends (rounded multiplication is monotonic), so its
 * answer lies in [guide[b], guide[b+1]]: the binary search over that range
 * returns exactly the plain search's answer.
 * synth_zipf_idx_range draws counters start .. start+n-1. */
void synth_zipf_table(double s, int64_t L, double* c) {
  double acc = 0.0;
  for (int64_t j = 0; j < L; ++j) { acc += pow((double)(j + 1), -s); c[j] = acc; }
}

static int64_t first_above(const double* c, int64_t lo, int64_t hi, double x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (c[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

void synth_zipf_guide(const double* c, int64_t L, int g, int64_t* guide) {
  const double total = c[L - 1];
  const int64_t B = (int64_t)1 << g;
  const double scale = 1.0 / (double)B;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b <= B; ++b) guide[b] = first_above(c, 0, L - 1, ((double)b * scale) * total);
}

void synth_zipf_idx_range(uint64_t seed, uint64_t stream, const double* c, const int64_t* guide, int g, int64_t L,
                          const int32_t* perm, int64_t start, int64_t n, int32_t* out) {
  const double total = c[L - 1];
  const uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t r = draw(k, (uint64_t)(start + i));
    const double x = u01(r) * total;
    const int64_t b = (int64_t)((r >> 11) >> (53 - g));
    out[i] = perm[first_above(c, guide[b], guide[b + 1], x)];
  }
}

/* Values lognormal(0, 1) rounded to float, counters start .. start+n-1. */
void synth_lognormal_f32_range(uint64_t seed, uint64_t stream, int64_t start, int64_t n, float* out) {
  uint64_t k = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (float)exp(normal_at(k, (uint64_t)(start + i)));
}
