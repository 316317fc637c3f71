/*
 * Seeded synthetic workload generators for the shortest-path benchmarks.
 *
 * This module only draws random numbers and lays out graph topologies,
 * weights and loss coefficients.  It contains no shortest-path arithmetic:
 * both the CPU oracle and the GPU library consume the arrays it writes.
 *
 * Random numbers: a counter-based form of splitmix64 (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).  Every
 * value is mix64(key(seed, stream) + (ctr + 1) * GOLDEN), so any element of
 * any stream can be drawn independently and in parallel, and the output does
 * not depend on the thread count.
 *
 * Graph families (edge lists in COO order, vertex ids 0..n-1):
 *   random : edge i has tail and head uniform in [0, n), the head redrawn
 *            while it equals the tail; duplicates kept.
 *   grid   : rows x cols lattice, id = r * cols + c, every vertex emits its
 *            edges to up, down, left, right neighbours in that order.
 *   rmat   : R-MAT recursive quadrant choice (Chakrabarti, Zhan & Faloutsos,
 *            SDM 2004) with probabilities a, b, c, d per bit level, no noise,
 *            followed by an optional seeded Fisher-Yates relabelling of ids;
 *            duplicates and self-loops kept.
 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed + GOLDEN * (stream + 0x1000ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return mix64(key + (ctr + 1ULL) * GOLDEN);
}

/* Unbiased integer in [0, range) by rejection; element `idx` of the stream
 * owns counters idx*64 .. idx*64+63 (a rejection needs probability
 * range/2^64 per try, so 64 tries are never exhausted in practice; the last
 * try is accepted as is). */
static inline uint64_t uniform_below(uint64_t key, uint64_t idx, uint64_t range) {
  uint64_t thresh = (0ULL - range) % range; /* 2^64 mod range */
  uint64_t x = 0;
  for (uint64_t t = 0; t < 64; ++t) {
    x = draw(key, idx * 64ULL + t);
    if (x >= thresh) break;
  }
  return x % range;
}

uint64_t gen_draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return draw(stream_key(seed, stream), ctr);
}

uint64_t gen_uniform_below(uint64_t seed, uint64_t stream, uint64_t idx, uint64_t range) {
  return uniform_below(stream_key(seed, stream), idx, range);
}

/* ---------------------------------------------------------------- topology */

void gen_random_edges(uint64_t seed, int32_t n, int64_t m, int32_t *src, int32_t *dst) {
  uint64_t kt = stream_key(seed, 1), kh = stream_key(seed, 2);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t t = (int32_t)uniform_below(kt, (uint64_t)i, (uint64_t)n);
    int32_t h = t;
    if (n > 1) {
      /* head draws for edge i use counters i*64*64 ..; redraw on a self-loop */
      for (uint64_t r = 0; h == t; ++r)
        h = (int32_t)uniform_below(kh, (uint64_t)i * 64ULL + r, (uint64_t)n);
    }
    src[i] = t;
    dst[i] = h;
  }
}

int64_t gen_grid_edge_count(int32_t rows, int32_t cols) {
  return 2LL * rows * (cols - 1) + 2LL * cols * (rows - 1);
}

void gen_grid_edges(int32_t rows, int32_t cols, int32_t *src, int32_t *dst) {
  int64_t k = 0;
  for (int32_t r = 0; r < rows; ++r)
    for (int32_t c = 0; c < cols; ++c) {
      int32_t v = r * cols + c;
      if (r > 0)        { src[k] = v; dst[k] = v - cols; ++k; }
      if (r < rows - 1) { src[k] = v; dst[k] = v + cols; ++k; }
      if (c > 0)        { src[k] = v; dst[k] = v - 1;    ++k; }
      if (c < cols - 1) { src[k] = v; dst[k] = v + 1;    ++k; }
    }
}

/* R-MAT: level l of edge i uses counter i*scale + l of stream 3; the 53-bit
 * uniform u picks quadrant a (u<a), b (u<a+b), c (u<a+b+c) or d. */
void gen_rmat_edges(uint64_t seed, int32_t scale, int64_t m, double a, double b, double c,
                    int permute, int32_t *src, int32_t *dst, int32_t *perm_work) {
  uint64_t kq = stream_key(seed, 3);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t t = 0, h = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double u = (double)(draw(kq, (uint64_t)i * (uint64_t)scale + (uint64_t)l) >> 11) *
                 (1.0 / 9007199254740992.0);
      uint32_t tb, hb;
      if (u < a)        { tb = 0; hb = 0; }
      else if (u < ab)  { tb = 0; hb = 1; }
      else if (u < abc) { tb = 1; hb = 0; }
      else              { tb = 1; hb = 1; }
      t = (t << 1) | tb;
      h = (h << 1) | hb;
    }
    src[i] = (int32_t)t;
    dst[i] = (int32_t)h;
  }
  if (!permute) return;
  /* seeded Fisher-Yates relabelling: perm_work[old] = new */
  int32_t n = (int32_t)1 << scale;
  uint64_t kp = stream_key(seed, 4);
  for (int32_t v = 0; v < n; ++v) perm_work[v] = v;
  for (int32_t v = n - 1; v > 0; --v) {
    int32_t j = (int32_t)uniform_below(kp, (uint64_t)v, (uint64_t)v + 1ULL);
    int32_t tmp = perm_work[v]; perm_work[v] = perm_work[j]; perm_work[j] = tmp;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    src[i] = perm_work[src[i]];
    dst[i] = perm_work[dst[i]];
  }
}

/* ----------------------------------------------------------------- weights */

/* integer weights uniform in [lo, hi] (stream 5) */
void gen_weights_int(uint64_t seed, int64_t m, int32_t lo, int32_t hi, int32_t *w) {
  uint64_t kw = stream_key(seed, 5);
  uint64_t range = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) w[i] = lo + (int32_t)uniform_below(kw, (uint64_t)i, range);
}

/* float weights (k + 1) * 2^-24 with k uniform in [0, 2^24): exactly
 * representable values in (0, 1] (stream 6) */
void gen_weights_unit24(uint64_t seed, int64_t m, float *w) {
  uint64_t kw = stream_key(seed, 6);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint64_t k = draw(kw, (uint64_t)i) >> 40;
    w[i] = (float)((double)(k + 1) * (1.0 / 16777216.0));
  }
}

/* float weights 0.5 + k * 2^-23 with k uniform in [0, 2^23]: exactly
 * representable values in [0.5, 1.5] (stream 7) */
void gen_weights_half23(uint64_t seed, int64_t m, float *w) {
  uint64_t kw = stream_key(seed, 7);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint64_t k = uniform_below(kw, (uint64_t)i, (1ULL << 23) + 1ULL);
    w[i] = (float)(0.5 + (double)k * (1.0 / 8388608.0));
  }
}

/* ------------------------------------------------------------ other draws */

/* `count` distinct vertices uniform in [0, n), in draw order (stream 8) */
int gen_distinct_vertices(uint64_t seed, int32_t n, int32_t count, int32_t *out) {
  if (count > n) return -1;
  uint64_t ks = stream_key(seed, 8);
  int32_t got = 0;
  for (uint64_t t = 0; got < count; ++t) {
    int32_t v = (int32_t)uniform_below(ks, t, (uint64_t)n);
    int dup = 0;
    for (int32_t j = 0; j < got; ++j)
      if (out[j] == v) { dup = 1; break; }
    if (!dup) out[got++] = v;
  }
  return 0;
}

/* standard normal draws by Box-Muller, rounded to float (stream 9) */
void gen_normal_f32(uint64_t seed, int64_t count, float *out) {
  uint64_t kn = stream_key(seed, 9);
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    uint64_t x = draw(kn, 2ULL * (uint64_t)i), y = draw(kn, 2ULL * (uint64_t)i + 1ULL);
    double u1 = ((double)(x >> 11) + 1.0) * (1.0 / 9007199254740992.0); /* (0, 1] */
    double u2 = (double)(y >> 11) * (1.0 / 9007199254740992.0);         /* [0, 1) */
    out[i] = (float)(sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
  }
}

/* out-degree argmax, ties to the smallest id (source choice of the R-MAT
 * workload) */
int32_t gen_max_out_degree_vertex(int32_t n, int64_t m, const int32_t *src, int32_t *deg_work) {
  for (int32_t v = 0; v < n; ++v) deg_work[v] = 0;
  for (int64_t i = 0; i < m; ++i) deg_work[src[i]]++;
  int32_t best = 0;
  for (int32_t v = 1; v < n; ++v)
    if (deg_work[v] > deg_work[best]) best = v;
  return best;
}
