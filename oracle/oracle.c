/*
 * CPU oracle for the lower/upper-bound single-source shortest-path method
 * (V. K. Garg, "Removing Sequential Bottleneck of Dijkstra's Algorithm for
 * the Shortest Path Problem").
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct C.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header, table or helper with the GPU
 * library; the two meet only in the arrays written by the seeded generators.
 *
 * Built with plain SSE float arithmetic (no -ffast-math, no FMA
 * contraction), so every float add is one IEEE round-to-nearest-even add.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* Out-adjacency of a COO edge list: off[n+1] and adj[m], the COO indices of
 * each tail's edges in input order (a stable counting sort by tail). */
int oracle_out_adjacency(int32_t n, int64_t m, const int32_t *src, int64_t *off, int32_t *adj) {
  if (n <= 0 || m < 0) return -1;
  for (int32_t v = 0; v <= n; ++v) off[v] = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n) return -2;
    off[src[i] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!fill) return -2;
  for (int32_t v = 0; v < n; ++v) fill[v] = off[v];
  for (int64_t i = 0; i < m; ++i) adj[fill[src[i]]++] = (int32_t)i;
  free(fill);
  return 0;
}

/* --------------------------------------------------------- typed parts */
#define T int32_t
#define SFX i32
#define INF_V INT32_MAX
#define ADD(a, w) (((a) == INT32_MAX || (w) == INT32_MAX) ? INT32_MAX : (a) + (w))
#define ADDSAT(a, w) (((int64_t)(a) + (int64_t)(w) >= INT32_MAX) ? INT32_MAX : (a) + (w))
#include "oracle_typed.inc"
#undef T
#undef SFX
#undef INF_V
#undef ADD
#undef ADDSAT

#define T float
#define SFX f32
#define INF_V INFINITY
#define ADD(a, w) ((float)((float)(a) + (float)(w)))
#define ADDSAT(a, w) ADD(a, w)
#include "oracle_typed.inc"
#undef T
#undef SFX
#undef INF_V
#undef ADD
#undef ADDSAT

#define T double
#define SFX f64
#define INF_V ((double)INFINITY)
#define ADD(a, w) ((a) + (w))
#define ADDSAT(a, w) ADD(a, w)
#include "oracle_typed.inc"
#undef T
#undef SFX
#undef INF_V
#undef ADD
#undef ADDSAT

/* ------------------------------------------------------ stable CSR / CSC */
/*
 * The incoming-edge access the method assumes (Section I) as a CSC next to
 * the CSR.  Stable counting sorts:
 *   CSR by tail, ties in COO order: perm[k] = COO index of CSR position k,
 *     out_dst[k] = dst[perm[k]]; k is the edge id used everywhere.
 *   CSC by head over CSR positions in increasing order, so each in-list is
 *     ascending by edge id: in_eid[j] = CSR position, in_src[j] its tail.
 */
int oracle_csr(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t *out_off,
               int32_t *out_dst, int64_t *perm, int64_t *in_off, int32_t *in_src,
               int64_t *in_eid) {
  if (n <= 0 || m < 0) return -1;
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int32_t *out_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  for (int32_t v = 0; v <= n; ++v) { out_off[v] = 0; in_off[v] = 0; }
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) { free(fill); free(out_src); return -2; }
    out_off[src[i] + 1]++;
    in_off[dst[i] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) { out_off[v + 1] += out_off[v]; in_off[v + 1] += in_off[v]; }
  for (int32_t v = 0; v < n; ++v) fill[v] = out_off[v];
  for (int64_t i = 0; i < m; ++i) {
    int64_t k = fill[src[i]]++;
    perm[k] = i;
    out_dst[k] = dst[i];
    out_src[k] = src[i];
  }
  for (int32_t v = 0; v < n; ++v) fill[v] = in_off[v];
  for (int64_t k = 0; k < m; ++k) {
    int64_t j = fill[out_dst[k]]++;
    in_eid[j] = k;
    in_src[j] = out_src[k];
  }
  free(fill);
  free(out_src);
  return 0;
}

/* ------------------------------------------------------------------- BFS */
/* hop distance from the source (-1 if unreachable): with unit weights the
 * SP_2 theorem says the method behaves as breadth-first search. */
int oracle_bfs(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t source,
               int32_t *hops) {
  if (n <= 0 || source < 0 || source >= n) return -1;
  int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < m; ++i) off[src[i] + 1]++;
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  {
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) fill[v] = off[v];
    for (int64_t i = 0; i < m; ++i) adj[fill[src[i]]++] = dst[i];
    free(fill);
  }
  for (int32_t v = 0; v < n; ++v) hops[v] = -1;
  int32_t head = 0, tail = 0;
  hops[source] = 0;
  queue[tail++] = source;
  while (head < tail) {
    int32_t v = queue[head++];
    for (int64_t q = off[v]; q < off[v + 1]; ++q)
      if (hops[adj[q]] < 0) { hops[adj[q]] = hops[v] + 1; queue[tail++] = adj[q]; }
  }
  free(off); free(adj); free(queue);
  return 0;
}

/* --------------------------------------------------- gradient reference */
/*
 * Gradient of L = sum_s sum_x g[s][x] * cost_s[x] with respect to each edge
 * weight, taking cost_s[x] as the sum of weights along the parent-pointer
 * path from source s to x (the tree the pred rule picks):
 *   acc_s[y] = g[s][y] + sum over tree children c of y of acc_s[c]
 *   dL/dw[e] = sum_s [e == pred_s[head(e)]] * acc_s[head(e)]
 * Unreachable vertices (pred = -1, not the source) contribute nothing.
 * fp64 throughout; tree children found from the CSR (out_off, out_dst) and
 * pred; subtree sums in reverse breadth-first order of the tree.
 */
int oracle_grad(int32_t n, int64_t m, const int64_t *out_off, const int32_t *out_dst,
                int32_t num_src, const int32_t *sources, const int64_t *pred, const double *g,
                double *grad) {
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *acc = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t e = 0; e < m; ++e) grad[e] = 0.0;
  for (int32_t s = 0; s < num_src; ++s) {
    const int64_t *ps = pred + (size_t)s * (size_t)n;
    const double *gs = g + (size_t)s * (size_t)n;
    int32_t head = 0, tail = 0;
    order[tail++] = sources[s];
    while (head < tail) {
      int32_t y = order[head++];
      for (int64_t k = out_off[y]; k < out_off[y + 1]; ++k) {
        int32_t c = out_dst[k];
        if (c != sources[s] && ps[c] == k) order[tail++] = c;
      }
    }
    for (int32_t i = 0; i < tail; ++i) acc[order[i]] = gs[order[i]];
    for (int32_t i = tail - 1; i > 0; --i) {
      int32_t y = order[i];
      int64_t e = ps[y];
      /* tail of edge e: the parent vertex */
      int32_t lo = 0, hi = n; /* find p with out_off[p] <= e < out_off[p+1] */
      while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        if (out_off[mid] <= e) lo = mid; else hi = mid;
      }
      acc[lo] += acc[y];
      grad[e] += acc[y];
    }
  }
  free(order);
  free(acc);
  return 0;
}
