/*
 * sssp.h -- C ABI of the MI355X (gfx950) lower/upper-bound single-source
 * shortest-path library.
 *
 * Method: V. K. Garg, "Removing Sequential Bottleneck of Dijkstra's
 * Algorithm for the Shortest Path Problem".  Every vertex x carries an upper
 * bound D[x] (a feasible path cost, as in Dijkstra's algorithm, Fig. 1) and
 * a lower bound C[x] (Section V: no path to x is cheaper than C[x]).  One
 * data-parallel round (the Section VI / Fig. 6 iteration, in the sound order
 * documented at sssp_solve) relaxes the out-edges of the vertices fixed in
 * the previous round, raises C of every discovered non-fixed vertex from its
 * in-edges (Eq. 1 with the global bound of Lemma crule2), and fixes every
 * vertex whose bounds meet or whose D is within the threshold of Lemma
 * crauser.  Many vertices settle per round instead of Dijkstra's one.
 *
 * Conventions shared by every call:
 *  - Graph and state pointers are DEVICE pointers owned by the caller; they
 *    must stay valid until the work queued on `stream` has completed.
 *    Pointers documented as host pointers are read before the call returns.
 *  - Vertex ids are int32 in [0, n).  Edge ids are positions in the CSR by
 *    tail (the builder's stable order: edges of one tail keep their input
 *    order).  m < 2^31.
 *  - Weights are strictly positive (Section I) and finite: int32 >= 1, or
 *    float32 > 0.  INF ("no path") is INT32_MAX for int32 and +inf for
 *    float32.  For int32 graphs the library requires (n-1) * w_max <
 *    INT32_MAX so that no finite path cost reaches INF.
 *  - Path costs are exact: int32 sums, or the float32 left fold of the path
 *    in path order with one round-to-nearest-even add per edge.  Since
 *    rounding is monotone, the float32 minimum over paths does not depend
 *    on the order in which edges are relaxed.
 *  - Calls are asynchronous on `stream` unless stated otherwise.  Errors a
 *    host can see (null pointers, bad sizes, ids out of range, dtype,
 *    overflow precondition) are returned synchronously and nothing is
 *    queued.  No C++ exception crosses this boundary.
 *  - The library keeps a per-device workspace cache (allocated with
 *    hipMalloc on first use or growth, freed by sssp_release_workspace).
 *    Concurrent calls on one device from several host threads are
 *    serialized by the library.
 */
#ifndef SSSP_H
#define SSSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SSSP_I32 = 0, SSSP_F32 = 1 } sssp_dtype;

typedef enum {
  SSSP_OK = 0,
  SSSP_ERR_ARG = 1,      /* null pointer, bad size, id out of range, dtype */
  SSSP_ERR_GRAPH = 2,    /* edge endpoint out of range in the input edges */
  SSSP_ERR_WEIGHT = 3,   /* weight <= 0, NaN or infinite */
  SSSP_ERR_OVERFLOW = 4, /* int32: (n-1) * w_max >= INT32_MAX */
  SSSP_ERR_NOMEM = 5,    /* workspace allocation failed */
  SSSP_ERR_HIP = 6,      /* a HIP runtime call failed */
  SSSP_ERR_INTERNAL = 7, /* round watchdog tripped (rounds > n + 1, see sssp_check) */
  SSSP_ERR_CAPACITY = 8  /* sssp_solve_noalloc: the solve's state exceeds its static scratch */
} sssp_status;

/*
 * Vertex numbering of the solver's working copy of a graph.  The rounds
 * gather lower and upper bounds of in- and out-neighbours; on skewed
 * degree distributions a numbering by descending degree packs the bounds
 * that are gathered most into few cache lines.  It changes no result:
 * every output and every edge id stays in the caller's numbering.
 *   SSSP_ORDER_AUTO    degree order when the largest total degree is at
 *                      least 16 times the mean, else the input order
 *   SSSP_ORDER_INPUT   the caller's vertex ids
 *   SSSP_ORDER_DEGREE  descending out-degree + in-degree, ties by vertex id
 */
typedef enum { SSSP_ORDER_AUTO = 0, SSSP_ORDER_INPUT = 1, SSSP_ORDER_DEGREE = 2 } sssp_order;

/*
 * Scope of the lower-bound step (C) of a round: the non-fixed vertices
 * whose C it raises.  No result changes (costs, parents); the number of
 * rounds and the work per round do.
 *   SSSP_SCOPE_OPEN  the discovered vertices only (D < INF); undiscovered
 *                    vertices keep C = 0
 *   SSSP_SCOPE_ALL   every non-fixed vertex, as step 4 of SP_4 (Section VI,
 *                    Fig. 6) reads: an undiscovered y gets
 *                    C'[y] = max(C[y], minD, m_y), m_y over all its
 *                    in-edges; unreachable vertices reach C = INF and stop
 *                    holding their out-neighbours' bounds down
 *   SSSP_SCOPE_AUTO  ALL when the largest total degree is at least 3m/n
 *                    (1.5 times the mean), else OPEN.  Graphs with uniform
 *                    degrees (grids, road-like networks) have long diameters:
 *                    their vertices stay undiscovered for many rounds, and
 *                    raising C on all of them costs more than the rounds it
 *                    saves; skewed and random graphs finish discovery within
 *                    a few rounds.
 * Every solve honours the scope of its graph.
 */
typedef enum { SSSP_SCOPE_AUTO = 0, SSSP_SCOPE_OPEN = 1, SSSP_SCOPE_ALL = 2 } sssp_scope;

/*
 * Relax step (A) of a round.  No result changes; rounds and relax work do.
 *   SSSP_RELAX_SETTING     label-setting: the out-edges of the vertices the
 *                          previous round fixed, each once per solve
 *   SSSP_RELAX_CORRECTING  label-correcting, as step 3 of SP_4 (Section VI,
 *                          Fig. 6) explores every discovered vertex: also the
 *                          open vertices whose D fell since their last relax,
 *                          each from its D at the start of the step; a fixed
 *                          vertex already relaxed at its final D is skipped;
 *                          with a finite `delta` (sssp_csr) an open vertex
 *                          joins only while D < minD + delta, minD of the
 *                          round that found it open: the first bucket of
 *                          Delta-stepping (Section I), so delta = 0 is
 *                          label-setting
 *   SSSP_RELAX_AUTO        CORRECTING with delta = 0.4 w_max on graphs of
 *                          low degree spread (deg_max * n < 3m) and wide
 *                          weight spread (w_max >= 16 w_min), where the
 *                          threshold rule fixes few vertices per round;
 *                          SETTING otherwise
 * Honoured per graph by single and batched solves.
 */
typedef enum { SSSP_RELAX_AUTO = 0, SSSP_RELAX_SETTING = 1, SSSP_RELAX_CORRECTING = 2 } sssp_relax;

/*
 * A built graph: CSR by tail plus CSC by head (the incoming-edge access the
 * method assumes, Section I).  All arrays are device arrays in the caller's
 * build buffer.
 *   out_off[n+1], out_dst[m], out_w[m]        CSR; edge id = CSR position
 *   in_off[n+1],  in_src[m], in_eid[m], in_w[m]
 *       CSC; in_eid[j] is the edge id of CSC entry j, and each vertex's
 *       in-list is ascending by edge id; in_w[j] = out_w[in_eid[j]]
 *   out_wmin[n]   minimum out-edge weight per vertex, INF if none (the
 *                 outWeight array of SP_3 and SP_4, Figs. 5 and 6)
 *   w_max         largest weight (filled by the builder; used for the
 *                 int32 overflow precondition)
 *   w_min         smallest weight (filled by the builder; 0 with no edges)
 *   scope         sssp_scope of the single solves on this graph (the
 *                 builder sets SSSP_SCOPE_AUTO; the caller may change it)
 *   relax         sssp_relax of the solves on this graph (likewise AUTO)
 *   deg_max       largest out-degree + in-degree (filled by the builder)
 *   delta         bucket width of label-correcting relax as a key of the
 *                 graph's dtype (the int32 value, or the float32 bit
 *                 pattern); INF (0x7fffffff, or +inf's bits), the
 *                 builder's value, is no bound; must lie in [0, INF]
 * The solver's working copy.  Always: in-lists ordered by weight, so that
 * the in-edges a lower-bound step needs (minD + w < D[y]) form a prefix:
 *   s_in_off[n+1], s_in_src[m] (solver ids), s_in_eid[m], s_in_w[m]
 *       each in-list ascending by (weight, tail solver id, edge id);
 *       s_in_eid holds the edge id of each entry
 * With order == SSSP_ORDER_DEGREE also a renumbered CSR:
 *   vid[k]  vertex id of solver vertex k;  rank[v]  solver id of vertex v
 *   s_out_off[n+1], s_out_dst[m] (solver ids), s_out_w[m], s_out_eid[m]
 *       each out-list ascending by (head solver id, edge id)
 *   s_out_wmin[n]  out_wmin by solver id
 * Always, too:
 *   s_in_sw[2m]: s_in_src and s_in_w of each in-list entry side by side
 *     (entry j at 2j, 2j + 1), so that a scan reads an in-edge's tail and
 *     weight from one place;
 *   s_out_rec[4m]: per entry of the out-lists s_out_* (the CSR itself in
 *     input order), {head solver id, weight, edge id, out_wmin of the
 *     head}, so that a relax reads an out-edge and its head's out_wmin
 *     from one place;
 *   s_vrec[8n], one 32-byte record per solver vertex,
 *     {out_off, out_degree, in_off, in_degree, out_wmin, s_in_src and s_in_w
 *     of the first in-list entry (0, 0 with no in-edges), 0}, so that a
 *     round reads a vertex's offsets, out_wmin and lightest in-edge from one
 *     cache line;
 *   s_vin[4n], the record's in-side half {in_off, in_degree, s_in_src and
 *     s_in_w of the first in-list entry}, for passes that need only that.
 * sssp_set_weights rebuilds every weight-dependent array among them.
 * With SSSP_ORDER_INPUT, solver ids are vertex ids: vid, rank and
 * s_out_eid are NULL and s_out_off/dst/w/wmin alias the CSR arrays.
 * These arrays are library-internal; callers only keep them valid.
 */
typedef struct {
  int32_t n;
  int32_t m;
  int32_t dtype; /* sssp_dtype */
  int32_t order; /* sssp_order the builder applied: INPUT or DEGREE */
  int32_t scope; /* sssp_scope of single solves */
  int32_t relax; /* sssp_relax of every solve on this graph */
  int32_t deg_max; /* largest total degree */
  int32_t delta;   /* label-correcting bucket width (key); INF: none */
  const int32_t *out_off;
  const int32_t *out_dst;
  const void *out_w;
  const int32_t *in_off;
  const int32_t *in_src;
  const int32_t *in_eid;
  const void *in_w;
  const void *out_wmin;
  double w_max;
  double w_min;
  const int32_t *vid;
  const int32_t *rank;
  const int32_t *s_out_off;
  const int32_t *s_out_dst;
  const void *s_out_w;
  const int32_t *s_out_eid;
  const int32_t *s_in_off;
  const int32_t *s_in_src;
  const int32_t *s_in_eid;
  const void *s_in_w;
  const void *s_out_wmin;
  const int32_t *s_vrec;
  const int32_t *s_in_sw;
  const int32_t *s_out_rec;
  const int32_t *s_vin;
} sssp_csr;

/*
 * What the AUTO settings of a graph resolve to, for its single solves on the
 * calling device under that device's default launch geometry
 * (sssp_set_launch): the C scope (SSSP_SCOPE_OPEN or SSSP_SCOPE_ALL), the
 * relax step (SSSP_RELAX_SETTING or SSSP_RELAX_CORRECTING), the bucket width
 * as a key (INF when there is none or the relax is label-setting) and the
 * round kernel that runs.
 */
typedef enum {
  SSSP_KERNEL_PERSISTENT = 0, /* rounds_kernel: cooperative grid, grid barriers */
  SSSP_KERNEL_WORKGROUP = 1,  /* wg_rounds_kernel: one workgroup per solve */
  SSSP_KERNEL_SMALL = 2       /* small_rounds_kernel: one workgroup, state in LDS */
} sssp_kernel;

typedef struct {
  int32_t scope;
  int32_t relax;
  int32_t delta;
  int32_t kernel; /* sssp_kernel */
} sssp_policy;

/* Fills *out for graph g (host pointers); SSSP_ERR_ARG on a malformed graph. */
sssp_status sssp_policy_of(const sssp_csr *g, sssp_policy *out);

/* Per-solve counters (host struct). */
typedef struct {
  int32_t rounds;            /* rounds of the method: runs of step (A), each
                                followed by the loop test (see sssp_solve) */
  int32_t settled;           /* reachable vertices (Dijkstra's removeMin count) */
  int64_t relaxed_edges;     /* out-edges of fixed vertices relaxed (once each) */
  int64_t scanned_in_edges;  /* in-edges the lower-bound step covers: the in-degree
                                summed over open vertices and rounds (an edge with
                                minD + w >= D[y] is covered without gathering C) */
  int64_t open_visits;       /* sum over rounds of |O| (open vertices processed) */
} sssp_stats;

/*
 * Bytes of the device buffer sssp_build_csr fills for a graph of n vertices,
 * m edges, the given dtype and vertex order (AUTO and DEGREE reserve room
 * for the renumbered CSR).  Returns 0 for invalid arguments.
 */
size_t sssp_build_csr_bytes(int32_t n, int32_t m, sssp_dtype dtype, sssp_order order);

/*
 * Build the CSR/CSC of a directed graph from COO edges on the GPU, plus the
 * solver's working copy in the requested vertex order.
 * Inputs (device): src[m], dst[m] vertex ids; w[m] weights (int32 or
 * float32 per dtype).  Self-loops and duplicate edges are kept.
 * buffer: device buffer of at least sssp_build_csr_bytes(n, m, dtype,
 * order) bytes, owned by the caller; *out receives pointers into it.
 * perm (device, nullable): perm[k] = COO index of edge id k.
 * Validates endpoints (SSSP_ERR_GRAPH), weights (SSSP_ERR_WEIGHT) and the
 * int32 overflow precondition (SSSP_ERR_OVERFLOW).  SYNCHRONOUS: returns
 * after the stream work has completed.
 */
sssp_status sssp_build_csr(int32_t n, int32_t m, sssp_dtype dtype, sssp_order order,
                           const int32_t *src, const int32_t *dst, const void *w, void *buffer,
                           size_t buffer_bytes, sssp_csr *out, int32_t *perm, void *stream);

/*
 * Replace the weights of a built graph: w[m] (device) is given in edge-id
 * order; every weight array of *g and w_max are rewritten in place and the
 * working copy's weight-ordered in-lists are rebuilt (the arrays live in the
 * caller's build buffer).  Validates weights and the overflow precondition;
 * on an error nothing is written.  SYNCHRONOUS.
 */
sssp_status sssp_set_weights(sssp_csr *g, const void *w, void *stream);

/*
 * Per-edge values between the caller's COO order and edge-id order, for
 * the weights w(e) of the problem statement (Section I) and gradients with
 * respect to them: the edge ids are CSR positions, and perm (device, m
 * entries, as sssp_build_csr writes it) holds perm[k] = COO index of edge
 * id k, a permutation of 0 .. m-1.
 *   to_coo = 0: out[k] = in[perm[k]]   (COO order -> edge-id order);
 *   to_coo = 1: out[perm[k]] = in[k]   (edge-id order -> COO order).
 * in, out: device arrays of m 4-byte values (float32 or int32), caller
 * owned; they must not overlap.  SSSP_ERR_ARG for m < 0, or a null pointer
 * or in == out with m > 0.  A perm that is not a permutation of 0 .. m-1
 * is not checked (out-of-range entries read or write out of bounds).
 * Asynchronous on `stream`.
 */
sssp_status sssp_permute_edges(const int32_t *perm, int64_t m, const void *in, void *out,
                               int32_t to_coo, void *stream);

/*
 * Single-source shortest paths by rounds of the lower/upper-bound method.
 *   cost[n] (device, dtype of g): cost[x] = minimum path cost (Section I),
 *           INF if x is unreachable.
 *   pred[n] (device, nullable): parent pointer (Section I) as an edge id:
 *           the smallest id among tight in-edges (cost[v] + w == cost[x])
 *           with cost[v] < cost[x]; for float32 graphs where only
 *           equal-cost tight in-edges exist (w below half an ulp of cost),
 *           the smallest id among those whose tail is one breadth-first
 *           level closer to a vertex with a strict tight in-edge inside the
 *           equal-cost class.  -1 for the source and unreachable vertices.
 *   stats (host, nullable): if non-null the call synchronizes the stream
 *           and fills *stats.
 * One round, with O the discovered non-fixed vertices:
 *   (A) relax out-edges of the previous round's newly fixed vertices;
 *   (B) minD = min D over O; thr = min over O of D[y] + out_wmin[y];
 *   (C) for y in O: m_y = min over in-edges (v,y,w), v not fixed, of
 *       max(C[v], minD) + w;  C'[y] = max(C[y], minD, min(D[y], m_y))
 *       (all reads of C before any write);
 *   (D) fix y iff C'[y] >= D[y] or D[y] <= thr.
 * The loop test (is a discovered vertex still not fixed?) follows step (A),
 * as the test of Fig. 6 follows its relax step: the solve stops when (A)
 * leaves O empty, and stats->rounds counts the runs of (A).  Under
 * label-setting relax each run relaxes a non-empty frontier (the last one
 * the final frontier); under label-correcting relax the last run's relax
 * set can be empty, when every vertex the previous round fixed was already
 * relaxed at its final D.  rounds <= settled.
 */
sssp_status sssp_solve(const sssp_csr *g, int32_t source, void *cost, int32_t *pred,
                       sssp_stats *stats, void *stream);

/*
 * sssp_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, same results and counters, with all of its state in one
 * static region of 64 MiB per device that the library's code object holds
 * from load to process end, instead of the workspace cache.  The call makes
 * no hipMalloc, hipFree, event creation or other allocating runtime call
 * (its first call on a device only looks the region's address up).
 *   Arguments, semantics and errors as for sssp_solve, plus
 *   SSSP_ERR_CAPACITY (nothing queued) when the solve's state does not fit
 *   the region: it needs about 148 bytes per vertex plus 0.4 MB, so every
 *   graph with n <= 450,000 fits, whatever its scope and relax step.
 * Every call on one device shares that device's region and leaves its
 * contents behind (each solve initializes what it reads first): calls that
 * overlap on one device race, so order them (one stream, or events).  Calls
 * are not ordered against sssp_solve's workspace use either; neither shares
 * memory with the other.  The round trace and the profiler do not apply.
 */
sssp_status sssp_solve_noalloc(const sssp_csr *g, int32_t source, void *cost, int32_t *pred,
                               sssp_stats *stats, void *stream);

/*
 * Single-target early exit (Section I: a shortest path to one destination
 * can be known as soon as that vertex's bounds meet, before Dijkstra's
 * algorithm would settle it).  The rounds of sssp_solve run until the round
 * whose step (D) fixes `target` (or, if the target is unreachable, to the
 * end); the frontier that round produced is not relaxed.
 *   target in [0, n) (caller's id); target == source stops before round 1.
 *   cost[n] (device): D when the rounds stop: the exact cost for every
 *           vertex fixed by then (the target among them), an upper bound
 *           for the other discovered vertices, INF for the rest.
 *   stats (host, nullable, synchronizes): rounds = rounds to the target,
 *           settled = vertices fixed when the rounds stop, relaxed_edges and
 *           scanned_in_edges = the work of those rounds.
 * No parent pointers: the parent rule needs every in-edge of a vertex
 * offered from a fixed tail, which a stopped solve has not done (call
 * sssp_solve for them).  Errors as for sssp_solve; a target outside [0, n)
 * is SSSP_ERR_ARG.
 */
sssp_status sssp_solve_target(const sssp_csr *g, int32_t source, int32_t target, void *cost,
                              sssp_stats *stats, void *stream);

/*
 * Many independent solves in one persistent launch.
 *   graphs[num_graphs] (host array of built graphs, all of one dtype)
 *   inst_graph[num_inst], inst_source[num_inst] (host): instance i solves
 *           graph inst_graph[i] from inst_source[i].
 *   cost, pred (device): instance i occupies entries
 *           [base_i, base_i + n_i) with base_i = sum_{j<i} n of graph
 *           inst_graph[j]; pred is nullable.  sum of n_i < 2^31.
 *   stats (host, nullable): num_inst entries; synchronizes.
 * Results are identical, instance by instance, to sssp_solve.
 */
sssp_status sssp_solve_batch(const sssp_csr *graphs, int32_t num_graphs,
                             const int32_t *inst_graph, const int32_t *inst_source,
                             int32_t num_inst, void *cost, int32_t *pred, sssp_stats *stats,
                             void *stream);

/*
 * Gradient of L = sum_i sum_x grad_cost[base_i + x] * cost_i[x] with respect
 * to every edge weight, taking cost_i[x] as the weight sum along the pred
 * tree path (an exact derivative where shortest paths are unique).
 *   graphs, inst_graph, inst_source, num_inst as in sssp_solve_batch;
 *   pred (device): the pred output of the forward solve, same layout.
 *   grad_cost (device float32, same layout): entries of unreachable
 *           vertices are ignored.
 *   grad_w (device float32, overwritten): graph g's edges occupy
 *           [ebase_g, ebase_g + m_g) with ebase_g = sum_{h<g} m_h, in edge-id
 *           order; each graph's gradient is summed over its instances in
 *           instance order, so results are deterministic.
 */
sssp_status sssp_backward(const sssp_csr *graphs, int32_t num_graphs, const int32_t *inst_graph,
                          const int32_t *inst_source, int32_t num_inst, const int32_t *pred,
                          const float *grad_cost, float *grad_w, void *stream);

/*
 * Launch geometry of the persistent round kernel.  Geometry changes only
 * the speed of a solve: costs, parents and counters are the same under
 * every setting.  A zero field takes the default.
 *   blocks:      grid size, 1 .. the co-resident maximum (default: that
 *                maximum, one 1024-thread block per compute unit);
 *   solo_edges:  a phase with at most this many edges runs on one block
 *                with block barriers only (default 8192; negative: never);
 *   block_units: otherwise the phase runs on about (work units) /
 *                block_units blocks, a power of two (default 2048);
 *   small_n:     a single solve (sssp_solve, sssp_solve_target, the
 *                sequence plan) of a graph with at most this many vertices
 *                runs all its rounds in one workgroup with the per-vertex
 *                state in LDS (default and maximum 4096; negative: never);
 *   wg:          solves whose graphs all run C scope OPEN run each instance
 *                in a workgroup of its own, with block barriers only (up to
 *                `blocks` workgroups at a time), and so does the tree pass
 *                of sssp_backward: 0 (default) when every graph has low
 *                degree spread (deg_max * n < 3m: many small rounds, deep
 *                trees), 1 always, negative never.
 */
typedef struct {
  int32_t blocks;
  int32_t solo_edges;
  int32_t block_units;
  int32_t small_n;
  int32_t wg;
} sssp_launch;

/*
 * Default geometry of the calling device's sssp_solve, sssp_solve_target
 * and sssp_solve_batch calls (null: back to the defaults).  A blocks value
 * above the co-resident maximum is SSSP_ERR_ARG.
 */
sssp_status sssp_set_launch(const sssp_launch *launch);

/*
 * Replayable solves.  A plan fixes the graphs, instances and output buffers
 * of a batch (the layout of sssp_solve_batch) and records every kernel of
 * the solve once into a HIP graph; sssp_plan_run replays it with one
 * launch.  The round kernel's node is cooperative, as in the direct call.
 *   kind SSSP_PLAN_BATCH:    one persistent launch for all instances, as
 *                            sssp_solve_batch;
 *   kind SSSP_PLAN_SEQUENCE: one single solve (sssp_solve) per instance,
 *                            back to back, into the same layout.
 *   cost, pred (device; pred nullable): written by every run; they, the
 *           graphs' buffers and the graphs' contents must stay valid until
 *           the plan is destroyed (new weights via sssp_set_weights are
 *           picked up by the next run: the plan holds pointers, not values;
 *           each graph's C scope, relax step, bucket width and kernel path
 *           are those it had when the plan was created).
 *   with_stats: non-zero to keep the per-instance counters that
 *           sssp_plan_stats reads (the batch kind counts them in the
 *           kernel, at some cost; the sequence kind always has them).
 *   launch (nullable): geometry of the plan's round kernels.
 * Ownership: the plan allocates its own device state (it shares nothing
 * with the workspace cache or other plans) when created, on the current
 * device; run allocates nothing.  Runs of one plan must not overlap (its
 * state is reused): replay it on one stream, or order the streams.
 * Creation synchronizes the device; errors as for sssp_solve_batch.
 */
typedef enum { SSSP_PLAN_BATCH = 0, SSSP_PLAN_SEQUENCE = 1 } sssp_plan_kind;
typedef struct sssp_plan_s *sssp_plan;

sssp_status sssp_plan_create(const sssp_csr *graphs, int32_t num_graphs,
                             const int32_t *inst_graph, const int32_t *inst_source,
                             int32_t num_inst, sssp_plan_kind kind, void *cost, int32_t *pred,
                             int32_t with_stats, const sssp_launch *launch, sssp_plan *plan);
/* Replay on `stream` (asynchronous).  SSSP_ERR_ARG on another device. */
sssp_status sssp_plan_run(sssp_plan plan, void *stream);
/* Counters of the last run, num_inst entries (host); synchronizes the
 * stream.  SSSP_ERR_ARG for a batch plan created without with_stats. */
sssp_status sssp_plan_stats(sssp_plan plan, sssp_stats *stats, void *stream);
/* Waits for the device, then frees the plan's graph and state. */
sssp_status sssp_plan_destroy(sssp_plan plan);

/*
 * Launch-geometry autotuner: builds a plan for the given solves and times
 * its replays (HIP events on `stream`, `reps` timed runs after one warm-up,
 * mean taken) under candidate geometries, one field at a time (blocks:
 * maximum, 1/2, 1/4; solo_edges: 2048, 8192, 32768; block_units: 1024,
 * 2048, 4096; small_n: the default, never; wg: the default, never, and
 * always when there are at least a quarter as many instances as compute
 * units), keeping a candidate only when it beats the best so far.
 * *best receives the fastest geometry, *best_ms its mean run time.  Writes
 * cost and pred like a run; synchronizes.  Arguments as for
 * sssp_plan_create; reps in [1, 100].
 */
sssp_status sssp_autotune(const sssp_csr *graphs, int32_t num_graphs, const int32_t *inst_graph,
                          const int32_t *inst_source, int32_t num_inst, sssp_plan_kind kind,
                          void *cost, int32_t *pred, int32_t reps, sssp_launch *best,
                          double *best_ms, void *stream);

/*
 * Status of the solves queued so far: waits for `stream`, then returns
 * SSSP_ERR_INTERNAL if any solve on the calling device since the previous
 * sssp_check (direct calls and plan runs, on any stream) ended with a fault
 * status -- the round watchdog tripped (rounds beyond n + 1, or beyond the
 * sssp_set_round_limit limit), or a float32 equal-cost vertex got no parent
 * -- and clears that condition; SSSP_OK otherwise.  Calls given a stats
 * pointer also report the condition in their own return value (and still
 * count for the next sssp_check); this call is how the others (stats ==
 * NULL, plan runs) learn of it.
 */
sssp_status sssp_check(void *stream);

/*
 * Diagnostics: caps the round watchdog of every later solve and plan
 * creation at `limit` rounds (when below the solve's own limit of n + 1);
 * 0 restores the default.  A solve that reaches the cap stops there with
 * incomplete results and reports SSSP_ERR_INTERNAL (through stats or
 * sssp_check).  Process-wide; negative is SSSP_ERR_ARG.
 */
sssp_status sssp_set_round_limit(int32_t limit);

/* Free the calling device's workspace cache and events, and the profiler's
 * events (synchronizes the device).  Later calls set the device up again. */
sssp_status sssp_release_workspace(void);

/*
 * Diagnostics for measurement.  While enabled (on != 0), every launch of
 * the persistent round kernel by sssp_solve / sssp_solve_batch is bracketed
 * by a pair of HIP events recorded on the caller's stream (at most 4096
 * pairs are kept; later launches are not timed until the next read).
 * sssp_profile_read waits for the recorded events, returns the number of
 * timed launches and their summed duration in milliseconds since the last
 * read, and starts a new count.  Both pointers are host pointers.
 */
sssp_status sssp_profile_enable(int on);
sssp_status sssp_profile_read(int64_t *launches, double *total_ms);

/* Static message for a status code. */
const char *sssp_strerror(sssp_status status);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_H */
