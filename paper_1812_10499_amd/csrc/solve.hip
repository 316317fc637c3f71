// Persistent gfx950 kernel for the data-parallel round of the
// lower/upper-bound SSSP method, plus its init and pred post-pass kernels.
//
// One round (D = upper bound, C = lower bound, O = discovered non-fixed
// vertices, F = vertices fixed in the previous round):
//   relax : out-edges of F into D with atomicMin on keys; a head whose old
//           D was INF joins O.  Successful candidates also seed minD
//           (Fig. 1's relaxation; the label-setting form of Fig. 5 step 3).
//   LB    : for y in O, m_y = min over in-edges (v,y,w) of max(C[v],minD)+w
//           (Eq. 1 with the global bound of Lemma crule2; a fixed v has
//           C[v] = INF and drops out); also thr = min D[y] + out_wmin[y]
//           (Lemma crauser).
//   fix   : C'[y] = max(C[y], minD, min(D[y], m_y)); y is fixed iff
//           C'[y] >= D[y] or D[y] <= thr; fixed vertices become the next F
//           (with C = INF), the others stay in O and seed the next minD.
// The three phases are separated by grid barriers, so every read of C in
// LB happens before any write of C in fix (Jacobi), and the round structure
// is deterministic: rounds and per-round fixed sets do not depend on thread
// timing.
//
// Lists (F, O) are compacted arrays of state indices with an exclusive
// prefix of the degree that the next phase expands (out-degree for F,
// in-degree for O).  Blocks append through an LDS staging buffer and one
// 64-bit atomicAdd per flush that reserves both the slots and the degree
// range, so the prefix stays consistent.  The relax and LB phases split the
// list's total edge count evenly across blocks (edge-balanced), so a
// million-edge hub and a degree-2 vertex cost the same per edge.  The
// global minima (minD, thr) of a single solve go through per-block slots
// reduced by every reader, never through one contended word.
#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

constexpr int RBS = kRoundBlock;  // threads per block of the round kernel
constexpr int EPT = 4;            // edges per thread per sub-chunk
constexpr int WIN = RBS;          // list items per window
constexpr int CAP_R = RBS * EPT;  // relax staging capacity (>= one sub-chunk)
constexpr int CAP_F = RBS;        // fix staging capacity per list (>= one pass)

// ----------------------------------------------------------- LDS layouts
template <int CAP>
struct Stager {
  int32_t v[CAP];
  int32_t d[CAP];  // local exclusive degree prefix
  int32_t inst[CAP];
  int32_t cnt;
  uint32_t deg;
  unsigned long long base;
};

struct SmemRelax {
  int32_t pfx[WIN + 1];
  int32_t base[WIN];
  int32_t dx[WIN];
  int32_t sb[WIN];
  int32_t gi[WIN];
  int32_t inst[WIN];
  Stager<CAP_R> st;
};

struct SmemLB {
  int32_t pfx[WIN + 1];
  int32_t base[WIN];
  int32_t acc[WIN];
  int32_t mind[WIN];
  int32_t sb[WIN];
  int32_t gi[WIN];
  int32_t inst[WIN];
};

struct SmemFix {
  Stager<CAP_F> fr;
  Stager<CAP_F> op;
};

struct SmemAll {
  union {
    SmemRelax r;
    SmemLB l;
    SmemFix f;
  } u;
  uint64_t scan[2 * (RBS / SSSP_WAVE + 1)];
  int32_t red[RBS / SSSP_WAVE];
  int32_t tmax;
};

template <bool BATCH>
__device__ __forceinline__ const GraphDev &graph_of(const RoundArgs &a, int gi) {
  if constexpr (BATCH) return a.graphs[gi];
  else return a.g;
}

__device__ __forceinline__ int32_t *part_slot(const RoundArgs &a, int k) {
  return a.part + (size_t)k * kMaxBlocks;
}

// min over the per-block partial slots p0[0..nb) (and p1 if given)
template <class V>
__device__ int32_t reduce_parts(const int32_t *p0, const int32_t *p1, uint32_t nb,
                                SmemAll &sm) {
  int32_t m = V::INF;
  for (uint32_t b = threadIdx.x; b < nb; b += RBS) {
    m = kmin(m, p0[b]);
    if (p1) m = kmin(m, p1[b]);
  }
  return block_min<RBS>(m, sm.red);
}

// -------------------------------------------------------------- staging
// Block-collective flush of an LDS stager into the global list: one 64-bit
// atomicAdd reserves (slots, degree range).  All threads call, after a
// barrier that made st.cnt current.
template <int CAP>
__device__ void stage_flush(Stager<CAP> &st, unsigned long long *ctr, int32_t *lv, int32_t *lp,
                            int32_t *li, bool batch) {
  const int cnt = st.cnt;
  if (cnt == 0) return;
  if (threadIdx.x == 0) {
    unsigned long long inc = ((unsigned long long)cnt << 32) | (unsigned long long)st.deg;
    st.base = atomicAdd(ctr, inc);
  }
  __syncthreads();
  const unsigned long long b = st.base;
  const int32_t bc = (int32_t)(b >> 32);
  const int32_t bd = (int32_t)(uint32_t)(b & 0xffffffffull);
  for (int j = threadIdx.x; j < cnt; j += RBS) {
    lv[bc + j] = st.v[j];
    lp[bc + j] = bd + st.d[j];
    if (batch) li[bc + j] = st.inst[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st.cnt = 0;
    st.deg = 0;
  }
  __syncthreads();
}

// Block-collective push: entry j of the thread's v/d/ins arrays is pushed
// iff bit j of `mask` is set (arrays are indexed by compile-time j only, so
// they stay in VGPRs).  Flushes first when the stager would overflow.
template <int CAP, int K>
__device__ void stage_push(Stager<CAP> &st, uint32_t mask, const int32_t (&v)[K],
                           const int32_t (&d)[K], const int32_t (&ins)[K],
                           unsigned long long *ctr, int32_t *lv, int32_t *lp, int32_t *li,
                           bool batch, SmemAll &sm) {
  uint32_t dsum = 0;
  int n_local = 0;
#pragma unroll
  for (int j = 0; j < K; ++j)
    if ((mask >> j) & 1u) {
      dsum += (uint32_t)d[j];
      ++n_local;
    }
  uint64_t tot;
  const uint64_t ex = block_excl_scan64<RBS>(((uint64_t)n_local << 32) | dsum, sm.scan, &tot);
  const int tcnt = (int)(tot >> 32);
  if (tcnt == 0) return;  // uniform
  if (st.cnt + tcnt > CAP) stage_flush(st, ctr, lv, lp, li, batch);
  int pos = st.cnt + (int)(ex >> 32);
  uint32_t dpos = st.deg + (uint32_t)(ex & 0xffffffffull);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if ((mask >> j) & 1u) {
      st.v[pos] = v[j];
      st.d[pos] = (int32_t)dpos;
      st.inst[pos] = ins[j];
      dpos += (uint32_t)d[j];
      ++pos;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st.cnt += tcnt;
    st.deg += (uint32_t)(tot & 0xffffffffull);
  }
  __syncthreads();
}

// One item per thread into each of two stagers, with a single scan.
struct ListRef {
  unsigned long long *ctr;
  int32_t *v, *p, *i;
};

__device__ void stage_push2(Stager<CAP_F> &s1, bool h1, int32_t v1, int32_t d1, int32_t i1,
                            const ListRef &l1, Stager<CAP_F> &s2, bool h2, int32_t v2,
                            int32_t d2, int32_t i2, const ListRef &l2, bool batch,
                            SmemAll &sm) {
  const uint64_t m1 = h1 ? ((1ull << 32) | (uint32_t)d1) : 0ull;
  const uint64_t m2 = h2 ? ((1ull << 32) | (uint32_t)d2) : 0ull;
  uint64_t ex1, ex2, t1, t2;
  block_excl_scan64x2<RBS>(m1, m2, sm.scan, &ex1, &ex2, &t1, &t2);
  const int c1 = (int)(t1 >> 32), c2 = (int)(t2 >> 32);
  if (c1 && s1.cnt + c1 > CAP_F) stage_flush(s1, l1.ctr, l1.v, l1.p, l1.i, batch);
  if (c2 && s2.cnt + c2 > CAP_F) stage_flush(s2, l2.ctr, l2.v, l2.p, l2.i, batch);
  if (h1) {
    const int pos = s1.cnt + (int)(ex1 >> 32);
    s1.v[pos] = v1;
    s1.d[pos] = (int32_t)(s1.deg + (uint32_t)(ex1 & 0xffffffffull));
    s1.inst[pos] = i1;
  }
  if (h2) {
    const int pos = s2.cnt + (int)(ex2 >> 32);
    s2.v[pos] = v2;
    s2.d[pos] = (int32_t)(s2.deg + (uint32_t)(ex2 & 0xffffffffull));
    s2.inst[pos] = i2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s1.cnt += c1;
    s1.deg += (uint32_t)(t1 & 0xffffffffull);
    s2.cnt += c2;
    s2.deg += (uint32_t)(t2 & 0xffffffffull);
  }
  __syncthreads();
}

// ------------------------------------------- edge-balanced list expansion
// The list has N items whose exclusive degree prefix is lp[] and E edges in
// total.  Block b takes edges [e0, e1) with e0 = E*b/nb.  Returns the first
// item whose edge range contains e0 (last item with lp <= e0), found by a
// block-cooperative RBS-ary search (3 steps for millions of items).
__device__ int find_start_item(const int32_t *lp, int N, uint32_t e0, SmemAll &sm) {
  int lo = 0, hi = N;
  while (hi - lo > 1) {
    const int span = hi - lo;
    const int pos = lo + (int)(((int64_t)span * threadIdx.x) / RBS);
    const bool le = (uint32_t)lp[pos] <= e0;  // pos < hi always; pos == lo for thread 0
    if (threadIdx.x == 0) sm.tmax = 0;
    __syncthreads();
    if (le) atomicMax(&sm.tmax, (int)threadIdx.x);
    __syncthreads();
    const int t = sm.tmax;
    const int nlo = lo + (int)(((int64_t)span * t) / RBS);
    const int nhi = (t == RBS - 1) ? hi : lo + (int)(((int64_t)span * (t + 1)) / RBS);
    __syncthreads();
    lo = nlo;
    hi = nhi;
  }
  return lo;
}

// last window position p in [0, WIN) with pfx[p] <= e
__device__ __forceinline__ int window_item(const int32_t *pfx, uint32_t e) {
  int lo = 0, len = WIN;
  while (len > 1) {
    const int half = len >> 1;
    if ((uint32_t)pfx[lo + half] <= e) lo += half;
    len -= half;
  }
  return lo;
}

// ------------------------------------------------------------ the kernel
template <class V, bool BATCH>
__global__ __launch_bounds__(RBS) void rounds_kernel(RoundArgs a) {
  __shared__ SmemAll sm;
  const int tid = threadIdx.x;
  const uint32_t nb = gridDim.x, bid = blockIdx.x;
  Ctl *ctl = a.ctl;
  const int I = a.num_inst;
  unsigned int epoch = 0;
  int r = 0;
  // single-instance counters, kept by block 0 thread 0
  long long st_settled = 0, st_relaxed = 0, st_scanned = 0, st_open = 0;

  for (;;) {
    ++r;
    const int cur = r & 1;
    int32_t *Ov = cur ? a.open_v1 : a.open_v0;
    int32_t *Op = cur ? a.open_p1 : a.open_p0;
    int32_t *Oi = cur ? a.open_i1 : a.open_i0;
    const ListRef next_open = {&ctl->open_ctr[cur ^ 1], cur ? a.open_v0 : a.open_v1,
                               cur ? a.open_p0 : a.open_p1, cur ? a.open_i0 : a.open_i1};
    const ListRef front = {&ctl->front_ctr, a.front_v, a.front_p, a.front_i};
    const int s_now = r % 3, s_next = (r + 1) % 3;

    if (r > a.max_rounds) {  // watchdog: rounds never exceed the reachable count
      if (bid == 0 && tid == 0) ctl->status = 7;
      break;
    }

    // =============================================================== relax
    const uint64_t fc = ld_relaxed64(&ctl->front_ctr);
    const int NF = (int)(fc >> 32);
    const uint32_t EF = (uint32_t)(fc & 0xffffffffull);
    long long *tr = (a.trace && r <= a.trace_rounds) ? a.trace + (size_t)(r - 1) * kTraceFields
                                                      : nullptr;
    if (tr && bid == 0 && tid == 0) {
      tr[TR_START] = (long long)wall_clock64();
      tr[TR_NF] = NF;
      tr[TR_EF] = EF;
    }
    if (bid == 0) {
      if (tid == 0) {
        ctl->open_ctr[cur ^ 1] = 0ull;
        st_settled += NF;
        st_relaxed += EF;
      }
      if constexpr (BATCH) {
        for (int i = tid; i < I; i += RBS) {
          a.imin[s_next * I + i] = V::INF;
          a.ithr[s_next * I + i] = V::INF;
        }
      }
    }
    if constexpr (BATCH) {
      // per-instance round count: the last round with a non-empty frontier
      for (int i = bid * RBS + tid; i < NF; i += nb * RBS) a.irounds[a.front_i[i]] = r;
    }
    {
      int32_t lmin = V::INF;
      const uint32_t e0 = (uint32_t)(((uint64_t)EF * bid) / nb);
      const uint32_t e1 = (uint32_t)(((uint64_t)EF * (bid + 1)) / nb);
      SmemRelax &S = sm.u.r;
      if (tid == 0) {
        S.st.cnt = 0;
        S.st.deg = 0;
      }
      __syncthreads();
      if (e0 < e1) {
        int i = find_start_item(a.front_p, NF, e0, sm);
        uint32_t k = e0;
        while (k < e1) {
          const int idx = i + tid;
          if (idx < NF) {
            const int32_t gx = a.front_v[idx];
            S.pfx[tid] = a.front_p[idx];
            int32_t sb = 0, gi = 0, ins = 0;
            if constexpr (BATCH) {
              ins = a.front_i[idx];
              const InstDev id = a.insts[ins];
              sb = id.sbase;
              gi = id.graph;
            }
            const GraphDev &G = graph_of<BATCH>(a, gi);
            S.base[tid] = G.out_off[gx - sb];
            S.dx[tid] = a.D[gx];
            S.sb[tid] = sb;
            S.gi[tid] = gi;
            S.inst[tid] = ins;
          } else {
            S.pfx[tid] = (int32_t)EF;
          }
          if (tid == 0) S.pfx[WIN] = (i + WIN < NF) ? a.front_p[i + WIN] : (int32_t)EF;
          __syncthreads();
          const uint32_t wend = min((uint32_t)S.pfx[WIN], e1);
          for (uint32_t cb = k; cb < wend; cb += RBS * EPT) {
            // gathers for all EPT edges are issued before any result is used
            int it[EPT];
            int32_t pos[EPT], y[EPT], wt[EPT], cand[EPT], gy[EPT], dy[EPT];
            bool val[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              const uint32_t e = cb + (uint32_t)(j * RBS + tid);
              val[j] = e < wend;
              it[j] = val[j] ? window_item(S.pfx, e) : 0;
              pos[j] = S.base[it[j]] + (int32_t)(e - (uint32_t)S.pfx[it[j]]);
            }
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              if (val[j]) {
                const GraphDev &G = graph_of<BATCH>(a, S.gi[it[j]]);
                y[j] = G.out_dst[pos[j]];
                wt[j] = G.out_w[pos[j]];
              }
            }
            if (a.coherent_filter) {
#pragma unroll
              for (int j = 0; j < EPT; ++j) {
                if (val[j]) {
                  cand[j] = V::add(S.dx[it[j]], wt[j]);
                  gy[j] = S.sb[it[j]] + y[j];
                  dy[j] = ld_relaxed(&a.D[gy[j]]);
                }
              }
            } else {
#pragma unroll
              for (int j = 0; j < EPT; ++j) {
                if (val[j]) {
                  cand[j] = V::add(S.dx[it[j]], wt[j]);
                  gy[j] = S.sb[it[j]] + y[j];
                  dy[j] = a.D[gy[j]];
                }
              }
            }
            int32_t nv[EPT], nd[EPT], ni[EPT];
            uint32_t nmask = 0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              if (val[j] && cand[j] < dy[j]) {
                const int32_t old = atomicMin(&a.D[gy[j]], cand[j]);
                if constexpr (BATCH) {
                  atomicMin(&a.imin[s_now * I + S.inst[it[j]]], cand[j]);
                } else {
                  lmin = kmin(lmin, cand[j]);
                }
                if (old == V::INF) nmask |= 1u << j;
              }
            }
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              if ((nmask >> j) & 1u) {
                const GraphDev &G = graph_of<BATCH>(a, S.gi[it[j]]);
                nv[j] = gy[j];
                nd[j] = G.in_off[y[j] + 1] - G.in_off[y[j]];
                ni[j] = S.inst[it[j]];
              } else {
                nv[j] = nd[j] = ni[j] = 0;
              }
            }
            stage_push<CAP_R, EPT>(S.st, nmask, nv, nd, ni, &ctl->open_ctr[cur], Ov, Op, Oi,
                                   BATCH, sm);
          }
          __syncthreads();
          k = wend;
          i += WIN;
        }
      }
      __syncthreads();
      stage_flush(S.st, &ctl->open_ctr[cur], Ov, Op, Oi, BATCH);
      if constexpr (!BATCH) {
        const int32_t bm = block_min<RBS>(lmin, sm.red);
        if (tid == 0) part_slot(a, P_CAND0 + cur)[bid] = bm;
      }
    }
    long long *tb = (a.trace_blk && r <= a.trace_blk_rounds)
                        ? a.trace_blk + (size_t)(r - 1) * 3 * kMaxBlocks + bid
                        : nullptr;
    if (tb && tid == 0) tb[0] = (long long)wall_clock64();
    if (tr && bid == 0 && tid == 0) tr[TR_ARR_RELAX] = (long long)wall_clock64();
    grid_barrier(a.flags, &ctl->go, epoch);

    const uint64_t oc = ld_relaxed64(&ctl->open_ctr[cur]);
    const int NO = (int)(oc >> 32);
    const uint32_t EO = (uint32_t)(oc & 0xffffffffull);
    if (tr && bid == 0 && tid == 0) {
      tr[TR_END_RELAX] = (long long)wall_clock64();
      tr[TR_NO] = NO;
      tr[TR_EO] = EO;
    }
    if (NO == 0) break;  // nothing left open: every reachable vertex is fixed

    // ================================================================== LB
    if (bid == 0 && tid == 0) {
      ctl->front_ctr = 0ull;
      st_scanned += EO;
      st_open += NO;
    }
    int32_t mind_all = V::INF;
    if constexpr (!BATCH)
      mind_all = reduce_parts<V>(part_slot(a, P_SURV0 + cur), part_slot(a, P_CAND0 + cur), nb, sm);
    {
      int32_t lthr = V::INF;
      const uint32_t e0 = (uint32_t)(((uint64_t)EO * bid) / nb);
      const uint32_t e1 = (uint32_t)(((uint64_t)EO * (bid + 1)) / nb);
      SmemLB &S = sm.u.l;
      if (e0 < e1) {
        int i = find_start_item(Op, NO, e0, sm);
        uint32_t k = e0;
        while (k < e1) {
          const int idx = i + tid;
          S.acc[tid] = V::INF;
          if (idx < NO) {
            const int32_t gy = Ov[idx];
            S.pfx[tid] = Op[idx];
            int32_t sb = 0, gi = 0, ins = 0;
            int32_t md = mind_all;
            if constexpr (BATCH) {
              ins = Oi[idx];
              const InstDev id = a.insts[ins];
              sb = id.sbase;
              gi = id.graph;
              md = ld_relaxed(&a.imin[s_now * I + ins]);
            }
            const GraphDev &G = graph_of<BATCH>(a, gi);
            S.base[tid] = G.in_off[gy - sb];
            S.mind[tid] = md;
            S.sb[tid] = sb;
            S.gi[tid] = gi;
            S.inst[tid] = ins;
          } else {
            S.pfx[tid] = (int32_t)EO;
          }
          if (tid == 0) S.pfx[WIN] = (i + WIN < NO) ? Op[i + WIN] : (int32_t)EO;
          __syncthreads();
          const uint32_t wend = min((uint32_t)S.pfx[WIN], e1);
          for (uint32_t cb = k; cb < wend; cb += RBS * EPT) {
            int it[EPT];
            int32_t pos[EPT], v[EPT], wt[EPT], cv[EPT];
            bool val[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              const uint32_t e = cb + (uint32_t)(j * RBS + tid);
              val[j] = e < wend;
              it[j] = val[j] ? window_item(S.pfx, e) : 0;
              pos[j] = S.base[it[j]] + (int32_t)(e - (uint32_t)S.pfx[it[j]]);
            }
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              if (val[j]) {
                const GraphDev &G = graph_of<BATCH>(a, S.gi[it[j]]);
                v[j] = G.in_src[pos[j]];
                wt[j] = G.in_w[pos[j]];
              }
            }
#pragma unroll
            for (int j = 0; j < EPT; ++j)
              if (val[j]) cv[j] = a.C[S.sb[it[j]] + v[j]];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              const int32_t t = val[j] ? V::add(kmax(cv[j], S.mind[it[j]]), wt[j]) : V::INF;
              const int myit = val[j] ? it[j] : -1;
              // segmented min into LDS; one LDS atomic per wave when the
              // whole wave works on one item (hub vertices)
              const uint64_t act = __ballot(val[j]);
              if (act) {
                const int lead = __ffsll((unsigned long long)act) - 1;
                const int it0 = __shfl(myit, lead, SSSP_WAVE);
                const uint64_t same = __ballot(val[j] && myit == it0);
                if (same == act) {
                  const int32_t wm = wave_min(t);
                  if (lane_id() == lead && wm < V::INF) atomicMin(&S.acc[it0], wm);
                } else if (val[j] && t < V::INF) {
                  atomicMin(&S.acc[myit], t);
                }
              }
            }
          }
          __syncthreads();
          // flush the window: item tid of this window
          if (idx < NO) {
            const uint32_t p0 = (uint32_t)S.pfx[tid], p1 = (uint32_t)S.pfx[tid + 1];
            const bool touched = p0 < e1 && p1 > e0 && p1 > p0;
            if (touched) {
              const int32_t acc = S.acc[tid];
              if (p0 >= e0 && p1 <= e1) a.mtmp[idx] = acc;
              else if (acc < V::INF) atomicMin(&a.mtmp[idx], acc);
            }
            if (p0 >= e0 && p0 < e1) {  // owner of the item's first edge
              const GraphDev &G = graph_of<BATCH>(a, S.gi[tid]);
              const int32_t gy = Ov[idx];
              const int32_t yl = gy - S.sb[tid];
              const int32_t th = V::add(a.D[gy], G.out_wmin[yl]);
              if constexpr (BATCH) {
                atomicMin(&a.ithr[s_now * I + S.inst[tid]], th);
                atomicAdd(&a.iscanned[2 * S.inst[tid]], (unsigned long long)(p1 - p0));
                atomicAdd(&a.iscanned[2 * S.inst[tid] + 1], 1ull);
              } else {
                lthr = kmin(lthr, th);
              }
            }
          }
          __syncthreads();
          k = wend;
          i += WIN;
        }
      }
      if constexpr (!BATCH) {
        const int32_t bm = block_min<RBS>(lthr, sm.red);
        if (tid == 0) part_slot(a, P_THR0 + cur)[bid] = bm;
      }
    }
    if (tb && tid == 0) tb[kMaxBlocks] = (long long)wall_clock64();
    if (tr && bid == 0 && tid == 0) tr[TR_ARR_LB] = (long long)wall_clock64();
    grid_barrier(a.flags, &ctl->go, epoch);
    if (tr && bid == 0 && tid == 0) tr[TR_END_LB] = (long long)wall_clock64();

    // ================================================================= fix
    {
      SmemFix &S = sm.u.f;
      if (tid == 0) {
        S.fr.cnt = 0;
        S.fr.deg = 0;
        S.op.cnt = 0;
        S.op.deg = 0;
      }
      int32_t thr_all = V::INF;
      if constexpr (!BATCH) thr_all = reduce_parts<V>(part_slot(a, P_THR0 + cur), nullptr, nb, sm);
      __syncthreads();
      int32_t lnext = V::INF;
      for (int b0 = (int)bid * RBS; b0 < NO; b0 += (int)nb * RBS) {
        const int idx = b0 + tid;
        bool hf = false, ho = false;
        int32_t gy = 0, fd = 0, od = 0, ins = 0;
        if (idx < NO) {
          gy = Ov[idx];
          const int32_t m = a.mtmp[idx];
          a.mtmp[idx] = V::INF;
          const uint32_t p0 = (uint32_t)Op[idx];
          const uint32_t p1 = (idx + 1 < NO) ? (uint32_t)Op[idx + 1] : EO;
          int32_t sb = 0, gi = 0;
          int32_t md = mind_all, th = thr_all;
          if constexpr (BATCH) {
            ins = Oi[idx];
            const InstDev id = a.insts[ins];
            sb = id.sbase;
            gi = id.graph;
            md = ld_relaxed(&a.imin[s_now * I + ins]);
            th = ld_relaxed(&a.ithr[s_now * I + ins]);
          }
          const int32_t Dy = a.D[gy];
          const int32_t Cy = a.C[gy];
          const int32_t Cn = kmax(kmax(Cy, md), kmin(Dy, m));
          if (Cn >= Dy || Dy <= th) {
            a.C[gy] = V::INF;  // fixed: drops out of every later lower-bound scan
            const GraphDev &G = graph_of<BATCH>(a, gi);
            const int32_t yl = gy - sb;
            fd = G.out_off[yl + 1] - G.out_off[yl];
            hf = true;
          } else {
            a.C[gy] = Cn;
            od = (int32_t)(p1 - p0);
            ho = true;
            if constexpr (BATCH) atomicMin(&a.imin[s_next * I + ins], Dy);
            else lnext = kmin(lnext, Dy);
          }
        }
        stage_push2(S.fr, hf, gy, fd, ins, front, S.op, ho, gy, od, ins, next_open, BATCH, sm);
      }
      stage_flush(S.fr, front.ctr, front.v, front.p, front.i, BATCH);
      stage_flush(S.op, next_open.ctr, next_open.v, next_open.p, next_open.i, BATCH);
      if constexpr (!BATCH) {
        const int32_t bm = block_min<RBS>(lnext, sm.red);
        if (tid == 0) part_slot(a, P_SURV0 + (cur ^ 1))[bid] = bm;
      }
    }
    if (tb && tid == 0) tb[2 * kMaxBlocks] = (long long)wall_clock64();
    if (tr && bid == 0 && tid == 0) tr[TR_ARR_FIX] = (long long)wall_clock64();
    grid_barrier(a.flags, &ctl->go, epoch);
    if (tr && bid == 0 && tid == 0) tr[TR_END_FIX] = (long long)wall_clock64();
  }

  if (bid == 0 && tid == 0) {
    ctl->rounds = r > a.max_rounds ? a.max_rounds : r;
    ctl->settled = st_settled;
    ctl->relaxed = st_relaxed;
    ctl->scanned = st_scanned;
    ctl->open_visits = st_open;
  }
}

// ------------------------------------------------------------------ init
// D = INF, C = 0, mtmp = INF over all state entries; barrier flags and the
// per-block partial slots are reset.
template <class V>
__global__ void init_fill_kernel(int32_t *D, int32_t *C, int32_t *mtmp, int32_t total,
                                 unsigned int *flags, int32_t *part) {
  const int32_t stride = gridDim.x * blockDim.x;
  const int32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int32_t i = t0; i < total; i += stride) {
    D[i] = V::INF;
    C[i] = 0;
    mtmp[i] = V::INF;
  }
  for (int32_t i = t0; i < kMaxBlocks; i += stride) flags[i * kFlagStride] = 0u;
  for (int32_t i = t0; i < kParts * kMaxBlocks; i += stride) part[i] = V::INF;
}

// One block: seeds every instance's source, the first frontier (with its
// out-degree prefix) and the control block.
template <class V, bool BATCH>
__global__ void init_seed_kernel(RoundArgs a) {
  __shared__ uint64_t scan[RBS / SSSP_WAVE + 1];
  const int I = a.num_inst;
  uint64_t run = 0;
  for (int b0 = 0; b0 < I; b0 += RBS) {
    const int i = b0 + threadIdx.x;
    uint32_t deg = 0;
    int32_t gs = 0;
    if (i < I) {
      int32_t sb = 0, gi = 0, s = a.source;
      if constexpr (BATCH) {
        const InstDev id = a.insts[i];
        sb = id.sbase;
        gi = id.graph;
        s = id.source;
      }
      const GraphDev &G = graph_of<BATCH>(a, gi);
      gs = sb + s;
      deg = (uint32_t)(G.out_off[s + 1] - G.out_off[s]);
      a.D[gs] = 0;
      a.C[gs] = V::INF;
    }
    uint64_t tot;
    const uint64_t ex = block_excl_scan64<RBS>((uint64_t)deg, scan, &tot);
    if (i < I) {
      a.front_v[i] = gs;
      a.front_p[i] = (int32_t)(run + ex);
      if constexpr (BATCH) {
        a.front_i[i] = i;
        for (int s = 0; s < 3; ++s) {
          a.imin[s * I + i] = V::INF;
          a.ithr[s * I + i] = V::INF;
        }
        a.irounds[i] = 0;
        a.iscanned[2 * i] = 0ull;
        a.iscanned[2 * i + 1] = 0ull;
        if (a.istat) {
          a.istat[4 * i + 0] = 0;
          a.istat[4 * i + 1] = 0;
          a.istat[4 * i + 2] = 0;
          a.istat[4 * i + 3] = 0;
        }
      }
    }
    run += tot;
  }
  if (threadIdx.x == 0) {
    Ctl *c = a.ctl;
    c->front_ctr = ((unsigned long long)I << 32) | (run & 0xffffffffull);
    c->open_ctr[0] = 0ull;
    c->open_ctr[1] = 0ull;
    c->go = 0u;
    c->status = 0;
    c->rounds = 0;
    c->settled = c->relaxed = c->scanned = c->open_visits = 0;
    c->deg_count = 0;
    c->heavy_count = 0;
  }
}

// ------------------------------------------------------------------ pred
// pred[y] = smallest edge id among in-edges (v,y,w) with D[v] + w == D[y]
// and D[v] < D[y] (in-lists are ascending by edge id, so the first hit in
// list order).  Thread per vertex for in-degree <= PRED_LIGHT; heavier
// vertices are queued for a wave each; float32 vertices with only
// equal-cost tight edges are queued for the level pass.
constexpr int PRED_LIGHT = 32;

template <class V, bool BATCH>
__global__ __launch_bounds__(256) void pred_light_kernel(RoundArgs a, int32_t *pred,
                                                         int32_t *heavy, int32_t *degen,
                                                         int32_t *lvl, long long *istat) {
  const int inst = BATCH ? (int)blockIdx.y : 0;
  int32_t sb = 0, gi = 0, s = a.source, n = a.g.n;
  if constexpr (BATCH) {
    const InstDev id = a.insts[inst];
    sb = id.sbase;
    gi = id.graph;
    s = id.source;
    n = id.n;
  }
  const GraphDev &G = graph_of<BATCH>(a, gi);
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  long long c_settled = 0, c_relaxed = 0;
  if (y < n) {
    const int32_t gy = sb + y;
    const int32_t dy = a.D[gy];
    int32_t p = -1;
    if (dy != V::INF) {
      c_settled = 1;
      c_relaxed = G.out_off[y + 1] - G.out_off[y];
    }
    if (y != s && dy != V::INF) {
      const int32_t j0 = G.in_off[y], j1 = G.in_off[y + 1];
      if (j1 - j0 > PRED_LIGHT) {
        p = -3;
        const int q = atomicAdd(&a.ctl->heavy_count, 1);
        heavy[q] = gy;
        heavy[a.total + q] = inst;
      } else {
        for (int32_t j = j0; j < j1; ++j) {
          const int32_t dv = a.D[sb + G.in_src[j]];
          if (dv < dy && V::add(dv, G.in_w[j]) == dy) {
            p = G.in_eid[j];
            break;
          }
        }
        if (p < 0) {
          // reachable with no strict tight in-edge: only equal-cost ones
          p = -2;
          const int q = atomicAdd(&a.ctl->deg_count, 1);
          degen[q] = gy;
          degen[a.total + q] = inst;
          lvl[gy] = -1;
        }
      }
    }
    pred[gy] = p;
  }
  if (istat) {
    const long long s1 = wave_sum64(c_settled), s2 = wave_sum64(c_relaxed);
    if (lane_id() == 0 && (s1 | s2)) {
      atomicAdd((unsigned long long *)&istat[4 * inst + 1], (unsigned long long)s1);
      atomicAdd((unsigned long long *)&istat[4 * inst + 2], (unsigned long long)s2);
    }
  }
}

template <class V, bool BATCH>
__global__ __launch_bounds__(256) void pred_heavy_kernel(RoundArgs a, int32_t *pred,
                                                         const int32_t *heavy, int32_t *degen,
                                                         int32_t *lvl) {
  const int nh = ld_relaxed(&a.ctl->heavy_count);
  const int wpb = blockDim.x / SSSP_WAVE;
  for (int q = blockIdx.x * wpb + threadIdx.x / SSSP_WAVE; q < nh; q += gridDim.x * wpb) {
    const int32_t gy = heavy[q];
    const int inst = heavy[a.total + q];
    int32_t sb = 0, gi = 0;
    if constexpr (BATCH) {
      const InstDev id = a.insts[inst];
      sb = id.sbase;
      gi = id.graph;
    }
    const GraphDev &G = graph_of<BATCH>(a, gi);
    const int32_t y = gy - sb;
    const int32_t dy = a.D[gy];
    const int32_t j0 = G.in_off[y], j1 = G.in_off[y + 1];
    int32_t p = -2;
    for (int32_t jb = j0; jb < j1; jb += SSSP_WAVE) {
      const int32_t j = jb + lane_id();
      bool hit = false;
      if (j < j1) {
        const int32_t dv = a.D[sb + G.in_src[j]];
        hit = (dv < dy) && (V::add(dv, G.in_w[j]) == dy);
      }
      const uint64_t bal = __ballot(hit);
      if (bal) {
        const int src_lane = __ffsll((unsigned long long)bal) - 1;
        p = __shfl(j < j1 ? G.in_eid[j] : 0, src_lane, SSSP_WAVE);
        break;
      }
    }
    if (lane_id() == 0) {
      pred[gy] = p;
      if (p == -2) {
        const int qq = atomicAdd(&a.ctl->deg_count, 1);
        degen[qq] = gy;
        degen[a.total + qq] = inst;
        lvl[gy] = -1;
      }
    }
  }
}

// Equal-cost tie pass (float32 only; one block).  level 0: the source and
// every vertex with a strict tight in-edge; a queued vertex y gets
// level(y) = 1 + min level over tails v with D[v] == D[y] and D[v] + w ==
// D[y]; pred[y] = smallest such edge id with level(v) = level(y) - 1.
template <class V, bool BATCH>
__global__ __launch_bounds__(1024) void pred_degen_kernel(RoundArgs a, int32_t *pred,
                                                          const int32_t *degen, int32_t *lvl,
                                                          int32_t *flag) {
  __shared__ int changed;
  const int nd = ld_relaxed(&a.ctl->deg_count);
  if (nd == 0) return;
  for (int lv = 0;; ++lv) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < nd; q += blockDim.x) {
      flag[q] = 0;
      const int32_t gy = degen[q];
      if (lvl[gy] != -1) continue;
      const int inst = degen[a.total + q];
      int32_t sb = 0, gi = 0;
      if constexpr (BATCH) {
        const InstDev id = a.insts[inst];
        sb = id.sbase;
        gi = id.graph;
      }
      const GraphDev &G = graph_of<BATCH>(a, gi);
      const int32_t y = gy - sb, dy = a.D[gy];
      for (int32_t j = G.in_off[y]; j < G.in_off[y + 1]; ++j) {
        const int32_t gv = sb + G.in_src[j];
        const int32_t dv = a.D[gv];
        if (dv == dy && V::add(dv, G.in_w[j]) == dy) {
          const int32_t lv_v = (pred[gv] == -2) ? lvl[gv] : 0;
          if (lv_v == lv) {
            flag[q] = 1;
            break;
          }
        }
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nd; q += blockDim.x) {
      if (flag[q]) {
        lvl[degen[q]] = lv + 1;
        changed = 1;
      }
    }
    __syncthreads();
    if (!changed) break;
  }
  for (int q = threadIdx.x; q < nd; q += blockDim.x) {
    const int32_t gy = degen[q];
    const int inst = degen[a.total + q];
    int32_t sb = 0, gi = 0;
    if constexpr (BATCH) {
      const InstDev id = a.insts[inst];
      sb = id.sbase;
      gi = id.graph;
    }
    const GraphDev &G = graph_of<BATCH>(a, gi);
    const int32_t y = gy - sb, dy = a.D[gy], ly = lvl[gy];
    int32_t best = -1;
    if (ly >= 1) {
      for (int32_t j = G.in_off[y]; j < G.in_off[y + 1]; ++j) {
        const int32_t gv = sb + G.in_src[j];
        const int32_t dv = a.D[gv];
        if (dv == dy && V::add(dv, G.in_w[j]) == dy) {
          const int32_t lv_v = (pred[gv] == -2) ? lvl[gv] : 0;
          if (lv_v == ly - 1) {
            best = G.in_eid[j];
            break;
          }
        }
      }
    }
    flag[q] = best;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nd; q += blockDim.x) {
    pred[degen[q]] = flag[q];
    if (flag[q] < 0) a.ctl->status = 7;
  }
}

// ------------------------------------------------------- host launchers
template <class V, bool BATCH>
static hipError_t launch_solve_t(const RoundArgs &a, int32_t *pred, const LaunchGeom &geo,
                                 long long *istat, int32_t max_n, const KernelTimer *timer,
                                 hipStream_t stream) {
  hipError_t e;
  if (geo.blocks > kMaxBlocks) return hipErrorInvalidConfiguration;
  {
    int blocks = (int)((a.total + 255) / 256);
    if (blocks < (kParts * kMaxBlocks) / 256) blocks = (kParts * kMaxBlocks) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(init_fill_kernel<V>, dim3(blocks), dim3(256), 0, stream, a.D, a.C,
                       a.mtmp, a.total, a.flags, a.part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((init_seed_kernel<V, BATCH>), dim3(1), dim3(RBS), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    RoundArgs arg = a;
    void *params[] = {&arg};
    if (timer && (e = hipEventRecord(timer->start, stream)) != hipSuccess) return e;
    e = hipLaunchCooperativeKernel((const void *)rounds_kernel<V, BATCH>, dim3(geo.blocks),
                                   dim3(RBS), params, 0, stream);
    if (e != hipSuccess) return e;
    if (timer && (e = hipEventRecord(timer->stop, stream)) != hipSuccess) return e;
  }
  if (pred || istat) {
    int32_t *p = pred ? pred : a.scratch_pred;
    const dim3 grid((max_n + 255) / 256, BATCH ? a.num_inst : 1);
    hipLaunchKernelGGL((pred_light_kernel<V, BATCH>), grid, dim3(256), 0, stream, a, p,
                       a.heavy, a.degen, a.lvl, istat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pred) {
      hipLaunchKernelGGL((pred_heavy_kernel<V, BATCH>), dim3(geo.cus * 4), dim3(256), 0, stream,
                         a, p, a.heavy, a.degen, a.lvl);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (V::INF == KeyF32::INF) {
        hipLaunchKernelGGL((pred_degen_kernel<V, BATCH>), dim3(1), dim3(1024), 0, stream, a, p,
                           a.degen, a.lvl, a.flag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
  }
  return hipSuccess;
}

hipError_t launch_solve(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                        const LaunchGeom &geo, long long *istat, int32_t max_n,
                        const KernelTimer *timer, hipStream_t stream) {
  if (f32) {
    return batch ? launch_solve_t<KeyF32, true>(a, pred, geo, istat, max_n, timer, stream)
                 : launch_solve_t<KeyF32, false>(a, pred, geo, istat, max_n, timer, stream);
  }
  return batch ? launch_solve_t<KeyI32, true>(a, pred, geo, istat, max_n, timer, stream)
               : launch_solve_t<KeyI32, false>(a, pred, geo, istat, max_n, timer, stream);
}

hipError_t round_kernel_occupancy(bool f32, bool batch, int *blocks_per_cu) {
  const void *k = f32 ? (batch ? (const void *)rounds_kernel<KeyF32, true>
                               : (const void *)rounds_kernel<KeyF32, false>)
                      : (batch ? (const void *)rounds_kernel<KeyI32, true>
                               : (const void *)rounds_kernel<KeyI32, false>);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, RBS, 0);
}

}  // namespace sssp
