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
// million-edge hub and a degree-2 vertex cost the same per edge.
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
  uint64_t scan[RBS / SSSP_WAVE + 1];
  int32_t red[RBS / SSSP_WAVE];
  int32_t tmax;
};

template <bool BATCH>
__device__ __forceinline__ const GraphDev &graph_of(const RoundArgs &a, int gi) {
  if constexpr (BATCH) return a.graphs[gi];
  else return a.g;
}

// -------------------------------------------------------------- staging
// Block-collective push of up to K items per thread into an LDS stager;
// flushes to the global list when it would overflow.  All threads call.
template <int CAP>
__device__ void stage_flush(Stager<CAP> &st, unsigned long long *ctr, int32_t *lv, int32_t *lp,
                            int32_t *li, bool batch, SmemAll &sm) {
  // st.cnt is read by all threads after the caller's barrier
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

// Entry j of the thread's v/d/ins arrays is pushed iff bit j of `mask` is
// set (arrays are indexed by compile-time j only, so they stay in VGPRs).
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
  uint64_t mine = ((uint64_t)n_local << 32) | dsum;
  uint64_t tot;
  uint64_t ex = block_excl_scan64<RBS>(mine, sm.scan, &tot);
  const int tcnt = (int)(tot >> 32);
  if (tcnt == 0) return;  // uniform
  if (st.cnt + tcnt > CAP) stage_flush(st, ctr, lv, lp, li, batch, sm);
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
  long long st_settled = 0, st_relaxed = 0, st_scanned = 0;

  for (;;) {
    ++r;
    const int cur = r & 1;
    int32_t *Ov = cur ? a.open_v1 : a.open_v0;
    int32_t *Op = cur ? a.open_p1 : a.open_p0;
    int32_t *Oi = cur ? a.open_i1 : a.open_i0;
    int32_t *Nv = cur ? a.open_v0 : a.open_v1;
    int32_t *Np = cur ? a.open_p0 : a.open_p1;
    int32_t *Ni = cur ? a.open_i0 : a.open_i1;
    const int s_now = r % 3, s_next = (r + 1) % 3;

    if (r > a.max_rounds) {  // watchdog: rounds never exceed the reachable count
      if (bid == 0 && tid == 0) ctl->status = 7;
      break;
    }

    // =============================================================== relax
    const uint64_t fc = ld_relaxed64(&ctl->front_ctr);
    const int NF = (int)(fc >> 32);
    const uint32_t EF = (uint32_t)(fc & 0xffffffffull);
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
      } else {
        if (tid == 0) {
          ctl->minD[s_next] = V::INF;
          ctl->thr[s_next] = V::INF;
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
            int32_t nv[EPT], nd[EPT], ni[EPT];
            uint32_t nmask = 0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              const uint32_t e = cb + (uint32_t)(j * RBS + tid);
              if (e < wend) {
                const int it = window_item(S.pfx, e);
                const GraphDev &G = graph_of<BATCH>(a, S.gi[it]);
                const int32_t pos = S.base[it] + (int32_t)(e - (uint32_t)S.pfx[it]);
                const int32_t y = G.out_dst[pos];
                const int32_t cand = V::add(S.dx[it], G.out_w[pos]);
                const int32_t gy = S.sb[it] + y;
                if (cand < a.D[gy]) {
                  const int32_t old = atomicMin(&a.D[gy], cand);
                  if constexpr (BATCH) {
                    atomicMin(&a.imin[s_now * I + S.inst[it]], cand);
                  } else {
                    lmin = kmin(lmin, cand);
                  }
                  if (old == V::INF) {
                    nv[j] = gy;
                    nd[j] = G.in_off[y + 1] - G.in_off[y];
                    ni[j] = S.inst[it];
                    nmask |= 1u << j;
                  }
                }
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
      stage_flush(S.st, &ctl->open_ctr[cur], Ov, Op, Oi, BATCH, sm);
      if constexpr (!BATCH) {
        const int32_t bm = block_min<RBS>(lmin, sm.red);
        if (tid == 0 && bm < V::INF) atomicMin(&ctl->minD[s_now], bm);
      }
    }
    grid_barrier(&ctl->barrier, epoch);

    const uint64_t oc = ld_relaxed64(&ctl->open_ctr[cur]);
    const int NO = (int)(oc >> 32);
    const uint32_t EO = (uint32_t)(oc & 0xffffffffull);
    if (NO == 0) break;  // nothing left open: every reachable vertex is fixed

    // ================================================================== LB
    if (bid == 0 && tid == 0) {
      ctl->front_ctr = 0ull;
      st_scanned += EO;
    }
    {
      int32_t lthr = V::INF;
      int32_t mind_all = V::INF;
      if constexpr (!BATCH) mind_all = ld_relaxed(&ctl->minD[s_now]);
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
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              const uint32_t e = cb + (uint32_t)(j * RBS + tid);
              const bool valid = e < wend;
              int it = -1;
              int32_t t = V::INF;
              if (valid) {
                it = window_item(S.pfx, e);
                const GraphDev &G = graph_of<BATCH>(a, S.gi[it]);
                const int32_t pos = S.base[it] + (int32_t)(e - (uint32_t)S.pfx[it]);
                const int32_t v = G.in_src[pos];
                const int32_t cv = a.C[S.sb[it] + v];
                t = V::add(kmax(cv, S.mind[it]), G.in_w[pos]);
              }
              // segmented min into LDS; one LDS atomic per wave when the
              // whole wave works on one item (hub vertices)
              const uint64_t act = __ballot(valid);
              if (act) {
                const int lead = __ffsll((unsigned long long)act) - 1;
                const int it0 = __shfl(it, lead, SSSP_WAVE);
                const uint64_t same = __ballot(valid && it == it0);
                if (same == act) {
                  const int32_t wm = wave_min(t);
                  if (lane_id() == lead && wm < V::INF) atomicMin(&S.acc[it0], wm);
                } else if (valid && t < V::INF) {
                  atomicMin(&S.acc[it], t);
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
              const int32_t y = gy - S.sb[tid];
              const int32_t th = V::add(a.D[gy], G.out_wmin[y]);
              if constexpr (BATCH) {
                atomicMin(&a.ithr[s_now * I + S.inst[tid]], th);
                atomicAdd(&a.iscanned[S.inst[tid]], (unsigned long long)(p1 - p0));
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
        if (tid == 0 && bm < V::INF) atomicMin(&ctl->thr[s_now], bm);
      }
    }
    grid_barrier(&ctl->barrier, epoch);

    // ================================================================= fix
    {
      SmemFix &S = sm.u.f;
      if (tid == 0) {
        S.fr.cnt = 0;
        S.fr.deg = 0;
        S.op.cnt = 0;
        S.op.deg = 0;
      }
      __syncthreads();
      int32_t lnext = V::INF;
      int32_t mind_all = V::INF, thr_all = V::INF;
      if constexpr (!BATCH) {
        mind_all = ld_relaxed(&ctl->minD[s_now]);
        thr_all = ld_relaxed(&ctl->thr[s_now]);
      }
      for (int b0 = (int)bid * RBS; b0 < NO; b0 += (int)nb * RBS) {
        const int idx = b0 + tid;
        int32_t fv[1] = {0}, fd[1] = {0}, fi[1] = {0}, ov[1] = {0}, od[1] = {0}, oi[1] = {0};
        uint32_t nf = 0, no = 0;
        if (idx < NO) {
          const int32_t gy = Ov[idx];
          const int32_t m = a.mtmp[idx];
          a.mtmp[idx] = V::INF;
          const uint32_t p0 = (uint32_t)Op[idx];
          const uint32_t p1 = (idx + 1 < NO) ? (uint32_t)Op[idx + 1] : EO;
          int32_t sb = 0, gi = 0, ins = 0;
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
            const int32_t y = gy - sb;
            fv[0] = gy;
            fd[0] = G.out_off[y + 1] - G.out_off[y];
            fi[0] = ins;
            nf = 1;
          } else {
            a.C[gy] = Cn;
            ov[0] = gy;
            od[0] = (int32_t)(p1 - p0);
            oi[0] = ins;
            no = 1;
            if constexpr (BATCH) atomicMin(&a.imin[s_next * I + ins], Dy);
            else lnext = kmin(lnext, Dy);
          }
        }
        stage_push<CAP_F, 1>(S.fr, nf, fv, fd, fi, &ctl->front_ctr, a.front_v, a.front_p,
                             a.front_i, BATCH, sm);
        stage_push<CAP_F, 1>(S.op, no, ov, od, oi, &ctl->open_ctr[cur ^ 1], Nv, Np, Ni, BATCH,
                             sm);
      }
      stage_flush(S.fr, &ctl->front_ctr, a.front_v, a.front_p, a.front_i, BATCH, sm);
      stage_flush(S.op, &ctl->open_ctr[cur ^ 1], Nv, Np, Ni, BATCH, sm);
      if constexpr (!BATCH) {
        const int32_t bm = block_min<RBS>(lnext, sm.red);
        if (tid == 0 && bm < V::INF) atomicMin(&ctl->minD[s_next], bm);
      }
    }
    grid_barrier(&ctl->barrier, epoch);
  }

  if (bid == 0 && tid == 0) {
    ctl->rounds = r > a.max_rounds ? a.max_rounds : r;
    ctl->settled = st_settled;
    ctl->relaxed = st_relaxed;
    ctl->scanned = st_scanned;
  }
}

// ------------------------------------------------------------------ init
// D = INF, C = 0, mtmp = INF over all state entries; each instance's
// source gets D = 0 and the fixed marker C = INF.
template <class V>
__global__ void init_fill_kernel(int32_t *D, int32_t *C, int32_t *mtmp, int32_t total) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += gridDim.x * blockDim.x) {
    D[i] = V::INF;
    C[i] = 0;
    mtmp[i] = V::INF;
  }
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
        a.imin[0 * I + i] = V::INF;
        a.imin[1 * I + i] = V::INF;
        a.imin[2 * I + i] = V::INF;
        a.ithr[0 * I + i] = V::INF;
        a.ithr[1 * I + i] = V::INF;
        a.ithr[2 * I + i] = V::INF;
        a.irounds[i] = 0;
        a.iscanned[i] = 0ull;
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
    c->barrier = 0u;
    c->status = 0;
    for (int s = 0; s < 3; ++s) {
      c->minD[s] = V::INF;
      c->thr[s] = V::INF;
    }
    c->rounds = 0;
    c->settled = c->relaxed = c->scanned = 0;
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
        bool eq = false;
        for (int32_t j = j0; j < j1; ++j) {
          const int32_t dv = a.D[sb + G.in_src[j]];
          if (V::add(dv, G.in_w[j]) == dy) {
            if (dv < dy) {
              p = G.in_eid[j];
              break;
            }
            eq = true;
          }
        }
        if (p < 0) {
          // reachable, no strict tight edge: only equal-cost tight edges
          (void)eq;
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
                                 long long *istat, int32_t max_n, hipStream_t stream) {
  hipError_t e;
  {
    const int blocks = (int)((a.total + 255) / 256 < 4096 ? (a.total + 255) / 256 : 4096);
    hipLaunchKernelGGL(init_fill_kernel<V>, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream,
                       a.D, a.C, a.mtmp, a.total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((init_seed_kernel<V, BATCH>), dim3(1), dim3(RBS), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    RoundArgs arg = a;
    void *params[] = {&arg};
    e = hipLaunchCooperativeKernel((const void *)rounds_kernel<V, BATCH>, dim3(geo.blocks),
                                   dim3(RBS), params, 0, stream);
    if (e != hipSuccess) return e;
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
                        hipStream_t stream) {
  if (f32) {
    return batch ? launch_solve_t<KeyF32, true>(a, pred, geo, istat, max_n, stream)
                 : launch_solve_t<KeyF32, false>(a, pred, geo, istat, max_n, stream);
  }
  return batch ? launch_solve_t<KeyI32, true>(a, pred, geo, istat, max_n, stream)
               : launch_solve_t<KeyI32, false>(a, pred, geo, istat, max_n, stream);
}

hipError_t round_kernel_occupancy(bool f32, bool batch, int *blocks_per_cu) {
  const void *k = f32 ? (batch ? (const void *)rounds_kernel<KeyF32, true>
                               : (const void *)rounds_kernel<KeyF32, false>)
                      : (batch ? (const void *)rounds_kernel<KeyI32, true>
                               : (const void *)rounds_kernel<KeyI32, false>);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, RBS, 0);
}

}  // namespace sssp
