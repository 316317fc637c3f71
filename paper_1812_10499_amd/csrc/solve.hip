// Persistent gfx950 kernel for the data-parallel round of the
// lower/upper-bound SSSP method, and its init kernels.
//
// One round r (D = upper bound, C = lower bound, O = discovered non-fixed
// vertices, F = vertices fixed in round r-1), in two phases:
//   relax : out-edges of F into D with atomicMin on keys (the relaxation of
//           Fig. 1; label-setting form of Fig. 6 step 3).  A head whose old D
//           was INF joins O.  Each successful candidate c for head y also
//           offers c to minD and c + out_wmin[y] to thr.
//   bound-and-fix, for y in O:
//           m_y = min over in-edges (v,y,w) of max(C[v], minD) + w
//                 (Eq. 1 with the global bound of Lemma crule2; a fixed v
//                 has C[v] = INF and drops out);
//           C'[y] = max(C[y], minD, min(D[y], m_y));
//           y is fixed iff C'[y] >= D[y] or D[y] <= thr (Lemma crauser);
//           fixed vertices form the next F, the others stay in O and offer
//           D[y] to the next minD and D[y] + out_wmin[y] to the next thr.
// minD = min D over O and thr = min over O of D[y] + out_wmin[y] are
// complete once relax ends, because D only changes in relax and every value
// that D[y] takes there is offered.  C is double-buffered by round parity:
// the bound step reads the previous round's C and writes the other buffer,
// so all reads precede all writes (Jacobi) and rounds are deterministic.
//
// Lists (F, O) are compacted arrays of state indices with an exclusive
// prefix of the work the next phase expands: the out-degree for F; for O
// the number of in-edges (v, y, w) with minD + w < D[y], the only ones that
// can move C'[y] (weight-ordered in-lists make them a prefix).  Blocks append through an LDS staging buffer and one 64-bit
// atomicAdd per flush that reserves slots and degree range together.  Each
// phase splits the list's edge count into equal contiguous chunks, one per
// block (edge-balanced): a million-edge hub and a degree-2 vertex cost the
// same per edge.  An item whose in-edges span several chunks is finished by
// the last block to arrive (per-item arrival counter), so bound-and-fix
// needs no barrier of its own: two grid barriers per round.
//
// A phase runs on as many blocks as its work needs: block 0 alone (block
// barriers only) for at most `solo_edges` edges, else a power of two near
// work / block_units; the other blocks park and block 0 wakes them when a
// phase grows.  A barrier among k blocks costs far less than one across
// the whole grid, which matters for the long tails of small rounds (grids,
// the end of every solve).
#include <cstring>
#include <type_traits>

#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

constexpr int RBS = kRoundBlock;  // threads per block of the round kernel
constexpr int EPT = 4;            // edges per thread per sub-chunk
constexpr int WIN = RBS;          // list items per window
// relax: block staging capacity of first discoveries (what does not fit
// goes to the open list without a payload, its work counted inline)
constexpr int CAP_R = RBS * 7;
constexpr int CAP_F = RBS;        // bound-and-fix staging capacity per list (>= one window)
constexpr uint32_t CW_RELAX = 4;  // work units per frontier item (its loads and list entry)
constexpr uint32_t CW_FUSED = 16; // work units per open item (loads, decision, list entry)
constexpr uint32_t CW_LIVE = 8;   // work units per live undiscovered vertex (scope ALL)
constexpr int CAP_L = 8 * RBS;    // live-list staging capacity
constexpr int kLivePT = 4;        // live-list entries per thread and tile
static_assert(kLivePT * RBS <= CAP_L && RBS < 65536 && kLivePT <= 4,
              "a tile fits the stager; per-slot counts fit 16-bit fields of one 64-bit scan");

// ----------------------------------------------------------- LDS layouts
// LDS staging of list appends: vertex, local exclusive work prefix,
// instance, and NX payload words per item.
template <int CAP, int NX>
struct Stager {
  int32_t v[CAP];
  int32_t d[CAP];  // local exclusive degree prefix
  int32_t inst[CAP];
  int32_t x[NX > 0 ? NX : 1][NX > 0 ? CAP : 1];
  int32_t cnt;
  uint32_t deg;
  unsigned long long base;
};



// LDS staging of the first discoveries of a relax phase.  A wave reserves
// places with one LDS atomic (no block barrier per batch of edges); places
// beyond the capacity go straight to the global list.  d holds the
// discovering candidate, an upper bound of the vertex's D this round; the
// block flush turns it into the entry's work count.
struct RelaxStage {
  int32_t v[CAP_R];
  int32_t d[CAP_R];
  int32_t inst[CAP_R];
  int32_t cnt;  // places reserved (may exceed CAP_R: the rest went global)
  unsigned long long base;
};

struct SmemRelax {
  int32_t pfx[WIN + 1];
  int32_t epfx[WIN];  // edge prefix of the window's edge sub-ranges
  int32_t epos[WIN];  // CSR position where an item's sub-range starts
  int32_t base[WIN];
  int32_t dx[WIN];
  int32_t sb[WIN];
  int32_t gi[WIN];
  int32_t inst[WIN];
  RelaxStage st;
};

struct SmemFused {
  int32_t pfx[WIN + 1];  // work-unit prefix of the window's items (balancing)
  int32_t epfx[WIN];     // edge prefix of the window's in-chunk edge segments
  int32_t eoff[WIN];     // where an item's segment starts in its in-list
  int32_t base[WIN];
  int32_t ideg[WIN];     // in-degree (statistics), out-offset, out-degree, out_wmin
  int32_t ooff[WIN];
  int32_t odeg[WIN];
  int32_t owm[WIN];
  int32_t acc[WIN];
  // 1 + the largest list position among the item's edges that pass this
  // round's weight test (they form a prefix: its length, the item's work
  // next round), or kNoCount when the scan may have stopped short of that
  // prefix (a first discovery cut by the probe)
  int32_t cnt[WIN];
  int32_t dy[WIN];
  int32_t cy[WIN];
  int32_t mind[WIN];
  int32_t thr[WIN];
  int32_t sb[WIN];
  int32_t gi[WIN];
  int32_t inst[WIN];
  Stager<CAP_F, kFX> fr;
  Stager<CAP_F, kOX> op;
};

// The live pass of a bound step runs after the open items' stagers are
// flushed, so it reuses their LDS.
struct SmemLive {
  int32_t v[CAP_L];  // staged survivors
  int32_t cnt;
  int32_t base;
};

struct SmemAll {
  union {
    SmemRelax r;
    SmemFused f;
    SmemLive l;
  } u;
  uint64_t scan[2 * (RBS / SSSP_WAVE + 1)];
  int32_t red[2 * (RBS / SSSP_WAVE)];
  int32_t tmax;
  // block 0, thread 0: the solve's counters, written out at the end
  long long n_relaxed, n_open, n_solo, n_bound;
  unsigned long long n_fixed;  // this block's fixes (single solve)
  unsigned long long n_scanned;  // this block's share of the scanned in-edge count
  // single solve: minima a one-block phase produced, and their rounds
  int32_t solo_cand_min, solo_cand_thr, solo_surv_min, solo_surv_thr;
  int32_t solo_cand_r, solo_surv_r;
  int32_t res_round, res_phase, res_done, res_act;
  unsigned int res_go, res_aep;
};

// Batched solves: each block gathers the per-instance minima (minD and thr
// candidates) and statistics of a phase in LDS and adds them to the global
// per-instance words once per touched instance at the phase end, instead of
// one device atomic per candidate on a handful of hot addresses.  Batches
// with more instances than kLdsInst use the device atomics directly.
constexpr int kLdsInst = 2048;

template <bool BATCH>
struct BatchLds {};

template <>
struct BatchLds<true> {
  int32_t mn[kLdsInst];
  int32_t th[kLdsInst];
  uint32_t scan[kLdsInst];
  uint32_t visit[kLdsInst];
};

template <class V>
__device__ void batch_lds_reset(BatchLds<true> &bl, int I) {
  for (int i = threadIdx.x; i < I && i < kLdsInst; i += RBS) {
    bl.mn[i] = V::INF;
    bl.th[i] = V::INF;
    bl.scan[i] = 0u;
    bl.visit[i] = 0u;
  }
}

// Offer (v, t) to instance ins's minD / thr candidates of slot `slot`.  One
// LDS atomic per wave when every offering lane of the wave has the same
// instance (the usual case: lanes walk the edges of neighbouring items).
template <class V>
__device__ __forceinline__ void batch_offer(BatchLds<true> &bl, const RoundArgs &a, int slot,
                                            bool on, int ins, int32_t v, int32_t t) {
  const int I = a.num_inst;
  if (I > kLdsInst) {
    if (on) {
      atomicMin(&a.imin[slot * I + ins], v);
      atomicMin(&a.ithr[slot * I + ins], t);
    }
    return;
  }
  const uint64_t act = __ballot(on);
  if (!act) return;
  const int lead = __ffsll((unsigned long long)act) - 1;
  const int i0 = __builtin_amdgcn_readlane(ins, lead);
  if (__ballot(on && ins == i0) == act) {
    const int32_t wv = wave_min(on ? v : V::INF);
    const int32_t wt = wave_min(on ? t : V::INF);
    if (lane_id() == lead) {
      atomicMin(&bl.mn[i0], wv);
      atomicMin(&bl.th[i0], wt);
    }
  } else if (on) {
    atomicMin(&bl.mn[ins], v);
    atomicMin(&bl.th[ins], t);
  }
}

// After a barrier: the block's per-instance minima and counts into the
// global words (slot < 0: no minima this phase).  Per instance the counts
// are iscanned[3i] scanned in-edges and [3i + 1] open visits (bound step),
// [3i + 2] relaxed edges (relax step, accumulated in `scan`).
template <class V>
__device__ void batch_lds_flush(BatchLds<true> &bl, const RoundArgs &a, int slot, bool relax) {
  const int I = a.num_inst;
  for (int i = threadIdx.x; i < I && i < kLdsInst; i += RBS) {
    if (slot >= 0) {
      if (bl.mn[i] != V::INF) atomicMin(&a.imin[slot * I + i], bl.mn[i]);
      if (bl.th[i] != V::INF) atomicMin(&a.ithr[slot * I + i], bl.th[i]);
    }
    if (relax) {
      if (bl.scan[i]) atomicAdd(&a.iscanned[3 * i + 2], (unsigned long long)bl.scan[i]);
    } else {
      // the live pass adds scanned counts for instances with no open item here
      if (bl.scan[i]) atomicAdd(&a.iscanned[3 * i], (unsigned long long)bl.scan[i]);
      if (bl.visit[i]) atomicAdd(&a.iscanned[3 * i + 1], (unsigned long long)bl.visit[i]);
    }
  }
}

// A value every lane of the block holds alike, moved to a scalar register.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v);
}

// Round-trace checkpoint k of a phase: one chosen block's wall-clock (when
// enabled).
__device__ __forceinline__ void mark(const RoundArgs &a, int r, int phase, int k) {
  if (a.marks && blockIdx.x == (uint32_t)a.mark_block && threadIdx.x == 0 && r <= a.mark_rounds)
    a.marks[((size_t)(r - 1) * 2 + phase) * kMarks + k] = (long long)wall_clock64();
}

// The portion of the grid a phase runs on: all blocks, or block 0 alone.
struct PhaseCtx {
  uint32_t vnb, vbid;
  bool solo;
  int32_t target;  // single-target solve: the target's solver id, else -1
};

// What a block's share of a phase was (for the round trace).
struct PhaseWork {
  int windows = 0;
  int first_item = -1;
  uint32_t units = 0;
  long long t_mid = 0;  // wall-clock after the list windows (before the flush or live pass)
  int32_t bmin = 0, bthr = 0;  // single solve: the block's minD / thr offers
};

__device__ __forceinline__ int32_t *part_slot(const RoundArgs &a, int k) {
  return a.part + (size_t)k * kMaxBlocks;
}

// This round's minD and thr: minima over all per-block partial slots of the
// survivors (last bound step) and the candidates (this relax), in one pass.
template <class V>
__device__ void reduce_parts(const RoundArgs &a, int cur, int32_t &mind, int32_t &thr,
                             SmemAll &sm) {
  const int32_t *s0 = part_slot(a, P_SURV0 + cur), *c0 = part_slot(a, P_CAND0 + cur);
  const int32_t *s1 = part_slot(a, P_TSURV0 + cur), *c1 = part_slot(a, P_TCAND0 + cur);
  int32_t m = V::INF, t = V::INF;
  for (uint32_t b = threadIdx.x; b < gridDim.x; b += RBS) {
    m = kmin(m, kmin(s0[b], c0[b]));
    t = kmin(t, kmin(s1[b], c1[b]));
  }
  block_min2<RBS>(m, t, sm.red);
  mind = m;
  thr = t;
}

// A block's partial.  With k active blocks, block b also clears the slots
// b + k, b + 2k, ... of the parked blocks, so readers can reduce all slots.
template <class V>
__device__ void put_part(const RoundArgs &a, int k, int32_t v, const PhaseCtx &pc) {
  int32_t *p = part_slot(a, k);
  const uint32_t b0 = pc.vbid;
  if (threadIdx.x == 0) p[b0] = v;
  for (uint32_t b = b0 + pc.vnb * (threadIdx.x + 1); b < gridDim.x; b += pc.vnb * RBS)
    p[b] = V::INF;
}

// -------------------------------------------------------------- staging
// A global list: its append counter ((items << 32) | work units) and its
// arrays.  x[k] receives payload word k; a list fed by a payload-free
// stager gets -1 in x[0] when x[0] is set (the "no payload" mark).
struct ListRef {
  unsigned long long *ctr;
  int32_t *v, *p, *i;
  int32_t *x[kOX];
};

// Block-collective flush of an LDS stager into the global list: one 64-bit
// atomicAdd reserves (slots, degree range).  All threads call, after a
// barrier that made st.cnt current.
template <int CAP, int NX>
__device__ void stage_flush(Stager<CAP, NX> &st, const ListRef &l, bool batch) {
  const int cnt = st.cnt;
  if (cnt == 0) return;
  if (threadIdx.x == 0) {
    unsigned long long inc = ((unsigned long long)cnt << 32) | (unsigned long long)st.deg;
    st.base = atomicAdd(l.ctr, inc);
  }
  __syncthreads();
  const unsigned long long b = st.base;
  const int32_t bc = (int32_t)(b >> 32);
  const int32_t bd = (int32_t)(uint32_t)(b & 0xffffffffull);
  for (int j = threadIdx.x; j < cnt; j += RBS) {
    l.v[bc + j] = st.v[j];
    l.p[bc + j] = bd + st.d[j];
    if (batch) l.i[bc + j] = st.inst[j];
    if constexpr (NX > 0) {
#pragma unroll
      for (int k = 0; k < NX; ++k) l.x[k][bc + j] = st.x[k][j];
    } else {
      if (l.x[0]) l.x[0][bc + j] = -1;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st.cnt = 0;
    st.deg = 0;
  }
  __syncthreads();
}

// Both stagers of the bound step flushed together: the two reservations are
// issued from different waves before either is waited for, so their
// device-atomic latencies overlap.
template <int CAP, int N1, int N2>
__device__ void stage_flush2(Stager<CAP, N1> &s1, const ListRef &l1, Stager<CAP, N2> &s2,
                             const ListRef &l2, bool batch) {
  const int c1 = s1.cnt, c2 = s2.cnt;
  if (c1 == 0 && c2 == 0) return;
  if (threadIdx.x == 0 && c1)
    s1.base = atomicAdd(l1.ctr, ((unsigned long long)c1 << 32) | (unsigned long long)s1.deg);
  if (threadIdx.x == SSSP_WAVE && c2)
    s2.base = atomicAdd(l2.ctr, ((unsigned long long)c2 << 32) | (unsigned long long)s2.deg);
  __syncthreads();
  const unsigned long long b1 = s1.base, b2 = s2.base;
  const int32_t bc1 = (int32_t)(b1 >> 32), bd1 = (int32_t)(uint32_t)(b1 & 0xffffffffull);
  const int32_t bc2 = (int32_t)(b2 >> 32), bd2 = (int32_t)(uint32_t)(b2 & 0xffffffffull);
  for (int j = threadIdx.x; j < c1; j += RBS) {
    l1.v[bc1 + j] = s1.v[j];
    l1.p[bc1 + j] = bd1 + s1.d[j];
    if (batch) l1.i[bc1 + j] = s1.inst[j];
#pragma unroll
    for (int k = 0; k < N1; ++k) l1.x[k][bc1 + j] = s1.x[k][j];
  }
  for (int j = threadIdx.x; j < c2; j += RBS) {
    l2.v[bc2 + j] = s2.v[j];
    l2.p[bc2 + j] = bd2 + s2.d[j];
    if (batch) l2.i[bc2 + j] = s2.inst[j];
#pragma unroll
    for (int k = 0; k < N2; ++k) l2.x[k][bc2 + j] = s2.x[k][j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s1.cnt = 0;
    s1.deg = 0;
    s2.cnt = 0;
    s2.deg = 0;
  }
  __syncthreads();
}

// One item per thread into each of two payload stagers, with a single scan.
template <int N1, int N2>
__device__ void stage_push2(Stager<CAP_F, N1> &s1, bool h1, int32_t v1, int32_t d1, int32_t i1,
                            const int32_t (&x1)[N1], const ListRef &l1,
                            Stager<CAP_F, N2> &s2, bool h2, int32_t v2, int32_t d2, int32_t i2,
                            const int32_t (&x2)[N2], const ListRef &l2, bool batch,
                            SmemAll &sm) {
  const uint64_t m1 = h1 ? ((1ull << 32) | (uint32_t)d1) : 0ull;
  const uint64_t m2 = h2 ? ((1ull << 32) | (uint32_t)d2) : 0ull;
  uint64_t ex1, ex2, t1, t2;
  block_excl_scan64x2<RBS>(m1, m2, sm.scan, &ex1, &ex2, &t1, &t2);
  const int c1 = (int)(t1 >> 32), c2 = (int)(t2 >> 32);
  if (c1 && s1.cnt + c1 > CAP_F) stage_flush(s1, l1, batch);
  if (c2 && s2.cnt + c2 > CAP_F) stage_flush(s2, l2, batch);
  if (h1) {
    const int pos = s1.cnt + (int)(ex1 >> 32);
    s1.v[pos] = v1;
    s1.d[pos] = (int32_t)(s1.deg + (uint32_t)(ex1 & 0xffffffffull));
    s1.inst[pos] = i1;
#pragma unroll
    for (int k = 0; k < N1; ++k) s1.x[k][pos] = x1[k];
  }
  if (h2) {
    const int pos = s2.cnt + (int)(ex2 >> 32);
    s2.v[pos] = v2;
    s2.d[pos] = (int32_t)(s2.deg + (uint32_t)(ex2 & 0xffffffffull));
    s2.inst[pos] = i2;
#pragma unroll
    for (int k = 0; k < N2; ++k) s2.x[k][pos] = x2[k];
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

// ------------------------------------------- work-balanced list expansion
// A list has N items whose exclusive degree prefix is lp[] and E edges in
// total.  Each item weighs its degree plus c units of per-item work, so
// item i spans the work range [lp[i] + c*i, lp[i+1] + c*(i+1)): c virtual
// units (the item's own loads and bookkeeping) followed by its edges.  The
// phase's block b takes work units [b*chunk, min(W, (b+1)*chunk)) with
// W = E + c*N, which balances edges and items together.
// Returns the item whose work range contains e0, found by a
// block-cooperative RBS-ary search (3 steps for millions of items).
__device__ int find_start_item(const int32_t *lp, int N, uint32_t c, uint32_t e0, SmemAll &sm) {
  if (e0 == 0) return 0;  // the first chunk (and every one-block phase)
  int lo = 0, hi = N;
  while (hi - lo > 1) {
    const int span = hi - lo;
    const int pos = lo + (int)(((int64_t)span * threadIdx.x) / RBS);
    // pos < hi always; pos == lo for thread 0
    const bool le = (uint32_t)lp[pos] + c * (uint32_t)pos <= e0;
    if (threadIdx.x == 0) sm.tmax = 0;
    __syncthreads();
    // the last thread with le (they form a prefix): one LDS atomic per wave
    const uint64_t bl = __ballot(le);
    if (lane_id() == 0 && bl)
      atomicMax(&sm.tmax, (int)(threadIdx.x + 63u - (uint32_t)__clzll((long long)bl)));
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

// last window position p in [0, WIN) with pfx[p] <= e (pfx ascending, with
// pfx[0] <= e)
static_assert(WIN == 1024, "the window search covers 1024 positions");
__device__ __forceinline__ int window_item(const int32_t *pfx, uint32_t e) {
  return search1024(pfx, e);
}

__device__ __forceinline__ uint32_t chunk_of(uint32_t E, uint32_t vnb) {
  return (E + vnb - 1) / vnb;
}

// A prefix search below stops once its interval [lo, hi) holds at most
// kSearchSlack edges and takes hi: the count then covers the prefix and at
// most kSearchSlack edges that fail the weight test.  The bound step reads
// an item's in-edges contiguously and gathers C only for edges that pass,
// so each extra edge costs a share of a coalesced read, where every search
// step saved is a dependent random read (a CU issues about one random
// line per clock, and these searches run in the lists' flushes and
// finishes).
constexpr int32_t kSearchSlack = 32;

// Work of an open vertex y in the bound step: its in-edges (v, y, w) with
// md + w < dy.  The working copy's in-lists are ascending by weight and the
// rounded add is monotone, so they are a prefix of y's list; a binary
// search bounds its length from above, to within kSearchSlack (short lists
// are taken whole).  With md at most the minD of the round that scans y and
// dy at least that round's D[y], the prefix covers every edge the bound
// step needs.
template <class V>
__device__ __forceinline__ int32_t useful_in_edges_at(const GraphDev &G, int32_t b, int32_t deg,
                                                      int32_t md, int32_t dy) {
  int32_t lo = 0, hi = deg;
  if (hi <= 16) return hi;
  while (hi - lo > kSearchSlack) {
    const int32_t mid = (lo + hi) >> 1;
    if (V::add(md, G.in_w[b + mid]) < dy) lo = mid + 1;
    else hi = mid;
  }
  return hi;
}

// Work of a vertex y first discovered in this round's relax step: the
// weight prefix above, cut after the first of y's kProbe lightest in-edges
// whose tail v has C[v] <= md in the C the bound step will read (so v is not
// fixed: fixed vertices carry C = INF).  With minD >= md that edge's term
// max(C[v], minD) + w is minD + w, and every later edge of the list is at
// least as heavy, so its term is no smaller: m_y is decided by the edges up
// to the probe hit, and the probe's own weights give the prefix among them
// (no search).  Cold must be stable for the whole relax step (the bound step
// writes the other C buffer).
constexpr int kProbe = 2;
constexpr int32_t kNoCount = 0x40000000;  // above any list position

// The work of K first discoveries (bit k of `valid`: entry k is one), the
// rule above taken one step at a time for all K entries, so that their
// dependent loads overlap: the vertex record (in-offset, in-degree and the
// lightest in-edge), the second lightest in-edge and both tails' lower
// bounds, then the weight searches in lockstep.  gy is a state index, dy
// the discovering candidate; md is the minD of an earlier round (md_prev, or
// per instance in a batch).  With a payload array, entry k's open-list
// payload is returned too (read with the vertex record): in-offset,
// in-degree as -1 - in-degree (the mark of a first discovery), out-offset,
// out-degree, out_wmin and C (0, or under scope ALL what the live pass
// raised it to).
template <class V, bool BATCH, int K>
__device__ void discovery_work_x(const RoundArgs &a, const int32_t *Cold, uint32_t valid,
                                 const int32_t (&gy)[K], const int32_t (&dy)[K],
                                 const int32_t (&ins)[K], int32_t md_prev, int r,
                                 int32_t (&out)[K], int32_t (*pay)[K] = nullptr) {
  int32_t sb[K], gi[K], md[K], b[K], deg[K], v0[K], w0[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    out[k] = 0;
    sb[k] = gi[k] = 0;
    md[k] = md_prev;
    b[k] = deg[k] = v0[k] = w0[k] = 0;
    if ((valid >> k) & 1u) {
      if constexpr (BATCH) {
        const InstDev id = a.insts[ins[k]];
        sb[k] = id.sbase;
        gi[k] = id.graph;
        md[k] = 0;
        if (r > 1) {
          md[k] = ld_relaxed(&a.imin[((r + 2) % 3) * a.num_inst + ins[k]]);
          if (md[k] == V::INF) md[k] = 0;
        }
      }
      const GraphDev &G = graph_of<BATCH>(a, gi[k]);
      const int32_t y = gy[k] - sb[k];
      const int4 rec = G.vrec[2 * y], rec2 = G.vrec[2 * y + 1];
      b[k] = rec.z;
      deg[k] = rec.w;
      v0[k] = rec2.y;  // the lightest in-edge's tail and weight
      w0[k] = rec2.z;
      if (pay) {
        pay[OX_BASE][k] = rec.z;
        pay[OX_IDEG][k] = -1 - rec.w;
        pay[OX_OOFF][k] = rec.x;
        pay[OX_ODEG][k] = rec.y;
        pay[OX_OWM][k] = rec2.x;
        pay[OX_C][k] = G.all ? Cold[gy[k]] : 0;
      }
    }
  }
  // short lists are taken whole; longer ones probe their two lightest edges
  uint32_t probe = 0;
  int32_t v1[K], w1[K], c0[K], c1[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v1[k] = w1[k] = 0;
    if ((valid >> k) & 1u) {
      if (deg[k] > 16) {
        const GraphDev &G = graph_of<BATCH>(a, gi[k]);
        probe |= 1u << k;
        const int2 e1 = G.in_sw[b[k] + 1];
        v1[k] = e1.x;
        w1[k] = e1.y;
      } else {
        out[k] = deg[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    c0[k] = c1[k] = V::INF;
    if ((probe >> k) & 1u) {
      c0[k] = Cold[sb[k] + v0[k]];
      c1[k] = Cold[sb[k] + v1[k]];
    }
  }
  uint32_t search = 0, bylim = 0;
  int32_t lo[K], hi[K], lim[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    lo[k] = hi[k] = lim[k] = 0;
    if (!((probe >> k) & 1u)) continue;
    const int hit = c0[k] <= md[k] ? 0 : (c1[k] <= md[k] ? 1 : kProbe);
    if (hit < kProbe) {
      // the edges that pass the weight test form a prefix of the list
      int32_t p = V::add(md[k], w0[k]) < dy[k] ? 1 : 0;
      if (hit == 1 && V::add(md[k], w1[k]) < dy[k]) ++p;
      out[k] = p;
      continue;
    }
    lo[k] = 0;
    hi[k] = deg[k];
    search |= 1u << k;
    if constexpr (std::is_same<V, KeyI32>::value) {
      // Integer weights: a probed tail j with C[j] > md still bounds the
      // scan.  For every minD >= md its term max(C[j], minD) + w_j is at
      // most minD + w_j + (C[j] - md), so each edge with weight at least
      // W* = min_j (w_j + C[j] - md) has minD + w >= that term: only the
      // edges lighter than W*, and the probe edge j* that attains it, can
      // set m_y.  One search then finds the weight bound min(dy - md, W*):
      // md + w < dy is w < dy - md (dy <= INF, so the saturating add hides
      // nothing), and j* itself lies below W* (C[j*] > md here).  The bound
      // is at most dy - md, so it fits an int32.
      long long ws = (long long)V::INF + V::INF;
      if (c0[k] != V::INF) ws = (long long)w0[k] + (c0[k] - md[k]);
      if (c1[k] != V::INF) {
        const long long t = (long long)w1[k] + (c1[k] - md[k]);
        if (t < ws) ws = t;
      }
      if (c0[k] != V::INF || c1[k] != V::INF) {
        bylim |= 1u << k;
        const long long dm = (long long)dy[k] - md[k];
        lim[k] = (int32_t)(ws < dm ? ws : dm);
      }
    }
  }
  // the weight searches, one step for every searching entry per pass
  while (search) {
    int32_t x[K], mid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      mid[k] = (lo[k] + hi[k]) >> 1;
      x[k] = ((search >> k) & 1u) ? graph_of<BATCH>(a, gi[k]).in_w[b[k] + mid[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!((search >> k) & 1u)) continue;
      const bool pass = ((bylim >> k) & 1u) ? x[k] < lim[k] : V::add(md[k], x[k]) < dy[k];
      if (pass) lo[k] = mid[k] + 1;
      else hi[k] = mid[k];
      if (hi[k] - lo[k] <= kSearchSlack) {
        search &= ~(1u << k);
        out[k] = hi[k];
      }
    }
  }
}

// One pass of the flush below: the stager's entries [off, off + cnt),
// thread t taking off + 4t .. off + 4t + 3.
template <class V, bool BATCH>
__device__ void relax_flush_pass(const RoundArgs &a, RelaxStage &st, const ListRef &l,
                                 const int32_t *Cold, int32_t md_prev, int r, SmemAll &sm,
                                 int off, int cnt) {
  constexpr int PER = 4;
  const int j0 = threadIdx.x * PER;
  int32_t work[PER], gy[PER], dy[PER], ins[PER], pay[kOX][PER];
  uint32_t valid = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    gy[k] = dy[k] = ins[k] = 0;
    if (j0 + k < cnt) {
      valid |= 1u << k;
      gy[k] = st.v[off + j0 + k];
      dy[k] = st.d[off + j0 + k];
      ins[k] = st.inst[off + j0 + k];
    }
  }
  discovery_work_x<V, BATCH, PER>(a, Cold, valid, gy, dy, ins, md_prev, r, work, pay);
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) sum += (uint32_t)work[k];
  uint64_t tot;
  const uint64_t ex = block_excl_scan64<RBS>((uint64_t)sum, sm.scan, &tot);
  if (threadIdx.x == 0)
    st.base = atomicAdd(l.ctr, ((unsigned long long)cnt << 32) | (tot & 0xffffffffull));
  __syncthreads();
  const unsigned long long b = st.base;
  const int32_t bc = (int32_t)(b >> 32);
  uint32_t p = (uint32_t)(b & 0xffffffffull) + (uint32_t)ex;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int j = j0 + k;
    if (j < cnt) {
      l.v[bc + j] = gy[k];
      l.p[bc + j] = (int32_t)p;
      if (BATCH) l.i[bc + j] = ins[k];
#pragma unroll
      for (int q = 0; q < kOX; ++q) l.x[q][bc + j] = pay[q][k];
      p += (uint32_t)work[k];
    }
  }
  __syncthreads();  // st.base is read before the next pass writes it
}

// Block-collective flush of the relax stager (all threads, after a barrier
// that made its contents current), in passes of four entries per thread:
// a thread counts the useful in-edges of its four side by side; one block
// scan and one atomicAdd per pass reserve the list slots and the work
// range.  Entries carry their payload, read with the count, so the bound
// step need not read the vertex record.
template <class V, bool BATCH>
__device__ void relax_flush(const RoundArgs &a, RelaxStage &st, const ListRef &l,
                            const int32_t *Cold, int32_t md_prev, int r, SmemAll &sm) {
  const int all = st.cnt < CAP_R ? st.cnt : CAP_R;
  for (int off = 0; off < all; off += 4 * RBS)
    relax_flush_pass<V, BATCH>(a, st, l, Cold, md_prev, r, sm, off, min(all - off, 4 * RBS));
  if (threadIdx.x == 0) st.cnt = 0;
  __syncthreads();
}

// Discoveries a wave could not place in the stager (it was full): straight
// to the global list, one atomicAdd for the wave, with the "no payload"
// mark (the bound step reads their vertex records).  All lanes of the wave
// call it; mask selects the lane's entries among its EPT candidates.
template <class V, bool BATCH>
__device__ void relax_push_global(const RoundArgs &a, const ListRef &l, const int32_t *Cold,
                                  int32_t md_prev, int r, uint32_t mask,
                                  const int32_t (&gy)[EPT], const int32_t (&dy)[EPT],
                                  const int32_t (&ins)[EPT]) {
  int32_t work[EPT];
  discovery_work_x<V, BATCH, EPT>(a, Cold, mask, gy, dy, ins, md_prev, r, work);
  uint32_t n = 0, wsum = 0;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    if ((mask >> j) & 1u) {
      ++n;
      wsum += (uint32_t)work[j];
    }
  }
  const uint64_t mine = ((uint64_t)n << 32) | wsum;
  const uint64_t inc = wave_incl_scan64(mine);
  const uint64_t tot = (uint64_t)readlane64((int64_t)inc, SSSP_WAVE - 1);
  unsigned long long base = 0;
  if (lane_id() == 0 && tot) base = atomicAdd(l.ctr, (unsigned long long)tot);
  base = (unsigned long long)readlane64((int64_t)base, 0);
  const uint64_t ex = inc - mine;
  int32_t pos = (int32_t)(base >> 32) + (int32_t)(ex >> 32);
  uint32_t p = (uint32_t)(base & 0xffffffffull) + (uint32_t)(ex & 0xffffffffull);
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    if ((mask >> j) & 1u) {
      l.v[pos] = gy[j];
      l.p[pos] = (int32_t)p;
      if (BATCH) l.i[pos] = ins[j];
      if (l.x[0]) l.x[0][pos] = -1;
      ++pos;
      p += (uint32_t)work[j];
    }
  }
}

// ================================================================== relax
// md_prev: a minD of an earlier round (0 before the first), a lower bound of
// this round's minD for the work counts of newly discovered vertices.
template <class V, bool BATCH>
__device__ void relax_phase(const RoundArgs &a, SmemAll &sm, BatchLds<BATCH> &bl,
                            const PhaseCtx &pc, int r, int NF, uint32_t EF, int32_t md_prev,
                            PhaseWork &pw) {
  const int tid = threadIdx.x;
  const int cur = r & 1, s_now = r % 3;
  const int I = a.num_inst;
  Ctl *ctl = a.ctl;
  // first discoveries go to this round's open list, marked "no payload"
  int32_t *const *Oxw = cur ? a.open_x1 : a.open_x0;
  const ListRef olist = {&ctl->open_ctr[cur], cur ? a.open_v1 : a.open_v0,
                         cur ? a.open_p1 : a.open_p0, cur ? a.open_i1 : a.open_i0,
                         {Oxw[0], Oxw[1], Oxw[2], Oxw[3], Oxw[4], Oxw[5]}};
  int32_t *Cnew = cur ? a.C0 : a.C1;
  const int32_t *Cold = cur ? a.C1 : a.C0;  // what this round's bound step reads
  if constexpr (BATCH) {
    // per-instance round count: the last round with a non-empty frontier
    for (int i = (int)(pc.vbid * RBS) + tid; i < NF; i += (int)(pc.vnb * RBS))
      a.irounds[a.front_i[i]] = r;
  }
  int32_t lmin = V::INF, ltmin = V::INF;
  SmemRelax &S = sm.u.r;
  if (tid == 0) S.st.cnt = 0;
  if constexpr (BATCH) batch_lds_reset<V>(bl, I);
  __syncthreads();
  mark(a, r, 0, 2);
  const uint32_t WT = EF + CW_RELAX * (uint32_t)NF;
  const uint32_t chunk = chunk_of(WT, pc.vnb);
  const uint32_t e0 = pc.vbid * chunk;
  const uint32_t e1 = min(WT, e0 + chunk);
  if (e0 < e1) {
    int i = uni(find_start_item(a.front_p, NF, CW_RELAX, e0, sm));
    uint32_t k = e0;
    pw.first_item = i;
    pw.units = e1 - e0;
    mark(a, r, 0, 3);
    while (k < e1) {
      const int idx = i + tid;
      if (idx < NF) {
        const int32_t gx = a.front_v[idx];
        S.pfx[tid] = a.front_p[idx] + (int32_t)(CW_RELAX * (uint32_t)idx);
        int32_t sb = 0, gi = 0, ins = 0;
        if constexpr (BATCH) {
          ins = a.front_i[idx];
          const InstDev id = a.insts[ins];
          sb = id.sbase;
          gi = id.graph;
        }
        // out-offset and relax D travel with the entry (bit 31: x is open)
        const int32_t dxr = a.front_x[FX_D][idx];
        const int32_t dx = dxr & 0x7fffffff;
        S.base[tid] = a.front_x[FX_OOFF][idx];
        S.dx[tid] = dx;
        S.sb[tid] = sb;
        S.gi[tid] = gi;
        S.inst[tid] = ins;
        // a fixed x was fixed last round; the buffer the next bound step
        // reads must say so too (every item is in some block's window: each
        // weighs CW_RELAX units even with no edges)
        if (dxr >= 0) Cnew[gx] = V::INF;
        if (graph_of<BATCH>(a, gi).lc) a.DR[gx] = dx;  // relaxed from dx
      } else {
        S.pfx[tid] = (int32_t)WT;
      }
      if (tid == 0)
        S.pfx[WIN] = (i + WIN < NF)
                         ? a.front_p[i + WIN] + (int32_t)(CW_RELAX * (uint32_t)(i + WIN))
                         : (int32_t)WT;
      __syncthreads();
      if (pw.windows == 0) mark(a, r, 0, 4);
      if constexpr (BATCH) {
        // relaxed-edge count per instance: an item's out-degree, counted by
        // the block whose chunk holds the item's first unit
        if (idx < NF) {
          const uint32_t p0 = (uint32_t)S.pfx[tid];
          const uint32_t deg = (uint32_t)S.pfx[tid + 1] - p0 - CW_RELAX;
          if (p0 >= e0 && p0 < e1 && deg) {
            if (I > kLdsInst) atomicAdd(&a.iscanned[3 * S.inst[tid] + 2], (unsigned long long)deg);
            else atomicAdd(&bl.scan[S.inst[tid]], deg);
          }
        }
      }
      const uint32_t wend = uni(min((uint32_t)S.pfx[WIN], e1));
      // Each item's units are CW_RELAX of bookkeeping, then one per
      // out-edge; lanes walk only the edges that fall in [k, wend).
      uint64_t etot;
      {
        uint32_t ecnt = 0;
        if (idx < NF) {
          const uint32_t p0 = (uint32_t)S.pfx[tid] + CW_RELAX, p1 = (uint32_t)S.pfx[tid + 1];
          const uint32_t lo = max(p0, k), hi = min(p1, wend);
          if (hi > lo) {
            ecnt = hi - lo;
            S.epos[tid] = S.base[tid] + (int32_t)(lo - p0);
          }
        }
        S.epfx[tid] = (int32_t)block_excl_scan64<RBS>((uint64_t)ecnt, sm.scan, &etot);
        __syncthreads();
      }
      const uint32_t ET = uni((uint32_t)etot);
      for (uint32_t cb = 0; cb < ET; cb += RBS * EPT) {
        // Each step below issues the loads (or atomics) of all EPT edges
        // before any result is read, so the EPT accesses of a lane overlap.
        // Lanes past the window's last edge repeat it (a valid position)
        // rather than branch around the loads: a conditional load whose
        // result is merged back makes the compiler wait for it at once.
        int it[EPT];
        int32_t pos[EPT], y[EPT], wt[EPT], cand[EPT], gy[EPT], eid[EPT], wm[EPT];
        unsigned long long key[EPT], dk[EPT], old[EPT];
        bool val[EPT], doa[EPT], off[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const uint32_t q = cb + (uint32_t)(j * RBS + tid);
          val[j] = q < ET;
          const uint32_t qc = val[j] ? q : ET - 1u;
          it[j] = window_item(S.epfx, qc);
          pos[j] = S.epos[it[j]] + (int32_t)(qc - (uint32_t)S.epfx[it[j]]);
        }
        // one record per edge: head, weight, edge id (the caller's CSR
        // position) and the head's out_wmin
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int4 e = graph_of<BATCH>(a, S.gi[it[j]]).out_rec[pos[j]];
          y[j] = e.x;
          wt[j] = e.y;
          eid[j] = e.z;
          wm[j] = e.w;
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          cand[j] = V::add(S.dx[it[j]], wt[j]);
          gy[j] = S.sb[it[j]] + y[j];
        }
        // The key read may be stale: it only filters the atomic, against
        // contention on hot heads in the big rounds; a one-block phase goes
        // straight to the atomic and saves the dependent load.
        if (pc.solo) {
#pragma unroll
          for (int j = 0; j < EPT; ++j) dk[j] = 0x7fffffffffffffffull;
        } else {
#pragma unroll
          for (int j = 0; j < EPT; ++j) dk[j] = a.D64[gy[j]];
        }
        wait_vector_memory();  // then the EPT atomics issue back to back
        // A float edge that leaves the cost unchanged (w below half an ulp)
        // is an equal-cost parent.  Every in-edge of a reachable vertex is
        // offered once, from a tail with its final cost, so the key ends at
        // (cost, best parent).
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          key[j] = make_key(cand[j], eid[j], cand[j] == S.dx[it[j]]);
          doa[j] = val[j] && cand[j] <= (int32_t)(dk[j] >> 32) && key[j] < dk[j];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (doa[j]) old[j] = atomicMin(&a.D64[gy[j]], key[j]);
        // Offers to minD and thr.  With the key read first, every candidate
        // below the D it read is offered, with its head's out_wmin (from the
        // edge record), while the atomics are in flight.  That covers every value D[y] takes in
        // the phase (the candidate that first brings D[y] to a value read a
        // larger D), and a candidate that lost a race to a smaller one is
        // at least y's final D, itself offered: both minima are exact.
        // Without the key read, the atomic's old value decides.
        if (!pc.solo) {
#pragma unroll
          for (int j = 0; j < EPT; ++j) off[j] = val[j] && cand[j] < (int32_t)(dk[j] >> 32);
        } else {
#pragma unroll
          for (int j = 0; j < EPT; ++j) off[j] = doa[j] && cand[j] < (int32_t)(old[j] >> 32);
        }
        uint32_t nmask = 0;
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (doa[j] && (int32_t)(old[j] >> 32) == V::INF) nmask |= 1u << j;  // first discovery
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          int32_t th = V::INF;
          if (off[j]) {
            th = V::add(cand[j], wm[j]);
            if constexpr (!BATCH) {
              lmin = kmin(lmin, cand[j]);
              ltmin = kmin(ltmin, th);
            }
          }
          if constexpr (BATCH)
            batch_offer<V>(bl, a, s_now, off[j], off[j] ? S.inst[it[j]] : 0,
                           off[j] ? cand[j] : V::INF, th);
        }
        // first discoveries (queued for this round's bound step; D[y] can
        // only drop below cand before it runs): places in the stager by one
        // LDS atomic per wave; what does not fit goes to the global list
        {
          static_assert(EPT < 8, "a lane's discoveries fit three bits");
          uint32_t utot;
          const uint32_t ex = wave_excl_small<3>((uint32_t)__popc(nmask), &utot);
          const int tot = (int)utot;
          if (tot) {
            int wbase = 0;
            if (lane_id() == 0) wbase = atomicAdd(&S.st.cnt, tot);
            wbase = __builtin_amdgcn_readlane(wbase, 0);
            int sp = wbase + (int)ex;
            int32_t ni[EPT];
            uint32_t over = 0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
              ni[j] = S.inst[it[j]];
              if ((nmask >> j) & 1u) {
                if (sp < CAP_R) {
                  S.st.v[sp] = gy[j];
                  S.st.d[sp] = cand[j];
                  S.st.inst[sp] = ni[j];
                } else {
                  over |= 1u << j;
                }
                ++sp;
              }
            }
            if (wbase + tot > CAP_R)  // wave-uniform
              relax_push_global<V, BATCH>(a, olist, Cold, md_prev, r, over, gy, cand, ni);
          }
        }
      }
      __syncthreads();
      if (pw.windows == 0) mark(a, r, 0, 5);
      k = wend;
      i += WIN;
      ++pw.windows;
    }
  }
  __syncthreads();
  if (a.trace_blk) pw.t_mid = (long long)wall_clock64();
  // the phase's discoveries to the open list (S.st.cnt is current); what
  // did not fit went to the list during the phase
  relax_flush<V, BATCH>(a, S.st, olist, Cold, md_prev, r, sm);
  mark(a, r, 0, 6);
  if constexpr (!BATCH) {
    block_min2<RBS>(lmin, ltmin, sm.red);
    put_part<V>(a, P_CAND0 + cur, lmin, pc);
    put_part<V>(a, P_TCAND0 + cur, ltmin, pc);
    pw.bmin = lmin;
    pw.bthr = ltmin;
  } else {
    __syncthreads();
    batch_lds_flush<V>(bl, a, s_now, true);
  }
  mark(a, r, 0, 7);
}

// ================================================ live pass (C scope ALL)
// Step (C) for the undiscovered vertices (SP_4's step-4 scope, Section VI):
// C'[y] = max(C[y], minD, m_y), m_y over all in-edges (no in-neighbour of
// an undiscovered vertex is fixed: fixed tails were relaxed), reading the C
// of the round start (Cold) and writing Cnew.  The round's live list holds
// the undiscovered vertices whose C may still be finite (round 1: every
// vertex, by index).  Each thread takes one vertex:
//   discovered since (D < INF): dropped, it is an open item now;
//   C = INF: C' = INF, dropped (it was kept one round so that both C
//     buffers hold INF; an undiscovered vertex with C = INF is unreachable);
//   else its weight-ordered in-list is scanned, the lightest edge alone and
//     then four edges at a time, until minD + w of the last edge read
//     reaches the running minimum (no later, heavier edge can lower it),
//     and the vertex is kept.
// The method's scanned count takes every undiscovered vertex's whole
// in-degree each round; dropped unreachable ones are settled at the end
// from dead_deg and dead_deg_r.
template <class V, bool BATCH>
__device__ void live_pass(const RoundArgs &a, SmemAll &sm, BatchLds<BATCH> &bl,
                          const PhaseCtx &pc, int r, int NL, int32_t md, const int32_t *Cold,
                          int32_t *Cnew) {
  const int tid = threadIdx.x;
  const int cur = r & 1, s_now = r % 3;
  const int I = a.num_inst;
  SmemLive &L = sm.u.l;
  const int32_t *Lv = cur ? a.live_v1 : a.live_v0;
  int32_t *Ln = cur ? a.live_v0 : a.live_v1;
  unsigned long long *lctr = &a.ctl->live_ctr[cur ^ 1];
  if (tid == 0) L.cnt = 0;
  __syncthreads();
  // Tiles of LPT * RBS list entries go round-robin to the blocks (the lists
  // keep solver order, and under degree order the costly vertices come
  // first); thread tid takes entries tid, tid + RBS, ... of a tile and
  // issues the loads of all of them before any test (an entry leaves the
  // list only at the compaction after its discovery, so its own words are
  // read unconditionally).  A batch takes kLivePT entries per thread: its
  // long lists of low-degree vertices pay the tile's scan and barriers once
  // for all of them.  A single solve takes one: a thread's in-edge loops run
  // one after another, and a degree-ordered list starts with the hubs.
  long long scanned = 0, ddeg = 0, ddeg_r = 0;
  constexpr int LPT = BATCH ? kLivePT : 1;
  constexpr uint32_t TILE = LPT * RBS;
  for (uint32_t b0 = pc.vbid * TILE; b0 < (uint32_t)NL; b0 += pc.vnb * TILE) {
    int32_t y[LPT], ins[LPT], sb[LPT], gi[LPT], mdi[LPT], c[LPT];
    int32_t c0[LPT];
    unsigned long long dk[LPT];
    int4 rec[LPT];  // in_off, in_degree, lightest in-edge's tail and weight
    bool val[LPT], keep[LPT];
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const uint32_t i = b0 + (uint32_t)(k * RBS + tid);
      val[k] = i < (uint32_t)NL;
      keep[k] = false;
      y[k] = (r == 1) ? (int32_t)(val[k] ? i : 0u) : Lv[val[k] ? i : 0u];
    }
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      sb[k] = 0;
      gi[k] = 0;
      ins[k] = 0;
      mdi[k] = md;
      if constexpr (BATCH) ins[k] = a.inst_of[y[k]];
      dk[k] = a.D64[y[k]];
      // round 1: every C is still 0 but the sources', and they are
      // discovered (their entries drop at the test below)
      c[k] = (r == 1) ? 0 : Cold[y[k]];
    }
    if constexpr (BATCH) {
      // the entry's instance, and that instance's minD this round (INF:
      // its rounds have ended, so its undiscovered vertices are done)
#pragma unroll
      for (int k = 0; k < LPT; ++k) {
        const InstDev id = a.insts[ins[k]];
        sb[k] = id.sbase;
        gi[k] = id.graph;
        mdi[k] = ld_relaxed(&a.imin[s_now * I + ins[k]]);
      }
    }
    // the in-side half of the vertex record: in_off, in_degree, the
    // lightest in-edge's tail and weight (16 bytes, not the 32 of vrec)
#pragma unroll
    for (int k = 0; k < LPT; ++k) rec[k] = graph_of<BATCH>(a, gi[k]).vin[y[k] - sb[k]];
    // A batch also gathers the lightest in-edge's tail C here; a single
    // solve only where the tests below pass (measured faster there).  Round
    // 1 reads the initial C: 0 for every vertex but the source, and the
    // source is no tail of an undiscovered vertex, its out-edges having been
    // relaxed.
#pragma unroll
    for (int k = 0; k < LPT; ++k) c0[k] = (r == 1 || !BATCH) ? 0 : Cold[sb[k] + rec[k].z];
#pragma unroll
    for (int k = 0; k < LPT; ++k)
      asm volatile("" : "+v"(dk[k]), "+v"(c[k]), "+v"(c0[k]), "+v"(rec[k].x), "+v"(rec[k].y),
                   "+v"(rec[k].w));
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const GraphDev &G = graph_of<BATCH>(a, gi[k]);
      if (!(val[k] && G.all && mdi[k] != V::INF && (int32_t)(dk[k] >> 32) == V::INF)) continue;
      const int32_t b = rec[k].x, deg = rec[k].y;
      const int32_t *Cg = Cold + sb[k];  // the instance's C, by graph-local id
      if constexpr (BATCH) {
        if (I > kLdsInst) atomicAdd(&a.iscanned[3 * ins[k]], (unsigned long long)deg);
        else atomicAdd(&bl.scan[ins[k]], (uint32_t)deg);
      } else {
        scanned += deg;
      }
      if (c[k] == V::INF) {
        Cnew[y[k]] = V::INF;
        if constexpr (BATCH) {
          if (deg) {
            atomicAdd(&a.idead[2 * ins[k]], (unsigned long long)deg);
            atomicAdd(&a.idead[2 * ins[k] + 1], (unsigned long long)deg * (unsigned long long)r);
          }
        } else {
          ddeg += deg;
          ddeg_r += (long long)deg * r;
        }
        continue;
      }
      int32_t m = V::INF;
      int32_t j = 0;
      const int32_t mk = mdi[k];
      if (deg > 0) {
        // the lightest in-edge alone first: its tail usually decides m
        const int32_t w0 = rec[k].w;
        const int32_t cz = (BATCH || r == 1) ? c0[k] : Cg[rec[k].z];
        if (cz != V::INF) m = V::add(kmax(cz, mk), w0);
        j = (V::add(mk, w0) >= m) ? deg : 1;
      }
      for (; j < deg; j += 4) {
        int32_t vs[4], ws[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int2 e = (j + q < deg) ? G.in_sw[b + j + q] : make_int2(0, 0);
          vs[q] = e.x;
          ws[q] = e.y;
        }
        int32_t cs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) cs[q] = (j + q < deg) ? Cg[vs[q]] : V::INF;
        int32_t wl = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (j + q < deg) {
            if (cs[q] != V::INF) m = kmin(m, V::add(kmax(cs[q], mk), ws[q]));
            wl = ws[q];
          }
        }
        if (V::add(mk, wl) >= m) break;
      }
      Cnew[y[k]] = kmax(kmax(c[k], mk), m);
      keep[k] = true;
    }
    // stage the kept vertices in list order (entry k * RBS + tid of the
    // tile): one scan of the per-slot keep flags packed in 16-bit fields;
    // flush to the next live list when full
    uint64_t packed = 0;
#pragma unroll
    for (int k = 0; k < LPT; ++k) packed |= (uint64_t)(keep[k] ? 1u : 0u) << (16 * k);
    uint64_t tot;
    const uint64_t ex = block_excl_scan64<RBS>(packed, sm.scan, &tot);
    int tcnt = 0;
#pragma unroll
    for (int k = 0; k < LPT; ++k) tcnt += (int)((tot >> (16 * k)) & 0xffffu);
    if (L.cnt + tcnt > CAP_L) {
      const int cnt = L.cnt;
      if (tid == 0) L.base = (int32_t)atomicAdd(lctr, (unsigned long long)cnt);
      __syncthreads();
      for (int j = tid; j < cnt; j += RBS) Ln[L.base + j] = L.v[j];
      __syncthreads();
      if (tid == 0) L.cnt = 0;
      __syncthreads();
    }
    int before = L.cnt;
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      if (keep[k]) L.v[before + (int)((ex >> (16 * k)) & 0xffffu)] = y[k];
      before += (int)((tot >> (16 * k)) & 0xffffu);
    }
    __syncthreads();
    if (tid == 0) L.cnt += tcnt;
    __syncthreads();
  }
  {
    const int cnt = L.cnt;
    if (cnt > 0) {
      if (tid == 0) L.base = (int32_t)atomicAdd(lctr, (unsigned long long)cnt);
      __syncthreads();
      for (int j = tid; j < cnt; j += RBS) Ln[L.base + j] = L.v[j];
    }
  }
  if constexpr (!BATCH) {
    const long long s1 = wave_sum64(scanned), s2 = wave_sum64(ddeg), s3 = wave_sum64(ddeg_r);
    if (lane_id() == 0) {
      if (s1) atomicAdd(&sm.n_scanned, (unsigned long long)s1);
      if (s2) atomicAdd(&a.ctl->dead_deg, (unsigned long long)s2);
      if (s3) atomicAdd(&a.ctl->dead_deg_r, (unsigned long long)s3);
    }
  }
  __syncthreads();
}

// ========================================================== bound-and-fix
template <class V, bool BATCH>
__device__ void fused_phase(const RoundArgs &a, SmemAll &sm, const PhaseCtx &pc, int r, int NO,
                            uint32_t EO, int NL, int32_t mind_all, int32_t thr_all,
                            BatchLds<BATCH> &bl, PhaseWork &pw) {
  const int tid = threadIdx.x;
  const int cur = r & 1, s_now = r % 3, s_next = (r + 1) % 3;
  const int I = a.num_inst;
  Ctl *ctl = a.ctl;
  const int32_t *Ov = cur ? a.open_v1 : a.open_v0;
  const int32_t *Op = cur ? a.open_p1 : a.open_p0;
  const int32_t *Oi = cur ? a.open_i1 : a.open_i0;
  const int32_t *Cold = cur ? a.C1 : a.C0;
  int32_t *Cnew = cur ? a.C0 : a.C1;
  int32_t *const *Ox = cur ? a.open_x1 : a.open_x0;
  int32_t *const *Nx = cur ? a.open_x0 : a.open_x1;
  const ListRef next_open = {&ctl->open_ctr[cur ^ 1], cur ? a.open_v0 : a.open_v1,
                             cur ? a.open_p0 : a.open_p1, cur ? a.open_i0 : a.open_i1,
                             {Nx[0], Nx[1], Nx[2], Nx[3], Nx[4], Nx[5]}};
  const ListRef front = {&ctl->front_ctr[cur ^ 1], a.front_v, a.front_p, a.front_i,
                         {a.front_x[FX_OOFF], a.front_x[FX_D]}};
  SmemFused &S = sm.u.f;
  if (tid == 0) {
    S.fr.cnt = 0;
    S.fr.deg = 0;
    S.op.cnt = 0;
    S.op.deg = 0;
  }
  if constexpr (BATCH) batch_lds_reset<V>(bl, I);
  __syncthreads();
  mark(a, r, 1, 3);
  int32_t lnext = V::INF, ltnext = V::INF;
  const uint32_t WT = EO + CW_FUSED * (uint32_t)NO;
  const uint32_t chunk = chunk_of(WT, pc.vnb);
  const uint32_t e0 = pc.vbid * chunk;
  const uint32_t e1 = min(WT, e0 + chunk);
  if (e0 < e1) {
    int i = uni(find_start_item(Op, NO, CW_FUSED, e0, sm));
    uint32_t k = e0;
    pw.first_item = i;
    pw.units = e1 - e0;
    mark(a, r, 1, 4);
    while (k < e1) {
      const int idx = i + tid;
      S.acc[tid] = V::INF;
      S.cnt[tid] = 0;
      if (idx < NO) {
        const int32_t gy = Ov[idx];
        S.pfx[tid] = Op[idx] + (int32_t)(CW_FUSED * (uint32_t)idx);
        int32_t sb = 0, gi = 0, ins = 0;
        if constexpr (BATCH) {
          ins = Oi[idx];
          const InstDev id = a.insts[ins];
          sb = id.sbase;
          gi = id.graph;
          S.mind[tid] = ld_relaxed(&a.imin[s_now * I + ins]);
          S.thr[tid] = ld_relaxed(&a.ithr[s_now * I + ins]);
        }
        const GraphDev &G = graph_of<BATCH>(a, gi);
        S.dy[tid] = ld_relaxed(key_d(&a.D64[gy]));
        // everything the item's finish needs, carried by its entry (a first
        // discovery's in-degree as -1 - in-degree), or (first discovery, no
        // payload) one vertex record with C = 0
        int32_t xv[kOX];
#pragma unroll
        for (int k = 0; k < kOX; ++k) xv[k] = Ox[k][idx];
        // (the no-payload mark first: the other words of such an entry are
        // left over from an earlier list)
        if (xv[OX_BASE] >= 0 && xv[OX_IDEG] < 0) {
          xv[OX_IDEG] = -1 - xv[OX_IDEG];
          // the probe may have cut its scan short of the weight prefix
          if (xv[OX_IDEG] > 16) S.cnt[tid] = kNoCount;
        } else if (xv[OX_BASE] < 0) {
          const int32_t yl = gy - sb;
          const int4 rec = G.vrec[2 * yl];  // out_off, out_degree, in_off, in_degree
          xv[OX_BASE] = rec.z;
          xv[OX_IDEG] = rec.w;
          xv[OX_OOFF] = rec.x;
          xv[OX_ODEG] = rec.y;
          xv[OX_OWM] = G.vrec[2 * yl + 1].x;
          // C of an undiscovered vertex: 0, or under scope ALL what the
          // live pass raised it to
          xv[OX_C] = G.all ? Cold[gy] : 0;
          // the probe may have cut its scan short of the weight prefix
          if (xv[OX_IDEG] > 16) S.cnt[tid] = kNoCount;
        }
        S.base[tid] = xv[OX_BASE];
        S.ideg[tid] = xv[OX_IDEG];
        S.ooff[tid] = xv[OX_OOFF];
        S.odeg[tid] = xv[OX_ODEG];
        S.owm[tid] = xv[OX_OWM];
        S.cy[tid] = xv[OX_C];
        S.sb[tid] = sb;
        S.gi[tid] = gi;
        S.inst[tid] = ins;
      } else {
        S.pfx[tid] = (int32_t)WT;
      }
      if (tid == 0)
        S.pfx[WIN] = (i + WIN < NO) ? Op[i + WIN] + (int32_t)(CW_FUSED * (uint32_t)(i + WIN))
                                    : (int32_t)WT;
      __syncthreads();
      if (pw.windows == 0) mark(a, r, 1, 5);
      const uint32_t wend = uni(min((uint32_t)S.pfx[WIN], e1));
      // The units of an item are CW_FUSED of bookkeeping and then its
      // edges; lanes walk only the edges that fall in [k, wend).
      uint64_t etot;
      {
        uint32_t ecnt = 0;
        if (idx < NO) {
          const uint32_t p0 = (uint32_t)S.pfx[tid] + CW_FUSED, p1 = (uint32_t)S.pfx[tid + 1];
          const uint32_t lo = max(p0, k), hi = min(p1, wend);
          if (hi > lo) {
            ecnt = hi - lo;
            S.eoff[tid] = (int32_t)(lo - p0);
          }
        }
        S.epfx[tid] = (int32_t)block_excl_scan64<RBS>((uint64_t)ecnt, sm.scan, &etot);
        __syncthreads();
      }
      const uint32_t ET = uni((uint32_t)etot);
      for (uint32_t cb = 0; cb < ET; cb += RBS * EPT) {
        // As in the relax step: lanes past the window's last edge repeat it,
        // so that the EPT loads of a step issue together, unconditionally.
        int it[EPT];
        int32_t pos[EPT], v[EPT], wt[EPT], cv[EPT], sbv[EPT], dyv[EPT];
        bool val[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const uint32_t q = cb + (uint32_t)(j * RBS + tid);
          val[j] = q < ET;
          const uint32_t qc = val[j] ? q : ET - 1u;
          it[j] = window_item(S.epfx, qc);
          pos[j] = S.base[it[j]] + S.eoff[it[j]] + (int32_t)(qc - (uint32_t)S.epfx[it[j]]);
          sbv[j] = S.sb[it[j]];
          dyv[j] = S.dy[it[j]];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int2 e = graph_of<BATCH>(a, S.gi[it[j]]).in_sw[pos[j]];
          v[j] = e.x;
          wt[j] = e.y;
        }
        // the loaded values count as used here: no load moves into the
        // gather's condition below
#pragma unroll
        for (int j = 0; j < EPT; ++j) asm volatile("" : "+v"(v[j]), "+v"(wt[j]));
        // An in-edge can only lower min(D[y], m_y) below D[y] if
        // minD + w < D[y]: its term max(C[v], minD) + w is at least
        // minD + w (rounding is monotone).  Every other edge leaves C'[y]
        // exactly as it is, so its tail's lower bound is not gathered.
        // Every lane gathers (a filtered one reads entry 0: one line for all
        // of them), so that no load sits in a branch.
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int32_t md = BATCH ? S.mind[it[j]] : mind_all;
          val[j] = val[j] & (V::add(md, wt[j]) < dyv[j]);
          cv[j] = Cold[val[j] ? sbv[j] + v[j] : 0];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int32_t md = BATCH ? (val[j] ? S.mind[it[j]] : 0) : mind_all;
          const int32_t t = val[j] ? V::add(kmax(cv[j], md), wt[j]) : V::INF;
          const int myit = val[j] ? it[j] : -1;
          // 1 + the edge's position in the item's list
          const int32_t c1 = val[j] ? pos[j] - S.base[it[j]] + 1 : 0;
          // segmented min (and position max) into LDS; one LDS atomic per
          // wave when the whole wave works on one item (hub vertices)
          const uint64_t act = __ballot(val[j]);
          if (act) {
            const int lead = __ffsll((unsigned long long)act) - 1;
            const int it0 = __builtin_amdgcn_readlane(myit, lead);
            const uint64_t same = __ballot(val[j] && myit == it0);
            if (same == act) {
              const int32_t wm = wave_min(t);
              const int32_t wc = wave_max(c1);
              if (lane_id() == lead) {
                if (wm < V::INF) atomicMin(&S.acc[it0], wm);
                atomicMax(&S.cnt[it0], wc);
              }
            } else if (val[j]) {
              if (t < V::INF) atomicMin(&S.acc[myit], t);
              atomicMax(&S.cnt[myit], c1);
            }
          }
        }
      }
      __syncthreads();
      if (pw.windows == 0) mark(a, r, 1, 6);
      // finish the window's items: thread tid handles window item tid
      bool hf = false, ho = false;
      int32_t gy = 0, fd = 0, od = 0, ins = 0, nfix = 0;
      int32_t sv = V::INF, st = V::INF;  // a survivor's offers to the next minD / thr
      int32_t sdeg = 0;                  // in-degree of a finished item (statistics)
      int32_t fx[kFX] = {0, 0}, ox[kOX] = {0, 0, 0, 0, 0, 0};  // payloads of the pushes
      if (idx < NO) {
        const uint32_t p0 = (uint32_t)S.pfx[tid], p1 = (uint32_t)S.pfx[tid + 1];
        const uint32_t fb = p0 / chunk, lb = (p1 - 1) / chunk;  // p1 > p0 always
        if (fb <= pc.vbid && pc.vbid <= lb) {
          int32_t m = S.acc[tid];
          bool fin = (fb == lb);
          if (!fin) {
            // Split item: the last block to arrive sees every partial.  All
            // three operations are device-scope atomics, performed at one
            // point per address; each block's atomicMin has completed
            // (vmcnt(0)) before its arrival is counted, and the last
            // arriver reads the minimum only after counting, so no cache
            // write-back or invalidate is needed.
            int32_t prev = V::INF;
            if (m < V::INF) prev = atomicMin(&a.mtmp[idx], m);
            __asm__ volatile("" : : "v"(prev));  // the atomic has returned (is performed)
            const unsigned int old = atomicAdd(&a.arrive[idx], 1u);
            if (old == lb - fb) {
              fin = true;
              m = atomicMin(&a.mtmp[idx], V::INF);  // reads the final minimum
              a.mtmp[idx] = V::INF;
              a.arrive[idx] = 0u;
            }
          }
          ins = S.inst[tid];
          if (fin) {
            gy = Ov[idx];
            const int32_t md = BATCH ? S.mind[tid] : mind_all;
            const int32_t th = BATCH ? S.thr[tid] : thr_all;
            const int32_t Dy = S.dy[tid], Cy = S.cy[tid];
            const int32_t Cn = kmax(kmax(Cy, md), kmin(Dy, m));
            const GraphDev &G = graph_of<BATCH>(a, S.gi[tid]);
            // the method's count: every in-edge of an open vertex is covered
            const long long deg = S.ideg[tid];
            if constexpr (BATCH) {
              if (a.istat) {  // statistics requested
                if (I > kLdsInst) {
                  atomicAdd(&a.iscanned[3 * ins], (unsigned long long)deg);
                  atomicAdd(&a.iscanned[3 * ins + 1], 1ull);
                } else {
                  atomicAdd(&bl.scan[ins], (uint32_t)deg);
                  atomicAdd(&bl.visit[ins], 1u);
                }
              }
            } else {
              sdeg = (int32_t)deg;
            }
            // label-correcting: the D y was last relaxed with (INF if never)
            const int32_t dr = G.lc ? a.DR[gy] : V::INF;
            if (Cn >= Dy || Dy <= th) {
              Cnew[gy] = V::INF;  // fixed: drops out of every later bound step
              if (gy == pc.target) ctl->target_hit = 1;
              // next round's relax list; a vertex already relaxed at its
              // final D comes with no edges, only to mark its C
              fd = Dy < dr ? S.odeg[tid] : 0;
              hf = true;
              nfix = 1;
              fx[FX_OOFF] = S.ooff[tid];
              fx[FX_D] = Dy;
            } else {
              Cnew[gy] = Cn;
              // Next round (minD >= md, D[y] <= Dy) needs at most the
              // edges that passed this round's weight test, a prefix of the
              // list; the scan counted it, unless the item was split over
              // blocks or its scan may have stopped short (then a search)
              const int32_t sc = S.cnt[tid];
              od = (fb == lb && sc < kNoCount)
                       ? sc
                       : useful_in_edges_at<V>(G, S.base[tid], S.ideg[tid], md, Dy);
              ho = true;
              ox[OX_BASE] = S.base[tid];
              ox[OX_IDEG] = S.ideg[tid];
              ox[OX_OOFF] = S.ooff[tid];
              ox[OX_ODEG] = S.odeg[tid];
              ox[OX_OWM] = S.owm[tid];
              ox[OX_C] = Cn;
              const int32_t tn = V::add(Dy, S.owm[tid]);
              sv = Dy;
              st = tn;
              if (G.lc && Dy < dr && Dy < V::add(md, G.delta)) {
                // label-correcting: relaxed again from its lower D (while in
                // the first bucket above minD)
                hf = true;
                fd = S.odeg[tid];
                fx[FX_OOFF] = S.ooff[tid];
                fx[FX_D] = Dy | kOpenRelax;
              }
              if constexpr (!BATCH) {
                lnext = kmin(lnext, Dy);
                ltnext = kmin(ltnext, tn);
              }
            }
          }
        }
      }
      if constexpr (BATCH) {
        batch_offer<V>(bl, a, s_next, ho, ins, sv, st);
      } else {
        const long long ws = wave_sum64(sdeg), wf = wave_sum64(nfix);
        if (lane_id() == 0 && ws) atomicAdd(&sm.n_scanned, (unsigned long long)ws);
        if (lane_id() == 0 && wf) atomicAdd(&sm.n_fixed, (unsigned long long)wf);
      }
      stage_push2(S.fr, hf, gy, fd, ins, fx, front, S.op, ho, gy, od, ins, ox, next_open, BATCH,
                  sm);
      if (pw.windows == 0) mark(a, r, 1, 7);
      k = wend;
      i += WIN;
      ++pw.windows;
    }
  }
  stage_flush2(S.fr, front, S.op, next_open, BATCH);
  if (a.trace_blk) pw.t_mid = (long long)wall_clock64();
  if (NL > 0) {
    __syncthreads();  // the live pass reuses the stagers' LDS
    live_pass<V, BATCH>(a, sm, bl, pc, r, NL, mind_all, Cold, Cnew);
  }
  mark(a, r, 1, 8);
  if constexpr (!BATCH) {
    block_min2<RBS>(lnext, ltnext, sm.red);
    put_part<V>(a, P_SURV0 + (cur ^ 1), lnext, pc);
    put_part<V>(a, P_TSURV0 + (cur ^ 1), ltnext, pc);
    pw.bmin = lnext;
    pw.bthr = ltnext;
  } else {
    __syncthreads();
    batch_lds_flush<V>(bl, a, s_next, false);
  }
  mark(a, r, 1, 9);
}

// ------------------------------------------------ active blocks, parking
// A phase runs on blocks [0, k): k = 1 for phases of at most `solo_edges`
// edges (block barriers only), else a power of two near work / block_units,
// at most the grid.  Every active block derives the same k from the list
// counter.  Blocks outside the active set park on `go`; block 0 wakes them
// when the set grows.  All blocks count `go` bumps (epoch) and active
// barriers (aep) alike, so a parked block adopts both on waking.
__device__ __forceinline__ uint32_t active_for(const RoundArgs &a, uint32_t E, uint32_t WT,
                                               uint32_t nb) {
  if (a.solo_edges > 0 && E <= (uint32_t)a.solo_edges) return 1u;
  const uint32_t u = a.block_units > 0 ? (uint32_t)a.block_units : 1u;
  const uint32_t want = (WT + u - 1) / u;
  uint32_t k = 2;
  while (k < want && k < nb) k <<= 1;
  return k < nb ? k : nb;
}

// Block 0 publishes the resume point in the next hand-over's slot and moves
// `go` one epoch on.
__device__ void wake_parked(Ctl *ctl, unsigned int &epoch, int r, int phase, int done,
                            uint32_t act, unsigned int aep) {
  wait_own_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    ResumeSlot &s = ctl->resume[(epoch + 1u) % kResumeSlots];
    s.round = r;
    s.phase = phase;
    s.done = done;
    s.act = (int32_t)act;
    s.aep = aep;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&ctl->go, epoch + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  epoch += 1u;
  __syncthreads();
}

// A parked block sleeps until a hand-over names it active (or the solve
// ends) and adopts the resume point.  Returns true when the solve is done.
// It reads the slot of the hand-over it saw and keeps it only if no more
// than kResumeSlots - 2 hand-overs followed meanwhile (block 0 writes the
// slot of hand-over e + 1 before announcing it, so slot g is intact while
// go < g + kResumeSlots - 1).  Hand-overs can follow only while this block
// is not among their active blocks (block 0 waits for every active block
// at the phase's end), so the slot it keeps names it active only if it is
// the latest; otherwise it waits for the next one.
__device__ bool park(Ctl *ctl, unsigned int &epoch, unsigned int &aep, int &r, int &phase,
                     uint32_t &act, SmemAll &sm) {
  for (;;) {
    if (threadIdx.x == 0) {
      unsigned int g, g2;
      for (;;) {
        while ((int)((g = ld_flag(&ctl->go)) - epoch) <= 0) __builtin_amdgcn_s_sleep(2);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const ResumeSlot *s = &ctl->resume[g % kResumeSlots];
        sm.res_round = ld_relaxed(&s->round);
        sm.res_phase = ld_relaxed(&s->phase);
        sm.res_done = ld_relaxed(&s->done);
        sm.res_act = ld_relaxed(&s->act);
        sm.res_aep = (unsigned int)ld_relaxed((const int32_t *)&s->aep);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        g2 = ld_flag(&ctl->go);
        if ((int)(g2 - g) <= kResumeSlots - 2) break;
      }
      sm.res_go = g;
    }
    __syncthreads();
    epoch = sm.res_go;
    r = sm.res_round;
    phase = sm.res_phase;
    act = (uint32_t)sm.res_act;
    aep = sm.res_aep;
    const bool done = sm.res_done != 0;
    __syncthreads();
    if (done) return true;
    if (blockIdx.x < act) return false;
  }
}

// ------------------------------------------------------------ the kernel
template <class V, bool BATCH>
__global__ __launch_bounds__(RBS) void rounds_kernel(RoundArgs a) {
  __shared__ SmemAll sm;
  __shared__ BatchLds<BATCH> bl;
  const int tid = threadIdx.x;
  const uint32_t nb = gridDim.x, bid = blockIdx.x;
  Ctl *ctl = a.ctl;
  const int I = a.num_inst;
  unsigned int epoch = 0;  // hand-overs so far (bumps of ctl->go)
  unsigned int aep = 0;    // barriers of the active blocks so far
  int r = 1, phase = 0;    // phase 0: relax, 1: bound-and-fix
  uint32_t act = nb;       // active blocks
  int32_t md_prev = 0;     // the last minD this block computed (0 before round 1)
  const int32_t tgt = (!BATCH && a.target >= 0) ? uni(ld_relaxed(&ctl->target_id)) : -1;
  if (tid == 0) {
    sm.n_relaxed = sm.n_open = sm.n_solo = sm.n_bound = 0;
    sm.n_fixed = 0ull;
    sm.n_scanned = 0ull;
    sm.solo_cand_r = sm.solo_surv_r = -1;
  }
  __syncthreads();

  for (;;) {
    const int cur = r & 1;
    mark(a, r, phase, 0);
    const uint64_t ctr =
        ld_relaxed64(phase == 0 ? &ctl->front_ctr[cur] : &ctl->open_ctr[cur]);
    const int N = uni((int)(ctr >> 32));
    const uint32_t E = uni((uint32_t)(ctr & 0xffffffffull));
    if (N >= 0) mark(a, r, phase, 1);  // the counter has arrived
    // termination: the relax left nothing open, the target has been fixed
    // (single-target solve: the frontier it joined is not relaxed), or the
    // watchdog (rounds never exceed the reachable count)
    const bool watchdog = phase == 0 && r > a.max_rounds;
    const bool reached = phase == 0 && tgt >= 0 && uni(ld_relaxed(&ctl->target_hit)) != 0;
    if (watchdog || reached || (phase == 1 && N == 0)) {
      if (bid == 0 && tid == 0) {
        if (watchdog) ctl->status = 7;
        ctl->rounds = watchdog ? a.max_rounds : (reached ? r - 1 : r);
      }
      if (act < nb && bid == 0) wake_parked(ctl, epoch, r, phase, 1, act, aep);
      break;
    }
    // scope ALL: the bound step also walks the live list (round 1: all n)
    const int NL = (phase == 1 && a.scope_all)
                       ? (r == 1 ? a.total : uni((int)ld_relaxed64(&ctl->live_ctr[cur])))
                       : 0;
    const uint32_t WL = CW_LIVE * (uint32_t)NL;
    const uint32_t WT = E + (phase == 0 ? CW_RELAX : CW_FUSED) * (uint32_t)N + WL;
    const uint32_t want = active_for(a, E + WL, WT, nb);
    if (want < act) {
      if (bid >= want) {
        if (park(ctl, epoch, aep, r, phase, act, sm)) break;
        continue;  // resume where block 0 left off
      }
      act = want;
    } else if (want > act) {
      if (bid == 0) wake_parked(ctl, epoch, r, phase, 0, want, aep);
      else epoch += 1u;
      act = want;
    }
    const bool solo = act == 1;
    const PhaseCtx pc = {act, bid, solo, tgt};
    long long *tr = (a.trace && r <= a.trace_rounds) ? a.trace + (size_t)(r - 1) * kTraceFields
                                                      : nullptr;
    long long *tb = (a.trace_blk && r <= a.trace_blk_rounds)
                        ? a.trace_blk + (((size_t)(r - 1) * 2 + phase) * kMaxBlocks + bid) *
                                            kBlkFields
                        : nullptr;
    if (bid == 0) {
      if (tid == 0) {
        if (phase == 0) {
          // counters the coming bound-and-fix appends to (last read a round ago)
          ctl->open_ctr[cur ^ 1] = 0ull;
          ctl->front_ctr[cur ^ 1] = 0ull;
          ctl->live_ctr[cur ^ 1] = 0ull;
          sm.n_relaxed += E;
        } else {
          sm.n_open += N;
          sm.n_bound += 1;
        }
        if (solo) sm.n_solo += 1;
        if (tr) {
          if (phase == 0) {
            tr[TR_START] = (long long)wall_clock64();
            tr[TR_NF] = N;
            tr[TR_EF] = E;
          } else {
            tr[TR_NO] = N;
            tr[TR_EO] = E;
            tr[TR_NL] = NL;
          }
          // active blocks of the relax (low half) and bound-and-fix phases
          tr[TR_MODE] |= (long long)act << (16 * phase);
        }
      }
      if constexpr (BATCH) {
        if (phase == 0) {
          const int s_next = (r + 1) % 3;
          for (int i = tid; i < I; i += RBS) {
            a.imin[s_next * I + i] = V::INF;
            a.ithr[s_next * I + i] = V::INF;
          }
        }
      }
    }
    PhaseWork pw;
    if (phase == 0) {
      relax_phase<V, BATCH>(a, sm, bl, pc, r, N, E, md_prev, pw);
      if (!BATCH && solo && tid == 0) {
        // block 0 alone wrote every partial slot: keep the values
        sm.solo_cand_min = pw.bmin;
        sm.solo_cand_thr = pw.bthr;
        sm.solo_cand_r = r;
      }
    } else {
      int32_t mind_all = V::INF, thr_all = V::INF;
      if constexpr (!BATCH) {
        if (solo && sm.solo_cand_r == r && sm.solo_surv_r == r - 1) {
          // both halves of this round's minima came from block 0 alone
          mind_all = kmin(sm.solo_cand_min, sm.solo_surv_min);
          thr_all = kmin(sm.solo_cand_thr, sm.solo_surv_thr);
        } else {
          reduce_parts<V>(a, cur, mind_all, thr_all, sm);
        }
        mind_all = uni(mind_all);
        thr_all = uni(thr_all);
        if (mind_all != V::INF) md_prev = mind_all;  // minD never decreases over rounds
      }
      mark(a, r, 1, 2);
      fused_phase<V, BATCH>(a, sm, pc, r, N, E, NL, mind_all, thr_all, bl, pw);
      if (!BATCH && solo && tid == 0) {
        sm.solo_surv_min = pw.bmin;
        sm.solo_surv_thr = pw.bthr;
        sm.solo_surv_r = r;
      }
    }
    if (tb && tid == 0) {
      tb[0] = (long long)wall_clock64();
      tb[1] = pw.windows;
      tb[2] = pw.first_item;
      tb[3] = pw.units;
      tb[4] = pw.t_mid;
    }
    if (tr && bid == 0 && tid == 0) tr[phase == 0 ? TR_ARR_RELAX : TR_ARR_FUSED] = (long long)wall_clock64();
    if (solo) {
      wait_own_stores();
      __syncthreads();
    } else {
      grid_barrier(a.flags, &ctl->go_a, aep, act);
    }
    if (tr && bid == 0 && tid == 0) tr[phase == 0 ? TR_END_RELAX : TR_END_FUSED] = (long long)wall_clock64();
    mark(a, r, phase, 10);
    if (phase == 0) {
      phase = 1;
    } else {
      phase = 0;
      ++r;
    }
  }
  __syncthreads();
  if (!BATCH && a.scope_all && bid == 0 && tid == 0) {
    // unreachable vertices dropped from the live list in round r_d are
    // still scanned in every later round with a bound step
    const unsigned long long dd = ld_relaxed64(&ctl->dead_deg);
    const unsigned long long ddr = ld_relaxed64(&ctl->dead_deg_r);
    sm.n_scanned += dd * (unsigned long long)sm.n_bound - ddr;
  }
  if (!BATCH && tid == 0 && sm.n_scanned)
    atomicAdd((unsigned long long *)&ctl->scanned, sm.n_scanned);
  // settled: the source plus every vertex a bound step fixed
  if (!BATCH && tid == 0 && (sm.n_fixed || bid == 0))
    atomicAdd((unsigned long long *)&ctl->settled, sm.n_fixed + (bid == 0 ? 1ull : 0ull));
  if (bid == 0 && tid == 0) {
    ctl->relaxed = sm.n_relaxed;
    ctl->open_visits = sm.n_open;
    ctl->solo_phases = sm.n_solo;
  }
}

// ------------------------------------------------------------------ init
// D = INF, C = 0 (both buffers), mtmp = INF, arrive = 0 (and, with
// label-correcting relax, DR = INF) over all state entries; barrier flags
// and the per-block partial slots are reset.
template <class V>
__global__ void init_fill_kernel(RoundArgs a) {
  const int32_t stride = gridDim.x * blockDim.x;
  const int32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int32_t i = t0; i < a.total; i += stride) {
    a.D64[i] = make_key(V::INF, -1, false);
    a.C0[i] = 0;
    a.C1[i] = 0;
    a.mtmp[i] = V::INF;
    a.arrive[i] = 0u;
    if (a.DR) a.DR[i] = V::INF;
  }
  for (int32_t i = t0; i < kMaxBlocks; i += stride) a.flags[i * kFlagStride] = 0u;
  for (int32_t i = t0; i < kParts * kMaxBlocks; i += stride) a.part[i] = V::INF;
}

// Batched solves with a scope-ALL graph: the instance of every state entry
// (block b fills instance b's range).
__global__ void inst_of_kernel(RoundArgs a) {
  for (int i = blockIdx.x; i < a.num_inst; i += gridDim.x) {
    const InstDev id = a.insts[i];
    for (int32_t j = threadIdx.x; j < id.n; j += blockDim.x) a.inst_of[id.sbase + j] = i;
  }
}

// One block: seeds every instance's source, the first frontier (with its
// out-degree prefix, read by round 1 at parity 1) and the control block.
template <class V, bool BATCH>
__global__ void init_seed_kernel(RoundArgs a) {
  __shared__ uint64_t scan[RBS / SSSP_WAVE + 1];
  const int I = a.num_inst;
  uint64_t run = 0;
  for (int b0 = 0; b0 < I; b0 += RBS) {
    const int i = b0 + threadIdx.x;
    uint32_t deg = 0;
    int32_t gs = 0, ooff = 0;
    if (i < I) {
      int32_t sb = 0, gi = 0, s = a.source;
      if constexpr (BATCH) {
        const InstDev id = a.insts[i];
        sb = id.sbase;
        gi = id.graph;
        s = id.source;
      }
      const GraphDev &G = graph_of<BATCH>(a, gi);
      if (G.rank) s = G.rank[s];  // the solver's id of the source
      gs = sb + s;
      if constexpr (!BATCH) {
        int32_t t = a.target;
        if (t >= 0 && G.rank) t = G.rank[t];
        a.ctl->target_id = t;
        a.ctl->target_hit = (t >= 0 && t == s) ? 1 : 0;  // the source is fixed at the start
      }
      ooff = G.out_off[s];
      deg = (uint32_t)(G.out_off[s + 1] - ooff);
      a.D64[gs] = make_key(0, -1, false);
      a.C0[gs] = V::INF;
      a.C1[gs] = V::INF;
    }
    uint64_t tot;
    const uint64_t ex = block_excl_scan64<RBS>((uint64_t)deg, scan, &tot);
    if (i < I) {
      a.front_v[i] = gs;
      a.front_p[i] = (int32_t)(run + ex);
      a.front_x[FX_OOFF][i] = ooff;
      a.front_x[FX_D][i] = 0;
      if constexpr (BATCH) {
        a.front_i[i] = i;
        for (int s = 0; s < 3; ++s) {
          a.imin[s * I + i] = V::INF;
          a.ithr[s * I + i] = V::INF;
        }
        a.irounds[i] = 0;
        a.iscanned[3 * i] = 0ull;
        a.iscanned[3 * i + 1] = 0ull;
        a.iscanned[3 * i + 2] = 0ull;
        if (a.idead) {
          a.idead[2 * i] = 0ull;
          a.idead[2 * i + 1] = 0ull;
        }
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
    c->front_ctr[1] = ((unsigned long long)I << 32) | (run & 0xffffffffull);
    c->front_ctr[0] = 0ull;
    c->open_ctr[0] = 0ull;
    c->open_ctr[1] = 0ull;
    c->go = 0u;
    c->go_a = 0u;
    c->status = 0;
    c->rounds = 0;
    c->deg_count = 0;
    c->settled = c->relaxed = c->scanned = c->open_visits = 0;
    c->solo_phases = 0;
    c->live_ctr[0] = c->live_ctr[1] = 0ull;
    c->dead_deg = c->dead_deg_r = 0ull;
  }
}

// ------------------------------------------------------- host launchers
hipError_t launch_kernel(Launcher &L, const void *fn, dim3 grid, dim3 block, void **args,
                         bool cooperative) {
  if (!L.graph) {
    return cooperative ? hipLaunchCooperativeKernel(fn, grid, block, args, 0, L.stream)
                       : hipLaunchKernel(fn, grid, block, args, 0, L.stream);
  }
  hipKernelNodeParams p;
  memset(&p, 0, sizeof(p));
  p.func = const_cast<void *>(fn);
  p.gridDim = grid;
  p.blockDim = block;
  p.kernelParams = args;
  hipGraphNode_t node;
  hipError_t e = hipGraphAddKernelNode(&node, L.graph, L.last ? &L.last : nullptr,
                                       L.last ? 1 : 0, &p);
  if (e != hipSuccess) return e;
  if (cooperative) {
    hipKernelNodeAttrValue v;
    memset(&v, 0, sizeof(v));
    v.cooperative = 1;
    if ((e = hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v)) !=
        hipSuccess)
      return e;
  }
  L.last = node;
  return hipSuccess;
}

template <class V, bool BATCH>
static hipError_t launch_solve_t(const RoundArgs &a, int32_t *pred, const LaunchGeom &geo,
                                 long long *istat, int32_t max_n, const KernelTimer *timer,
                                 Launcher &L) {
  hipError_t e;
  if (geo.blocks > kMaxBlocks) return hipErrorInvalidConfiguration;
  if (!BATCH && a.total <= geo.small_n) return launch_small(V::INF == KeyF32::INF, a, pred, timer, L);
  if (geo.wg && !a.scope_all)
    return launch_wg(V::INF == KeyF32::INF, BATCH, a, pred, geo, istat, max_n, timer, L);
  RoundArgs arg = a;
  void *params[] = {&arg};
  {
    int blocks = (int)((a.total + 255) / 256);
    if (blocks < (kParts * kMaxBlocks) / 256) blocks = (kParts * kMaxBlocks) / 256;
    if (blocks > 4096) blocks = 4096;
    if ((e = launch_kernel(L, (const void *)init_fill_kernel<V>, dim3(blocks), dim3(256), params,
                           false)) != hipSuccess)
      return e;
    if ((e = launch_kernel(L, (const void *)init_seed_kernel<V, BATCH>, dim3(1), dim3(RBS),
                           params, false)) != hipSuccess)
      return e;
    if (BATCH && a.inst_of) {
      const int nbk = a.num_inst < 1024 ? a.num_inst : 1024;
      if ((e = launch_kernel(L, (const void *)inst_of_kernel, dim3(nbk), dim3(256), params,
                             false)) != hipSuccess)
        return e;
    }
  }
  if (L.graph) timer = nullptr;
  if (timer && (e = hipEventRecord(timer->start, L.stream)) != hipSuccess) return e;
  if ((e = launch_kernel(L, (const void *)rounds_kernel<V, BATCH>, dim3(geo.blocks), dim3(RBS),
                         params, true)) != hipSuccess)
    return e;
  if (timer && (e = hipEventRecord(timer->stop, L.stream)) != hipSuccess) return e;
  // the emit pass writes the costs (and parents) out of the keys
  return launch_pred(V::INF == KeyF32::INF, BATCH, a, pred, geo, istat, max_n, L);
}

hipError_t launch_solve(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                        const LaunchGeom &geo, long long *istat, int32_t max_n,
                        const KernelTimer *timer, Launcher &L) {
  if (f32) {
    return batch ? launch_solve_t<KeyF32, true>(a, pred, geo, istat, max_n, timer, L)
                 : launch_solve_t<KeyF32, false>(a, pred, geo, istat, max_n, timer, L);
  }
  return batch ? launch_solve_t<KeyI32, true>(a, pred, geo, istat, max_n, timer, L)
               : launch_solve_t<KeyI32, false>(a, pred, geo, istat, max_n, timer, L);
}

// ------------------------------------------------ static scratch region
// The state of an allocation-free solve (sssp_solve_noalloc) lives here:
// one region per device, part of this code object, held until the process
// ends.  In host code the array's name stands for no device address; the
// address comes from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void **ptr) {
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t round_kernel_occupancy(bool f32, bool batch, int *blocks_per_cu) {
  const void *k = f32 ? (batch ? (const void *)rounds_kernel<KeyF32, true>
                               : (const void *)rounds_kernel<KeyF32, false>)
                      : (batch ? (const void *)rounds_kernel<KeyI32, true>
                               : (const void *)rounds_kernel<KeyI32, false>);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, RBS, 0);
}

}  // namespace sssp
