// The rounds of each solve in one workgroup: instance i of a launch runs on
// block i (blocks loop over the instances when there are more), with its
// state in global memory (the (D, parent) keys, both C buffers, the relax
// set, the open lists by parity with their payload) and block barriers
// only: no grid barrier, no hand-over, and no instance waits for another.
// For graphs of low degree spread under C scope OPEN (meshes, grids), whose
// rounds are many and small; the rounds, counters and keys are those of the
// persistent kernel (Section VI's rounds in the adopted order: relax, minD
// and the threshold, the lower bounds of Eq. 1, fix).
#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

constexpr int WBS = 1024;  // threads of the workgroup
static_assert(WBS == 1024, "the relax window search covers 1024 items");
constexpr int kWgItems = 2;  // open-list entries per thread and pass of the bound step
// relax items kept in LDS (x, D to relax from, out-offset, out-degree); the
// rest of a longer relax set lives in the global arrays
constexpr int kRelLds = 2048;

struct WgLds {
  int32_t pfx[WBS + 1];  // out-degree prefix of a window of relax items
  int32_t wbase[WBS];    // out-list start of a window item
  int32_t wdx[WBS];      // its relax D
  uint64_t scan[WBS / SSSP_WAVE + 1];
  int32_t red[2 * (WBS / SSSP_WAVE)];
  int32_t nF, nF2, nO, nO2, target_hit;
  unsigned long long relaxed, scanned, visits, settled;
  int4 rel[kRelLds];  // relax items [0, kRelLds): written by the fix step, read by the relax
};

// The open entries' payload by list parity, as two int4 arrays of
// a.total entries each (in the open-list payload words, kOXMem per entry):
// the vertex record's two halves, with C in the last word (where the
// record holds 0).
__device__ __forceinline__ int4 *wg_payload(const RoundArgs &a, int parity, int32_t sb) {
  return (int4 *)(parity ? a.open_x1[0] : a.open_x0[0]) + sb;
}

// Relax item q of the next round: in LDS when it fits, else in the global
// arrays.
__device__ __forceinline__ void push_rel(WgLds &s, int32_t *F, int32_t *FD, int32_t *FO,
                                         int32_t *FG, int q, int32_t x, int32_t fd, int32_t fo,
                                         int32_t fg) {
  if (q < kRelLds) {
    s.rel[q] = make_int4(x, fd, fo, fg);
  } else {
    F[q] = x;
    FD[q] = fd;
    FO[q] = fo;
    FG[q] = fg;
  }
}

template <class V, bool BATCH>
__global__ __launch_bounds__(WBS) void wg_rounds_kernel(RoundArgs a) {
  __shared__ WgLds s;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) {
    // the control block the emit pass and the host read
    Ctl *c = a.ctl;
    c->front_ctr[0] = c->front_ctr[1] = 0ull;
    c->open_ctr[0] = c->open_ctr[1] = 0ull;
    c->live_ctr[0] = c->live_ctr[1] = 0ull;
    c->go = c->go_a = 0u;
    c->deg_count = 0;
    c->solo_phases = 0;
    c->dead_deg = c->dead_deg_r = 0ull;
    c->status = 0;
  }
  for (int inst = blockIdx.x; inst < a.num_inst; inst += gridDim.x) {
    int32_t sb = 0, gi = 0, src = a.source, n = a.g.n;
    if constexpr (BATCH) {
      const InstDev id = a.insts[inst];
      sb = id.sbase;
      gi = id.graph;
      src = id.source;
      n = id.n;
    }
    // by value: the fields stay in registers rather than being reloaded
    // from the graph table after every store
    const GraphDev G = graph_of<BATCH>(a, gi);
    const bool lc = G.lc != 0;
    int32_t tgt = BATCH ? -1 : a.target;
    if (G.rank) {
      src = G.rank[src];
      if (tgt >= 0) tgt = G.rank[tgt];
    }
    // D is updated by atomics (performed in L2): its reads after a barrier
    // bypass the CU's L1 (agent-scope loads); the other arrays are written
    // and read by plain accesses of this workgroup only
    unsigned long long *D = a.D64 + sb;
    int32_t *C[2] = {a.C0 + sb, a.C1 + sb};
    // relax items beyond the first kRelLds (those stay in LDS): vertex, D
    // to relax from, out-offset, out-degree
    int32_t *F = a.front_v + sb, *FD = a.front_x[FX_D] + sb;
    int32_t *FO = a.front_x[FX_OOFF] + sb, *FG = a.front_p + sb;
    // open entries by parity: the vertex, its payload (wg_payload) and the
    // D it was last relaxed with (INF before its first relax): everything
    // its bound step reads but D and the tails' C, loaded coalesced rather
    // than gathered
    int32_t *O[2] = {a.open_v0 + sb, a.open_v1 + sb};
    int32_t *OR[2] = {a.open_p0 + sb, a.open_p1 + sb};
    for (int y = tid; y < n; y += WBS) {
      const bool is_s = y == src;
      D[y] = make_key(is_s ? 0 : V::INF, -1, false);
      C[0][y] = C[1][y] = is_s ? V::INF : 0;  // the source is fixed from the start
    }
    if (tid == 0) {
      const int32_t o0 = G.out_off[src];
      s.rel[0] = make_int4(src, 0, o0, G.out_off[src + 1] - o0);
      s.nF = 1;
      s.nO = 0;
      s.target_hit = (tgt >= 0 && tgt == src) ? 1 : 0;
      s.relaxed = s.scanned = s.visits = 0ull;
      s.settled = 1ull;  // the source
    }
    __syncthreads();
    // minD / thr offers of this thread's survivors of the last fix step:
    // with the relax's successful candidates they cover every open vertex's
    // current D (a survivor whose D fell offered the lower value as a
    // candidate), so no pass over the open list is needed for them
    int32_t smd = V::INF, sth = V::INF;
    int r = 0, o = 0, status = 0;  // o: the open list being built this round
    for (;;) {
      if (tgt >= 0 && s.target_hit) break;  // the frontier that fixed it is not relaxed
      ++r;
      if (r > n + 1 || r > a.max_rounds) {
        status = 7;
        break;
      }
      const int cur = r & 1;  // the bound step reads C[cur] and writes C[cur ^ 1]
      const int32_t *Cold = C[cur];
      int32_t *Cnew = C[cur ^ 1];
      // (A) relax the relax set's out-edges, each from its D at the start of
      // the step; first discoveries join the open list.  Relax items:
      // FD = the D to relax from (bit 31 set: an open vertex, label-
      // correcting), or INF: a vertex fixed at a D it was already relaxed
      // with (no edges).  A fixed item also marks its C in the buffer this
      // round writes (the other buffer has it since the fix).
      const int nF = s.nF;
      const int nS = s.nO;  // the open entries with a payload: last round's survivors
      unsigned long long nrel = 0;
      int32_t md = smd, th = sth;
      for (int i0 = 0; i0 < nF; i0 += WBS) {
        const int i = i0 + tid;
        int32_t deg = 0;
        if (i < nF) {
          // (x, relax D, out-offset, out-degree), from LDS for the first
          // kRelLds items
          const int4 f = i < kRelLds ? s.rel[i] : make_int4(F[i], FD[i], 0, 0);
          const int32_t x = f.x;
          const int32_t fd = f.y;
          const int32_t dx = fd & 0x7fffffff;
          if (fd >= 0) Cnew[x] = V::INF;
          if (dx != V::INF) {
            deg = i < kRelLds ? f.w : FG[i];
            s.wbase[tid] = i < kRelLds ? f.z : FO[i];
            s.wdx[tid] = dx;
          }
        }
        uint64_t tot;
        s.pfx[tid] = (int32_t)block_excl_scan64<WBS>((uint64_t)deg, s.scan, &tot);
        __syncthreads();
        const int ET = (int)tot;
        nrel += (unsigned long long)ET;
        for (int e = tid; e < ET; e += WBS) {
          // the last window item with pfx <= e (an 8-ary search: four LDS steps)
          const int lo = search1024(s.pfx, (uint32_t)e);
          const int32_t pos = s.wbase[lo] + (e - s.pfx[lo]);
          const int4 er = G.out_rec[pos];  // head, weight, edge id, the head's out_wmin
          const int32_t y = er.x;
          const int32_t w = er.y;
          const int32_t eid = er.z;
          const int32_t dx = s.wdx[lo];
          const int32_t cand = V::add(dx, w);
          // one workgroup: little contention, so straight to the atomic
          const unsigned long long old = atomicMin(&D[y], make_key(cand, eid, cand == dx));
          const int32_t od = (int32_t)(old >> 32);
          if (cand < od) {  // D[y] fell: offer it to minD and thr
            md = kmin(md, cand);
            th = kmin(th, V::add(cand, er.w));
          }
          // a first discovery joins the open list after the survivors, with
          // no payload: its bound step reads the vertex record
          if (od == V::INF) O[o][atomicAdd(&s.nO, 1)] = y;
        }
        __syncthreads();
      }
      const int nO = s.nO;
      if (tid == 0) s.relaxed += nrel;
      if (nO == 0) break;  // (A) left nothing open
      // (B) minD and the threshold over the open list
      block_min2<WBS>(md, th, s.red);
      if (tid == 0) {
        s.nF2 = 0;
        s.nO2 = 0;
      }
      __syncthreads();
      // (C) lower bounds (Eq. 1), Jacobi: read C[cur], write C[cur ^ 1];
      // then (D) for the same vertex: it only needs the vertex's own C'.
      // In-lists are ascending by weight and every term max(C[v], minD) + w
      // is at least minD + w, so a scan stops at the first edge with
      // minD + w >= min(D[y], m_y); the counters take whole in-degrees.
      // Fixed vertices get C = INF (C[cur] at the next relax); the next
      // relax set is the newly fixed vertices (label-correcting: those and,
      // within the first bucket above minD, the survivors whose D fell since
      // their last relax; a fixed one at a D it was relaxed with comes with
      // no edges, to mark its C)
      unsigned long long nscan = 0, nfix = 0;
      smd = sth = V::INF;
      // Each thread takes kWgItems list entries per pass and issues the
      // loads of all of them before any decision: the entries with their
      // payload (coalesced), then D and the lightest tail's C together
      // (lanes past the list read entry 0), then the rest of the in-list.
      // First discoveries (the list's tail, from nS on) have no payload yet:
      // a wave that holds one reads their vertex records beside D (the
      // record's last word is 0, the C of an undiscovered vertex; never
      // relaxed), and the tails' C after.
      const int4 *Pc = wg_payload(a, o, sb), *Qc = Pc + a.total;
      int4 *Pn = wg_payload(a, o ^ 1, sb), *Qn = Pn + a.total;
      static_assert(kWgItems == 2, "slot 1 of a pass is the optional one");
      for (int i0 = 0; i0 < nO; i0 += kWgItems * WBS) {
        // (wave-uniform) a wave past the list's end sits the pass out, and
        // one whose second slot is past it issues no loads for that slot
        const int wb = i0 + (tid & ~(SSSP_WAVE - 1));
        if (wb >= nO) continue;
        const bool two = wb + WBS < nO;
        int32_t y[kWgItems] = {0, 0}, dy[kWgItems], dr[kWgItems] = {0, 0}, c0[kWgItems] = {0, 0};
        int4 ra[kWgItems] = {}, rb[kWgItems] = {};  // out_off, out_deg, in_off, in_deg; out_wmin, tail0, w0, C
        unsigned long long dk[kWgItems] = {0, 0};
        bool ok[kWgItems];
#pragma unroll
        for (int u = 0; u < kWgItems; ++u) ok[u] = i0 + u * WBS + tid < nO;
#pragma unroll
        for (int u = 0; u < kWgItems; ++u) {
          if (u == 0 || two) {
            const int i = i0 + u * WBS + tid;
            const int ic = ok[u] ? i : 0;
            const int ip = i < nS ? i : 0;  // (first discoveries: one line for all)
            y[u] = O[o][ic];
            ra[u] = Pc[ip];
            rb[u] = Qc[ip];
            dr[u] = OR[o][ip];
          }
        }
        bool fdw = false;
#pragma unroll
        for (int u = 0; u < kWgItems; ++u) fdw |= ok[u] && i0 + u * WBS + tid >= nS;
        // (the empty asm statements mark the loaded values as used there:
        // every load of a step issues before the wave waits for any)
        if (__ballot(fdw) == 0ull) {
#pragma unroll
          for (int u = 0; u < kWgItems; ++u) {
            if (u == 0 || two) {
              dk[u] = ld_relaxed64(&D[y[u]]);
              // (0 for a vertex with no in-edge; lanes past the list read
              // entry 0, whose payload is unset when it is a first discovery)
              c0[u] = Cold[ok[u] ? rb[u].y : 0];
            }
          }
#pragma unroll
          for (int u = 0; u < kWgItems; ++u) asm volatile("" : "+v"(dk[u]), "+v"(c0[u]));
        } else {
          int4 va[kWgItems] = {}, vb[kWgItems] = {};
#pragma unroll
          for (int u = 0; u < kWgItems; ++u) {
            if (u == 0 || two) {
              dk[u] = ld_relaxed64(&D[y[u]]);
              va[u] = G.vrec[2 * y[u]];
              vb[u] = G.vrec[2 * y[u] + 1];
            }
          }
#pragma unroll
          for (int u = 0; u < kWgItems; ++u)
            asm volatile("" : "+v"(dk[u]), "+v"(va[u].x), "+v"(va[u].y), "+v"(va[u].z),
                         "+v"(va[u].w), "+v"(vb[u].x), "+v"(vb[u].y), "+v"(vb[u].z));
#pragma unroll
          for (int u = 0; u < kWgItems; ++u) {
            if (i0 + u * WBS + tid >= nS) {
              ra[u] = va[u];
              rb[u] = vb[u];
              dr[u] = V::INF;
            }
          }
#pragma unroll
          for (int u = 0; u < kWgItems; ++u)
            if (u == 0 || two) c0[u] = Cold[rb[u].y];
#pragma unroll
          for (int u = 0; u < kWgItems; ++u) asm volatile("" : "+v"(c0[u]));
        }
#pragma unroll
        for (int u = 0; u < kWgItems; ++u) dy[u] = (int32_t)(dk[u] >> 32);
#pragma unroll
        for (int u = 0; u < kWgItems; ++u) {
          if (!ok[u]) continue;
          const int32_t ioff = ra[u].z, ideg = ra[u].w, w0 = rb[u].z;
          int32_t m = V::INF;
          if (ideg > 0 && V::add(md, w0) < dy[u]) {
            if (c0[u] != V::INF) m = V::add(kmax(c0[u], md), w0);
            for (int32_t j = 1; j < ideg; ++j) {  // the rest from the in-list
              const int2 e = G.in_sw[ioff + j];  // tail, weight
              const int32_t w = e.y;
              if (V::add(md, w) >= kmin(dy[u], m)) break;
              const int32_t cv = Cold[e.x];
              if (cv != V::INF) m = kmin(m, V::add(kmax(cv, md), w));
            }
          }
          const int32_t cn = kmax(kmax(rb[u].w, md), kmin(dy[u], m));
          nscan += (unsigned long long)ideg;
          const bool relax_again = !lc || dy[u] < dr[u];
          if (cn >= dy[u] || dy[u] <= th) {
            Cnew[y[u]] = V::INF;
            ++nfix;
            if (y[u] == tgt) s.target_hit = 1;
            const int q = atomicAdd(&s.nF2, 1);
            push_rel(s, F, FD, FO, FG, q, y[u], relax_again ? dy[u] : V::INF, ra[u].x, ra[u].y);
          } else {
            Cnew[y[u]] = cn;
            // label-correcting: relaxed again from its lower D (while in the
            // first bucket above minD)
            const bool again = lc && relax_again && dy[u] < V::add(md, G.delta);
            const int q = atomicAdd(&s.nO2, 1);
            O[o ^ 1][q] = y[u];
            rb[u].w = cn;
            Pn[q] = ra[u];
            Qn[q] = rb[u];
            OR[o ^ 1][q] = again ? dy[u] : dr[u];
            smd = kmin(smd, dy[u]);
            sth = kmin(sth, V::add(dy[u], rb[u].x));
            if (again) {
              const int p = atomicAdd(&s.nF2, 1);
              push_rel(s, F, FD, FO, FG, p, y[u], dy[u] | kOpenRelax, ra[u].x, ra[u].y);
            }
          }
        }
      }
      const long long f = wave_sum64((long long)nfix), sc = wave_sum64((long long)nscan);
      if (lane_id() == 0) {
        if (f) atomicAdd(&s.settled, (unsigned long long)f);
        if (sc) atomicAdd(&s.scanned, (unsigned long long)sc);
      }
      __syncthreads();
      if (tid == 0) {
        s.visits += (unsigned long long)nO;
        s.nF = s.nF2;
        s.nO = s.nO2;
      }
      o ^= 1;
      __syncthreads();
    }
    if (tid == 0) {
      if constexpr (BATCH) {
        a.irounds[inst] = r;
        a.iscanned[3 * inst] = s.scanned;
        a.iscanned[3 * inst + 1] = s.visits;
        a.iscanned[3 * inst + 2] = s.relaxed;
        if (a.istat) {  // the emit pass adds the reachable count (= settled)
          a.istat[4 * inst + 0] = 0;
          a.istat[4 * inst + 1] = 0;
          a.istat[4 * inst + 2] = 0;
          a.istat[4 * inst + 3] = 0;
        }
        if (status) atomicMax(&a.ctl->status, status);
      } else {
        Ctl *c = a.ctl;
        c->rounds = r;
        c->status = status;
        c->settled = (long long)s.settled;
        c->relaxed = (long long)s.relaxed;
        c->scanned = (long long)s.scanned;
        c->open_visits = (long long)s.visits;
        c->target_id = tgt;
        c->target_hit = s.target_hit;
      }
    }
    __syncthreads();  // the next instance reuses the LDS
  }
}

template <class V, bool BATCH>
static hipError_t launch_wg_t(const RoundArgs &a, int32_t *pred, const LaunchGeom &geo,
                              long long *istat, int32_t max_n, const KernelTimer *timer,
                              Launcher &L) {
  hipError_t e;
  if (a.scope_all) return hipErrorInvalidValue;  // the live pass is not here
  RoundArgs arg = a;
  void *params[] = {&arg};
  int blocks = a.num_inst < geo.blocks ? a.num_inst : geo.blocks;
  if (blocks < 1) blocks = 1;
  if (L.graph) timer = nullptr;
  if (timer && (e = hipEventRecord(timer->start, L.stream)) != hipSuccess) return e;
  if ((e = launch_kernel(L, (const void *)wg_rounds_kernel<V, BATCH>, dim3(blocks), dim3(WBS),
                         params, false)) != hipSuccess)
    return e;
  if (timer && (e = hipEventRecord(timer->stop, L.stream)) != hipSuccess) return e;
  return launch_pred(V::INF == KeyF32::INF, BATCH, a, pred, geo, istat, max_n, L);
}

hipError_t launch_wg(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                     const LaunchGeom &geo, long long *istat, int32_t max_n,
                     const KernelTimer *timer, Launcher &L) {
  if (f32)
    return batch ? launch_wg_t<KeyF32, true>(a, pred, geo, istat, max_n, timer, L)
                 : launch_wg_t<KeyF32, false>(a, pred, geo, istat, max_n, timer, L);
  return batch ? launch_wg_t<KeyI32, true>(a, pred, geo, istat, max_n, timer, L)
               : launch_wg_t<KeyI32, false>(a, pred, geo, istat, max_n, timer, L);
}

}  // namespace sssp
