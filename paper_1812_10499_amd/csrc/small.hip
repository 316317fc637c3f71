// The rounds of a single solve on a small graph (n <= kSmallN) in one
// workgroup, with the whole per-vertex state in LDS: the (D, parent) keys,
// both C buffers, the relax set, the open lists and the last-relaxed D of
// label-correcting relax.  Only the graph arrays are read from global memory
// (through this CU's L2).  The phases are separated by block barriers alone,
// so a round costs a few microseconds instead of the grid barriers and
// hand-overs of the persistent kernel; results and counters are the same
// round for round (Section VI's rounds in the adopted order: relax, minD and
// the threshold, the lower bounds of Eq. 1, fix).  The keys are written back
// to global memory at the end for the emit pass.
#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

constexpr int SBS = 1024;  // threads of the workgroup
static_assert(SBS == 1024, "the relax window search covers 1024 items");
constexpr int kSlots = kSmallN / SBS;     // vertices per thread: y = tid + k * SBS
static_assert(kSlots * SBS == kSmallN, "whole slots");

// The open set O is implicit: y is open iff it is discovered (D < INF) and
// not fixed (C < INF; fixed vertices carry C = INF in both buffers, and a
// discovered vertex never has C = INF otherwise, as C <= D).
struct SmallLds {
  unsigned long long D[kSmallN];  // (D << 32) | equal-cost flag << 31 | edge id
  int32_t C[2][kSmallN];          // lower bounds by round parity (INF: fixed)
  int32_t F[kSmallN];             // relax set: vertex ...
  int32_t FD[kSmallN];            // ... and the D it is relaxed with
  int32_t DR[kSmallN];            // label-correcting: D of the last relax (INF: never)
  int32_t pfx[SBS + 1];           // out-degree prefix of a window of relax items
  int32_t wbase[SBS];             // out-list start of a window item
  int32_t wdx[SBS];               // its relax D
  uint64_t scan[SBS / SSSP_WAVE + 1];
  int32_t red[2 * (SBS / SSSP_WAVE)];
  int32_t nF, nF2, nO, target_hit;
  unsigned long long relaxed, scanned, visits, settled;
};

// m_y of Eq. 1 over y's weight-ordered in-list (first edge from registers):
// the scan stops at the first edge with minD + w >= lim, as every later term
// max(C[v], minD) + w is at least minD + w.
template <class V>
__device__ __forceinline__ int32_t small_m(const GraphDev &G, const int32_t *Cold, int32_t b,
                                           int32_t deg, int32_t s0, int32_t w0, int32_t md,
                                           int32_t lim) {
  int32_t m = V::INF;
  if (deg == 0 || V::add(md, w0) >= lim) return m;
  {
    const int32_t cv = Cold[s0];
    if (cv != V::INF) m = V::add(kmax(cv, md), w0);
  }
  for (int32_t j = 1; j < deg; ++j) {
    const int2 e = G.in_sw[b + j];  // tail, weight
    const int32_t w = e.y;
    if (V::add(md, w) >= kmin(lim, m)) break;
    const int32_t cv = Cold[e.x];
    if (cv != V::INF) m = kmin(m, V::add(kmax(cv, md), w));
  }
  return m;
}

template <class V>
__global__ __launch_bounds__(SBS) void small_rounds_kernel(RoundArgs a) {
  __shared__ SmallLds s;
  const int tid = threadIdx.x;
  const GraphDev &G = a.g;
  const int n = G.n;
  const bool lc = G.lc != 0, all = a.scope_all != 0;
  Ctl *ctl = a.ctl;
  int32_t src = a.source, tgt = a.target;
  if (G.rank) {
    src = G.rank[src];
    if (tgt >= 0) tgt = G.rank[tgt];
  }
  // this thread's vertices: in-list offset and length, lightest in-edge, out_wmin
  int32_t ib[kSlots], id[kSlots], s0[kSlots], w0[kSlots], owm[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const int y = tid + k * SBS;
    ib[k] = id[k] = s0[k] = 0;
    w0[k] = owm[k] = V::INF;
    if (y < n) {
      const int4 rec = G.vrec[2 * y];  // out_off, out_degree, in_off, in_degree
      ib[k] = rec.z;
      id[k] = rec.w;
      owm[k] = G.vrec[2 * y + 1].x;
      if (rec.w > 0) {
        s0[k] = G.in_src[rec.z];
        w0[k] = G.in_w[rec.z];
      }
      const bool is_s = y == src;
      s.D[y] = make_key(is_s ? 0 : V::INF, -1, false);
      s.C[0][y] = s.C[1][y] = is_s ? V::INF : 0;  // the source is fixed from the start
      s.DR[y] = V::INF;
    }
  }
  if (tid == 0) {
    s.F[0] = src;
    s.FD[0] = 0;
    s.nF = 1;
    s.nO = 0;
    s.target_hit = (tgt >= 0 && tgt == src) ? 1 : 0;
    s.relaxed = s.scanned = s.visits = 0ull;
    s.settled = 1ull;  // the source
  }
  __syncthreads();
  int r = 0, status = 0;
  for (;;) {
    if (tgt >= 0 && s.target_hit) break;  // the frontier that fixed it is not relaxed
    ++r;
    if (r > a.max_rounds) {
      status = 7;
      break;
    }
    const int cur = r & 1;  // the bound step reads C[cur] and writes C[cur ^ 1]
    // (A) relax the relax set's out-edges, each from its D at the start of
    // the step (first discoveries join O by getting a finite D)
    const int nF = s.nF;
    unsigned long long nrel = 0;
    for (int i0 = 0; i0 < nF; i0 += SBS) {
      const int i = i0 + tid;
      int32_t deg = 0;
      if (i < nF) {
        const int32_t x = s.F[i];
        const int32_t b = G.out_off[x];
        deg = G.out_off[x + 1] - b;
        s.wbase[tid] = b;
        s.wdx[tid] = s.FD[i];
        if (lc) s.DR[x] = s.FD[i];
      }
      uint64_t tot;
      s.pfx[tid] = (int32_t)block_excl_scan64<SBS>((uint64_t)deg, s.scan, &tot);
      __syncthreads();
      const int ET = (int)tot;
      nrel += (unsigned long long)ET;
      for (int e = tid; e < ET; e += SBS) {
        // the last window item with pfx <= e (an 8-ary search: four LDS steps)
        const int lo = search1024(s.pfx, (uint32_t)e);
        const int32_t pos = s.wbase[lo] + (e - s.pfx[lo]);
        const int4 er = G.out_rec[pos];  // head, weight, edge id, the head's out_wmin
        const int32_t y = er.x;
        const int32_t w = er.y;
        const int32_t eid = er.z;
        const int32_t dx = s.wdx[lo];
        const int32_t cand = V::add(dx, w);
        atomicMin(&s.D[y], make_key(cand, eid, cand == dx));
      }
      __syncthreads();
    }
    const int32_t *Cold = s.C[cur];
    int32_t *Cnew = s.C[cur ^ 1];
    // (B) minD and the threshold over O, and |O|
    int32_t md = V::INF, th = V::INF;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const int y = tid + k * SBS;
      if (y < n) {
        const int32_t dy = (int32_t)(s.D[y] >> 32);
        if (dy != V::INF && Cold[y] != V::INF) {
          md = kmin(md, dy);
          th = kmin(th, V::add(dy, owm[k]));
          ++cnt;
        }
      }
    }
    {
      const long long c = wave_sum64((long long)cnt);
      if (lane_id() == 0 && c) atomicAdd(&s.nO, (int32_t)c);
    }
    block_min2<SBS>(md, th, s.red);  // its barriers also publish nO
    const int nO = s.nO;
    if (tid == 0) s.relaxed += nrel;
    if (nO == 0) break;  // (A) left nothing open
    // (C) lower bounds (Eq. 1), Jacobi over C[cur]; SP_4's scope also
    // raises C of undiscovered vertices (an unreachable one, C = INF, keeps
    // it).  The counters take whole in-degrees.
    unsigned long long nscan = 0;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const int y = tid + k * SBS;
      if (y < n) {
        const int32_t dy = (int32_t)(s.D[y] >> 32);
        const int32_t c = Cold[y];
        const bool open = dy != V::INF && c != V::INF;
        const bool undiscovered = dy == V::INF && all;
        if (open || undiscovered) {
          // m_y matters below min(D[y], m_y); D = INF for undiscovered ones
          const int32_t m = c == V::INF ? V::INF
                                        : small_m<V>(G, Cold, ib[k], id[k], s0[k], w0[k], md, dy);
          Cnew[y] = kmax(kmax(c, md), kmin(dy, m));
          nscan += (unsigned long long)id[k];
        }
      }
    }
    if (tid == 0) s.nF2 = 0;
    __syncthreads();
    // (D) fix: C' >= D or D <= thr.  Fixed vertices get C = INF in both
    // buffers; the next relax set is the newly fixed vertices (label-
    // correcting: those and the survivors whose D fell since their last
    // relax, the fixed ones only if it fell)
    unsigned long long nfix = 0;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const int y = tid + k * SBS;
      if (y < n) {
        const int32_t dy = (int32_t)(s.D[y] >> 32);
        if (dy != V::INF && Cold[y] != V::INF) {
          const int32_t cn = Cnew[y];
          const bool relax_again = !lc || dy < s.DR[y];
          const bool fix = cn >= dy || dy <= th;
          if (fix) {
            s.C[0][y] = s.C[1][y] = V::INF;
            ++nfix;
            if (y == tgt) s.target_hit = 1;
          }
          // an open vertex only while in the first bucket above minD
          if (relax_again && (fix || (lc && dy < V::add(md, G.delta)))) {
            const int q = atomicAdd(&s.nF2, 1);
            s.F[q] = y;
            s.FD[q] = dy;
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
      s.nO = 0;
    }
    __syncthreads();
  }
  __syncthreads();
  // the keys for the emit pass, and the control block it and the host read
  for (int y = tid; y < n; y += SBS) a.D64[y] = s.D[y];
  if (tid == 0) {
    ctl->front_ctr[0] = ctl->front_ctr[1] = 0ull;
    ctl->open_ctr[0] = ctl->open_ctr[1] = 0ull;
    ctl->live_ctr[0] = ctl->live_ctr[1] = 0ull;
    ctl->go = ctl->go_a = 0u;
    ctl->deg_count = 0;
    ctl->solo_phases = 0;
    ctl->dead_deg = ctl->dead_deg_r = 0ull;
    ctl->rounds = r;
    ctl->status = status;
    ctl->settled = (long long)s.settled;
    ctl->relaxed = (long long)s.relaxed;
    ctl->scanned = (long long)s.scanned;
    ctl->open_visits = (long long)s.visits;
    ctl->target_id = tgt;
    ctl->target_hit = s.target_hit;
  }
}

template <class V>
static hipError_t launch_small_t(const RoundArgs &a, int32_t *pred, const KernelTimer *timer,
                                 Launcher &L) {
  hipError_t e;
  if (a.total > kSmallN || a.num_inst != 1) return hipErrorInvalidValue;
  RoundArgs arg = a;
  void *params[] = {&arg};
  if (L.graph) timer = nullptr;
  if (timer && (e = hipEventRecord(timer->start, L.stream)) != hipSuccess) return e;
  if ((e = launch_kernel(L, (const void *)small_rounds_kernel<V>, dim3(1), dim3(SBS), params,
                         false)) != hipSuccess)
    return e;
  if (timer && (e = hipEventRecord(timer->stop, L.stream)) != hipSuccess) return e;
  LaunchGeom geo = {1, 1};
  return launch_pred(V::INF == KeyF32::INF, false, a, pred, geo, nullptr, a.total, L);
}

hipError_t launch_small(bool f32, const RoundArgs &a, int32_t *pred, const KernelTimer *timer,
                        Launcher &L) {
  return f32 ? launch_small_t<KeyF32>(a, pred, timer, L)
             : launch_small_t<KeyI32>(a, pred, timer, L);
}

}  // namespace sssp
