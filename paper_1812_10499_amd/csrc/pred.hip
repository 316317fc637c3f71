// Emit pass of a solve (single or batched): costs and parent pointers from
// the 64-bit (D, parent) keys the relax phase leaves behind, and the
// equal-cost level pass for float32 ties.  Runs after the persistent round
// kernel on the same stream.
//
// Parent rule (parent pointers, Section I): pred[y] is the smallest edge id
// among tight in-edges (v, y, w), D[v] + w == D[y], with D[v] < D[y].  The
// key's atomicMin already selected it: every in-edge of a reachable vertex
// was offered exactly once, from a tail with its final cost, with the
// equal-cost flag set when D[v] + w == D[v].  If the minimum key carries the
// flag, y has no strict tight in-edge (only float32 edges below half an ulp
// of the cost reach it at equal cost); such vertices get the level rule:
// level 0 holds the source and every vertex with a strict tight in-edge, a
// queued y gets level(y) = 1 + min level over equal-cost tight tails, and
// pred[y] = the smallest such edge id with level(v) = level(y) - 1.
#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

// Fault flag of this device: the emit pass of any solve whose rounds tripped
// the watchdog (or whose level rule left a vertex without a parent) sets it;
// fault_flag_take reads and clears it.  One word per device, in the code
// object's own memory, so plan replays set it too.
__device__ int32_t g_fault_flag;

template <class V, bool BATCH>
__global__ __launch_bounds__(256) void emit_kernel(RoundArgs a, int32_t *pred, int32_t *degen,
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
  // one thread per caller id: the outputs are written in order and a
  // renumbered graph's keys are gathered through rank
  const int uy = blockIdx.x * blockDim.x + threadIdx.x;  // the caller's id
  long long c_settled = 0, c_relaxed = 0;
  if (uy == 0 && inst == 0 && ld_relaxed(&a.ctl->status) != 0) atomicOr(&g_fault_flag, 1);
  if (uy < n) {
    const int32_t y = G.rank ? G.rank[uy] : uy;  // solver id
    const unsigned long long k = a.D64[sb + y];
    const int32_t gy = sb + uy;
    const int32_t d = (int32_t)(k >> 32);
    a.D[gy] = d;
    if (d != V::INF) {
      c_settled = 1;
      c_relaxed = G.u_out_off[uy + 1] - G.u_out_off[uy];
    }
    if (pred) {
      int32_t p = -1;
      if (uy != s && d != V::INF) {
        if (k & kKeyEqualCost) {
          p = -2;
          const int q = atomicAdd(&a.ctl->deg_count, 1);
          degen[q] = gy;
          degen[a.total + q] = inst;
          lvl[gy] = -1;
        } else {
          p = (int32_t)(k & kKeyEidMask);
        }
      }
      pred[gy] = p;
    }
  }
  if (istat) {
    const long long s1 = wave_sum64(c_settled), s2 = wave_sum64(c_relaxed);
    if (lane_id() == 0 && (s1 | s2)) {
      atomicAdd((unsigned long long *)&istat[4 * inst + 1], (unsigned long long)s1);
      atomicAdd((unsigned long long *)&istat[4 * inst + 2], (unsigned long long)s2);
    }
  }
}

// Equal-cost tie pass (float32 only; one block; the queue is tiny in
// practice).
template <class V, bool BATCH>
__global__ __launch_bounds__(1024) void pred_degen_kernel(RoundArgs a, int32_t *pred,
                                                          const int32_t *degen, int32_t *lvl,
                                                          int32_t *flag) {
  const int nd = ld_relaxed(&a.ctl->deg_count);
  if (nd == 0) return;
  // every level adds at least one vertex or ends the loop, so it runs at
  // most nd + 1 times; the loop test is a block-wide vote, taken by every
  // thread at the same barrier
  for (int lv = 0;; ++lv) {
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
      for (int32_t j = G.u_in_off[y]; j < G.u_in_off[y + 1]; ++j) {
        const int32_t gv = sb + G.u_in_src[j];
        const int32_t dv = a.D[gv];
        if (dv == dy && V::add(dv, G.u_in_w[j]) == dy) {
          const int32_t lv_v = (pred[gv] == -2) ? lvl[gv] : 0;
          if (lv_v == lv) {
            flag[q] = 1;
            break;
          }
        }
      }
    }
    __syncthreads();
    int changed = 0;
    for (int q = threadIdx.x; q < nd; q += blockDim.x) {
      if (flag[q]) {
        lvl[degen[q]] = lv + 1;
        changed = 1;
      }
    }
    if (!__syncthreads_or(changed)) break;
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
      for (int32_t j = G.u_in_off[y]; j < G.u_in_off[y + 1]; ++j) {
        const int32_t gv = sb + G.u_in_src[j];
        const int32_t dv = a.D[gv];
        if (dv == dy && V::add(dv, G.u_in_w[j]) == dy) {
          const int32_t lv_v = (pred[gv] == -2) ? lvl[gv] : 0;
          if (lv_v == ly - 1) {
            best = G.u_in_eid[j];
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
    if (flag[q] < 0) {
      a.ctl->status = 7;
      atomicOr(&g_fault_flag, 1);
    }
  }
}

template <class V, bool BATCH>
static hipError_t launch_emit_t(const RoundArgs &a, int32_t *pred, long long *istat,
                                int32_t max_n, Launcher &L) {
  hipError_t e;
  RoundArgs arg = a;
  int32_t *p = pred, *degen = a.degen, *lvl = a.lvl, *flag = a.flag;
  long long *st = istat;
  const dim3 grid((max_n + 255) / 256, BATCH ? a.num_inst : 1);
  void *eargs[] = {&arg, &p, &degen, &lvl, &st};
  if ((e = launch_kernel(L, (const void *)emit_kernel<V, BATCH>, grid, dim3(256), eargs,
                         false)) != hipSuccess)
    return e;
  if (pred && V::INF == KeyF32::INF) {
    void *dargs[] = {&arg, &p, &degen, &lvl, &flag};
    if ((e = launch_kernel(L, (const void *)pred_degen_kernel<V, BATCH>, dim3(1), dim3(1024),
                           dargs, false)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

hipError_t fault_flag_take(int32_t *out, hipStream_t stream) {
  int32_t v = 0;
  hipError_t e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  if ((e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_fault_flag), sizeof(v))) != hipSuccess) return e;
  *out = v;
  if (v) {
    const int32_t zero = 0;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_fault_flag), &zero, sizeof(zero))) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

hipError_t launch_pred(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                       const LaunchGeom &geo, long long *istat, int32_t max_n, Launcher &L) {
  (void)geo;
  if (f32)
    return batch ? launch_emit_t<KeyF32, true>(a, pred, istat, max_n, L)
                 : launch_emit_t<KeyF32, false>(a, pred, istat, max_n, L);
  return batch ? launch_emit_t<KeyI32, true>(a, pred, istat, max_n, L)
               : launch_emit_t<KeyI32, false>(a, pred, istat, max_n, L);
}

}  // namespace sssp
