// Backward pass of the shortest-path costs with respect to edge weights.
//
// The source of an instance is the root of its tree whatever its pred entry
// says: it is never taken as a child, and no edge into it gets a gradient.
// Every other vertex has one parent entry, so a walk down from the root
// meets each vertex at most once (a vertex on a parent cycle that avoids the
// root is reachable from no vertex outside that cycle), and the level lists
// never hold more than the instance's n entries.
//
// With cost_i[x] the weight sum along the pred-tree path from instance i's
// source to x, L = sum_i sum_x g_i[x] * cost_i[x] has
//   dL/dw[e] = sum_i [e == pred_i[head(e)]] * acc_i[head(e)],
//   acc_i[y] = g_i[y] + sum over tree children c of y of acc_i[c].
// The tree's children of y are the heads of y's out-edges e with
// pred[head(e)] == e, so no child lists are built: a top-down pass records
// the tree level by level (persistent kernel, one grid barrier per level),
// and a bottom-up pass computes acc deepest level first, each vertex adding
// its children in edge-id order (or, for deep trees, each instance in a
// workgroup of its own).  A final edge-parallel kernel sums the instances of
// each graph in instance order.  Every sum has a fixed order,
// so the result is deterministic.
#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

constexpr int BBS = kBackBlock;

// acc = 0 everywhere, so a vertex whose parent entry names an edge from
// outside the tree contributes nothing
__global__ void bw_zero_kernel(BackArgs a) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < a.total;
       i += gridDim.x * blockDim.x)
    a.acc[i] = 0.0f;
}

__global__ void bw_init_kernel(BackArgs a) {
  for (int i = threadIdx.x; i < a.num_inst; i += blockDim.x) {
    const InstDev id = a.insts[i];
    a.lv_v[i] = id.sbase + id.source;
    a.lv_i[i] = i;
  }
  for (int b = threadIdx.x; b < kMaxBlocks; b += blockDim.x) a.flags[b * kFlagStride] = 0u;
  if (threadIdx.x == 0) {
    *a.go = 0u;
    *a.ctr = (unsigned int)a.num_inst;
    a.lv_off[0] = 0;
    a.lv_off[1] = a.num_inst;
    *a.nlevels = 0;
  }
}

__global__ __launch_bounds__(BBS) void bw_levels_kernel(BackArgs a) {
  __shared__ uint64_t scan[BBS / SSSP_WAVE + 1];
  __shared__ unsigned int sbase;
  const int tid = threadIdx.x;
  const int nb = gridDim.x, bid = blockIdx.x;
  unsigned int epoch = 0;
  // ---- top-down: level L occupies [s, e) of the level list
  int s = 0, e = a.num_inst, L = 0;
  while (s < e) {
    for (int b0 = s + bid * BBS; b0 < e; b0 += nb * BBS) {
      const int idx = b0 + tid;
      int32_t x = 0, ins = 0, sb = 0, vx = 0, k0 = 0, k1 = 0, root = -1;
      const GraphDev *G = nullptr;
      uint32_t nch = 0;
      // the children among the first four out-edges (bit q: edge k0 + q)
      uint32_t cm = 0;
      int32_t cc[4] = {0, 0, 0, 0};
      if (idx < e) {
        x = a.lv_v[idx];
        ins = a.lv_i[idx];
        const InstDev id = a.insts[ins];
        sb = id.sbase;
        root = id.source;
        G = &a.graphs[id.graph];
        vx = x - sb;
        k0 = G->u_out_off[vx];
        k1 = G->u_out_off[vx + 1];
        // four out-edges at a time: their heads, then the heads' parent
        // entries, each step's loads issued together (past the list's end a
        // lane reads edge kb again and its test fails)
        for (int32_t kb = k0; kb < k1; kb += 4) {
          int32_t c[4], pr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) c[q] = G->u_out_dst[kb + q < k1 ? kb + q : kb];
#pragma unroll
          for (int q = 0; q < 4; ++q) pr[q] = a.pred[sb + c[q]];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (kb + q < k1 && c[q] != root && pr[q] == kb + q) {
              ++nch;
              if (kb == k0) {
                cm |= 1u << q;
                cc[q] = c[q];
              }
            }
          }
        }
      }
      uint64_t tot;
      const uint64_t ex = block_excl_scan64<BBS>((uint64_t)nch, scan, &tot);
      if (tot > 0) {
        if (tid == 0) sbase = atomicAdd(a.ctr, (unsigned int)tot);
        __syncthreads();
        uint32_t p = sbase + (uint32_t)ex;
        if (idx < e && nch) {
          if (k1 - k0 <= 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if ((cm >> q) & 1u) {
                a.lv_v[p] = sb + cc[q];
                a.lv_i[p] = ins;
                ++p;
              }
            }
          } else {
            for (int32_t k = k0; k < k1; ++k) {
              const int32_t c = G->u_out_dst[k];
              if (c != root && a.pred[sb + c] == k) {
                a.lv_v[p] = sb + c;
                a.lv_i[p] = ins;
                ++p;
              }
            }
          }
        }
        __syncthreads();
      }
    }
    grid_barrier(a.flags, a.go, epoch);
    s = e;
    e = (int)__hip_atomic_load(a.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++L;
    if (bid == 0 && tid == 0) a.lv_off[L + 1] = e;
  }
  // levels 0..L-1 are non-empty; lv_off[0..L] are their bounds
  grid_barrier(a.flags, a.go, epoch);
  // ---- bottom-up: deepest level first
  for (int lv = L - 1; lv >= 0; --lv) {
    const int ls = a.lv_off[lv], le = a.lv_off[lv + 1];
    for (int idx = ls + bid * BBS + tid; idx < le; idx += nb * BBS) {
      const int32_t y = a.lv_v[idx];
      const InstDev id = a.insts[a.lv_i[idx]];
      const GraphDev &G = a.graphs[id.graph];
      const int32_t sb = id.sbase, vy = y - sb;
      float acc = a.gcost[y];
      const int32_t k0 = G.u_out_off[vy], k1 = G.u_out_off[vy + 1];
      // as in the top-down pass, four out-edges at a time; a head's subtree
      // sum loads with its parent entry and counts only for a child (in
      // edge order)
      for (int32_t kb = k0; kb < k1; kb += 4) {
        int32_t lc[4], pr[4];
        float av[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) lc[q] = G.u_out_dst[kb + q < k1 ? kb + q : kb];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          pr[q] = a.pred[sb + lc[q]];
          av[q] = a.acc[sb + lc[q]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (kb + q < k1 && lc[q] != id.source && pr[q] == kb + q) acc = __fadd_rn(acc, av[q]);
      }
      a.acc[y] = acc;
    }
    grid_barrier(a.flags, a.go, epoch);
  }
  if (bid == 0 && tid == 0) *a.nlevels = L;
}

// The same two passes with each instance's tree in a workgroup of its own
// (blocks loop over the instances) and block barriers only: for deep trees
// (grids, meshes), whose levels are many and small.  Instance i's level
// list occupies lv_v[sbase_i, sbase_i + n_i) and the ends of its levels
// lv_i[sbase_i + l] (a tree has at most n_i levels).  The top-down pass
// appends each entry's children together, in edge order, and entries'
// children in list order, so the children of the entry at position p are
// the list positions [lv_cs[p], lv_cs[p + 1]) (the list's end for the last
// entry); the bottom-up pass sums them from lv_acc, the subtree sums by
// list position, in that order (edge order, as the grid-wide pass does).
// The top-down step also keeps the level it builds in LDS (the first
// kLevelLds entries, double-buffered by level parity), so the next step reads
// its entries there instead of from the global list it has just written.
constexpr int kLevelLds = 4096;

__global__ __launch_bounds__(BBS) void bw_wg_kernel(BackArgs a) {
  __shared__ uint64_t scan[BBS / SSSP_WAVE + 1];
  __shared__ int32_t cnt;
  __shared__ int32_t lvl[2][kLevelLds];
  const int tid = threadIdx.x;
  int lmax = 0;
  for (int ins = blockIdx.x; ins < a.num_inst; ins += gridDim.x) {
    const InstDev id = a.insts[ins];
    const GraphDev G = a.graphs[id.graph];  // by value: its fields stay in registers
    const int32_t sb = id.sbase;
    int32_t *V = a.lv_v + sb, *LE = a.lv_i + sb, *CS = a.lv_cs + sb;
    float *AL = a.lv_acc + sb;
    if (tid == 0) {
      V[0] = id.source;  // graph-local ids in this path
      lvl[0][0] = id.source;
      cnt = 1;
    }
    __syncthreads();
    // ---- top-down: level L occupies [s, e) of V, and its first kLevelLds
    // entries lvl[L & 1]
    int s = 0, e = 1, L = 0;
    while (s < e) {
      const int32_t *cur = lvl[L & 1];
      int32_t *nxt = lvl[(L & 1) ^ 1];
      for (int b0 = s; b0 < e; b0 += BBS) {
        const int idx = b0 + tid;
        int32_t k0 = 0, k1 = 0;
        uint32_t nch = 0;
        // the children among the first four out-edges (bit q: edge k0 + q)
        uint32_t cm = 0;
        int32_t cc[4] = {0, 0, 0, 0};
        if (idx < e) {
          const int32_t x = idx - s < kLevelLds ? cur[idx - s] : V[idx];
          k0 = G.u_out_off[x];
          k1 = G.u_out_off[x + 1];
          // four out-edges at a time: their heads, then the heads' parent
          // entries, each step's loads issued together (past the list's
          // end a lane reads edge kb again and its test fails)
          for (int32_t kb = k0; kb < k1; kb += 4) {
            int32_t c[4], pr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) c[q] = G.u_out_dst[kb + q < k1 ? kb + q : kb];
#pragma unroll
            for (int q = 0; q < 4; ++q) pr[q] = a.pred[sb + c[q]];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if (kb + q < k1 && c[q] != id.source && pr[q] == kb + q) {
                ++nch;
                if (kb == k0) {
                  cm |= 1u << q;
                  cc[q] = c[q];
                }
              }
            }
          }
        }
        uint64_t tot;
        const uint64_t ex = block_excl_scan64<BBS>((uint64_t)nch, scan, &tot);
        if (idx < e) CS[idx] = cnt + (int32_t)ex;  // (cnt is current: the scan's barriers)
        if (tot > 0) {
          uint32_t p = (uint32_t)cnt + (uint32_t)ex;
          if (idx < e && nch) {
            // the next level starts at e: entry p is its entry p - e
            if (k1 - k0 <= 4) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                if ((cm >> q) & 1u) {
                  V[p] = cc[q];
                  if (p - (uint32_t)e < (uint32_t)kLevelLds) nxt[p - e] = cc[q];
                  ++p;
                }
              }
            } else {
              for (int32_t k = k0; k < k1; ++k) {
                const int32_t c = G.u_out_dst[k];
                if (c != id.source && a.pred[sb + c] == k) {
                  V[p] = c;
                  if (p - (uint32_t)e < (uint32_t)kLevelLds) nxt[p - e] = c;
                  ++p;
                }
              }
            }
          }
          __syncthreads();
          if (tid == 0) cnt += (int32_t)tot;
          __syncthreads();
        }
      }
      if (tid == 0) LE[L] = e;
      ++L;
      s = e;
      e = cnt;  // every thread reads it after the barriers above
      __syncthreads();
    }
    lmax = L > lmax ? L : lmax;
    // ---- bottom-up: deepest level first; an entry's children are the
    // list range its top-down step recorded, summed in list (edge) order
    const int nv = e;  // the tree's size: the list's end
    for (int lv = L - 1; lv >= 0; --lv) {
      const int ls = lv == 0 ? 0 : LE[lv - 1], le = LE[lv];
      for (int idx = ls + tid; idx < le; idx += BBS) {
        const int32_t y = V[idx];
        const int32_t c0 = CS[idx], c1 = idx + 1 < nv ? CS[idx + 1] : nv;
        float acc = a.gcost[sb + y];
        for (int32_t p = c0; p < c1; ++p) acc = __fadd_rn(acc, AL[p]);
        AL[idx] = acc;
        a.acc[sb + y] = acc;
      }
      __syncthreads();
    }
  }
  if (tid == 0 && lmax) atomicMax(a.nlevels, lmax);
}

// grad_w[ebase[g] + e] = sum over instances i of graph g (instance order) of
// acc_i[head(e)] if pred_i[head(e)] == e
__global__ void bw_grad_kernel(BackArgs a, const int32_t *goff, const int32_t *ginst,
                               const int32_t *ebase, int32_t num_graphs, int32_t total_m,
                               float *grad_w) {
  for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total_m;
       q += gridDim.x * blockDim.x) {
    int lo = 0, hi = num_graphs;  // ebase[lo] <= q < ebase[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (ebase[mid] <= q) lo = mid;
      else hi = mid;
    }
    const GraphDev &G = a.graphs[lo];
    const int32_t e = q - ebase[lo];
    const int32_t y = G.u_out_dst[e];
    float sum = 0.0f;
    for (int32_t j = goff[lo]; j < goff[lo + 1]; ++j) {
      const InstDev id = a.insts[ginst[j]];
      if (y != id.source && a.pred[id.sbase + y] == e) sum = __fadd_rn(sum, a.acc[id.sbase + y]);
    }
    grad_w[q] = sum;
  }
}

hipError_t launch_backward(const BackArgs &a, const LaunchGeom &geo, const int32_t *goff,
                           const int32_t *ginst, const int32_t *ebase, int32_t num_graphs,
                           int32_t total_m, float *grad_w, hipStream_t stream) {
  hipError_t e;
  {
    int zb = (a.total + 255) / 256;
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(bw_zero_kernel, dim3(zb < 1 ? 1 : zb), dim3(256), 0, stream, a);
  }
  hipLaunchKernelGGL(bw_init_kernel, dim3(1), dim3(256), 0, stream, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (geo.wg) {
    int nbk = a.num_inst < geo.blocks ? a.num_inst : geo.blocks;
    if (nbk < 1) nbk = 1;
    hipLaunchKernelGGL(bw_wg_kernel, dim3(nbk), dim3(BBS), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    int occ = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)bw_levels_kernel,
                                                          BBS, 0)) != hipSuccess)
      return e;
    int per_cu = geo.blocks / (geo.cus > 0 ? geo.cus : 1);
    if (occ < per_cu) per_cu = occ;
    if (per_cu < 1) return hipErrorLaunchFailure;
    BackArgs arg = a;
    void *params[] = {&arg};
    e = hipLaunchCooperativeKernel((const void *)bw_levels_kernel, dim3(geo.cus * per_cu),
                                   dim3(BBS), params, 0, stream);
    if (e != hipSuccess) return e;
  }
  int blocks = (total_m + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(bw_grad_kernel, dim3(blocks), dim3(256), 0, stream, a, goff, ginst, ebase,
                     num_graphs, total_m, grad_w);
  return hipGetLastError();
}

}  // namespace sssp
