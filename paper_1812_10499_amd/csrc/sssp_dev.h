// Device-side building blocks shared by the gfx950 kernels of the SSSP
// library: value traits in the int32 "key" domain, wave/block scans and
// reductions for 64-wide wavefronts, a grid barrier for the persistent
// round kernel, and the descriptors the kernels read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SSSP_WAVE 64

namespace sssp {

// ---------------------------------------------------------------- values
// Every value the kernels keep (D, C, minD, thr, m_y, weights) is stored as
// an int32 key.  For int32 graphs the key is the value.  For float32 graphs
// the key is the IEEE bit pattern: all values are >= +0, and non-negative
// floats (with +inf) order exactly like their int32 bit patterns, so min,
// max, compare and atomicMin all work on keys.  Only the path-sum
// extension needs the value type.
struct KeyI32 {
  static constexpr int32_t INF = 0x7fffffff;
  // a + b saturating at INF.  Both operands are in [0, INF], so the sum
  // fits in uint32 without wrapping.
  __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) {
    uint32_t s = (uint32_t)a + (uint32_t)b;
    return s >= (uint32_t)INF ? INF : (int32_t)s;
  }
};

struct KeyF32 {
  static constexpr int32_t INF = 0x7f800000;  // +inf
  // one IEEE round-to-nearest-even float add; inf + x = inf.
  __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) {
    return __float_as_int(__fadd_rn(__int_as_float(a), __int_as_float(b)));
  }
};

__device__ __forceinline__ int32_t kmin(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ __forceinline__ int32_t kmax(int32_t a, int32_t b) { return a > b ? a : b; }

// ---------------------------------------------------------- descriptors
struct GraphDev {
  const int32_t *out_off, *out_dst, *out_w;
  const int32_t *in_off, *in_src, *in_eid, *in_w;
  const int32_t *out_wmin;
  int32_t n, m;
};

// Instance i of a batch: graph index, source vertex (graph-local), base of
// its entries in the state arrays, vertex count.
struct InstDev {
  int32_t graph, source, sbase, n;
};

// ------------------------------------------------------------ wave ops
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int32_t wave_min(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = kmin(v, __shfl_xor(v, o, SSSP_WAVE));
  return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, SSSP_WAVE);
  return v;
}

// inclusive prefix sum across the wave
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < SSSP_WAVE; o <<= 1) {
    uint64_t t = __shfl_up(v, o, SSSP_WAVE);
    if (l >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < SSSP_WAVE; o <<= 1) {
    uint32_t t = __shfl_up(v, o, SSSP_WAVE);
    if (l >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of a uint64 per thread.  `scratch` must hold
// BS/64 + 1 entries of LDS.  Returns the exclusive prefix; *total gets the
// block sum.  Contains __syncthreads(); call from all threads.
template <int BS>
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v, uint64_t *scratch,
                                                     uint64_t *total) {
  constexpr int NW = BS / SSSP_WAVE;
  const int w = threadIdx.x / SSSP_WAVE, l = lane_id();
  uint64_t inc = wave_incl_scan64(v);
  if (l == SSSP_WAVE - 1) scratch[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    for (int i = 0; i < NW; ++i) {
      uint64_t t = scratch[i];
      scratch[i] = run;
      run += t;
    }
    scratch[NW] = run;
  }
  __syncthreads();
  uint64_t res = scratch[w] + inc - v;
  *total = scratch[NW];
  __syncthreads();
  return res;
}

// Block-wide min; result valid in all threads.  scratch: BS/64 entries.
template <int BS>
__device__ __forceinline__ int32_t block_min(int32_t v, int32_t *scratch) {
  constexpr int NW = BS / SSSP_WAVE;
  const int w = threadIdx.x / SSSP_WAVE;
  v = wave_min(v);
  if (lane_id() == 0) scratch[w] = v;
  __syncthreads();
  int32_t r = scratch[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r = kmin(r, scratch[i]);
  __syncthreads();
  return r;
}

// ------------------------------------------------------- grid barrier
// Sense-free barrier for a cooperative (all blocks co-resident) launch:
// `counter` only grows; the k-th barrier completes when it reaches
// k * gridDim.x.  Thread 0 of each block publishes the block's writes with
// an agent-scope release (write-back of this XCD's L2) and, once all blocks
// arrived, acquires (invalidate) before the block continues.  `epoch` is
// the block's own count of barriers passed (same in every block).
// The counter may wrap past 2^32 on very long solves; the wait compares the
// signed difference, which stays correct while fewer than 2^31 arrivals
// separate any two blocks (they are at most one barrier apart).
__device__ __forceinline__ void grid_barrier(unsigned int *counter, unsigned int &epoch) {
  // every wave publishes its own stores before the block meets
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  epoch += 1;
  if (threadIdx.x == 0) {
    const unsigned int target = epoch * gridDim.x;
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    while ((int)(__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) -
                 target) < 0)
      __builtin_amdgcn_s_sleep(1);
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_relaxed64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sssp
