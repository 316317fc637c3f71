// Measurement probes for MI355X (gfx950): the access rates and latencies
// that bound the round kernels.  Not part of a solve; built into its own
// library (libsssp_probe.so) and driven by paper_1812_10499_amd.probe.
//
//  - random gathers of 8- or 4-byte values at indices read from a stream
//    (U independent gathers in flight per thread), as the relax and bound
//    steps gather D and C;
//  - gather then 64-bit atomicMin where the key is smaller (the relax
//    step's pre-filtered update), also with a set share of atomics;
//  - gathers folded into per-XCD ranges of the array (L2 locality);
//  - a dependent-load chain (one lane follows next[] pointers), the latency
//    of one step of a round's critical path at a given working-set size;
//  - block barriers (__syncthreads) in one 1024-thread workgroup, and the
//    round kernel's grid barrier over a cooperative grid;
//  - what one CU's memory pipeline pays per wave instruction (one
//    1024-thread workgroup): random 4-byte gathers, coalesced 4- and
//    16-byte loads and stores (the one-workgroup kernel's trade).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sssp_dev.h"

namespace {

constexpr int U = 8;

template <class T>
__global__ __launch_bounds__(256) void gather_k(const T *__restrict__ arr,
                                                const uint32_t *__restrict__ idx, int64_t n,
                                                T *out) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  T acc = (T)-1;
  for (int64_t b = tid; b < n; b += stride * U) {
    uint32_t ix[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + (int64_t)u * stride;
      ix[u] = i < n ? idx[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = arr[ix[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) acc = v[u] < acc ? v[u] : acc;
  }
  out[tid] = acc;
}

__global__ __launch_bounds__(256) void gather_atomic_k(unsigned long long *arr,
                                                       const uint32_t *__restrict__ idx,
                                                       int64_t n, unsigned long long *out) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long acc = 0;
  for (int64_t b = tid; b < n; b += stride * U) {
    uint32_t ix[U];
    unsigned long long k[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + (int64_t)u * stride;
      ix[u] = i < n ? idx[i] : 0u;
      k[u] = ((unsigned long long)(uint32_t)(i * 2654435761u) << 20) | (uint64_t)(i & 0xfffff);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) d[u] = arr[ix[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + (int64_t)u * stride;
      if (i < n && k[u] < d[u]) acc += atomicMin(&arr[ix[u]], k[u]);
    }
  }
  out[tid] = acc;
}

// Gathers whose indices are folded into one of `parts` equal ranges of the
// array, the range chosen by the block: part (block / div) % parts.  With
// div = 1 the blocks of one XCD (workgroups go to the XCDs round-robin)
// share one range; with div = parts, every range is read from every XCD.
template <class T>
__global__ __launch_bounds__(256) void gather_part_k(const T *__restrict__ arr,
                                                     const uint32_t *__restrict__ idx, int64_t n,
                                                     T *out, uint32_t span, int parts, int div) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint32_t lo = ((blockIdx.x / div) % parts) * span;
  T acc = (T)-1;
  for (int64_t b = tid; b < n; b += stride * U) {
    uint32_t ix[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + (int64_t)u * stride;
      ix[u] = i < n ? lo + idx[i] % span : lo;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = arr[ix[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) acc = v[u] < acc ? v[u] : acc;
  }
  out[tid] = acc;
}

// The relax step's update with a given share of atomics: every edge's key
// is gathered, and one edge in `every` whose index is at least `cut`
// carries the key 0, at most every stored one, so it issues a 64-bit
// atomicMin (the others carry the largest key and are filtered out).  With
// the cut above the hubs, a vertex takes few atomics, as in the relax step
// (its pre-filter keeps nearly all atomics off the hubs).
__global__ __launch_bounds__(256) void gather_atomic_every_k(unsigned long long *arr,
                                                             const uint32_t *__restrict__ idx,
                                                             int64_t n, unsigned long long *out,
                                                             int every, uint32_t cut) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long acc = 0;
  for (int64_t b = tid; b < n; b += stride * U) {
    uint32_t ix[U];
    unsigned long long k[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + (int64_t)u * stride;
      ix[u] = i < n ? idx[i] : 0u;
      k[u] = (i % every == 0 && ix[u] >= cut) ? 0ull : ~0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) d[u] = arr[ix[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + (int64_t)u * stride;
      if (i < n && k[u] <= d[u]) acc += atomicMin(&arr[ix[u]], k[u]);
    }
  }
  out[tid] = acc;
}

// Each of the 64 lanes of one wave follows next[] for `steps` dependent
// loads from its own start (a per-lane address keeps them vector loads);
// the wave waits for its slowest lane at every step.
__global__ __launch_bounds__(64) void chase_k(const uint32_t *next, const uint32_t *start,
                                              int64_t steps, uint32_t *out) {
  uint32_t p = start[threadIdx.x];
  for (int64_t s = 0; s < steps; ++s) p = next[p];
  out[threadIdx.x] = p;
}

// `iters` block barriers, with an LDS store and load between them so that
// none can be dropped.
__global__ __launch_bounds__(1024) void sync_k(int iters, int *out) {
  __shared__ int slot[1024];
  int v = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
    slot[threadIdx.x] = v;
    __syncthreads();
    v += slot[(threadIdx.x + 1) & 1023];
    __syncthreads();
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = v;
}

// `iters` grid barriers of the round kernel (sssp::grid_barrier) over the
// whole cooperative grid.  flags (kMaxBlocks * kFlagStride) and go must be
// zero at launch.
__global__ __launch_bounds__(1024) void grid_sync_k(unsigned int *flags, unsigned int *go,
                                                    int iters) {
  unsigned int epoch = 0;
  for (int i = 0; i < iters; ++i) sssp::grid_barrier(flags, go, epoch);
}

// One workgroup, 8 accesses per thread and iteration, all issued before
// any is used.  Mode 0: random 4-byte gathers (indices from a per-lane LCG,
// masked to the array); 1: coalesced 4-byte loads; 2: coalesced 16-byte
// loads; 3: coalesced 4-byte stores; 4: coalesced 16-byte stores.  The
// array holds mask + 1 ints (a power of two, at least 4 * 8 * 1024).
template <int MODE>
__global__ __launch_bounds__(1024) void cu_access_k(int *__restrict__ a, uint32_t mask, int iters,
                                                    int *out) {
  int acc = 0;
  uint32_t x = threadIdx.x * 2654435761u + 12345u;
  for (int it = 0; it < iters; ++it) {
    int v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t lin = ((uint32_t)it * 8u + j) * 1024u + threadIdx.x;
      if (MODE == 0) {
        x = x * 1664525u + 1013904223u;
        v[j] = a[(x >> 4) & mask];
      } else if (MODE == 1) {
        v[j] = a[lin & mask];
      } else if (MODE == 2) {
        const int4 q = *(const int4 *)(a + ((lin * 4u) & mask));
        v[j] = q.x ^ q.y ^ q.z ^ q.w;
      } else if (MODE == 3) {
        a[lin & mask] = it + j;
      } else {
        *(int4 *)(a + ((lin * 4u) & mask)) = make_int4(it, j, 0, 0);
      }
    }
    if (MODE <= 2) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += v[j];
    }
  }
  out[threadIdx.x] = acc;
}

}  // namespace

extern "C" {

int probe_cu_access(int mode, int *a, uint32_t mask, int iters, int *out, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (mode) {
    case 0: hipLaunchKernelGGL(cu_access_k<0>, dim3(1), dim3(1024), 0, s, a, mask, iters, out); break;
    case 1: hipLaunchKernelGGL(cu_access_k<1>, dim3(1), dim3(1024), 0, s, a, mask, iters, out); break;
    case 2: hipLaunchKernelGGL(cu_access_k<2>, dim3(1), dim3(1024), 0, s, a, mask, iters, out); break;
    case 3: hipLaunchKernelGGL(cu_access_k<3>, dim3(1), dim3(1024), 0, s, a, mask, iters, out); break;
    case 4: hipLaunchKernelGGL(cu_access_k<4>, dim3(1), dim3(1024), 0, s, a, mask, iters, out); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}


int probe_gather(int width, const void *arr, const uint32_t *idx, int64_t n, void *out,
                 int blocks, void *stream) {
  if (width == 8)
    hipLaunchKernelGGL(gather_k<unsigned long long>, dim3(blocks), dim3(256), 0,
                       (hipStream_t)stream, (const unsigned long long *)arr, idx, n,
                       (unsigned long long *)out);
  else
    hipLaunchKernelGGL(gather_k<uint32_t>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint32_t *)arr, idx, n, (uint32_t *)out);
  return (int)hipGetLastError();
}

int probe_gather_atomic(void *arr, const uint32_t *idx, int64_t n, void *out, int blocks,
                        void *stream) {
  hipLaunchKernelGGL(gather_atomic_k, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (unsigned long long *)arr, idx, n, (unsigned long long *)out);
  return (int)hipGetLastError();
}

int probe_gather_part(int width, const void *arr, const uint32_t *idx, int64_t n, void *out,
                      int blocks, uint32_t span, int parts, int div, void *stream) {
  if (width == 8)
    hipLaunchKernelGGL(gather_part_k<unsigned long long>, dim3(blocks), dim3(256), 0,
                       (hipStream_t)stream, (const unsigned long long *)arr, idx, n,
                       (unsigned long long *)out, span, parts, div);
  else
    hipLaunchKernelGGL(gather_part_k<uint32_t>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint32_t *)arr, idx, n, (uint32_t *)out, span, parts, div);
  return (int)hipGetLastError();
}

int probe_gather_atomic_every(void *arr, const uint32_t *idx, int64_t n, void *out, int blocks,
                              int every, uint32_t cut, void *stream) {
  hipLaunchKernelGGL(gather_atomic_every_k, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (unsigned long long *)arr, idx, n, (unsigned long long *)out, every, cut);
  return (int)hipGetLastError();
}

int probe_chase(const uint32_t *next, const uint32_t *start, int64_t steps, uint32_t *out,
                void *stream) {
  hipLaunchKernelGGL(chase_k, dim3(1), dim3(64), 0, (hipStream_t)stream, next, start, steps,
                     out);
  return (int)hipGetLastError();
}

int probe_sync(int iters, int *out, void *stream) {
  hipLaunchKernelGGL(sync_k, dim3(1), dim3(1024), 0, (hipStream_t)stream, iters, out);
  return (int)hipGetLastError();
}

int probe_grid_sync(unsigned int *flags, unsigned int *go, int iters, int blocks,
                    void *stream) {
  void *args[] = {&flags, &go, &iters};
  return (int)hipLaunchCooperativeKernel((const void *)grid_sync_k, dim3(blocks), dim3(1024),
                                         args, 0, (hipStream_t)stream);
}
}
