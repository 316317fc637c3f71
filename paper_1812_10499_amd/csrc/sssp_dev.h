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
// The round kernel works on the solver numbering (out_*, in_*, out_wmin);
// out_eid maps a CSR position there to the caller's edge id, vid a solver
// vertex to the caller's vertex id, rank the reverse (all three null when
// the numberings coincide).  The u_ arrays are the caller-numbered CSR/CSC
// that the parent tie pass and the backward pass walk.
// vrec: per solver vertex {out_off, out_degree, in_off, in_degree,
// out_wmin, in_src and in_w of the lightest in-edge (0, 0 if none), 0}
// (one 32-byte record).  in_sw: (in_src, in_w) of each in-list entry side
// by side, one 8-byte read per in-edge where a scan needs both.  out_rec:
// per out-list entry {out_dst, out_w, edge id (out_eid, else the
// position), out_wmin of the head}, one 16-byte read per relaxed edge.
struct GraphDev {
  const int32_t *out_off, *out_dst, *out_w, *out_eid;
  const int32_t *in_off, *in_src, *in_w;
  const int2 *in_sw;
  const int4 *out_rec;
  const int4 *vin;  // per vertex {in_off, in_degree, lightest in-edge's tail, its weight}
  const int32_t *out_wmin;
  const int4 *vrec;
  const int32_t *vid, *rank;
  const int32_t *u_out_off, *u_out_dst;
  const int32_t *u_in_off, *u_in_src, *u_in_eid, *u_in_w;
  int32_t n, m;
  int32_t lc;     // label-correcting relax on this graph
  int32_t all;    // C scope ALL on this graph
  int32_t delta;  // label-correcting: open vertices join the relax set while D < minD + delta
};

// Instance i of a batch: graph index, source vertex (graph-local), base of
// its entries in the state arrays, vertex count.
struct InstDev {
  int32_t graph, source, sbase, n;
};

// ------------------------------------------------------------ wave ops
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Wave-wide reductions (every lane of the wave active; the result is
// wave-uniform): DPP lane moves combine within each row of 16 lanes (the
// quad swaps 1 and 2, then the half-row and row mirrors), then one lane of
// each of the four rows is read into scalar registers.  No LDS traffic and
// no waits on it, unlike a shuffle ladder.
enum : int {
  kDppQuadSwap1 = 0xB1,    // quad_perm [1,0,3,2]
  kDppQuadSwap2 = 0x4E,    // quad_perm [2,3,0,1]
  kDppRowMirror = 0x140,   // lane i of a row reads lane 15 - i
  kDppHalfMirror = 0x141,  // lane i of a half-row reads lane 7 - i
};

template <int CTRL>
__device__ __forceinline__ int32_t dpp_mov(int32_t v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

template <class Op>
__device__ __forceinline__ int32_t wave_reduce32(int32_t v, Op op) {
  v = op(v, dpp_mov<kDppQuadSwap1>(v));
  v = op(v, dpp_mov<kDppQuadSwap2>(v));
  v = op(v, dpp_mov<kDppHalfMirror>(v));
  v = op(v, dpp_mov<kDppRowMirror>(v));
  const int32_t r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int32_t r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}

__device__ __forceinline__ int32_t wave_min(int32_t v) {
  return wave_reduce32(v, [](int32_t x, int32_t y) { return kmin(x, y); });
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
  return wave_reduce32(v, [](int32_t x, int32_t y) { return kmax(x, y); });
}

template <int CTRL>
__device__ __forceinline__ int64_t dpp_mov64(int64_t v) {
  const int32_t lo = dpp_mov<CTRL>((int32_t)(uint32_t)v);
  const int32_t hi = dpp_mov<CTRL>((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Lane `lane` (wave-uniform) of v, in scalar registers.
__device__ __forceinline__ int64_t readlane64(int64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
  v += dpp_mov64<kDppQuadSwap1>(v);
  v += dpp_mov64<kDppQuadSwap2>(v);
  v += dpp_mov64<kDppHalfMirror>(v);
  v += dpp_mov64<kDppRowMirror>(v);
  return (readlane64(v, 0) + readlane64(v, 16)) + (readlane64(v, 32) + readlane64(v, 48));
}

// Inclusive prefix sums across the wave (every lane active), by DPP:
// Hillis-Steele steps within each row of 16 lanes (shifts right by 1, 2, 4,
// 8; lanes without a source add 0), then row 0's total into row 1 and row
// 2's into row 3 (broadcast of lane 15 of each row), then lane 31's total
// into rows 2 and 3.
enum : int { kDppRowShr = 0x110, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143 };

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, CTRL, ROWS, 0xF, true);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_or_zero64(uint64_t v) {
  const uint32_t lo = dpp_or_zero<CTRL, ROWS>((uint32_t)v);
  const uint32_t hi = dpp_or_zero<CTRL, ROWS>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
  v += dpp_or_zero64<kDppRowShr + 1, 0xF>(v);
  v += dpp_or_zero64<kDppRowShr + 2, 0xF>(v);
  v += dpp_or_zero64<kDppRowShr + 4, 0xF>(v);
  v += dpp_or_zero64<kDppRowShr + 8, 0xF>(v);
  v += dpp_or_zero64<kDppRowBcast15, 0xA>(v);
  v += dpp_or_zero64<kDppRowBcast31, 0xC>(v);
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v) {
  v += dpp_or_zero<kDppRowShr + 1, 0xF>(v);
  v += dpp_or_zero<kDppRowShr + 2, 0xF>(v);
  v += dpp_or_zero<kDppRowShr + 4, 0xF>(v);
  v += dpp_or_zero<kDppRowShr + 8, 0xF>(v);
  v += dpp_or_zero<kDppRowBcast15, 0xA>(v);
  v += dpp_or_zero<kDppRowBcast31, 0xC>(v);
  return v;
}

// Last position p in [0, 1024) with pfx[p] <= e, for pfx ascending with
// pfx[0] <= e (an LDS window's exclusive prefix): an 8-ary search, four
// dependent LDS steps instead of a binary search's ten.
__device__ __forceinline__ int search1024(const int32_t *pfx, uint32_t e) {
  int lo = 0;
#pragma unroll
  for (int s = 128; s >= 2; s /= 8) {  // spans 128, 16, 2
    int c = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) c += (uint32_t)pfx[lo + k * s] <= e ? 1 : 0;
    lo += c * s;
  }
  return (uint32_t)pfx[lo + 1] <= e ? lo + 1 : lo;
}

// Exclusive prefix over the wave of a per-lane count below 2^B, and the
// wave's total: one ballot and one lane-mask count per bit, no LDS.
template <int B>
__device__ __forceinline__ uint32_t wave_excl_small(uint32_t v, uint32_t *total) {
  uint32_t ex = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < B; ++k) {
    const unsigned long long m = __ballot((v >> k) & 1u);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    ex += below << k;
    tot += (uint32_t)__popcll(m) << k;
  }
  *total = tot;
  return ex;
}

// Block-wide exclusive scan of a uint64 per thread (BS a multiple of 64, at
// most 64 waves).  `scratch` must hold BS/64 + 1 entries of LDS.  Returns the exclusive prefix; *total gets the
// block sum.  Contains __syncthreads(); call from all threads.
template <int BS>
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v, uint64_t *scratch,
                                                     uint64_t *total) {
  constexpr int NW = BS / SSSP_WAVE;
  static_assert(NW * SSSP_WAVE == BS && NW <= SSSP_WAVE, "whole waves, one wave of totals");
  const int w = threadIdx.x / SSSP_WAVE, l = lane_id();
  uint64_t inc = wave_incl_scan64(v);
  if (l == SSSP_WAVE - 1) scratch[w] = inc;
  __syncthreads();
  if (w == 0) {  // the waves' totals, prefixed by wave 0 in one wave scan
    const uint64_t t = l < NW ? scratch[l] : 0ull;
    const uint64_t it = wave_incl_scan64(t);
    if (l < NW) scratch[l] = it - t;
    if (l == NW - 1) scratch[NW] = it;
  }
  __syncthreads();
  uint64_t res = scratch[w] + inc - v;
  *total = scratch[NW];
  __syncthreads();
  return res;
}

// Two independent block-wide exclusive scans in one pass (one barrier pair).
// scratch: 2 * (BS/64 + 1) entries.
template <int BS>
__device__ __forceinline__ void block_excl_scan64x2(uint64_t v1, uint64_t v2, uint64_t *scratch,
                                                    uint64_t *ex1, uint64_t *ex2,
                                                    uint64_t *tot1, uint64_t *tot2) {
  constexpr int NW = BS / SSSP_WAVE;
  static_assert(NW * SSSP_WAVE == BS && NW <= SSSP_WAVE, "whole waves, one wave of totals");
  const int w = threadIdx.x / SSSP_WAVE, l = lane_id();
  const uint64_t i1 = wave_incl_scan64(v1), i2 = wave_incl_scan64(v2);
  if (l == SSSP_WAVE - 1) {
    scratch[w] = i1;
    scratch[NW + 1 + w] = i2;
  }
  __syncthreads();
  if (w == 0) {  // both sets of wave totals, prefixed by wave 0
    const uint64_t t1 = l < NW ? scratch[l] : 0ull, t2 = l < NW ? scratch[NW + 1 + l] : 0ull;
    const uint64_t s1 = wave_incl_scan64(t1), s2 = wave_incl_scan64(t2);
    if (l < NW) {
      scratch[l] = s1 - t1;
      scratch[NW + 1 + l] = s2 - t2;
    }
    if (l == NW - 1) {
      scratch[NW] = s1;
      scratch[2 * NW + 1] = s2;
    }
  }
  __syncthreads();
  *ex1 = scratch[w] + i1 - v1;
  *ex2 = scratch[NW + 1 + w] + i2 - v2;
  *tot1 = scratch[NW];
  *tot2 = scratch[2 * NW + 1];
  __syncthreads();
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

// Two block-wide minima in one pass; results valid in all threads.
// scratch: 2 * BS/64 entries.
template <int BS>
__device__ __forceinline__ void block_min2(int32_t &a, int32_t &b, int32_t *scratch) {
  constexpr int NW = BS / SSSP_WAVE;
  const int w = threadIdx.x / SSSP_WAVE;
  a = wave_min(a);
  b = wave_min(b);
  if (lane_id() == 0) {
    scratch[w] = a;
    scratch[NW + w] = b;
  }
  __syncthreads();
  a = scratch[0];
  b = scratch[NW];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    a = kmin(a, scratch[i]);
    b = kmin(b, scratch[NW + i]);
  }
  __syncthreads();
}

// ------------------------------------------------------- grid barrier
// Barrier for a cooperative launch (all blocks co-resident) that uses no
// same-address atomics: 512 blocks incrementing one counter serialize at
// the memory side (tens of microseconds per barrier on MI355X).  Instead
// each block owns a flag word on its own 64-byte line:
//   1. every wave waits for its own stores (vmcnt(0)) so that they sit in
//      this XCD's L2; thread 0 writes the L2 back (agent release) and
//      stores the block's epoch into its flag;
//   2. block 0's threads poll all flags in parallel, then thread 0 stores
//      the epoch into `go`;
//   3. every block waits for `go`, then invalidates its L1/L2 (agent
//      acquire) so that later loads see the other XCDs' writes.
// `epoch` is the block's count of barriers passed (equal in all blocks);
// flags and `go` must be zero at launch.  Comparisons use the signed
// difference, so epoch wrap-around is harmless.
constexpr int kFlagStride = 16;  // ints between flags (64 bytes)

__device__ __forceinline__ void wait_own_stores() {
  // s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15): only vector memory counts
  __builtin_amdgcn_s_waitcnt(0x0F70);
}

// Waits for every vector memory access this wave has in flight.  Placed
// after a group of independent loads, it lets the accesses that depend on
// them issue back to back: the counter is in order, so a value needed
// between two of them would otherwise make the later wait for the earlier.
__device__ __forceinline__ void wait_vector_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ unsigned int ld_flag(const unsigned int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// nblocks: the participants are blocks [0, nblocks) (the whole grid by
// default); the others must not call it for this epoch.
__device__ __forceinline__ void grid_barrier(unsigned int *flags, unsigned int *go,
                                             unsigned int &epoch, unsigned int nblocks = 0) {
  if (nblocks == 0) nblocks = gridDim.x;
  wait_own_stores();
  __syncthreads();
  epoch += 1;
  const unsigned int ep = epoch;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&flags[blockIdx.x * kFlagStride], ep, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x == 0) {
    for (unsigned int b = threadIdx.x; b < nblocks; b += blockDim.x)
      while ((int)(ld_flag(&flags[b * kFlagStride]) - ep) < 0) __builtin_amdgcn_s_sleep(1);
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      __hip_atomic_store(go, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (threadIdx.x == 0) {
    while ((int)(ld_flag(go) - ep) < 0) __builtin_amdgcn_s_sleep(1);
  }
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
}

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_relaxed64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace sssp
