// Graph builder on gfx950: COO edges -> CSR by tail (stable: the edges of a
// tail keep their input order; edge id = CSR position) and CSC by head over
// edge ids in increasing order (so every in-list is ascending by edge id).
// This is the incoming-edge access the method assumes, built once per
// graph; out_wmin is the per-vertex minimum out-edge weight (outWeight of
// Figs. 5 and 6).
//
// The solver's working copy: an optional renumbering by descending total
// degree (CSR copy, vid/rank), and always a CSC whose in-lists are ascending
// by weight.  The lower-bound step only needs the in-edges (v, y, w) with
// minD + w < D[y]; with weight-ordered in-lists they are a prefix of y's
// list whose length one binary search finds.
//
// Sorting: LSD radix sort of (key, value) int32 pairs with 8-bit digits;
// each pass is a per-tile digit histogram, an exclusive scan over
// (digit, tile) in digit-major order, and a stable scatter that ranks equal
// digits inside a tile with 64-lane ballots.  Offsets come from the sorted
// keys (position of each key change), so no atomics decide any order.
#include "sssp_dev.h"
#include "sssp_kernels.h"

namespace sssp {

constexpr int SBS = 256;             // threads per sort block
constexpr int SKPT = 8;              // keys per thread per tile
constexpr int STILE = SBS * SKPT;    // keys per tile
constexpr int SCAN_BS = 256;
constexpr int SCAN_PT = 16;
constexpr int SCAN_TILE = SCAN_BS * SCAN_PT;

enum : int32_t { BAD_GRAPH = 1, BAD_WEIGHT = 2 };

static inline int tiles_of(int32_t m) { return (m + STILE - 1) / STILE; }

size_t build_hist_entries(int32_t m) {
  const size_t nt = (size_t)tiles_of(m > 0 ? m : 1);
  const size_t h = 256 * nt;
  return h + (h + SCAN_TILE - 1) / SCAN_TILE + 64;
}

// -------------------------------------------------------------- validate
// status: [0] error flags, [1] largest weight key, [3] INT32_MAX minus the
// smallest weight key (a maximum, so the zeroed word is its identity)
__global__ void validate_kernel(int32_t n, int32_t m, int f32, const int32_t *src,
                                const int32_t *dst, const int32_t *w, int32_t *status) {
  int32_t bad = 0, wmax = 0, wmin_c = 0;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const int32_t k = w[i];
    if (src) {
      const int32_t s = src[i], d = dst[i];
      if (s < 0 || s >= n || d < 0 || d >= n) bad |= BAD_GRAPH;
    }
    // int32: w >= 1.  float32 key: w > 0 and finite  <=>  0 < bits < 0x7f800000
    if (f32 ? (k <= 0 || k >= 0x7f800000) : (k < 1)) bad |= BAD_WEIGHT;
    else {
      wmax = kmax(wmax, k);
      wmin_c = kmax(wmin_c, 0x7fffffff - k);
    }
  }
  if (bad) atomicOr(&status[0], bad);
  if (wmax) atomicMax(&status[1], wmax);
  if (wmin_c) atomicMax(&status[3], wmin_c);
}

hipError_t launch_validate(int32_t n, int32_t m, bool f32, const int32_t *src,
                           const int32_t *dst, const int32_t *w, int32_t *status,
                           hipStream_t stream) {
  const int blocks = m > 0 ? ((m + 255) / 256 < 8192 ? (m + 255) / 256 : 8192) : 1;
  hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(256), 0, stream, n, m, f32 ? 1 : 0,
                     src, dst, w, status);
  return hipGetLastError();
}

// ------------------------------------------------------------------ scan
// exclusive prefix sum of int32 data[L] in place, three passes
__global__ void scan_reduce_kernel(const int32_t *data, int32_t L, int32_t *sums) {
  __shared__ uint64_t sc[SCAN_BS / SSSP_WAVE + 1];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int32_t s = 0;
  for (int j = 0; j < SCAN_PT; ++j) {
    const int64_t i = base + (int64_t)j * SCAN_BS + threadIdx.x;
    if (i < L) s += data[i];
  }
  uint64_t tot;
  block_excl_scan64<SCAN_BS>((uint64_t)(uint32_t)s, sc, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = (int32_t)tot;
}

__global__ void scan_sums_kernel(int32_t *sums, int32_t ns) {
  __shared__ uint64_t sc[SCAN_BS / SSSP_WAVE + 1];
  uint64_t run = 0;
  for (int b0 = 0; b0 < ns; b0 += SCAN_BS) {
    const int i = b0 + threadIdx.x;
    const uint32_t v = i < ns ? (uint32_t)sums[i] : 0u;
    uint64_t tot;
    const uint64_t ex = block_excl_scan64<SCAN_BS>((uint64_t)v, sc, &tot);
    if (i < ns) sums[i] = (int32_t)(run + ex);
    run += tot;
  }
}

__global__ void scan_apply_kernel(int32_t *data, int32_t L, const int32_t *sums) {
  __shared__ uint64_t sc[SCAN_BS / SSSP_WAVE + 1];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  // each thread owns SCAN_PT consecutive elements
  int32_t v[SCAN_PT];
  int32_t s = 0;
  const int64_t mine = base + (int64_t)threadIdx.x * SCAN_PT;
  for (int j = 0; j < SCAN_PT; ++j) {
    const int64_t i = mine + j;
    v[j] = i < L ? data[i] : 0;
    s += v[j];
  }
  uint64_t tot;
  const uint64_t ex = block_excl_scan64<SCAN_BS>((uint64_t)(uint32_t)s, sc, &tot);
  int32_t run = sums[blockIdx.x] + (int32_t)ex;
  for (int j = 0; j < SCAN_PT; ++j) {
    const int64_t i = mine + j;
    if (i < L) data[i] = run;
    run += v[j];
  }
}

static hipError_t exclusive_scan(int32_t *data, int32_t L, int32_t *sums, hipStream_t stream) {
  const int nb = (L + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(SCAN_BS), 0, stream, data, L, sums);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_BS), 0, stream, sums, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(SCAN_BS), 0, stream, data, L, sums);
  return hipGetLastError();
}

// ----------------------------------------------------------- radix sort
__global__ void iota_kernel(int32_t *v, int32_t m) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    v[i] = i;
}

__global__ __launch_bounds__(SBS) void radix_hist_kernel(const int32_t *keys, int32_t m,
                                                         int shift, int32_t *hist, int nt) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * STILE;
  for (int j = 0; j < SKPT; ++j) {
    const int64_t i = base + (int64_t)j * SBS + threadIdx.x;
    if (i < m) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nt + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(SBS) void radix_scatter_kernel(const int32_t *kin,
                                                            const int32_t *vin, int32_t *kout,
                                                            int32_t *vout, int32_t m, int shift,
                                                            const int32_t *offs, int nt) {
  constexpr int NW = SBS / SSSP_WAVE;
  __shared__ int32_t run[256];
  __shared__ int32_t wcnt[NW][256];
  const int t = threadIdx.x, w = t / SSSP_WAVE, l = lane_id();
  run[t] = offs[(int64_t)t * nt + blockIdx.x];
  const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
  const int64_t base = (int64_t)blockIdx.x * STILE;
  for (int j = 0; j < SKPT; ++j) {
    const int64_t i = base + (int64_t)j * SBS + t;
    const bool valid = i < m;
    int32_t key = 0, val = 0, d = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      d = (key >> shift) & 255;
    }
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(valid && bit);
      mask &= bit ? bb : ~bb;
    }
    const int rank = __popcll(mask & lt);
    const int cnt = __popcll(mask);
#pragma unroll
    for (int q = 0; q < NW; ++q) wcnt[q][t] = 0;
    __syncthreads();
    if (valid && rank == 0) wcnt[w][d] = cnt;
    __syncthreads();
    if (valid) {
      int32_t pos = run[d] + rank;
      for (int q = 0; q < w; ++q) pos += wcnt[q][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) add += wcnt[q][t];
    run[t] += add;
    __syncthreads();
  }
}

// Sorts (ka, va) by key; the result ends in (ka, va) again (even pass
// count) or is copied back.  Keys are < n.
static hipError_t radix_sort(int32_t *ka, int32_t *va, int32_t *kb, int32_t *vb, int32_t m,
                             int32_t n, int32_t *hist, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
  const int passes = (bits + 7) / 8;
  const int nt = tiles_of(m);
  const int32_t L = 256 * nt;
  int32_t *sums = hist + L;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nt), dim3(SBS), 0, stream, ka, m, shift, hist,
                       nt);
    hipError_t e = exclusive_scan(hist, L, sums, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nt), dim3(SBS), 0, stream, ka, va, kb, vb, m,
                       shift, hist, nt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t *t;
    t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  if (passes & 1) {
    // result is in the "b" buffers of the caller: copy back
    hipError_t e = hipMemcpyAsync(kb, ka, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice,
                                  stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vb, va, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------- assembling
// offsets from sorted keys: off[v] = first position with key >= v
// off[v] = the number of sorted keys below v (v = 0 .. n): one binary search
// per vertex, so a long run of vertices with no edges costs no thread more
// than the others
__global__ void offsets_kernel(const int32_t *skeys, int32_t m, int32_t n, int32_t *off) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = m;
    while (lo < hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      if (skeys[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    off[v] = lo;
  }
}

__global__ void gather_csr_kernel(const int32_t *perm, const int32_t *src, const int32_t *dst,
                                  const int32_t *w, int32_t m, int32_t *out_dst, int32_t *out_w,
                                  int32_t *tail, int32_t *perm_out) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
    const int32_t i = perm[k];
    out_dst[k] = dst[i];
    out_w[k] = w[i];
    tail[k] = src[i];
    if (perm_out) perm_out[k] = i;
  }
}

__global__ void gather_csc_kernel(const int32_t *eid, const int32_t *tail, const int32_t *out_w,
                                  int32_t m, int32_t *in_src, int32_t *in_w) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const int32_t e = eid[j];
    in_src[j] = tail[e];
    in_w[j] = out_w[e];
  }
}

template <bool F32>
__global__ void wmin_fill_kernel(int32_t n, int32_t *out_wmin) {
  constexpr int32_t INF = F32 ? KeyF32::INF : KeyI32::INF;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    out_wmin[v] = INF;
}

// the vertex whose out-list holds CSR position k (k < m): the largest v with
// out_off[v] <= k
__device__ int32_t owner_of(const int32_t *out_off, int32_t n, int32_t k) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo + 1) >> 1);
    if (out_off[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Minimum out-weight per vertex over fixed chunks of CSR positions (after
// wmin_fill_kernel; vertices with no out-edges keep INF).  A list wholly
// inside one chunk is stored; a list cut by a chunk boundary is combined by
// atomicMin (weights are positive, so float bits order like int32), so a
// hub's list costs no thread more than a chunk.
constexpr int32_t kWminChunk = 256;

template <bool F32>
__global__ void wmin_kernel(const int32_t *out_off, const int32_t *out_w, int32_t n, int32_t m,
                            int32_t *out_wmin) {
  constexpr int32_t INF = F32 ? KeyF32::INF : KeyI32::INF;
  const int64_t chunks = ((int64_t)m + kWminChunk - 1) / kWminChunk;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < chunks;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k0 = (int32_t)(c * kWminChunk);
    const int32_t k1 = (int32_t)min((int64_t)m, c * kWminChunk + kWminChunk);
    int32_t v = owner_of(out_off, n, k0);
    int32_t vend = out_off[v + 1];
    bool whole = out_off[v] >= k0;  // v's list starts in this chunk
    int32_t mn = INF;
    for (int32_t k = k0; k < k1; ++k) {
      mn = kmin(mn, out_w[k]);
      if (k + 1 == vend || k + 1 == k1) {
        if (whole && k + 1 == vend) out_wmin[v] = mn;
        else atomicMin(&out_wmin[v], mn);
        if (k + 1 < k1) {
          // the next non-empty list: usually v + 1's (k + 1 < m, so v + 2 <= n)
          v = out_off[v + 2] > k + 1 ? v + 1 : owner_of(out_off, n, k + 1);
          vend = out_off[v + 1];
          whole = true;
          mn = INF;
        }
      }
    }
  }
}

static inline int grid_for(int64_t work) {
  int64_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (int)b;
}

static void launch_wmin(bool f32, int32_t n, int32_t m, const int32_t *out_off,
                        const int32_t *out_w, int32_t *out_wmin, hipStream_t stream) {
  const int gc = grid_for(((int64_t)m + kWminChunk - 1) / kWminChunk);
  if (f32) {
    hipLaunchKernelGGL(wmin_fill_kernel<true>, dim3(grid_for(n)), dim3(256), 0, stream, n,
                       out_wmin);
    if (m > 0)
      hipLaunchKernelGGL(wmin_kernel<true>, dim3(gc), dim3(256), 0, stream, out_off, out_w, n,
                         m, out_wmin);
  } else {
    hipLaunchKernelGGL(wmin_fill_kernel<false>, dim3(grid_for(n)), dim3(256), 0, stream, n,
                       out_wmin);
    if (m > 0)
      hipLaunchKernelGGL(wmin_kernel<false>, dim3(gc), dim3(256), 0, stream, out_off, out_w, n,
                         m, out_wmin);
  }
}

hipError_t launch_build(int32_t n, int32_t m, bool f32, const int32_t *src, const int32_t *dst,
                        const int32_t *w, int32_t *out_off, int32_t *out_dst, int32_t *out_w,
                        int32_t *in_off, int32_t *in_src, int32_t *in_eid, int32_t *in_w,
                        int32_t *out_wmin, int32_t *perm, const BuildTemps &t,
                        hipStream_t stream) {
  hipError_t e;
  const int gm = grid_for(m), gn = grid_for((int64_t)n + 1);
  // CSR: sort edge indices by tail
  if (m > 0) {
    e = hipMemcpyAsync(t.ka, src, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(iota_kernel, dim3(gm), dim3(256), 0, stream, t.va, m);
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, n, t.hist, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(gather_csr_kernel, dim3(gm), dim3(256), 0, stream, t.va, src, dst, w, m,
                       out_dst, out_w, t.tail, perm);
  }
  hipLaunchKernelGGL(offsets_kernel, dim3(gn), dim3(256), 0, stream, t.ka, m, n, out_off);
  // CSC: sort edge ids (already increasing) by head
  if (m > 0) {
    e = hipMemcpyAsync(t.ka, out_dst, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice,
                       stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(iota_kernel, dim3(gm), dim3(256), 0, stream, t.va, m);
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, n, t.hist, stream)) != hipSuccess) return e;
    e = hipMemcpyAsync(in_eid, t.va, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice,
                       stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_csc_kernel, dim3(gm), dim3(256), 0, stream, in_eid, t.tail, out_w,
                       m, in_src, in_w);
  }
  hipLaunchKernelGGL(offsets_kernel, dim3(gn), dim3(256), 0, stream, t.ka, m, n, in_off);
  launch_wmin(f32, n, m, out_off, out_w, out_wmin, stream);
  return hipGetLastError();
}

// --------------------------------------------------- the working copy
// total degree per vertex, and its maximum into status[2]
__global__ void degree_kernel(const int32_t *out_off, const int32_t *in_off, int32_t n,
                              int32_t *deg, int32_t *status) {
  int32_t mx = 0;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int32_t d = (out_off[v + 1] - out_off[v]) + (in_off[v + 1] - in_off[v]);
    deg[v] = d;
    mx = kmax(mx, d);
  }
  if (mx) atomicMax(&status[2], mx);
}

// sort key for descending degree: dmax - deg; values = vertex ids
__global__ void degree_key_kernel(int32_t *key, int32_t *val, int32_t n, int32_t dmax) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    key[v] = dmax - key[v];
    val[v] = v;
  }
}

__global__ void rank_kernel(const int32_t *vid, int32_t n, int32_t *vid_out, int32_t *rank) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int32_t v = vid[k];
    vid_out[k] = v;
    rank[v] = k;
  }
}

// tail of every edge id from the CSR offsets
__global__ void tail_kernel(const int32_t *out_off, int32_t n, int32_t m, int32_t *tail) {
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n;  // out_off[lo] <= e < out_off[hi]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (out_off[mid] <= e) lo = mid;
      else hi = mid;
    }
    tail[e] = lo;
  }
}

// key[i] = solver id of ends[val[i]] (val: edge ids; ends: tail or head per
// edge id; rank null = identity); with iota the values are reset first
__global__ void edge_key_kernel(const int32_t *ends, const int32_t *rank, int32_t m,
                                int32_t *key, int32_t *val, bool iota) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    if (iota) val[i] = i;
    const int32_t v = ends[val[i]];
    key[i] = rank ? rank[v] : v;
  }
}

// key[i] = weight bits of edge val[i] (positive int32 or float32: the bit
// patterns order like the values)
__global__ void weight_key_kernel(const int32_t *w, int32_t m, int32_t *key,
                                  const int32_t *val) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    key[i] = w[val[i]];
}

// entry p of a solver-numbered list: edge id eid[p]; the neighbour's solver
// id and the weight come from the caller-numbered arrays (s_pair, when
// given, receives both side by side)
__global__ void copy_gather_kernel(const int32_t *eid, const int32_t *ends, const int32_t *rank,
                                   const int32_t *out_w, int32_t m, int32_t *s_nbr,
                                   int32_t *s_w, int2 *s_pair) {
  for (int32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    const int32_t e = eid[p];
    const int32_t v = ends[e];
    const int32_t nb = rank ? rank[v] : v, w = out_w[e];
    if (s_nbr) s_nbr[p] = nb;
    s_w[p] = w;
    if (s_pair) s_pair[p] = make_int2(nb, w);
  }
}

__global__ void copy_wmin_kernel(const int32_t *vid, const int32_t *out_wmin, int32_t n,
                                 int32_t *s_out_wmin) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    s_out_wmin[k] = out_wmin[vid[k]];
}

hipError_t launch_degree(int32_t n, const int32_t *out_off, const int32_t *in_off,
                         const BuildTemps &t, hipStream_t stream) {
  hipLaunchKernelGGL(degree_kernel, dim3(grid_for(n)), dim3(256), 0, stream, out_off, in_off, n,
                     t.ka, t.status);
  return hipGetLastError();
}

hipError_t launch_renumber(int32_t n, int32_t m, int32_t dmax, const int32_t *out_dst,
                           const int32_t *out_w, const int32_t *out_wmin, const SolverCopy &c,
                           const BuildTemps &t, hipStream_t stream) {
  hipError_t e;
  const int gm = grid_for(m), gn = grid_for((int64_t)n + 1);
  // vertex order: stable sort by dmax - degree (t.ka holds the degrees)
  hipLaunchKernelGGL(degree_key_kernel, dim3(grid_for(n)), dim3(256), 0, stream, t.ka, t.va, n,
                     dmax);
  if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, n, dmax + 1, t.hist, stream)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(rank_kernel, dim3(grid_for(n)), dim3(256), 0, stream, t.va, n, c.vid,
                     c.rank);
  if (m > 0) {
    // CSR: edges by (solver id of tail, solver id of head): LSD, head first
    hipLaunchKernelGGL(edge_key_kernel, dim3(gm), dim3(256), 0, stream, out_dst, c.rank, m, t.ka,
                       t.va, true);
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, n, t.hist, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(edge_key_kernel, dim3(gm), dim3(256), 0, stream, t.tail, c.rank, m, t.ka,
                       t.va, false);
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, n, t.hist, stream)) != hipSuccess) return e;
    e = hipMemcpyAsync(c.out_eid, t.va, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice,
                       stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(copy_gather_kernel, dim3(gm), dim3(256), 0, stream, c.out_eid, out_dst,
                       c.rank, out_w, m, c.out_dst, c.out_w, (int2 *)nullptr);
  }
  hipLaunchKernelGGL(offsets_kernel, dim3(gn), dim3(256), 0, stream, t.ka, m, n, c.out_off);
  hipLaunchKernelGGL(copy_wmin_kernel, dim3(grid_for(n)), dim3(256), 0, stream, c.vid, out_wmin,
                     n, c.out_wmin);
  return hipGetLastError();
}

hipError_t launch_in_lists(int32_t n, int32_t m, int32_t wkey_max, const int32_t *out_off,
                           const int32_t *out_dst, const int32_t *out_w, const SolverCopy &c,
                           const BuildTemps &t, hipStream_t stream) {
  hipError_t e;
  const int gm = grid_for(m), gn = grid_for((int64_t)n + 1);
  if (m > 0) {
    hipLaunchKernelGGL(tail_kernel, dim3(gm), dim3(256), 0, stream, out_off, n, m, t.tail);
    // edges by (solver id of head, weight, solver id of tail): LSD order
    hipLaunchKernelGGL(edge_key_kernel, dim3(gm), dim3(256), 0, stream, t.tail, c.rank, m, t.ka,
                       t.va, true);
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, n, t.hist, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(weight_key_kernel, dim3(gm), dim3(256), 0, stream, out_w, m, t.ka, t.va);
    const int32_t wb = wkey_max < 0x7fffffff ? wkey_max + 1 : 0x7fffffff;
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, wb, t.hist, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(edge_key_kernel, dim3(gm), dim3(256), 0, stream, out_dst, c.rank, m, t.ka,
                       t.va, false);
    if ((e = radix_sort(t.ka, t.va, t.kb, t.vb, m, n, t.hist, stream)) != hipSuccess) return e;
    e = hipMemcpyAsync(c.in_eid, t.va, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice,
                       stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(copy_gather_kernel, dim3(gm), dim3(256), 0, stream, c.in_eid, t.tail,
                       c.rank, out_w, m, c.in_src, c.in_w, (int2 *)c.in_sw);
  }
  hipLaunchKernelGGL(offsets_kernel, dim3(gn), dim3(256), 0, stream, t.ka, m, n, c.in_off);
  return hipGetLastError();
}

// The record also carries the head of the weight-ordered in-list (tail and
// weight of the lightest in-edge; 0, 0 with no in-edges), so that a pass
// over many vertices reads its first in-edge from the record's line instead
// of one line of in_src and one of in_w per vertex.
__global__ void vrec_kernel(int32_t n, const int32_t *out_off, const int32_t *in_off,
                            const int32_t *in_src, const int32_t *in_w,
                            const int32_t *out_wmin, int4 *vrec, int4 *vin) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int32_t o = out_off[v], i = in_off[v], ideg = in_off[v + 1] - i;
    const int32_t s0 = ideg ? in_src[i] : 0, w0 = ideg ? in_w[i] : 0;
    vrec[2 * v] = make_int4(o, out_off[v + 1] - o, i, ideg);
    vrec[2 * v + 1] = make_int4(out_wmin[v], s0, w0, 0);
    vin[v] = make_int4(i, ideg, s0, w0);
  }
}

hipError_t launch_vrec(int32_t n, const SolverCopy &c, hipStream_t stream) {
  hipLaunchKernelGGL(vrec_kernel, dim3(grid_for(n)), dim3(256), 0, stream, n, c.out_off,
                     c.in_off, c.in_src, c.in_w, c.out_wmin, (int4 *)c.vrec, (int4 *)c.vin);
  return hipGetLastError();
}

// Entry p of the working copy's out-lists as one record: head, weight, edge
// id (the position when the copy is the CSR itself), the head's out_wmin.
__global__ void out_rec_kernel(int32_t m, const int32_t *out_dst, const int32_t *out_w,
                               const int32_t *out_eid, const int32_t *out_wmin, int4 *rec) {
  for (int32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    const int32_t y = out_dst[p];
    rec[p] = make_int4(y, out_w[p], out_eid ? out_eid[p] : p, out_wmin[y]);
  }
}

hipError_t launch_out_rec(int32_t m, const SolverCopy &c, hipStream_t stream) {
  if (m > 0)
    hipLaunchKernelGGL(out_rec_kernel, dim3(grid_for(m)), dim3(256), 0, stream, m, c.out_dst,
                       c.out_w, c.out_eid, c.out_wmin, (int4 *)c.out_rec);
  return hipGetLastError();
}

// ---------------------------------------------------------- reweighting
__global__ void set_weights_kernel(const int32_t *w, const int32_t *in_eid, int32_t m,
                                   int32_t *out_w, int32_t *in_w, const int32_t *s_out_eid,
                                   int32_t *s_out_w) {
  for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    out_w[j] = w[j];
    in_w[j] = w[in_eid[j]];
    if (s_out_eid) s_out_w[j] = w[s_out_eid[j]];
  }
}

hipError_t launch_set_weights(int32_t n, int32_t m, bool f32, const int32_t *w,
                              const int32_t *out_off, const int32_t *in_eid, int32_t *out_w,
                              int32_t *in_w, int32_t *out_wmin, const SolverCopy &c,
                              hipStream_t stream) {
  hipLaunchKernelGGL(set_weights_kernel, dim3(grid_for(m)), dim3(256), 0, stream, w, in_eid, m,
                     out_w, in_w, c.out_eid, c.out_w);
  launch_wmin(f32, n, m, out_off, out_w, out_wmin, stream);
  if (c.vid)
    hipLaunchKernelGGL(copy_wmin_kernel, dim3(grid_for(n)), dim3(256), 0, stream, c.vid,
                       out_wmin, n, c.out_wmin);
  return hipGetLastError();
}

// ------------------------------------------------- COO <-> edge-id order
// out[k] = in[perm[k]] (gather into edge-id order) or out[perm[k]] = in[k]
// (scatter into COO order): consecutive k read perm and one side
// coalesced; the other side follows the permutation.
__global__ void permute_edges_kernel(const int32_t *perm, int64_t m, const int32_t *in,
                                     int32_t *out, bool to_coo) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride) {
    const int32_t p = perm[k];
    if (to_coo) out[p] = in[k];
    else out[k] = in[p];
  }
}

hipError_t launch_permute_edges(const int32_t *perm, int64_t m, const int32_t *in, int32_t *out,
                                bool to_coo, hipStream_t stream) {
  hipLaunchKernelGGL(permute_edges_kernel, dim3(grid_for(m)), dim3(256), 0, stream, perm, m, in,
                     out, to_coo);
  return hipGetLastError();
}

}  // namespace sssp
