// Host runtime behind the C ABI in include/sssp.h: argument checks, the
// per-device workspace cache, launch geometry, and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sssp.h"
#include "sssp_kernels.h"

using namespace sssp;

namespace {

enum Slot {
  S_C, S_C1, S_ARRIVE, S_MTMP, S_OV0, S_OP0, S_OI0, S_OV1, S_OP1, S_OI1, S_FV, S_FP, S_FI, S_CTL,
  S_IMIN, S_ITHR, S_IROUNDS, S_ISCAN, S_DEGEN, S_LVL, S_FLAG, S_SPRED, S_ISTAT,
  S_GTAB, S_ITAB,
  S_BK_KA, S_BK_KB, S_BK_VA, S_BK_VB, S_BK_HIST, S_BK_TAIL, S_BK_STATUS,
  S_BW_ACC, S_BW_LV, S_BW_LI, S_BW_LOFF, S_BW_CTL, S_BW_GOFF, S_BW_GINST, S_BW_EBASE,
  S_BW_CS, S_BW_LACC,
  S_TRACE, S_FLAGS, S_PART, S_D64, S_FX, S_OX0, S_OX1, S_LV0, S_LV1, S_DR, S_INSTOF, S_IDEAD,
  NSLOTS
};

struct DevWS {
  bool init = false;
  void *buf[NSLOTS] = {};
  size_t cap[NSLOTS] = {};
  int cus = 0;
  int bpc[4] = {0, 0, 0, 0};  // blocks per CU of the round kernel per (f32, batch)
  void *pinned = nullptr;     // host staging for tables and stats
  size_t pinned_cap = 0;
  hipEvent_t last = nullptr;  // completion of the previous call's work
  hipEvent_t staged = nullptr;
  sssp_launch cfg = {0, 0, 0, 0, 0};  // default geometry of direct solves (sssp_set_launch)
};

std::mutex g_mu;
DevWS g_ws[64];
int32_t g_round_limit = 0;  // sssp_set_round_limit: 0 is none

// The watchdog's limit for a solve whose largest instance has n vertices:
// n + 1 (rounds never exceed the reachable count), or a lower limit set for
// diagnostics.
int32_t round_limit(int32_t n) {
  const int32_t lim = n + 1;
  return (g_round_limit > 0 && g_round_limit < lim) ? g_round_limit : lim;
}

struct Guard {
  std::lock_guard<std::mutex> lk;
  Guard() : lk(g_mu) {}
};

sssp_status hip_status(hipError_t e) {
  if (e == hipSuccess) return SSSP_OK;
  if (e == hipErrorOutOfMemory) return SSSP_ERR_NOMEM;
  return SSSP_ERR_HIP;
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t _e = (x);                            \
    if (_e != hipSuccess) return hip_status(_e);    \
  } while (0)

sssp_status ws_get(DevWS &w, int slot, size_t bytes, void **out) {
  if (bytes == 0) bytes = 256;
  if (w.cap[slot] < bytes) {
    if (w.buf[slot]) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipFree(w.buf[slot]));
      w.buf[slot] = nullptr;
      w.cap[slot] = 0;
    }
    size_t want = bytes + bytes / 8;  // headroom against repeated growth
    if (hipMalloc(&w.buf[slot], want) != hipSuccess) {
      (void)hipGetLastError();
      w.buf[slot] = nullptr;
      return SSSP_ERR_NOMEM;
    }
    w.cap[slot] = want;
  }
  *out = w.buf[slot];
  return SSSP_OK;
}

template <class T>
sssp_status ws_arr(DevWS &w, int slot, size_t count, T **out) {
  void *p = nullptr;
  sssp_status s = ws_get(w, slot, count * sizeof(T), &p);
  *out = (T *)p;
  return s;
}

sssp_status pinned_get(DevWS &w, size_t bytes, void **out) {
  // the previous call's host->device table copy must have consumed the buffer
  if (w.staged) HIPCHK(hipEventSynchronize(w.staged));
  if (w.pinned_cap < bytes) {
    if (w.pinned) HIPCHK(hipHostFree(w.pinned));
    w.pinned = nullptr;
    w.pinned_cap = 0;
    if (hipHostMalloc(&w.pinned, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      w.pinned = nullptr;
      return SSSP_ERR_NOMEM;
    }
    w.pinned_cap = bytes;
  }
  *out = w.pinned;
  return SSSP_OK;
}

sssp_status ws_for_current(DevWS **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SSSP_ERR_ARG;
  DevWS &w = g_ws[dev];
  if (!w.init) {
    HIPCHK(hipDeviceGetAttribute(&w.cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipEventCreateWithFlags(&w.last, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&w.staged, hipEventDisableTiming));
    w.init = true;
  }
  *out = &w;
  return SSSP_OK;
}

int env_flag(const char *name, int dflt) {
  const char *s = getenv(name);
  return s ? atoi(s) : dflt;
}

// Persistent grid: co-resident blocks, capped at SSSP_BLOCKS_PER_CU (default 2).
sssp_status geometry(DevWS &w, bool f32, bool batch, LaunchGeom *geo) {
  const int k = (f32 ? 1 : 0) + (batch ? 2 : 0);
  if (w.bpc[k] == 0) {
    int occ = 0;
    HIPCHK(round_kernel_occupancy(f32, batch, &occ));
    int cap = 2;
    if (const char *s = getenv("SSSP_BLOCKS_PER_CU")) {
      int v = atoi(s);
      if (v >= 1 && v <= 16) cap = v;
    }
    w.bpc[k] = occ < cap ? occ : cap;
    if (w.bpc[k] < 1) return SSSP_ERR_HIP;
  }
  geo->blocks = w.cus * w.bpc[k];
  geo->cus = w.cus;
  return SSSP_OK;
}

// The round kernel's geometry under `L` (null or zero fields: defaults;
// the environment variables SSSP_SOLO_EDGES and SSSP_BLOCK_UNITS override
// the defaults for measurement).
// low_spread: every graph of the launch has low degree spread (the default
// condition of the one-workgroup-per-instance path, which also needs C
// scope OPEN: checked per launch).
sssp_status resolve_launch(DevWS &w, bool f32, bool batch, const sssp_launch *L,
                           LaunchGeom *geo, RoundArgs &a, bool low_spread = false) {
  sssp_status s;
  if ((s = geometry(w, f32, batch, geo))) return s;
  if (L && L->blocks) {
    if (L->blocks < 1 || L->blocks > geo->blocks) return SSSP_ERR_ARG;
    geo->blocks = L->blocks;
  }
  a.solo_edges = env_flag("SSSP_SOLO_EDGES", 8192);
  if (L && L->solo_edges) a.solo_edges = L->solo_edges < 0 ? 0 : L->solo_edges;
  a.block_units = env_flag("SSSP_BLOCK_UNITS", 2048);
  if (L && L->block_units) {
    if (L->block_units < 0) return SSSP_ERR_ARG;
    a.block_units = L->block_units;
  }
  geo->small_n = kSmallN;
  if (L && L->small_n) geo->small_n = L->small_n < 0 ? 0 : (L->small_n < kSmallN ? L->small_n : kSmallN);
  const int wg = L ? L->wg : 0;
  geo->wg = wg > 0 || (wg == 0 && low_spread) ? 1 : 0;
  return SSSP_OK;
}

bool csr_ok(const sssp_csr *g) {
  if (!(g && g->n > 0 && g->m >= 0 && (g->dtype == SSSP_I32 || g->dtype == SSSP_F32) &&
        g->scope >= SSSP_SCOPE_AUTO && g->scope <= SSSP_SCOPE_ALL &&
        g->relax >= SSSP_RELAX_AUTO && g->relax <= SSSP_RELAX_CORRECTING && g->delta >= 0 &&
        g->delta <= (g->dtype == SSSP_F32 ? 0x7f800000 : 0x7fffffff) &&
        g->out_off && g->in_off && g->out_wmin && g->s_out_off && g->s_in_off &&
        g->s_out_wmin && g->s_vrec && g->s_vin &&
        (g->m == 0 || (g->out_dst && g->out_w && g->in_src && g->in_eid && g->in_w &&
                       g->s_out_dst && g->s_out_w && g->s_in_src && g->s_in_eid && g->s_in_w &&
                       g->s_in_sw && g->s_out_rec))))
    return false;
  if (g->order == SSSP_ORDER_INPUT) return true;
  return g->order == SSSP_ORDER_DEGREE && g->vid && g->rank && (g->m == 0 || g->s_out_eid);
}

// The C scope a graph's solves use (SSSP_SCOPE_AUTO: ALL when the largest
// total degree is at least 3m/n).
// Low degree spread: the largest total degree below 3m/n (meshes, grids:
// many small rounds).
bool low_spread(const sssp_csr *g) {
  return g->m > 0 && (int64_t)g->deg_max * g->n < 3 * (int64_t)g->m;
}

bool scope_all_of(const sssp_csr *g) {
  if (g->scope == SSSP_SCOPE_AUTO) return g->m > 0 && !low_spread(g);
  return g->scope == SSSP_SCOPE_ALL;
}

// SSSP_RELAX_AUTO: label-correcting relax in buckets of 0.4 w_max on graphs
// of low degree spread (largest total degree below 3m/n: the AUTO scope's
// OPEN case) whose weights spread widely (w_max >= 16 w_min), label-setting
// otherwise.  Measured on grids: weights in [1, 1000] (the threshold rule
// fixes few vertices per round there) take 26 % fewer rounds and 21 % less
// time at 0.1 % more relaxed edges; weights in [0.5, 1.5] gain nothing.
bool auto_correcting(const sssp_csr *g) { return low_spread(g) && g->w_max >= 16.0 * g->w_min; }

// The relax step a graph's solves use.
bool relax_correcting(const sssp_csr *g) {
  if (g->relax == SSSP_RELAX_AUTO) return auto_correcting(g);
  return g->relax == SSSP_RELAX_CORRECTING;
}

// The bucket width (a key) of a graph's label-correcting relax.
int32_t relax_delta(const sssp_csr *g) {
  if (g->relax != SSSP_RELAX_AUTO) return g->delta;
  if (g->dtype == SSSP_F32) {
    const float d = (float)(0.4 * g->w_max);
    int32_t k;
    memcpy(&k, &d, sizeof(k));
    return k;
  }
  const int32_t d = (int32_t)(0.4 * g->w_max);
  return d > 1 ? d : 1;
}

// A weight key as the value it encodes.
double key_value(int32_t key, bool f32) {
  if (!f32) return (double)key;
  float f;
  memcpy(&f, &key, sizeof(f));
  return (double)f;
}

bool overflow_risk(const sssp_csr *g) {
  if (g->dtype != SSSP_I32) return false;
  return (double)(g->n - 1) * g->w_max >= (double)INT_MAX;
}

// Device view of a built graph: the working copy for the rounds, the
// caller-numbered arrays for the parent tie pass and the backward pass.
GraphDev graph_dev(const sssp_csr *g) {
  GraphDev d;
  d.out_off = g->s_out_off;
  d.out_dst = g->s_out_dst;
  d.out_w = (const int32_t *)g->s_out_w;
  d.out_eid = g->s_out_eid;
  d.in_off = g->s_in_off;
  d.in_src = g->s_in_src;
  d.in_w = (const int32_t *)g->s_in_w;
  d.in_sw = (const int2 *)g->s_in_sw;
  d.out_rec = (const int4 *)g->s_out_rec;
  d.vin = (const int4 *)g->s_vin;
  d.out_wmin = (const int32_t *)g->s_out_wmin;
  d.vrec = (const int4 *)g->s_vrec;
  d.vid = g->vid;
  d.rank = g->rank;
  d.u_out_off = g->out_off;
  d.u_out_dst = g->out_dst;
  d.u_in_off = g->in_off;
  d.u_in_src = g->in_src;
  d.u_in_eid = g->in_eid;
  d.u_in_w = (const int32_t *)g->in_w;
  d.n = g->n;
  d.m = g->m;
  d.lc = relax_correcting(g) ? 1 : 0;
  d.delta = relax_delta(g);
  d.all = scope_all_of(g) ? 1 : 0;
  return d;
}

// Build buffer: the caller-numbered CSR/CSC, the working copy's
// weight-ordered in-lists, then (degree order) the renumbered CSR.
enum BufArr {
  B_OUT_OFF, B_OUT_DST, B_OUT_W, B_IN_OFF, B_IN_SRC, B_IN_EID, B_IN_W, B_OUT_WMIN,
  B_S_IN_OFF, B_S_IN_SRC, B_S_IN_EID, B_S_IN_W, B_S_VREC, B_S_IN_SW, B_S_OUT_REC, B_S_VIN,
  B_VID, B_RANK, B_S_OUT_OFF, B_S_OUT_DST, B_S_OUT_W, B_S_OUT_EID, B_S_OUT_WMIN, B_COUNT
};

struct Layout {
  size_t off[B_COUNT];
  size_t total;
};

Layout build_layout(int32_t n, int32_t m, bool renumber) {
  Layout L;
  size_t o = 0;
  const size_t N = (size_t)n, M = (size_t)m;
  const size_t count[B_COUNT] = {N + 1, M, M, N + 1, M, M, M, N, N + 1, M, M, M, 8 * N, 2 * M,
                                 4 * M, 4 * N, N, N, N + 1, M, M, M, N};
  const int narr = renumber ? B_COUNT : B_VID;
  for (int i = 0; i < B_COUNT; ++i) {
    L.off[i] = o;
    if (i < narr) o += (sizeof(int32_t) * count[i] + 255) & ~(size_t)255;
  }
  L.total = o;
  return L;
}

// the working copy's arrays as recorded in a built graph
SolverCopy solver_copy(const sssp_csr *g) {
  SolverCopy c;
  c.vid = (int32_t *)g->vid;
  c.rank = (int32_t *)g->rank;
  c.out_off = (int32_t *)g->s_out_off;
  c.out_dst = (int32_t *)g->s_out_dst;
  c.out_w = (int32_t *)g->s_out_w;
  c.out_eid = (int32_t *)g->s_out_eid;
  c.in_off = (int32_t *)g->s_in_off;
  c.in_src = (int32_t *)g->s_in_src;
  c.in_eid = (int32_t *)g->s_in_eid;
  c.in_w = (int32_t *)g->s_in_w;
  c.in_sw = (int32_t *)g->s_in_sw;
  c.out_rec = (int32_t *)g->s_out_rec;
  c.vin = (int32_t *)g->s_vin;
  c.out_wmin = (int32_t *)g->s_out_wmin;
  c.vrec = (int32_t *)g->s_vrec;
  return c;
}

// Sort temporaries of the builder for n vertices and m edges.
sssp_status build_temps(DevWS &ws, int32_t n, int32_t m, BuildTemps *t) {
  sssp_status s;
  const size_t M = (size_t)(m > n ? m : n);
  if ((s = ws_arr(ws, S_BK_KA, M, &t->ka))) return s;
  if ((s = ws_arr(ws, S_BK_KB, M, &t->kb))) return s;
  if ((s = ws_arr(ws, S_BK_VA, M, &t->va))) return s;
  if ((s = ws_arr(ws, S_BK_VB, M, &t->vb))) return s;
  if ((s = ws_arr(ws, S_BK_TAIL, (size_t)(m > 0 ? m : 1), &t->tail))) return s;
  if ((s = ws_arr(ws, S_BK_HIST, build_hist_entries(m > n ? m : n), &t->hist))) return s;
  if ((s = ws_arr(ws, S_BK_STATUS, 4, &t->status))) return s;
  return SSSP_OK;
}

// Where a solve's state arrays come from: the per-device workspace cache
// (slots grown on demand) ...
struct WsAlloc {
  DevWS &w;
  template <class T>
  sssp_status operator()(int slot, size_t count, T **out) {
    return ws_arr(w, slot, count, out);
  }
};

// ... or consecutive 256-byte-aligned pieces of one fixed region (the
// static scratch of sssp_solve_noalloc); a region too small is
// SSSP_ERR_CAPACITY.  With base == nullptr it only measures.
struct CarveAlloc {
  char *base;
  size_t cap;
  size_t used = 0;
  template <class T>
  sssp_status operator()(int, size_t count, T **out) {
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    const size_t off = (used + 255) & ~(size_t)255;
    if (off > cap || bytes > cap - off) return SSSP_ERR_CAPACITY;
    *out = base ? (T *)(base + off) : nullptr;
    used = off + bytes;
    return SSSP_OK;
  }
};

// Round-state arrays for `total` state entries.
template <class Alloc>
sssp_status state_arrays(Alloc &al, int32_t total, int32_t num_inst, bool batch,
                         RoundArgs &a) {
  const size_t T = (size_t)total;
  sssp_status s;
  if ((s = al(S_D64, T, &a.D64))) return s;
  if ((s = al(S_C, T, &a.C0))) return s;
  if ((s = al(S_C1, T, &a.C1))) return s;
  if ((s = al(S_ARRIVE, T, &a.arrive))) return s;
  if ((s = al(S_MTMP, T, &a.mtmp))) return s;
  if ((s = al(S_OV0, T, &a.open_v0))) return s;
  if ((s = al(S_OP0, T, &a.open_p0))) return s;
  if ((s = al(S_OV1, T, &a.open_v1))) return s;
  if ((s = al(S_OP1, T, &a.open_p1))) return s;
  if ((s = al(S_FV, T, &a.front_v))) return s;
  if ((s = al(S_FP, T, &a.front_p))) return s;
  {
    // list payload words: kFX per frontier entry, kOXMem per open entry and parity
    int32_t *fx, *ox0, *ox1;
    if ((s = al(S_FX, kFX * T, &fx))) return s;
    if ((s = al(S_OX0, kOXMem * T, &ox0))) return s;
    if ((s = al(S_OX1, kOXMem * T, &ox1))) return s;
    for (int k = 0; k < kFX; ++k) a.front_x[k] = fx + (size_t)k * T;
    for (int k = 0; k < kOX; ++k) {
      a.open_x0[k] = ox0 + (size_t)k * T;
      a.open_x1[k] = ox1 + (size_t)k * T;
    }
  }
  if ((s = al(S_CTL, 1, &a.ctl))) return s;
  if ((s = al(S_FLAGS, (size_t)kMaxBlocks * kFlagStride, &a.flags))) return s;
  if ((s = al(S_PART, (size_t)kParts * kMaxBlocks, &a.part))) return s;
  if ((s = al(S_DEGEN, 2 * T, &a.degen))) return s;
  if ((s = al(S_LVL, T, &a.lvl))) return s;
  if ((s = al(S_FLAG, T, &a.flag))) return s;
  if (a.scope_all) {
    if ((s = al(S_LV0, T, &a.live_v0))) return s;
    if ((s = al(S_LV1, T, &a.live_v1))) return s;
    if (batch) {
      if ((s = al(S_INSTOF, T, &a.inst_of))) return s;
      if ((s = al(S_IDEAD, 2 * (size_t)num_inst, &a.idead))) return s;
    }
  }
  if (a.any_lc && (s = al(S_DR, T, &a.DR))) return s;
  if (batch) {
    if ((s = al(S_OI0, T, &a.open_i0))) return s;
    if ((s = al(S_OI1, T, &a.open_i1))) return s;
    if ((s = al(S_FI, T, &a.front_i))) return s;
    if ((s = al(S_IMIN, 3 * (size_t)num_inst, &a.imin))) return s;
    if ((s = al(S_ITHR, 3 * (size_t)num_inst, &a.ithr))) return s;
    if ((s = al(S_IROUNDS, (size_t)num_inst, &a.irounds))) return s;
    if ((s = al(S_ISCAN, 3 * (size_t)num_inst, &a.iscanned))) return s;
  }
  return SSSP_OK;
}

sssp_status state_buffers(DevWS &w, int32_t total, int32_t num_inst, bool batch,
                          RoundArgs &a) {
  WsAlloc al{w};
  return state_arrays(al, total, num_inst, batch, a);
}

// Round trace: with SSSP_TRACE=<path> in the environment, a solve records
// per-round timestamps and list sizes on the device and, after the kernel,
// appends them as CSV lines to <path> (synchronizes the stream).
constexpr int kTraceRounds = 100000;
constexpr int kTraceBlkRounds = 64;  // rounds with per-block phase end times

sssp_status trace_begin(DevWS &w, RoundArgs &a, hipStream_t stream) {
  if (!getenv("SSSP_TRACE")) return SSSP_OK;
  sssp_status s;
  const size_t cnt = (size_t)kTraceRounds * kTraceFields;
  const size_t bcnt = (size_t)kTraceBlkRounds * 2 * kMaxBlocks * kBlkFields;
  const size_t mcnt = (size_t)kTraceRounds * 2 * kMarks;
  if ((s = ws_arr(w, S_TRACE, cnt + bcnt + mcnt, &a.trace))) return s;
  a.trace_rounds = kTraceRounds;
  a.trace_blk = a.trace + cnt;
  a.trace_blk_rounds = kTraceBlkRounds;
  a.marks = a.trace + cnt + bcnt;
  a.mark_rounds = kTraceRounds;
  a.mark_block = env_flag("SSSP_MARK_BLOCK", 0);
  HIPCHK(hipMemsetAsync(a.trace, 0, (cnt + bcnt + mcnt) * sizeof(long long), stream));
  return SSSP_OK;
}

sssp_status trace_end(const RoundArgs &a, int nblocks, hipStream_t stream) {
  const char *path = getenv("SSSP_TRACE");
  if (!path || !a.trace) return SSSP_OK;
  Ctl c;
  HIPCHK(hipStreamSynchronize(stream));
  HIPCHK(hipMemcpy(&c, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  const int nr = c.rounds < kTraceRounds ? c.rounds : kTraceRounds;
  std::vector<long long> h((size_t)nr * kTraceFields);
  HIPCHK(hipMemcpy(h.data(), a.trace, h.size() * sizeof(long long), hipMemcpyDeviceToHost));
  FILE *f = fopen(path, "a");
  if (!f) return SSSP_ERR_ARG;
  fprintf(f, "round,start,arr_relax,end_relax,arr_fused,end_fused,nf,ef,no,eo,mode,nl\n");
  for (int r = 0; r < nr; ++r) {
    fprintf(f, "%d", r + 1);
    for (int k = 0; k < kTraceFields; ++k) fprintf(f, ",%lld", h[(size_t)r * kTraceFields + k]);
    fprintf(f, "\n");
  }
  fclose(f);
  // checkpoints: <path>.marks, one line per (round, phase): round,phase,m0..
  {
    std::vector<long long> hm((size_t)nr * 2 * kMarks);
    HIPCHK(hipMemcpy(hm.data(), a.marks, hm.size() * sizeof(long long),
                     hipMemcpyDeviceToHost));
    std::string mp = std::string(path) + ".marks";
    FILE *fm = fopen(mp.c_str(), "a");
    if (!fm) return SSSP_ERR_ARG;
    for (int r = 0; r < nr; ++r)
      for (int ph = 0; ph < 2; ++ph) {
        fprintf(fm, "%d,%d", r + 1, ph);
        for (int k = 0; k < kMarks; ++k)
          fprintf(fm, ",%lld", hm[((size_t)r * 2 + ph) * kMarks + k]);
        fprintf(fm, "\n");
      }
    fclose(fm);
  }
  // per-block records: <path>.blk, one line per (round, phase, block):
  // round,phase,block,end,windows,first_item,units,mid
  const int nbr = nr < kTraceBlkRounds ? nr : kTraceBlkRounds;
  std::vector<long long> hb((size_t)nbr * 2 * kMaxBlocks * kBlkFields);
  HIPCHK(hipMemcpy(hb.data(), a.trace_blk, hb.size() * sizeof(long long),
                   hipMemcpyDeviceToHost));
  std::string bp = std::string(path) + ".blk";
  f = fopen(bp.c_str(), "a");
  if (!f) return SSSP_ERR_ARG;
  for (int r = 0; r < nbr; ++r)
    for (int ph = 0; ph < 2; ++ph)
      for (int b = 0; b < nblocks; ++b) {
        const long long *e = &hb[(((size_t)r * 2 + ph) * kMaxBlocks + b) * kBlkFields];
        fprintf(f, "%d,%d,%d,%lld,%lld,%lld,%lld,%lld\n", r + 1, ph, b, e[0], e[1], e[2], e[3],
                e[4]);
      }
  fclose(f);
  return SSSP_OK;
}

// Event pairs bracketing round-kernel launches while profiling is enabled.
struct Profiler {
  bool on = false;
  std::vector<KernelTimer> pool;
  size_t used = 0;
};
Profiler g_prof;

const KernelTimer *prof_timer(KernelTimer *out) {
  if (!g_prof.on) return nullptr;
  if (g_prof.used == g_prof.pool.size()) {
    if (g_prof.pool.size() >= 4096) return nullptr;
    KernelTimer t;
    if (hipEventCreate(&t.start) != hipSuccess) return nullptr;
    if (hipEventCreate(&t.stop) != hipSuccess) return nullptr;
    g_prof.pool.push_back(t);
  }
  *out = g_prof.pool[g_prof.used++];
  return out;
}

}  // namespace

extern "C" {

sssp_status sssp_profile_enable(int on) {
  Guard guard;
  g_prof.on = on != 0;
  return SSSP_OK;
}

sssp_status sssp_profile_read(int64_t *launches, double *total_ms) {
  if (!launches || !total_ms) return SSSP_ERR_ARG;
  Guard guard;
  double tot = 0.0;
  for (size_t i = 0; i < g_prof.used; ++i) {
    HIPCHK(hipEventSynchronize(g_prof.pool[i].stop));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, g_prof.pool[i].start, g_prof.pool[i].stop));
    tot += ms;
  }
  *launches = (int64_t)g_prof.used;
  *total_ms = tot;
  g_prof.used = 0;
  return SSSP_OK;
}


const char *sssp_strerror(sssp_status st) {
  switch (st) {
    case SSSP_OK: return "ok";
    case SSSP_ERR_ARG: return "invalid argument";
    case SSSP_ERR_GRAPH: return "edge endpoint out of range";
    case SSSP_ERR_WEIGHT: return "weight not strictly positive and finite";
    case SSSP_ERR_OVERFLOW: return "int32 path costs could reach INT32_MAX ((n-1)*w_max too large)";
    case SSSP_ERR_NOMEM: return "device workspace allocation failed";
    case SSSP_ERR_HIP: return "HIP runtime error";
    case SSSP_ERR_INTERNAL: return "internal error (round watchdog)";
    case SSSP_ERR_CAPACITY: return "graph too large for the static scratch of sssp_solve_noalloc";
  }
  return "unknown status";
}

size_t sssp_build_csr_bytes(int32_t n, int32_t m, sssp_dtype dtype, sssp_order order) {
  if (n <= 0 || m < 0 || (dtype != SSSP_I32 && dtype != SSSP_F32)) return 0;
  if (order != SSSP_ORDER_AUTO && order != SSSP_ORDER_INPUT && order != SSSP_ORDER_DEGREE)
    return 0;
  return build_layout(n, m, order != SSSP_ORDER_INPUT).total;
}

sssp_status sssp_build_csr(int32_t n, int32_t m, sssp_dtype dtype, sssp_order order,
                           const int32_t *src, const int32_t *dst, const void *w, void *buffer,
                           size_t buffer_bytes, sssp_csr *out, int32_t *perm, void *stream_) {
  if (n <= 0 || m < 0 || (dtype != SSSP_I32 && dtype != SSSP_F32) || !out || !buffer)
    return SSSP_ERR_ARG;
  if (order != SSSP_ORDER_AUTO && order != SSSP_ORDER_INPUT && order != SSSP_ORDER_DEGREE)
    return SSSP_ERR_ARG;
  if (m > 0 && (!src || !dst || !w)) return SSSP_ERR_ARG;
  const Layout L = build_layout(n, m, order != SSSP_ORDER_INPUT);
  if (buffer_bytes < L.total) return SSSP_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_;
  const bool f32 = dtype == SSSP_F32;
  Guard guard;
  DevWS *wp;
  sssp_status s;
  if ((s = ws_for_current(&wp))) return s;
  DevWS &ws = *wp;
  HIPCHK(hipStreamWaitEvent(stream, ws.last, 0));
  char *b = (char *)buffer;
  auto arr = [&](int i) { return (int32_t *)(b + L.off[i]); };
  int32_t *out_off = arr(B_OUT_OFF), *out_dst = arr(B_OUT_DST), *out_w = arr(B_OUT_W);
  int32_t *in_off = arr(B_IN_OFF), *in_src = arr(B_IN_SRC), *in_eid = arr(B_IN_EID);
  int32_t *in_w = arr(B_IN_W), *out_wmin = arr(B_OUT_WMIN);
  BuildTemps t;
  if ((s = build_temps(ws, n, m, &t))) return s;
  HIPCHK(hipMemsetAsync(t.status, 0, 4 * sizeof(int32_t), stream));
  HIPCHK(launch_validate(n, m, f32, src, dst, (const int32_t *)w, t.status, stream));
  int32_t hs[4];
  HIPCHK(hipMemcpyAsync(hs, t.status, sizeof(hs), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (hs[0] & 1) return SSSP_ERR_GRAPH;
  if (hs[0] & 2) return SSSP_ERR_WEIGHT;
  const int32_t wkey_max = hs[1];
  memset(out, 0, sizeof(*out));
  out->n = n;
  out->m = m;
  out->dtype = dtype;
  out->order = SSSP_ORDER_INPUT;
  out->scope = SSSP_SCOPE_AUTO;
  out->relax = SSSP_RELAX_AUTO;
  out->deg_max = 0;
  out->delta = dtype == SSSP_F32 ? 0x7f800000 : 0x7fffffff;  // no bucket bound
  out->out_off = out_off;
  out->out_dst = out_dst;
  out->out_w = out_w;
  out->in_off = in_off;
  out->in_src = in_src;
  out->in_eid = in_eid;
  out->in_w = in_w;
  out->out_wmin = out_wmin;
  out->w_max = key_value(wkey_max, f32);
  out->w_min = m > 0 ? key_value(0x7fffffff - hs[3], f32) : 0.0;
  if (overflow_risk(out)) return SSSP_ERR_OVERFLOW;
  HIPCHK(launch_build(n, m, f32, src, dst, (const int32_t *)w, out_off, out_dst, out_w, in_off,
                      in_src, in_eid, in_w, out_wmin, perm, t, stream));
  SolverCopy c;
  memset(&c, 0, sizeof(c));
  c.out_off = out_off;
  c.out_dst = out_dst;
  c.out_w = out_w;
  c.out_wmin = out_wmin;
  c.in_off = arr(B_S_IN_OFF);
  c.in_src = arr(B_S_IN_SRC);
  c.in_eid = arr(B_S_IN_EID);
  c.in_w = arr(B_S_IN_W);
  c.in_sw = arr(B_S_IN_SW);
  c.out_rec = arr(B_S_OUT_REC);
  c.vin = arr(B_S_VIN);
  c.vrec = arr(B_S_VREC);
  if (m > 0) {
    HIPCHK(launch_degree(n, out_off, in_off, t, stream));
    HIPCHK(hipMemcpyAsync(hs, t.status, sizeof(hs), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    out->deg_max = hs[2];
  }
  if (order != SSSP_ORDER_INPUT && m > 0) {
    const int32_t dmax = out->deg_max;
    // skewed: largest total degree >= 16 x the mean 2m/n
    const bool skewed = (int64_t)dmax * n >= 32 * (int64_t)m;
    if (order == SSSP_ORDER_DEGREE || skewed) {
      c.vid = arr(B_VID);
      c.rank = arr(B_RANK);
      c.out_off = arr(B_S_OUT_OFF);
      c.out_dst = arr(B_S_OUT_DST);
      c.out_w = arr(B_S_OUT_W);
      c.out_eid = arr(B_S_OUT_EID);
      c.out_wmin = arr(B_S_OUT_WMIN);
      HIPCHK(launch_renumber(n, m, dmax, out_dst, out_w, out_wmin, c, t, stream));
      out->order = SSSP_ORDER_DEGREE;
    }
  }
  HIPCHK(launch_in_lists(n, m, wkey_max, out_off, out_dst, out_w, c, t, stream));
  HIPCHK(launch_vrec(n, c, stream));
  HIPCHK(launch_out_rec(m, c, stream));
  out->s_vrec = c.vrec;
  out->vid = c.vid;
  out->rank = c.rank;
  out->s_out_off = c.out_off;
  out->s_out_dst = c.out_dst;
  out->s_out_w = c.out_w;
  out->s_out_eid = c.out_eid;
  out->s_in_off = c.in_off;
  out->s_in_src = c.in_src;
  out->s_in_eid = c.in_eid;
  out->s_in_w = c.in_w;
  out->s_in_sw = c.in_sw;
  out->s_out_rec = c.out_rec;
  out->s_vin = c.vin;
  out->s_out_wmin = c.out_wmin;
  HIPCHK(hipStreamSynchronize(stream));
  HIPCHK(hipEventRecord(ws.last, stream));
  return SSSP_OK;
}

sssp_status sssp_permute_edges(const int32_t *perm, int64_t m, const void *in, void *out,
                               int32_t to_coo, void *stream_) {
  if (m < 0) return SSSP_ERR_ARG;
  if (m == 0) return SSSP_OK;
  if (!perm || !in || !out || in == out) return SSSP_ERR_ARG;
  Guard guard;
  HIPCHK(launch_permute_edges(perm, m, (const int32_t *)in, (int32_t *)out, to_coo != 0,
                              (hipStream_t)stream_));
  return SSSP_OK;
}

sssp_status sssp_set_weights(sssp_csr *g, const void *w, void *stream_) {
  if (!csr_ok(g) || (g->m > 0 && !w)) return SSSP_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_;
  const bool f32 = g->dtype == SSSP_F32;
  Guard guard;
  DevWS *wp;
  sssp_status s;
  if ((s = ws_for_current(&wp))) return s;
  DevWS &ws = *wp;
  HIPCHK(hipStreamWaitEvent(stream, ws.last, 0));
  BuildTemps t;
  if ((s = build_temps(ws, g->n, g->m, &t))) return s;
  // validate before anything is written: on error the graph is unchanged
  HIPCHK(hipMemsetAsync(t.status, 0, 4 * sizeof(int32_t), stream));
  HIPCHK(launch_validate(g->n, g->m, f32, nullptr, nullptr, (const int32_t *)w, t.status,
                         stream));
  int32_t hs[4];
  HIPCHK(hipMemcpyAsync(hs, t.status, sizeof(hs), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (hs[0] & 2) {
    HIPCHK(hipEventRecord(ws.last, stream));
    return SSSP_ERR_WEIGHT;
  }
  const double w_max = key_value(hs[1], f32);
  const double w_min = g->m > 0 ? key_value(0x7fffffff - hs[3], f32) : 0.0;
  if (g->dtype == SSSP_I32 && (double)(g->n - 1) * w_max >= (double)INT_MAX) {
    HIPCHK(hipEventRecord(ws.last, stream));
    return SSSP_ERR_OVERFLOW;
  }
  const SolverCopy c = solver_copy(g);
  HIPCHK(launch_set_weights(g->n, g->m, f32, (const int32_t *)w, g->out_off, g->in_eid,
                            (int32_t *)g->out_w, (int32_t *)g->in_w, (int32_t *)g->out_wmin, c,
                            stream));
  HIPCHK(launch_in_lists(g->n, g->m, hs[1], g->out_off, g->out_dst, (const int32_t *)g->out_w,
                         c, t, stream));
  HIPCHK(launch_vrec(g->n, c, stream));  // out_wmin and the in-list heads changed
  HIPCHK(launch_out_rec(g->m, c, stream));  // the weights and the heads' out_wmin
  HIPCHK(hipStreamSynchronize(stream));
  HIPCHK(hipEventRecord(ws.last, stream));
  g->w_max = w_max;
  g->w_min = w_min;
  return SSSP_OK;
}

}  // extern "C"

// Round arguments of one solve from `source` (target >= 0: stop once the
// target is fixed) into `cost`, with its state buffers.
static void single_fill(const sssp_csr *g, int32_t source, int32_t target, void *cost,
                        RoundArgs &a) {
  memset(&a, 0, sizeof(a));
  a.g = graph_dev(g);
  a.num_inst = 1;
  a.source = source;
  a.total = g->n;
  a.max_rounds = round_limit(g->n);
  a.D = (int32_t *)cost;
  a.target = target;
  a.scope_all = a.g.all;
  a.any_lc = a.g.lc;
}

static sssp_status single_args(DevWS &ws, const sssp_csr *g, int32_t source, int32_t target,
                               void *cost, RoundArgs &a) {
  single_fill(g, source, target, cost, a);
  return state_buffers(ws, g->n, 1, false, a);
}

static void single_stats(const Ctl *c, sssp_stats *stats) {
  stats->rounds = c->rounds;
  stats->settled = (int32_t)c->settled;
  stats->relaxed_edges = c->relaxed;
  stats->scanned_in_edges = c->scanned;
  stats->open_visits = c->open_visits;
}

// One solve from `source`; with target >= 0 the rounds stop once the target
// is fixed (no parent pointers then).
static sssp_status solve_one(const sssp_csr *g, int32_t source, int32_t target, void *cost,
                             int32_t *pred, sssp_stats *stats, void *stream_) {
  if (!csr_ok(g) || !cost || source < 0 || source >= g->n) return SSSP_ERR_ARG;
  if (target >= g->n || (target >= 0 && pred)) return SSSP_ERR_ARG;
  if (overflow_risk(g)) return SSSP_ERR_OVERFLOW;
  hipStream_t stream = (hipStream_t)stream_;
  const bool f32 = g->dtype == SSSP_F32;
  Guard guard;
  DevWS *wp;
  sssp_status s;
  if ((s = ws_for_current(&wp))) return s;
  DevWS &ws = *wp;
  RoundArgs a;
  if ((s = single_args(ws, g, source, target, cost, a))) return s;
  LaunchGeom geo;
  if ((s = resolve_launch(ws, f32, false, &ws.cfg, &geo, a, low_spread(g)))) return s;
  HIPCHK(hipStreamWaitEvent(stream, ws.last, 0));
  KernelTimer tm;
  const KernelTimer *timer = prof_timer(&tm);
  if ((s = trace_begin(ws, a, stream))) return s;
  Launcher L;
  L.stream = stream;
  HIPCHK(launch_solve(f32, false, a, pred, geo, nullptr, g->n, timer, L));
  if ((s = trace_end(a, geo.blocks, stream))) return s;
  if (stats) {
    void *hp;
    if ((s = pinned_get(ws, sizeof(Ctl), &hp))) return s;
    HIPCHK(hipMemcpyAsync(hp, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    const Ctl *c = (const Ctl *)hp;
    single_stats(c, stats);
    if (c->status) {
      HIPCHK(hipEventRecord(ws.last, stream));
      return SSSP_ERR_INTERNAL;
    }
  }
  HIPCHK(hipEventRecord(ws.last, stream));
  return SSSP_OK;
}

// Host checks of a batch; *total and *max_n receive the number of state
// entries and the largest instance.
static sssp_status check_batch(const sssp_csr *graphs, int32_t num_graphs,
                               const int32_t *inst_graph, const int32_t *inst_source,
                               int32_t num_inst, void *cost, int64_t *total, int32_t *max_n) {
  if (!graphs || num_graphs <= 0 || !inst_graph || !inst_source || num_inst <= 0 || !cost)
    return SSSP_ERR_ARG;
  const int32_t dtype = graphs[0].dtype;
  for (int32_t gi = 0; gi < num_graphs; ++gi) {
    if (!csr_ok(&graphs[gi]) || graphs[gi].dtype != dtype) return SSSP_ERR_ARG;
    if (overflow_risk(&graphs[gi])) return SSSP_ERR_OVERFLOW;
  }
  *total = 0;
  *max_n = 0;
  for (int32_t i = 0; i < num_inst; ++i) {
    const int32_t gi = inst_graph[i];
    if (gi < 0 || gi >= num_graphs) return SSSP_ERR_ARG;
    const int32_t n = graphs[gi].n;
    if (inst_source[i] < 0 || inst_source[i] >= n) return SSSP_ERR_ARG;
    *total += n;
    if (n > *max_n) *max_n = n;
  }
  if (*total >= (int64_t)INT_MAX) return SSSP_ERR_ARG;
  return SSSP_OK;
}

// Whether every graph a batch's instances use has low degree spread.
static bool all_low_spread(const sssp_csr *graphs, const int32_t *inst_graph, int32_t num_inst) {
  for (int32_t i = 0; i < num_inst; ++i)
    if (!low_spread(&graphs[inst_graph[i]])) return false;
  return true;
}

// The host copies of a batch's graph and instance tables.
static void fill_tables(const sssp_csr *graphs, int32_t num_graphs, const int32_t *inst_graph,
                        const int32_t *inst_source, int32_t num_inst, GraphDev *hg,
                        InstDev *hi) {
  for (int32_t gi = 0; gi < num_graphs; ++gi) hg[gi] = graph_dev(&graphs[gi]);
  int32_t base = 0;
  for (int32_t i = 0; i < num_inst; ++i) {
    hi[i].graph = inst_graph[i];
    hi[i].source = inst_source[i];
    hi[i].sbase = base;
    hi[i].n = graphs[inst_graph[i]].n;
    base += hi[i].n;
  }
}

// Round arguments and state buffers of a batch (the tables a.graphs and
// a.insts are allocated, not filled).  stats: count per-instance counters.
static sssp_status batch_args(DevWS &ws, const sssp_csr *graphs, int32_t num_graphs,
                              const int32_t *inst_graph, int32_t num_inst, int64_t total,
                              int32_t max_n, void *cost, int32_t *pred, bool stats,
                              RoundArgs &a) {
  memset(&a, 0, sizeof(a));
  a.num_inst = num_inst;
  a.total = (int32_t)total;
  a.max_rounds = round_limit(max_n);
  a.target = -1;
  a.D = (int32_t *)cost;
  for (int32_t i = 0; i < num_inst; ++i) {
    if (relax_correcting(&graphs[inst_graph[i]])) a.any_lc = 1;
    if (scope_all_of(&graphs[inst_graph[i]])) a.scope_all = 1;
  }
  sssp_status s;
  if ((s = state_buffers(ws, a.total, num_inst, true, a))) return s;
  GraphDev *dg;
  InstDev *di;
  if ((s = ws_arr(ws, S_GTAB, (size_t)num_graphs, &dg))) return s;
  if ((s = ws_arr(ws, S_ITAB, (size_t)num_inst, &di))) return s;
  a.graphs = dg;
  a.insts = di;
  if (stats) {
    if ((s = ws_arr(ws, S_ISTAT, 4 * (size_t)num_inst, &a.istat))) return s;
    if (!pred && (s = ws_arr(ws, S_SPRED, (size_t)a.total, &a.scratch_pred))) return s;
  }
  return SSSP_OK;
}

// Per-instance counters of a finished batch (synchronizes the stream).
static sssp_status batch_stats(const RoundArgs &a, int32_t num_inst, sssp_stats *stats,
                               hipStream_t stream) {
  HIPCHK(hipStreamSynchronize(stream));
  const size_t I = (size_t)num_inst;
  std::vector<long long> st(4 * I);
  std::vector<int32_t> rounds(I);
  std::vector<unsigned long long> sc(3 * I), dd(2 * I, 0ull);
  HIPCHK(hipMemcpy(st.data(), a.istat, sizeof(long long) * 4 * I, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(rounds.data(), a.irounds, sizeof(int32_t) * I, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(sc.data(), a.iscanned, sizeof(unsigned long long) * 3 * I,
                   hipMemcpyDeviceToHost));
  // scope ALL: unreachable vertices dropped from the live list in round
  // r_d are still scanned in every later bound step of their instance
  // (rounds - 1 of them)
  if (a.idead)
    HIPCHK(hipMemcpy(dd.data(), a.idead, sizeof(unsigned long long) * 2 * I,
                     hipMemcpyDeviceToHost));
  Ctl c;
  HIPCHK(hipMemcpy(&c, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < I; ++i) {
    const int32_t r = rounds[i];
    stats[i].rounds = r;
    stats[i].settled = (int32_t)st[4 * i + 1];
    stats[i].relaxed_edges = (int64_t)sc[3 * i + 2];
    stats[i].scanned_in_edges = (int64_t)(sc[3 * i] +
                                          dd[2 * i] * (unsigned long long)(r > 0 ? r - 1 : 0) -
                                          dd[2 * i + 1]);
    stats[i].open_visits = (int64_t)sc[3 * i + 1];
  }
  return c.status ? SSSP_ERR_INTERNAL : SSSP_OK;
}

extern "C" {

sssp_status sssp_solve(const sssp_csr *g, int32_t source, void *cost, int32_t *pred,
                       sssp_stats *stats, void *stream) {
  return solve_one(g, source, -1, cost, pred, stats, stream);
}

// Per-device set-up of sssp_solve_noalloc, done on its first call on a
// device: the static scratch region's address, the CU count and (cached on
// first use) the round kernel's co-residency, so that later calls make no
// allocating runtime call.
struct NoAllocDev {
  bool init = false;
  char *scratch = nullptr;
  int cus = 0;
  int bpc[4] = {0, 0, 0, 0};
};
static NoAllocDev g_na[64];

sssp_status sssp_solve_noalloc(const sssp_csr *g, int32_t source, void *cost, int32_t *pred,
                               sssp_stats *stats, void *stream_) {
  if (!csr_ok(g) || !cost || source < 0 || source >= g->n) return SSSP_ERR_ARG;
  if (overflow_risk(g)) return SSSP_ERR_OVERFLOW;
  hipStream_t stream = (hipStream_t)stream_;
  const bool f32 = g->dtype == SSSP_F32;
  Guard guard;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SSSP_ERR_ARG;
  NoAllocDev &nd = g_na[dev];
  if (!nd.init) {
    void *p = nullptr;
    HIPCHK(scratch_address(&p));
    HIPCHK(hipDeviceGetAttribute(&nd.cus, hipDeviceAttributeMultiprocessorCount, dev));
    nd.scratch = (char *)p;
    nd.init = true;
  }
  RoundArgs a;
  single_fill(g, source, -1, cost, a);
  CarveAlloc al{nd.scratch, kScratchBytes};
  sssp_status s;
  if ((s = state_arrays(al, g->n, 1, false, a))) return s;
  // the device's default geometry (sssp_set_launch), resolved on a stack
  // copy of the set-up values
  DevWS tmp;
  tmp.cus = nd.cus;
  memcpy(tmp.bpc, nd.bpc, sizeof(nd.bpc));
  tmp.cfg = g_ws[dev].cfg;
  LaunchGeom geo;
  if ((s = resolve_launch(tmp, f32, false, &tmp.cfg, &geo, a, low_spread(g)))) return s;
  memcpy(nd.bpc, tmp.bpc, sizeof(nd.bpc));
  Launcher L;
  L.stream = stream;
  HIPCHK(launch_solve(f32, false, a, pred, geo, nullptr, g->n, nullptr, L));
  if (stats) {
    Ctl c;
    HIPCHK(hipMemcpyAsync(&c, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    single_stats(&c, stats);
    if (c.status) return SSSP_ERR_INTERNAL;
  }
  return SSSP_OK;
}

sssp_status sssp_solve_target(const sssp_csr *g, int32_t source, int32_t target, void *cost,
                              sssp_stats *stats, void *stream) {
  if (target < 0) return SSSP_ERR_ARG;
  return solve_one(g, source, target, cost, nullptr, stats, stream);
}

sssp_status sssp_solve_batch(const sssp_csr *graphs, int32_t num_graphs,
                             const int32_t *inst_graph, const int32_t *inst_source,
                             int32_t num_inst, void *cost, int32_t *pred, sssp_stats *stats,
                             void *stream_) {
  int64_t total;
  int32_t max_n;
  sssp_status s;
  if ((s = check_batch(graphs, num_graphs, inst_graph, inst_source, num_inst, cost, &total,
                       &max_n)))
    return s;
  hipStream_t stream = (hipStream_t)stream_;
  const bool f32 = graphs[0].dtype == SSSP_F32;
  Guard guard;
  DevWS *wp;
  if ((s = ws_for_current(&wp))) return s;
  DevWS &ws = *wp;
  RoundArgs a;
  if ((s = batch_args(ws, graphs, num_graphs, inst_graph, num_inst, total, max_n, cost, pred,
                      stats != nullptr, a)))
    return s;
  const size_t tab_bytes = sizeof(GraphDev) * num_graphs + sizeof(InstDev) * num_inst;
  void *hp;
  if ((s = pinned_get(ws, tab_bytes, &hp))) return s;
  GraphDev *hg = (GraphDev *)hp;
  InstDev *hi = (InstDev *)(hg + num_graphs);
  fill_tables(graphs, num_graphs, inst_graph, inst_source, num_inst, hg, hi);
  LaunchGeom geo;
  if ((s = resolve_launch(ws, f32, true, &ws.cfg, &geo, a,
                          all_low_spread(graphs, inst_graph, num_inst))))
    return s;
  HIPCHK(hipStreamWaitEvent(stream, ws.last, 0));
  HIPCHK(hipMemcpyAsync((void *)a.graphs, hg, sizeof(GraphDev) * num_graphs,
                        hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync((void *)a.insts, hi, sizeof(InstDev) * num_inst, hipMemcpyHostToDevice,
                        stream));
  HIPCHK(hipEventRecord(ws.staged, stream));
  KernelTimer tm;
  const KernelTimer *timer = prof_timer(&tm);
  if ((s = trace_begin(ws, a, stream))) return s;
  Launcher L;
  L.stream = stream;
  HIPCHK(launch_solve(f32, true, a, pred, geo, a.istat, max_n, timer, L));
  if ((s = trace_end(a, geo.blocks, stream))) return s;
  if (stats) s = batch_stats(a, num_inst, stats, stream);
  HIPCHK(hipEventRecord(ws.last, stream));
  return s;
}

sssp_status sssp_set_launch(const sssp_launch *launch) {
  Guard guard;
  DevWS *wp;
  sssp_status s;
  if ((s = ws_for_current(&wp))) return s;
  if (!launch) {
    wp->cfg = sssp_launch{0, 0, 0, 0, 0};
    return SSSP_OK;
  }
  // the grid must fit both kernel variants of both dtypes
  for (int k = 0; k < 4; ++k) {
    LaunchGeom geo;
    RoundArgs a;
    if ((s = resolve_launch(*wp, k & 1, (k & 2) != 0, launch, &geo, a))) return s;
  }
  wp->cfg = *launch;
  return SSSP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ plans
struct sssp_plan_s {
  int dev = 0;
  int32_t kind = SSSP_PLAN_BATCH;
  int32_t num_inst = 0;
  bool with_stats = false;
  bool f32 = false;
  DevWS ws;  // the plan's own state (never the shared cache)
  RoundArgs a;                  // batch kind: the solve's arguments
  int32_t *batch_pred = nullptr;  // batch kind: the parent output (nullable)
  std::vector<RoundArgs> seq;   // sequence kind: one per instance
  std::vector<int32_t> seq_n;   // sequence kind: instance sizes
  std::vector<int32_t *> seq_pred;
  std::vector<char> seq_low;    // sequence kind: the instance's graph has low degree spread
  bool low_spread = false;      // batch kind: every graph has
  int32_t max_n = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void ws_free(DevWS &w) {
  for (int i = 0; i < NSLOTS; ++i) {
    if (w.buf[i]) (void)hipFree(w.buf[i]);
    w.buf[i] = nullptr;
    w.cap[i] = 0;
  }
  if (w.pinned) (void)hipHostFree(w.pinned);
  w.pinned = nullptr;
  w.pinned_cap = 0;
}

static void plan_drop_graph(sssp_plan_s *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

// (Re)records the plan's kernels into a new HIP graph under geometry `L`.
static sssp_status plan_record(sssp_plan_s *p, const sssp_launch *L) {
  plan_drop_graph(p);
  LaunchGeom geo;
  const bool batch = p->kind == SSSP_PLAN_BATCH;
  sssp_status s;
  RoundArgs probe;
  memset(&probe, 0, sizeof(probe));
  if ((s = resolve_launch(p->ws, p->f32, batch, L, &geo, probe, p->low_spread))) return s;
  HIPCHK(hipGraphCreate(&p->graph, 0));
  Launcher rec;
  rec.graph = p->graph;
  if (batch) {
    p->a.solo_edges = probe.solo_edges;
    p->a.block_units = probe.block_units;
    HIPCHK(launch_solve(p->f32, true, p->a, p->batch_pred, geo, p->a.istat, p->max_n, nullptr,
                        rec));
  } else {
    const int wg = L ? L->wg : 0;
    for (size_t i = 0; i < p->seq.size(); ++i) {
      p->seq[i].solo_edges = probe.solo_edges;
      p->seq[i].block_units = probe.block_units;
      LaunchGeom gi = geo;
      gi.wg = wg > 0 || (wg == 0 && p->seq_low[i]) ? 1 : 0;
      HIPCHK(launch_solve(p->f32, false, p->seq[i], p->seq_pred[i], gi, nullptr, p->seq_n[i],
                          nullptr, rec));
    }
  }
  HIPCHK(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  return SSSP_OK;
}

static sssp_status plan_build(const sssp_csr *graphs, int32_t num_graphs,
                              const int32_t *inst_graph, const int32_t *inst_source,
                              int32_t num_inst, sssp_plan_kind kind, void *cost, int32_t *pred,
                              int32_t with_stats, const sssp_launch *launch, sssp_plan_s *p) {
  int64_t total;
  int32_t max_n;
  sssp_status s;
  if (kind != SSSP_PLAN_BATCH && kind != SSSP_PLAN_SEQUENCE) return SSSP_ERR_ARG;
  if ((s = check_batch(graphs, num_graphs, inst_graph, inst_source, num_inst, cost, &total,
                       &max_n)))
    return s;
  HIPCHK(hipGetDevice(&p->dev));
  HIPCHK(hipDeviceGetAttribute(&p->ws.cus, hipDeviceAttributeMultiprocessorCount, p->dev));
  p->ws.init = true;
  p->kind = kind;
  p->num_inst = num_inst;
  p->with_stats = with_stats != 0;
  p->f32 = graphs[0].dtype == SSSP_F32;
  p->max_n = max_n;
  std::vector<GraphDev> hg((size_t)num_graphs);
  std::vector<InstDev> hi((size_t)num_inst);
  fill_tables(graphs, num_graphs, inst_graph, inst_source, num_inst, hg.data(), hi.data());
  if (kind == SSSP_PLAN_BATCH) {
    if ((s = batch_args(p->ws, graphs, num_graphs, inst_graph, num_inst, total, max_n, cost,
                        pred, p->with_stats, p->a)))
      return s;
    HIPCHK(hipMemcpy((void *)p->a.graphs, hg.data(), sizeof(GraphDev) * num_graphs,
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy((void *)p->a.insts, hi.data(), sizeof(InstDev) * num_inst,
                     hipMemcpyHostToDevice));
    p->batch_pred = pred;
    p->low_spread = all_low_spread(graphs, inst_graph, num_inst);
  } else {
    // one set of state buffers for the largest instance, reused solve
    // after solve, and one control block per instance for its counters
    RoundArgs base;
    memset(&base, 0, sizeof(base));
    for (int32_t i = 0; i < num_inst; ++i) {
      if (relax_correcting(&graphs[inst_graph[i]])) base.any_lc = 1;
      if (scope_all_of(&graphs[inst_graph[i]])) base.scope_all = 1;
    }
    if ((s = state_buffers(p->ws, max_n, 1, false, base))) return s;
    Ctl *ctls;
    if ((s = ws_arr(p->ws, S_CTL, (size_t)num_inst, &ctls))) return s;
    for (int32_t i = 0; i < num_inst; ++i) {
      const sssp_csr *g = &graphs[inst_graph[i]];
      RoundArgs a = base;
      a.g = graph_dev(g);
      a.num_inst = 1;
      a.source = inst_source[i];
      a.total = g->n;
      a.max_rounds = round_limit(g->n);
      a.D = (int32_t *)cost + hi[i].sbase;
      a.target = -1;
      a.scope_all = a.g.all;
      a.any_lc = a.g.lc;
      a.ctl = ctls + i;
      p->seq.push_back(a);
      p->seq_n.push_back(g->n);
      p->seq_pred.push_back(pred ? pred + hi[i].sbase : nullptr);
      p->seq_low.push_back(low_spread(g) ? 1 : 0);
    }
  }
  return plan_record(p, launch);
}

// Runs the plan once on `stream` (no synchronization).
static sssp_status plan_launch(sssp_plan_s *p, hipStream_t stream) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != p->dev) return SSSP_ERR_ARG;
  HIPCHK(hipGraphLaunch(p->exec, stream));
  return SSSP_OK;
}

extern "C" {

sssp_status sssp_plan_create(const sssp_csr *graphs, int32_t num_graphs,
                             const int32_t *inst_graph, const int32_t *inst_source,
                             int32_t num_inst, sssp_plan_kind kind, void *cost, int32_t *pred,
                             int32_t with_stats, const sssp_launch *launch, sssp_plan *plan) {
  if (!plan) return SSSP_ERR_ARG;
  *plan = nullptr;
  if (kind != SSSP_PLAN_BATCH && kind != SSSP_PLAN_SEQUENCE) return SSSP_ERR_ARG;
  {
    int64_t total;
    int32_t max_n;
    const sssp_status s = check_batch(graphs, num_graphs, inst_graph, inst_source, num_inst,
                                      cost, &total, &max_n);
    if (s) return s;
  }
  sssp_plan_s *p = new (std::nothrow) sssp_plan_s();
  if (!p) return SSSP_ERR_NOMEM;
  sssp_status s = plan_build(graphs, num_graphs, inst_graph, inst_source, num_inst, kind, cost,
                             pred, with_stats, launch, p);
  if (s == SSSP_OK && hipDeviceSynchronize() != hipSuccess) s = SSSP_ERR_HIP;
  if (s != SSSP_OK) {
    (void)hipDeviceSynchronize();
    plan_drop_graph(p);
    ws_free(p->ws);
    delete p;
    return s;
  }
  *plan = p;
  return SSSP_OK;
}

sssp_status sssp_plan_run(sssp_plan plan, void *stream) {
  if (!plan) return SSSP_ERR_ARG;
  return plan_launch(plan, (hipStream_t)stream);
}

sssp_status sssp_plan_stats(sssp_plan plan, sssp_stats *stats, void *stream_) {
  if (!plan || !stats) return SSSP_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_;
  if (plan->kind == SSSP_PLAN_BATCH) {
    if (!plan->with_stats) return SSSP_ERR_ARG;
    return batch_stats(plan->a, plan->num_inst, stats, stream);
  }
  HIPCHK(hipStreamSynchronize(stream));
  std::vector<Ctl> c((size_t)plan->num_inst);
  HIPCHK(hipMemcpy(c.data(), plan->seq[0].ctl, sizeof(Ctl) * c.size(), hipMemcpyDeviceToHost));
  sssp_status s = SSSP_OK;
  for (int32_t i = 0; i < plan->num_inst; ++i) {
    single_stats(&c[i], &stats[i]);
    if (c[i].status) s = SSSP_ERR_INTERNAL;
  }
  return s;
}

sssp_status sssp_plan_destroy(sssp_plan plan) {
  if (!plan) return SSSP_OK;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipSetDevice(plan->dev));
  const hipError_t e = hipDeviceSynchronize();
  plan_drop_graph(plan);
  ws_free(plan->ws);
  delete plan;
  HIPCHK(hipSetDevice(dev));
  HIPCHK(e);
  return SSSP_OK;
}

sssp_status sssp_autotune(const sssp_csr *graphs, int32_t num_graphs, const int32_t *inst_graph,
                          const int32_t *inst_source, int32_t num_inst, sssp_plan_kind kind,
                          void *cost, int32_t *pred, int32_t reps, sssp_launch *best,
                          double *best_ms, void *stream_) {
  if (!best || reps < 1 || reps > 100) return SSSP_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_;
  sssp_plan p = nullptr;
  sssp_status s = sssp_plan_create(graphs, num_graphs, inst_graph, inst_source, num_inst, kind,
                                   cost, pred, 0, nullptr, &p);
  if (s) return s;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  LaunchGeom full;
  RoundArgs probe;
  memset(&probe, 0, sizeof(probe));
  // mean replay time of the plan under geometry L (re-recorded)
  auto time_of = [&](const sssp_launch &L, double *ms) -> sssp_status {
    sssp_status st = plan_record(p, &L);
    if (st) return st;
    if ((st = plan_launch(p, stream))) return st;  // warm-up (uploads the graph)
    HIPCHK(hipEventRecord(t0, stream));
    for (int32_t k = 0; k < reps; ++k)
      if ((st = plan_launch(p, stream))) return st;
    HIPCHK(hipEventRecord(t1, stream));
    HIPCHK(hipEventSynchronize(t1));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, t0, t1));
    *ms = (double)f / reps;
    return SSSP_OK;
  };
  auto run = [&]() -> sssp_status {
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    sssp_status st;
    if ((st = resolve_launch(p->ws, p->f32, kind == SSSP_PLAN_BATCH, nullptr, &full, probe)))
      return st;
    sssp_launch cur = {full.blocks, probe.solo_edges, probe.block_units, full.small_n, 0};
    double cur_ms;
    if ((st = time_of(cur, &cur_ms))) return st;
    const int32_t blocks[3] = {full.blocks, full.blocks / 2, full.blocks / 4};
    const int32_t solo[3] = {2048, 8192, 32768};
    const int32_t units[3] = {1024, 2048, 4096};
    const int32_t small[3] = {full.small_n, -1, full.small_n};
    const int32_t wgs[3] = {0, -1, 1};
    for (int field = 0; field < 5; ++field) {
      for (int c = 0; c < 3; ++c) {
        sssp_launch cand = cur;
        if (field == 0) cand.blocks = blocks[c];
        if (field == 1) cand.solo_edges = solo[c];
        if (field == 2) cand.block_units = units[c];
        if (field == 3) cand.small_n = small[c];
        if (field == 4) {
          cand.wg = wgs[c];
          // forcing one workgroup per instance only pays with many instances
          if (cand.wg > 0 && num_inst < full.cus / 4) continue;
        }
        if (cand.blocks < 1 || (cand.blocks == cur.blocks && cand.solo_edges == cur.solo_edges &&
                                cand.block_units == cur.block_units &&
                                cand.small_n == cur.small_n && cand.wg == cur.wg))
          continue;
        double ms;
        if ((st = time_of(cand, &ms))) return st;
        if (ms < cur_ms) {
          cur = cand;
          cur_ms = ms;
        }
      }
    }
    // leave cost and pred as a run under the chosen geometry writes them
    if ((st = plan_record(p, &cur))) return st;
    if ((st = plan_launch(p, stream))) return st;
    HIPCHK(hipStreamSynchronize(stream));
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return SSSP_OK;
  };
  s = run();
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  const sssp_status s2 = sssp_plan_destroy(p);
  return s ? s : s2;
}

sssp_status sssp_backward(const sssp_csr *graphs, int32_t num_graphs, const int32_t *inst_graph,
                          const int32_t *inst_source, int32_t num_inst, const int32_t *pred,
                          const float *grad_cost, float *grad_w, void *stream_) {
  if (!graphs || num_graphs <= 0 || !inst_graph || !inst_source || num_inst <= 0 || !pred ||
      !grad_cost || !grad_w)
    return SSSP_ERR_ARG;
  for (int32_t gi = 0; gi < num_graphs; ++gi)
    if (!csr_ok(&graphs[gi])) return SSSP_ERR_ARG;
  int64_t total = 0, total_m = 0;
  for (int32_t gi = 0; gi < num_graphs; ++gi) total_m += graphs[gi].m;
  for (int32_t i = 0; i < num_inst; ++i) {
    const int32_t gi = inst_graph[i];
    if (gi < 0 || gi >= num_graphs) return SSSP_ERR_ARG;
    if (inst_source[i] < 0 || inst_source[i] >= graphs[gi].n) return SSSP_ERR_ARG;
    total += graphs[gi].n;
  }
  if (total >= (int64_t)INT_MAX || total_m >= (int64_t)INT_MAX) return SSSP_ERR_ARG;
  hipStream_t stream = (hipStream_t)stream_;
  Guard guard;
  DevWS *wp;
  sssp_status s;
  if ((s = ws_for_current(&wp))) return s;
  DevWS &ws = *wp;
  BackArgs b;
  memset(&b, 0, sizeof(b));
  b.num_inst = num_inst;
  b.total = (int32_t)total;
  b.pred = pred;
  b.gcost = grad_cost;
  GraphDev *dg;
  InstDev *di;
  int32_t *goff, *ginst, *ebase;
  unsigned int *bctl;
  if ((s = ws_arr(ws, S_GTAB, (size_t)num_graphs, &dg))) return s;
  if ((s = ws_arr(ws, S_ITAB, (size_t)num_inst, &di))) return s;
  if ((s = ws_arr(ws, S_BW_ACC, (size_t)total, &b.acc))) return s;
  if ((s = ws_arr(ws, S_BW_LV, (size_t)total, &b.lv_v))) return s;
  if ((s = ws_arr(ws, S_BW_LI, (size_t)total, &b.lv_i))) return s;
  if ((s = ws_arr(ws, S_BW_LOFF, (size_t)total + 2, &b.lv_off))) return s;
  if ((s = ws_arr(ws, S_BW_CS, (size_t)total, &b.lv_cs))) return s;
  if ((s = ws_arr(ws, S_BW_LACC, (size_t)total, &b.lv_acc))) return s;
  if ((s = ws_arr(ws, S_BW_CTL, 8, &bctl))) return s;
  if ((s = ws_arr(ws, S_BW_GOFF, (size_t)num_graphs + 1, &goff))) return s;
  if ((s = ws_arr(ws, S_BW_GINST, (size_t)num_inst, &ginst))) return s;
  if ((s = ws_arr(ws, S_BW_EBASE, (size_t)num_graphs + 1, &ebase))) return s;
  if ((s = ws_arr(ws, S_FLAGS, (size_t)kMaxBlocks * kFlagStride, &b.flags))) return s;
  b.go = bctl;
  b.ctr = bctl + 1;
  b.nlevels = (int32_t *)(bctl + 2);
  b.graphs = dg;
  b.insts = di;
  const size_t tab_bytes = sizeof(GraphDev) * num_graphs + sizeof(InstDev) * num_inst +
                           sizeof(int32_t) * (3 * (size_t)num_graphs + 2 + num_inst) + 64;
  void *hp;
  if ((s = pinned_get(ws, tab_bytes, &hp))) return s;
  GraphDev *hg = (GraphDev *)hp;
  InstDev *hi = (InstDev *)(hg + num_graphs);
  int32_t *hgoff = (int32_t *)(hi + num_inst);
  int32_t *hginst = hgoff + num_graphs + 1;
  int32_t *hebase = hginst + num_inst;
  for (int32_t gi = 0; gi < num_graphs; ++gi) hg[gi] = graph_dev(&graphs[gi]);
  int32_t base = 0;
  for (int32_t i = 0; i < num_inst; ++i) {
    hi[i].graph = inst_graph[i];
    hi[i].source = inst_source[i];
    hi[i].sbase = base;
    hi[i].n = graphs[inst_graph[i]].n;
    base += hi[i].n;
  }
  // instances grouped by graph, in instance order within a graph
  for (int32_t gi = 0; gi <= num_graphs; ++gi) hgoff[gi] = 0;
  for (int32_t i = 0; i < num_inst; ++i) hgoff[inst_graph[i] + 1]++;
  for (int32_t gi = 0; gi < num_graphs; ++gi) hgoff[gi + 1] += hgoff[gi];
  {
    std::vector<int32_t> fill(hgoff, hgoff + num_graphs);
    for (int32_t i = 0; i < num_inst; ++i) hginst[fill[inst_graph[i]]++] = i;
  }
  int32_t eb = 0;
  for (int32_t gi = 0; gi < num_graphs; ++gi) {
    hebase[gi] = eb;
    eb += graphs[gi].m;
  }
  hebase[num_graphs] = eb;
  LaunchGeom geo;
  if ((s = geometry(ws, true, true, &geo))) return s;
  {
    // deep trees (graphs of low degree spread): each instance in a workgroup
    const int wg = ws.cfg.wg;
    geo.wg = wg > 0 || (wg == 0 && all_low_spread(graphs, inst_graph, num_inst)) ? 1 : 0;
  }
  HIPCHK(hipStreamWaitEvent(stream, ws.last, 0));
  HIPCHK(hipMemcpyAsync(dg, hg, sizeof(GraphDev) * num_graphs, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(di, hi, sizeof(InstDev) * num_inst, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(goff, hgoff, sizeof(int32_t) * (num_graphs + 1), hipMemcpyHostToDevice,
                        stream));
  HIPCHK(hipMemcpyAsync(ginst, hginst, sizeof(int32_t) * num_inst, hipMemcpyHostToDevice,
                        stream));
  HIPCHK(hipMemcpyAsync(ebase, hebase, sizeof(int32_t) * (num_graphs + 1),
                        hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(ws.staged, stream));
  HIPCHK(launch_backward(b, geo, goff, ginst, ebase, num_graphs, (int32_t)total_m, grad_w,
                         stream));
  HIPCHK(hipEventRecord(ws.last, stream));
  return SSSP_OK;
}

sssp_status sssp_policy_of(const sssp_csr *g, sssp_policy *out) {
  if (!csr_ok(g) || !out) return SSSP_ERR_ARG;
  const bool f32 = g->dtype == SSSP_F32;
  const int32_t inf = f32 ? 0x7f800000 : 0x7fffffff;
  const bool all = scope_all_of(g), lc = relax_correcting(g);
  out->scope = all ? SSSP_SCOPE_ALL : SSSP_SCOPE_OPEN;
  out->relax = lc ? SSSP_RELAX_CORRECTING : SSSP_RELAX_SETTING;
  out->delta = lc ? relax_delta(g) : inf;
  Guard guard;
  DevWS *wp;
  sssp_status s;
  if ((s = ws_for_current(&wp))) return s;
  LaunchGeom geo;
  RoundArgs a;
  memset(&a, 0, sizeof(a));
  if ((s = resolve_launch(*wp, f32, false, &wp->cfg, &geo, a, low_spread(g)))) return s;
  // the choice launch_solve makes for a single solve
  if (g->n <= geo.small_n) out->kernel = SSSP_KERNEL_SMALL;
  else if (geo.wg && !all) out->kernel = SSSP_KERNEL_WORKGROUP;
  else out->kernel = SSSP_KERNEL_PERSISTENT;
  return SSSP_OK;
}

sssp_status sssp_check(void *stream) {
  Guard guard;
  int32_t f = 0;
  HIPCHK(fault_flag_take(&f, (hipStream_t)stream));
  return f ? SSSP_ERR_INTERNAL : SSSP_OK;
}

sssp_status sssp_set_round_limit(int32_t limit) {
  if (limit < 0) return SSSP_ERR_ARG;
  Guard guard;
  g_round_limit = limit;
  return SSSP_OK;
}

sssp_status sssp_release_workspace(void) {
  Guard guard;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SSSP_ERR_ARG;
  DevWS &w = g_ws[dev];
  if (!w.init) return SSSP_OK;
  HIPCHK(hipDeviceSynchronize());
  for (int i = 0; i < NSLOTS; ++i) {
    if (w.buf[i]) HIPCHK(hipFree(w.buf[i]));
    w.buf[i] = nullptr;
    w.cap[i] = 0;
  }
  if (w.pinned) HIPCHK(hipHostFree(w.pinned));
  w.pinned = nullptr;
  w.pinned_cap = 0;
  if (w.last) HIPCHK(hipEventDestroy(w.last));
  if (w.staged) HIPCHK(hipEventDestroy(w.staged));
  w.last = w.staged = nullptr;
  w.bpc[0] = w.bpc[1] = w.bpc[2] = w.bpc[3] = 0;
  w.init = false;  // the next call sets the device up again (its launch defaults stay)
  // the profiler's event pairs (created on whichever device was current)
  for (KernelTimer &t : g_prof.pool) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  g_prof.pool.clear();
  g_prof.used = 0;
  return SSSP_OK;
}

}  // extern "C"
