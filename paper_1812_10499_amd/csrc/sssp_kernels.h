// Declarations shared by the host runtime (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sssp_dev.h"

namespace sssp {

constexpr int kRoundBlock = 512;  // threads per block of the persistent kernels
constexpr int kMaxBlocks = 4096;  // upper bound on a persistent grid

// Per-block partial minima of a single solve, [kParts][kMaxBlocks]: every
// block overwrites its own slot each round and readers reduce over blocks,
// so no two blocks ever update the same word.
enum PartSlot {
  P_SURV0 = 0,  // min D of the open vertices that stay open (for the next round), by parity
  P_SURV1,
  P_CAND0,      // min successful relaxation candidate, by round parity
  P_CAND1,
  P_THR0,       // min D[y] + out_wmin[y] over the open set, by round parity
  P_THR1,
  kParts
};

// Control block of one persistent solve, in device memory.
struct Ctl {
  unsigned long long front_ctr;    // (items << 32) | out-degree sum of the next frontier
  unsigned long long open_ctr[2];  // same for the two open-list buffers
  unsigned int go;                 // grid barrier release word
  int32_t status;                  // 0, or an sssp_status code set on the device
  int32_t rounds;
  int32_t deg_count;    // pred: vertices queued for the equal-cost pass
  int32_t heavy_count;  // pred: vertices queued for the wave-per-vertex pass
  int32_t pad;
  long long settled, relaxed, scanned, open_visits;
};

// Optional event pair recorded around the persistent kernel launch.
struct KernelTimer {
  hipEvent_t start, stop;
};

struct RoundArgs {
  GraphDev g;                // single solve
  const GraphDev *graphs;    // batch: graph table
  const InstDev *insts;      // batch: instance table
  int32_t num_inst;
  int32_t source;            // single solve
  int32_t total;             // state entries (sum of instance vertex counts)
  int32_t max_rounds;
  int32_t *D, *C, *mtmp;
  int32_t *open_v0, *open_p0, *open_i0;
  int32_t *open_v1, *open_p1, *open_i1;
  int32_t *front_v, *front_p, *front_i;
  Ctl *ctl;
  int32_t *imin, *ithr, *irounds;  // batch: [3][I], [3][I], [I]
  unsigned long long *iscanned;    // batch: [I][2] scanned in-edges, open visits
  int32_t *heavy, *degen, *lvl, *flag, *scratch_pred;
  long long *istat;                // batch stats [4][I], zeroed by the seed kernel
  // optional round trace (SSSP_TRACE): per round kTraceFields entries
  long long *trace;
  int32_t trace_rounds;
  int32_t trace_blk_rounds;  // rounds with per-block phase end times
  long long *trace_blk;      // [round][3 phases][kMaxBlocks] wall-clock at each block's phase end
  unsigned int *flags;  // grid barrier flags, kMaxBlocks * kFlagStride
  int32_t *part;        // per-block partial minima, kParts * kMaxBlocks
  int32_t coherent_filter;  // relax reads D[head] with an agent-coherent load
};

// Trace record of one round: wall-clock (100 MHz) at relax start, the last
// block's arrival and the release of each of the three barriers, and the
// list sizes the round processed.
enum TraceField {
  TR_START = 0, TR_ARR_RELAX, TR_END_RELAX, TR_ARR_LB, TR_END_LB, TR_ARR_FIX, TR_END_FIX,
  TR_NF, TR_EF, TR_NO, TR_EO, kTraceFields
};

struct LaunchGeom {
  int blocks;  // persistent grid size (co-resident)
  int cus;
};

hipError_t launch_solve(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                        const LaunchGeom &geo, long long *istat, int32_t max_n,
                        const KernelTimer *timer, hipStream_t stream);
hipError_t round_kernel_occupancy(bool f32, bool batch, int *blocks_per_cu);

// ------------------------------------------------------------- builder
struct BuildTemps {
  int32_t *ka, *kb, *va, *vb;  // radix sort ping-pong, m each
  int32_t *hist;               // 256 * tiles (+ scan sums)
  int32_t *tail;               // m: tail of each edge id
  int32_t *status;             // [0] error flags, [1] max weight key
};
size_t build_hist_entries(int32_t m);
hipError_t launch_validate(int32_t n, int32_t m, bool f32, const int32_t *src,
                           const int32_t *dst, const int32_t *w, int32_t *status,
                           hipStream_t stream);
hipError_t launch_build(int32_t n, int32_t m, bool f32, const int32_t *src, const int32_t *dst,
                        const int32_t *w, int32_t *out_off, int32_t *out_dst, int32_t *out_w,
                        int32_t *in_off, int32_t *in_src, int32_t *in_eid, int32_t *in_w,
                        int32_t *out_wmin, int32_t *perm, const BuildTemps &t,
                        hipStream_t stream);
hipError_t launch_set_weights(int32_t n, int32_t m, bool f32, const int32_t *w,
                              const int32_t *out_off, const int32_t *in_eid, int32_t *out_w,
                              int32_t *in_w, int32_t *out_wmin, int32_t *status,
                              hipStream_t stream);

// ------------------------------------------------------------ backward
struct BackArgs {
  const GraphDev *graphs;
  const InstDev *insts;
  int32_t num_inst;
  int32_t total;
  const int32_t *pred;
  const float *gcost;
  float *acc;
  int32_t *lv_v, *lv_i;       // level lists (vertex state index, instance)
  int32_t *lv_off;            // level offsets, capacity total + 2
  int32_t *nlevels;           // device scalar: number of non-empty levels
  unsigned int *flags;        // grid barrier flags, kMaxBlocks * kFlagStride
  unsigned int *go;           // grid barrier release word
  unsigned int *ctr;          // append counter for the level being built
};
hipError_t launch_backward(const BackArgs &a, const LaunchGeom &geo, const int32_t *ginst_off,
                           const int32_t *ginst, const int32_t *ebase, int32_t num_graphs,
                           int32_t total_m, float *grad_w, hipStream_t stream);

}  // namespace sssp
