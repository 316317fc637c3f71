// Declarations shared by the host runtime (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sssp_dev.h"

namespace sssp {

// Threads per block of the persistent round kernel: one block per CU (16
// waves) keeps the grid barrier at 256 participants while filling the CU.
constexpr int kRoundBlock = 1024;
constexpr int kBackBlock = 512;   // threads per block of the backward kernels
constexpr int kMaxBlocks = 4096;  // upper bound on a persistent grid

// Per-block partial minima of a single solve, [kParts][kMaxBlocks]: every
// block overwrites its own slot in each phase and readers reduce over all
// slots, so no two blocks ever update the same word.  Slots come in pairs
// indexed by round parity.
enum PartSlot {
  P_SURV0 = 0,  // min D of the vertices that stay open, for the next round
  P_SURV1,
  P_TSURV0,     // min D + out_wmin of the vertices that stay open, next round
  P_TSURV1,
  P_CAND0,      // min successful relaxation candidate of this round's relax
  P_CAND1,
  P_TCAND0,     // min candidate + out_wmin of the head, this round's relax
  P_TCAND1,
  kParts
};

// Payload words carried by the lists.  A relax item carries its out-offset
// and the D it is relaxed from; a fixed vertex carries its final D as is,
// an open one (label-correcting relax) its D with bit 31 set (D keys are
// non-negative, so the bit is free).  An open item pushed as a survivor
// carries what its next bound step needs, so neither phase gathers them.
// An open item pushed by relax (a first discovery) carries the same words,
// read from its vertex record when the relax step counts its work, with
// OX_IDEG = -1 - in-degree (the mark of a first discovery); one pushed when
// the relax stager was full carries OX_BASE = -1 instead: the bound step
// then reads the vertex record, and C (0, or under scope ALL what the live
// pass raised it to).  The one-workgroup kernel lays the same memory out
// as two int4 arrays (the vertex record's halves, with C in its last word),
// so kOXMem words are allocated per open entry.
constexpr int32_t kOpenRelax = (int32_t)0x80000000;
enum { FX_OOFF = 0, FX_D, kFX };
enum { OX_BASE = 0, OX_IDEG, OX_OOFF, OX_ODEG, OX_OWM, OX_C, kOX };
constexpr int kOXMem = 8;

// One hand-over to parked blocks: where to resume, whether the solve is
// done, how many blocks are active from there, and the active barrier's
// epoch.  Hand-over e (the e-th bump of Ctl::go) lives in slot
// e % kResumeSlots, so a reader holding e reads a slot that no later
// hand-over rewrites until e + kResumeSlots.
constexpr int kResumeSlots = 8;
struct ResumeSlot {
  int32_t round, phase, done, act;
  unsigned int aep;
  int32_t pad[3];
};

// Control block of one persistent solve, in device memory.
struct Ctl {
  unsigned long long front_ctr[2];  // by round parity: (items << 32) | out-degree sum
  unsigned long long open_ctr[2];   // by round parity: (items << 32) | in-degree sum
  unsigned int go;                  // hand-over word: parked blocks wait on it
  unsigned int go_a;                // barrier release word of the active blocks
  int32_t status;                   // 0, or an sssp_status code set on the device
  int32_t rounds;
  int32_t deg_count;    // pred: vertices queued for the equal-cost pass
  ResumeSlot resume[kResumeSlots];  // hand-overs to parked blocks, by go % kResumeSlots
  long long settled, relaxed, scanned, open_visits;
  long long solo_phases;  // phases run by block 0 alone
  // single-target solve: the target's solver id (-1: none) and whether a
  // bound step (or the seed) has fixed it
  int32_t target_id, target_hit;
  // C scope ALL: live-list sizes by round parity, and the in-degree sums
  // (plain and times the drop round) of undiscovered vertices dropped with
  // C = INF, for the scanned-edge count of the rounds after their drop
  unsigned long long live_ctr[2];
  unsigned long long dead_deg, dead_deg_r;
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
  int32_t *D;                // the caller's cost array (written by the emit pass)
  // Upper bound and parent candidate per state entry, one 64-bit key:
  // (D << 32) | (equal-cost flag << 31) | edge id.  atomicMin on the key
  // keeps the least D and, among candidates that reach it, strict ones
  // (tail cost below D) before equal-cost ones, then the smallest edge id.
  unsigned long long *D64;
  int32_t *C0, *C1;          // lower bounds, double-buffered by round parity
  int32_t *mtmp;             // per open slot: partial m_y of items split over blocks
  unsigned int *arrive;      // per open slot: contributing blocks that finished
  int32_t *open_v0, *open_p0, *open_i0;
  int32_t *open_v1, *open_p1, *open_i1;
  int32_t *front_v, *front_p, *front_i;
  int32_t *front_x[kFX];              // frontier payload words
  int32_t *open_x0[kOX], *open_x1[kOX];  // open-list payload words, by parity
  Ctl *ctl;
  int32_t *imin, *ithr, *irounds;  // batch: [3][I], [3][I], [I]
  unsigned long long *iscanned;    // batch: [I][3] scanned in-edges, open visits, relaxed edges
  int32_t *degen, *lvl, *flag, *scratch_pred;
  long long *istat;                // batch stats [4][I], zeroed by the seed kernel
  // optional round trace (SSSP_TRACE): per round kTraceFields entries
  long long *trace;
  int32_t trace_rounds;
  int32_t trace_blk_rounds;  // rounds with per-block records
  // [round][2 phases][kMaxBlocks][kBlkFields]: per block, the wall-clock at
  // its phase end, the list windows it walked, its first list item, the
  // work units of its chunk and the wall-clock after its list windows
  long long *trace_blk;
  // optional checkpoints: one block's wall-clock at fixed points inside each
  // phase, [round][2 phases][kMarks]
  long long *marks;
  int32_t mark_rounds;
  int32_t mark_block;  // the block whose checkpoints are recorded
  unsigned int *flags;       // grid barrier flags, kMaxBlocks * kFlagStride
  int32_t *part;             // per-block partial minima, kParts * kMaxBlocks
  int32_t solo_edges;        // phases with at most this many edges run on block 0 alone
  int32_t block_units;       // otherwise: about this many work units per active block
  int32_t target;            // single solve: stop once this vertex (caller's id) is fixed, or -1
  // single solve, C scope ALL: the bound step also raises C of undiscovered
  // vertices; live lists (by round parity) hold those whose C is finite
  int32_t scope_all;  // some graph of the solve runs C scope ALL
  int32_t *live_v0, *live_v1;
  int32_t *inst_of;              // batch, scope ALL: the instance of each state entry
  unsigned long long *idead;     // batch, scope ALL: [I][2] dead_deg, dead_deg_r
  // label-correcting relax: per state entry the D it was last relaxed with
  // (INF before its first relax)
  int32_t *DR;
  int32_t any_lc;  // some graph of the solve relaxes label-correcting
};

// Trace record of one round: wall-clock (100 MHz) at the relax start, block
// 0's arrival at and release from each of the two barriers, the list sizes
// (fixed, open, and the live list of undiscovered vertices under scope ALL),
// and which phases ran on one block (bit 0 relax, bit 1 bound-and-fix).
enum TraceField {
  TR_START = 0, TR_ARR_RELAX, TR_END_RELAX, TR_ARR_FUSED, TR_END_FUSED,
  TR_NF, TR_EF, TR_NO, TR_EO, TR_MODE, TR_NL, kTraceFields
};

constexpr int kBlkFields = 5;
constexpr int kMarks = 12;

struct LaunchGeom {
  int blocks;  // persistent grid size (co-resident)
  int cus;
  int small_n = 0;  // single solves of at most this many vertices run in one workgroup
  int wg = 0;       // every instance in a workgroup of its own (scope OPEN only)
};

// Largest graph the one-workgroup solver holds in LDS.
constexpr int kSmallN = 4096;

constexpr unsigned long long kKeyEidMask = 0x7fffffffull;
constexpr unsigned long long kKeyEqualCost = 0x80000000ull;

__device__ __forceinline__ unsigned long long make_key(int32_t d, int32_t eid, bool equal_cost) {
  return ((unsigned long long)(uint32_t)d << 32) | (equal_cost ? kKeyEqualCost : 0ull) |
         (unsigned long long)(uint32_t)eid;
}

// address of the D half of a key (little-endian: the high word)
__device__ __forceinline__ int32_t *key_d(unsigned long long *k) {
  return reinterpret_cast<int32_t *>(k) + 1;
}

// Graph of an item: the kernel argument for a single solve, the table
// entry for a batch.
template <bool BATCH>
__device__ __forceinline__ const GraphDev &graph_of(const RoundArgs &a, int gi) {
  if constexpr (BATCH) return a.graphs[gi];
  else return a.g;
}

// Where a solve's kernels go: onto `stream` at once, or (graph non-null)
// appended to `graph` as a chain of kernel nodes in launch order, each
// depending on the one before (`last`).  The persistent kernel's node
// carries the cooperative attribute, so a replay keeps its blocks
// co-resident like the direct cooperative launch.
struct Launcher {
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphNode_t last = nullptr;
};
// args: one pointer per kernel parameter (copied when the node is added)
hipError_t launch_kernel(Launcher &L, const void *fn, dim3 grid, dim3 block, void **args,
                         bool cooperative);

// timer: eager launches only (a graph records no events)
hipError_t launch_solve(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                        const LaunchGeom &geo, long long *istat, int32_t max_n,
                        const KernelTimer *timer, Launcher &L);
hipError_t launch_pred(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                       const LaunchGeom &geo, long long *istat, int32_t max_n, Launcher &L);
// waits for `stream`, then reads (*out: 0 or 1) and clears the device's
// fault flag, which the emit pass sets for a solve whose status is non-zero
hipError_t fault_flag_take(int32_t *out, hipStream_t stream);
hipError_t round_kernel_occupancy(bool f32, bool batch, int *blocks_per_cu);

// Bytes of the static scratch region of allocation-free solves, and its
// device address on the current device (call once per device, with that
// device current).
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t scratch_address(void **ptr);
// every instance's rounds in a workgroup of its own (C scope OPEN), then the emit pass
hipError_t launch_wg(bool f32, bool batch, const RoundArgs &a, int32_t *pred,
                     const LaunchGeom &geo, long long *istat, int32_t max_n,
                     const KernelTimer *timer, Launcher &L);
// a single solve of a.total <= kSmallN vertices in one workgroup, then the emit pass
hipError_t launch_small(bool f32, const RoundArgs &a, int32_t *pred, const KernelTimer *timer,
                        Launcher &L);

// ------------------------------------------------------------- builder
struct BuildTemps {
  int32_t *ka, *kb, *va, *vb;  // radix sort ping-pong, max(m, n) each
  int32_t *hist;               // 256 * tiles (+ scan sums)
  int32_t *tail;               // m: tail of each edge id
  int32_t *status;             // [0] error flags, [1] max weight key, [2] max total degree
};
// The solver's working copy of a graph (arrays in the build buffer).  In
// the input numbering vid, rank, out_eid are null and out_* alias the CSR;
// the in-lists are always a copy, ascending by weight.
struct SolverCopy {
  int32_t *vid, *rank;
  int32_t *out_off, *out_dst, *out_w, *out_eid;
  int32_t *in_off, *in_src, *in_eid, *in_w;
  int32_t *in_sw;  // (in_src, in_w) pairs
  int32_t *out_rec;  // (out_dst, out_w, edge id, out_wmin of the head) per out-list entry
  int32_t *out_wmin;
  int32_t *vrec;  // 8 ints per vertex
  int32_t *vin;   // 4 ints per vertex: vrec's in_off, in_degree, lightest tail and weight
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
// degrees into t.ka, their maximum into t.status[2]
hipError_t launch_degree(int32_t n, const int32_t *out_off, const int32_t *in_off,
                         const BuildTemps &t, hipStream_t stream);
// vid, rank and the CSR copy in descending-degree order, from the built CSR
// and the degrees left in t.ka by launch_degree (dmax: their maximum)
hipError_t launch_renumber(int32_t n, int32_t m, int32_t dmax, const int32_t *out_dst,
                           const int32_t *out_w, const int32_t *out_wmin, const SolverCopy &c,
                           const BuildTemps &t, hipStream_t stream);
// the weight-ordered in-lists of the copy (c.rank null: input numbering);
// wkey_max: the largest weight's bit pattern.  Overwrites t.tail.
hipError_t launch_in_lists(int32_t n, int32_t m, int32_t wkey_max, const int32_t *out_off,
                           const int32_t *out_dst, const int32_t *out_w, const SolverCopy &c,
                           const BuildTemps &t, hipStream_t stream);
// the per-vertex records of the copy (after its offsets and out_wmin)
hipError_t launch_vrec(int32_t n, const SolverCopy &c, hipStream_t stream);
// c.out_rec from the working copy's out-lists and out_wmin (after launch_vrec's inputs are final)
hipError_t launch_out_rec(int32_t m, const SolverCopy &c, hipStream_t stream);
// new weights (validated by the caller) into the CSR/CSC, out_wmin and the
// copy's out-lists; the copy's in-lists are rebuilt by launch_in_lists
hipError_t launch_set_weights(int32_t n, int32_t m, bool f32, const int32_t *w,
                              const int32_t *out_off, const int32_t *in_eid, int32_t *out_w,
                              int32_t *in_w, int32_t *out_wmin, const SolverCopy &c,
                              hipStream_t stream);
// per-edge 4-byte values through the builder's permutation (perm[k] = COO
// index of edge id k): out[k] = in[perm[k]], or out[perm[k]] = in[k]
hipError_t launch_permute_edges(const int32_t *perm, int64_t m, const int32_t *in, int32_t *out,
                                bool to_coo, hipStream_t stream);

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
  // one-workgroup path, per list position: where the entry's children start
  // in the list, and the entry's subtree sum
  int32_t *lv_cs;
  float *lv_acc;
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
