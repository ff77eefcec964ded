// Internal declarations of libdi: device graph, solve workspace, control
// block and the kernel launchers. Not part of the public ABI (include/di.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "di.h"

namespace di {

// ---- launch geometry ------------------------------------------------------
// select tiles: pull direction 1024 threads x 4 nodes (a grid of at most
// kSelectGridPull blocks loops over tiles); push direction 256 x 2 (one tile
// per block; the push block of the same index moves its frontier)
// (the three pull-direction select shapes may be set at build time)
#ifndef DI_SELECT_BLOCK
#define DI_SELECT_BLOCK 1024
#endif
#ifndef DI_SELECT_PER_THREAD
#define DI_SELECT_PER_THREAD 4
#endif
#ifndef DI_SELECT_GRID
#define DI_SELECT_GRID 256
#endif
constexpr int kSelectBlockPull = DI_SELECT_BLOCK;
constexpr int kSelectPerThreadPull = DI_SELECT_PER_THREAD;
constexpr int kSelectTilePull = kSelectBlockPull * kSelectPerThreadPull;
constexpr int kSelectGridPull = DI_SELECT_GRID;
constexpr int kSelectBlockPush = 256;
constexpr int kSelectPerThreadPush = 2;
constexpr int kSelectTilePush = kSelectBlockPush * kSelectPerThreadPush;
constexpr int kPullBlock = 256;       // threads per pull block
#ifndef DI_PULL_CHUNK
#define DI_PULL_CHUNK 2048
#endif
constexpr int kPullChunk = DI_PULL_CHUNK;  // in-links per pull work item (LDS staged)
constexpr int kPullMaxRows = 2048;    // rows per pull work item
#ifndef DI_PULL_LONG_ROW
#define DI_PULL_LONG_ROW 32
#endif
constexpr int kPullLongRow = DI_PULL_LONG_ROW;  // rows with more in-links: summed by a wave
constexpr int kPullMaxGrid = 2048;    // pull blocks (grid-stride over items)
constexpr int kXcds = 8;              // XCDs; workgroups are dealt round-robin
constexpr int kPushBlock = 256;       // threads per push block
constexpr int kReduceBlock = 256;     // threads per reduction block
constexpr int kReduceGrid = 256;      // reduction blocks (push direction)

// Per-node word: out-degree (self-loop included) in bits 0..29, heavy-row
// flag (more than kPullChunk in-links) in bit 30, self-loop flag in bit 31.
constexpr uint32_t kLoopBit = 0x80000000u;
constexpr uint32_t kHeavyBit = 0x40000000u;
constexpr uint32_t kOutMask = 0x3fffffffu;
// Heavy rows completed deterministically by the select kernel (their values
// are kept in its LDS); graphs with more heavy rows add the segment sums of
// every heavy row to F with atomics instead.
constexpr int kHeavyLds = 4096;
constexpr int kHeavyChunkSegs = 16;   // segment sums per completion chunk

// Window push: one launch per cycle selects the nodes of a tile of
// consecutive ids (four per thread), claims them and pushes their links. A
// link i -> j is "near" when |i - j| <= kWinHalo: it lands in the tile's LDS
// window [a - kWinHalo, a + tile + kWinHalo); the parts of the window outside
// the tile (the halos) are handed to the neighbouring tiles' next cycle. A
// far link into one of the first `hubs` hub rows (the nodes ranked by their
// far in-links) is accumulated per block in LDS; any other far link is a
// device-scope atomic into the far accumulator of the next cycle.
constexpr int kWinShapes = 3;  // tile shapes: 256, 512 or 1024 threads, 4 nodes each
constexpr int kWinTileOf[kWinShapes] = {1024, 2048, 4096};
constexpr int kWinHalo = 512;
constexpr int kWinHubMax = 1024;   // hub rows ranked per graph
constexpr int kWinMaxGrid = 1024;  // blocks (grid-stride over tiles)
constexpr int kWinHubMinFar = 16;  // far in-links a node needs to be ranked
static_assert(kWinHalo <= 1024, "a near link must land in the tile or a neighbour");

// A window configuration: tile shape, active hub rows (<= the graph's
// ranked hubs) and the largest grid.
struct WinCfg {
  int shape = 1;
  int hubs = kWinHubMax;
  int grid_cap = kWinMaxGrid;
  int rounds = 2;  // DI-SOP diffusion rounds per cycle over each tile
};

// stride of the two far-accumulator copies (whole 256-byte lines, so that
// both copies take aligned vector accesses)
inline int64_t win_stride(int64_t n) { return (n + 63) & ~int64_t(63); }
// rows of one copy of the hub partials: one per block of the largest grid
// any tile shape can take (the smallest tile has the most tiles)
inline int64_t win_hub_rows(int64_t tiles_of_smallest_shape) {
  return tiles_of_smallest_shape < 1 ? 1
                                     : (tiles_of_smallest_shape < kWinMaxGrid ? tiles_of_smallest_shape
                                                                              : kWinMaxGrid);
}
// wp_info: the node word as in info (out-degree, self-loop bit) with bit 30
// (the pull's heavy-row bit there) the ranked-hub flag
constexpr uint32_t kHubBit = 0x40000000u;

// FP32 passes of a refined solve (single, batched or served) stop once
// their r is at most kInnerStop * tol (or the relative inner target): the
// FP64 residual after the pass differs from that r by the FP32 rounding of
// what the pass moved (about 1e-7 of it, far below 0.1 tol), and a pass
// whose FP64 residual is still above tol is followed by another.
constexpr double kInnerStop = 0.9;

// Control block: two copies. The select kernel of cycle c reads copy c & 1
// (the state after cycle c - 1) and its block 0 writes copy (c + 1) & 1; the
// pull (or push) of cycle c reads copy (c + 1) & 1.

// Device control block of one solve.
struct Ctl {
  double r;          // sum |F| after the last cycle: r of the next selection
  double psum;       // sum F after the last cycle
  double e;          // fluid absorbed by dangling nodes
  double final_r;    // sum |F| when the solve stopped
  double paper_err;  // last sum F / (1 - d - d e)
  double r_first;    // r used by the first cycle
  double r_last;     // r used by the last cycle
  double r_start;    // sum |F| at the first selection of the run
  int cycles;        // cycles run
  int fallback;      // DI-CYC cycles run after an empty DI-SOP cycle
  int done;          // 0 running, 1 converged, 2 max_cycles, 3 non-finite,
                     // 4 inner stop (the FP32 pass of a refined solve ended)
  int cyc_mode;      // next cycle selects: 0 by the DI-SOP threshold, 1 every |F_i| > 0, 2 every node
  unsigned long long edges_total;  // link operations (pushes along j != i)
  unsigned long long front_total;  // diffused nodes with links to push
  unsigned long long sel_total;    // diffused nodes
  // device wall clock (wall_clock64) at the run's first selection, and at
  // the first selection whose r, an L1 residual, was <= 1e-9 (0: not yet)
  unsigned long long t_start;
  unsigned long long t_1e9;
  // launches of the run that decided this copy (the selection of cycle c
  // writes c + 1): the host's check that its pinned copy is the new one
  unsigned long long seq;
};

// Per select tile: what its nodes did in the cycle.
struct SelStat {
  unsigned long long ops;  // link operations
  double e;                // fluid absorbed by dangling nodes
  unsigned int sel;        // diffused nodes
  unsigned int nfront;     // diffused nodes with links to push
};

// Per pull / reduce / start block: its rows' sums, and the select
// statistics of the select blocks it folded in.
struct Part {
  double pabs;             // sum |F| over the block's rows
  double psum;             // sum F over the block's rows
  double e;                // absorbed fluid
  unsigned long long ops;  // link operations
  unsigned int sel;        // diffused nodes
  unsigned int nfront;     // diffused nodes with links to push
};

enum Prec { kF64 = 0, kF32 = 1 };

struct BatchWs;
void free_batch_ws(BatchWs* ws);

// Buffers of one solve; pooled per graph so repeated solves do not allocate.
struct Workspace {
  int prec = kF64;
  void* F = nullptr;            // fluid, n values of the fluid type
  void* H = nullptr;            // history, n values
  void* sent = nullptr;         // pull: amount each diffused node sends per link
  unsigned long long* front_bits = nullptr;  // pull: bit i set = node i sends
  int64_t* fr_lstart = nullptr; // push: per-block frontier, local link offset
  int64_t* fr_base = nullptr;   // push: CSR offset of the entry's links
  void* fr_s = nullptr;         // push: amount sent along each link
  SelStat* tile_stat = nullptr; // select statistics (select_stat_records)
  Part* blk_part = nullptr;     // per pull/reduce/start block
  double* seg_val = nullptr;    // pull: sums of the heavy-row segments
  // pull: the heavy rows' fluid kept by the last selection, two copies by
  // cycle parity (the selection of cycle c reads copy c & 1 and writes copy
  // (c + 1) & 1), so no selection block reads a value another block of the
  // same launch writes; n_heavy values of the fluid type each
  void* hret = nullptr;
  // pull with heavy_atomic: the segment sums of each heavy row, added with
  // FP64 atomics by the pull of cycle c into copy (c + 1) & 1 and read by
  // the next selection; the pull of cycle c clears copy c & 1
  double* hacc = nullptr;
  // window push: far accumulators (two copies by parity, n values each),
  // halos (two copies, per tile 2 * kWinHalo values: left then right), hub
  // partials (two copies, per block kWinHubMax values) and per-block records
  // (two copies); all of the fluid type except the records
  void* wA = nullptr;
  void* whalo = nullptr;
  void* whub = nullptr;
  Part* wrec = nullptr;
  int* wflag = nullptr;         // device flag (any negative right-hand side)
  int* host_flag = nullptr;     // pinned copy
  Ctl* ctl = nullptr;           // two copies (see Ctl)
  // pinned host copies of both, for the stop check: the selection kernels
  // (k_select, k_wcycle) store each new copy here too
  Ctl* host_ctl = nullptr;
  double* Y64 = nullptr;        // refinement: d X_j / out_j
  Part* host_part = nullptr;    // pinned: the residual sums (pabs, psum) of k_sum_parts
  double* X64 = nullptr;        // host entry points: device copy of X
  double* B64 = nullptr;        // host entry points: device copy of B
  std::vector<hipEvent_t> events;
  hipEvent_t copied = nullptr;  // the control block is in host_ctl (no timing)
  di_cycle_rec* trace = nullptr;  // per-cycle records of a traced solve
  int trace_cap = 0;
};

}  // namespace di

struct di_graph {
  int64_t n = 0;
  int64_t L = 0;           // links, self-loops included
  int64_t Lp = 0;          // links without self-loops
  int64_t n_dangling = 0;
  int64_t n_loops = 0;
  int64_t max_out = 0;
  int64_t max_in = 0;
  int device = 0;
  // out-links (columns of P) without self-loops: CSR
  int64_t* row_ptr = nullptr;  // n + 1
  int32_t* col = nullptr;      // Lp
  uint32_t* info = nullptr;    // n: out-degree | self-loop bit
  // in-links (rows of P) without self-loops: CSC
  int64_t* csc_ptr = nullptr;  // n + 1
  int32_t* csc_idx = nullptr;  // Lp
  // n: first in-link of a light row within its pull item, csc_ptr[j] - l0
  // (at most kPullChunk: 16 bits); 0 for heavy rows
  uint16_t* row_lo = nullptr;
  // pull work items: light items cover rows [r0, r1) and their in-links
  // [l0, l1); a segment item (seg >= 0) covers links [l0, l1) of the heavy
  // row r0 and writes its sum to seg_val[seg] (or adds it to F[r0]
  // atomically when heavy_atomic)
  int64_t n_items = 0;
  int64_t* it_r0 = nullptr;
  int64_t* it_r1 = nullptr;
  int64_t* it_l0 = nullptr;
  int64_t* it_l1 = nullptr;
  int32_t* it_seg = nullptr;
  // heavy rows (more than kPullChunk in-links)
  int64_t n_heavy = 0;
  int64_t n_segs = 0;
  bool heavy_atomic = false;      // n_heavy or n_hchunks > kHeavyLds
  int32_t* seg_heavy = nullptr;   // n_segs: the heavy row (index) of each segment
  // window push: out-links per row (offsets row_ptr) with the near links
  // (|i - j| <= kWinHalo, ids) first and the far links after them (ids, or
  // -1 - r for the hub of rank r); wp_info per node (info's out-degree and
  // self-loop bit, and kHubBit); the ranked hubs: node of each rank, and the
  // hubs by ascending id (node, rank) with, per tile shape, each tile's
  // range of them
  int32_t* wp_col = nullptr;
  uint32_t* wp_info = nullptr;
  int64_t n_hubs = 0;
  int32_t* hub_rank_node = nullptr;  // n_hubs
  int32_t* hub_id_node = nullptr;    // n_hubs, ascending
  int32_t* hub_id_rank = nullptr;    // n_hubs
  int32_t* hub_tile[di::kWinShapes] = {};  // n_wtiles[s] + 1 each
  int64_t n_wtiles[di::kWinShapes] = {};
  bool window_ok[di::kWinShapes] = {};     // every tile's links fit 32-bit offsets
  int64_t near_links = 0;        // near links (statistics)
  // the window configuration picked by the tuner (tuned: it has run), and
  // its measured time per cycle next to the default configuration's
  bool win_tuned = false;
  di::WinCfg win_cfg;
  bool win_use_pull = false;  // the tuner found the pull faster on this graph
  double win_us_default = 0.0, win_us_tuned = 0.0, pull_us = 0.0;
  int32_t* heavy_row = nullptr;   // n_heavy, ascending
  int64_t* heavy_seg = nullptr;   // n_heavy + 1: segment range of each
  // completion chunks: chunk k sums segments [hc_seg0[k], hc_seg1[k]) of one
  // heavy row; row h owns chunks [hc_off[h], hc_off[h + 1])
  int64_t n_hchunks = 0;
  int32_t* hc_seg0 = nullptr;
  int32_t* hc_seg1 = nullptr;
  int32_t* hc_off = nullptr;
  std::mutex mu;
  std::vector<di::Workspace*> pool;
  std::vector<di::BatchWs*> bpool;  // batched solves (di_batch.h)
};

namespace di {

// thread-local error message
void set_error(const std::string& msg);

// HIP call check: records the message and returns DI_E_DEVICE.
#define DI_HIP(call)                                                            \
  do {                                                                          \
    hipError_t err_ = (call);                                                   \
    if (err_ != hipSuccess) {                                                   \
      ::di::set_error(std::string(#call) + ": " + hipGetErrorString(err_));     \
      return DI_E_DEVICE;                                                       \
    }                                                                           \
  } while (0)

// Propagates a non-OK di_status.
#define DI_TRY(call)                  \
  do {                                \
    di_status st_ = (call);           \
    if (st_ != DI_OK) return st_;     \
  } while (0)

di_status check_device(int* device_out);
void free_workspace(Workspace* ws);

// ---- kernel launchers (di_kernels.hip) ------------------------------------
enum Direction { kPull = 0, kPush = 1, kWindow = 2 };

struct CycleArgs {
  const di_graph* g;
  Workspace* ws;
  double d;
  double tol;      // converged when sum |F| <= tol (first selection of a
                   // refined run: the FP64 residual of X)
  double tol_in;   // refined runs (tol_rel >= 0): after a cycle, stop the
  double tol_rel;  // FP32 pass when sum |F| <= max(tol_in, tol_rel * r_start)
  int first_parts; // records the first selection sums
  int method;      // DI_SOP or DI_CYC
  int stop;        // DI_STOP_RESID or DI_STOP_PAPER
  int max_cycles;  // the solve stops after this many cycles
  int direction;   // kPull, kPush or kWindow
  int folded;      // kWindow: the fluid may be signed, so a fold pass after
                   // every cycle gathers it into F and sums |F| exactly
  WinCfg wcfg;     // kWindow: tile shape, active hubs, largest grid
  hipStream_t stream;
  di_cycle_rec* trace;  // device records of this run's cycles (or null)
  int trace_cap;        // records it has room for
};

int select_tiles(int64_t n, int direction);
// select statistics records: one per wave (pull direction) or per tile (push)
int select_stat_records(int64_t n, int direction);
int select_grid(int64_t n, int direction);
int pull_grid(const di_graph* g);
int reduce_grid(int64_t n);
int part_count(const CycleArgs& a);

hipError_t launch_reset_ctl(const CycleArgs& a);
// F = B (or the uniform value), H = 0, and the per-block records of sum |F|
// and sum F that the first selection reads.
template <typename T>
hipError_t launch_start(const CycleArgs& a, const double* B, double b_uniform);
// The same records for a state (F, H) already in the workspace buffers.
template <typename T>
hipError_t launch_start_state(const CycleArgs& a);
// The selection of cycle c (its stop test first; first != 0 for c = 0).
template <typename T>
hipError_t launch_select(const CycleArgs& a, int cycle, int first);
// The move of cycle c: pull, or push + reduction. With non-null events the
// pull (or push) launch is bracketed by them.
template <typename T>
hipError_t launch_move(const CycleArgs& a, int cycle, hipEvent_t ev0, hipEvent_t ev1);
template <typename T>
hipError_t launch_h_to_x(const CycleArgs& a, double* X);
// Sums |F| and F over the records blk_part[0, count) in a fixed order into
// out->pabs and out->psum (pinned host or device memory).
hipError_t launch_sum_parts(const CycleArgs& a, int count, Part* out);

// ---- window push (di_window.hip) --------------------------------------------
// Cycle c is one launch of the window kernel: its selection reads the
// records of cycle c - 1 (or, for c = 0, the start records in blk_part) and
// the fluid F + far accumulator + halos + hub partials of parity c & 1; it
// pushes into parity (c + 1) & 1. Without `folded` the next r is summed from
// the kept and pushed amounts (exact for a fluid that stays >= 0); with it a
// fold pass after each cycle gathers the fluid into F and sums |F|.
int win_grid(const di_graph* g, const WinCfg& c);
// F = B (or the uniform value), H = 0, both far accumulators 0, and the
// start records (part_count(a) + 1 of them) in blk_part.
template <typename T>
hipError_t launch_wstart(const CycleArgs& a, const double* B, double b_uniform);
// the same for a state (F, H) already in the workspace
template <typename T>
hipError_t launch_wstart_state(const CycleArgs& a);
template <typename T>
hipError_t launch_wcycle(const CycleArgs& a, int cycle, hipEvent_t ev0, hipEvent_t ev1);
// After the stop at cycle c (parity c & 1): gathers the fluid into F (unless
// the run folded every cycle) and writes its exact sums, one record per
// window block, to blk_part[0, win_grid).
template <typename T>
hipError_t launch_wfinal(const CycleArgs& a, int parity, int add);
// *flag = 1 when some B_i < 0 (flag cleared first)
hipError_t launch_any_negative(const double* B, int64_t n, int* flag, hipStream_t stream);

// Asynchronous Gauss-Seidel (DI_GS_ASYNC), FP64, x in ws->H and y = d x / out
// in ws->F: x = B; then one sweep = the in-place sweep, the heavy rows and
// the stop test on ctl[0] (every kernel returns at once after the stop).
hipError_t launch_gs_init(const CycleArgs& a, const double* B, double b_uniform);
hipError_t launch_gs_sweep(const CycleArgs& a, const double* B, double b_uniform);

// ---- step-driven FP64 solve (di_solve.cpp) ----------------------------------
// One DI-SOP (or DI-CYC) solve in FP64, queued a chunk at a time on the
// caller's stream so that a caller moving other work (the serving worker)
// never waits for it. DI-SOP takes the window push (the graph's window
// configuration) when the graph allows it and allow_window is set (unless
// the graph's tuning found the pull faster), DI-CYC the select + pull pair.
//   solo_start queues the start state (F = B, H = 0 with B >= 0), the first
//     selection and the read-back of the control block;
//   solo_next, once that work has finished, reads the control block: done
//     != 0 ends the run (1 converged, 2 max_cycles, 3 non-finite);
//     otherwise it queues the next chunk of cycles and the read-back;
//   solo_finish queues X = H and fills the statistics (seconds 0). With the
//     window push it first gathers the fluid and sums the residual exactly
//     (waiting for the stream); should rounding leave that sum above tol, it
//     queues a new run from the gathered fluid instead and sets *again.
// The workspace is the run's own (not pooled); solo_run_bytes is its size.
struct SoloRun {
  di_graph* g = nullptr;
  Workspace* ws = nullptr;
  CycleArgs a{};
  int last_sel = 0;
  int chunk = 8;
  bool window = false;
  Ctl tot{};         // counters of the runs before a restart
  int restarts = 0;
  int max_cycles = 0;
};
size_t workspace_bytes(const di_graph* g, int prec);
size_t solo_run_bytes(const di_graph* g);
di_status solo_create(di_graph* g, SoloRun** out);
void solo_destroy(SoloRun* r);
di_status solo_start(SoloRun* r, const double* B_dev, double b_uniform, double d, double tol,
                     int method, int max_cycles, bool allow_window, hipStream_t stream);
di_status solo_next(SoloRun* r, int* done);
// Tunes the graph's window push (once per graph; a no-op when tuned), with
// an FP64 workspace of the graph's pool and a stream of its own.
di_status tune_window_f64(di_graph* g, double d);
di_status solo_finish(SoloRun* r, double* X_dev, di_stats* st, bool* again);
// FP64 residual pass: with H, first X += H and H = 0; then y = d X / out and
// R = B + P.X - X (B == nullptr: b_uniform everywhere), written to R_out as
// T, with the records of sum |R| and sum R in blk_part[0, pull_grid] (the
// last one covers the heavy rows). Every record is FP64.
template <typename T>
hipError_t launch_refine(const CycleArgs& a, double* X, T* H, const double* B, double b_uniform,
                         T* R_out);

}  // namespace di
