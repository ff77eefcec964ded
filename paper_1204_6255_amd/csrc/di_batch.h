// Batched D-iteration (k right-hand sides on one graph): device state and
// launchers. Internal to libdi.
//
// The k fluids are stored node-major, [n][KP] (the KP >= k values of a node
// contiguous, KP a power of two in [8, 256]; columns k..KP-1 are idle), so a
// node's values move in one coalesced access. Every column has its own r,
// tolerance, pass state and counters (BCtl); the frontier bitmap marks the
// nodes that send in at least one column.
#pragma once

#include "di_internal.h"

namespace di {

constexpr int kBatchMaxKP = 256;   // columns per batch launch
constexpr int kBBlock = 256;       // threads per batched block
constexpr int kBSelectMaxGrid = 4096;
constexpr int kBHeavyMaxGrid = 256;
constexpr int kBMaxRefinements = 100;  // a column stops (max_cycles state) after this many

// column states
enum BState {
  kBRun = 0,        // selecting every cycle
  kBConv = 1,       // converged: residual <= tol
  kBMaxCyc = 2,     // max_cycles reached
  kBNonFinite = 3,  // non-finite fluid
  kBInner = 4,      // FP32 pass ended: waiting for a residual pass
  kBFresh = 6,      // loaded: the next first-selection reduction starts it
  kBIdle = 7        // padding column or free slot
};

// Per-column control block (entries 0..KP-1), and one more entry (KP)
// holding node-level totals of the batch.
struct BCtl {
  double r;           // sum |F_c| at the start of the next cycle
  double r_start;     // sum |F_c| when the current pass started
  double final_r;     // r (or the FP64 residual) when the column stopped
  double tol;         // converged when the residual is <= tol
  double e;           // fluid absorbed by dangling nodes
  unsigned long long edges;      // link operations (entry KP: links gathered)
  unsigned long long sel_total;  // diffused nodes (entry KP: frontier nodes)
  int cycles;         // cycles run (entry KP: cycles with a running column)
  int pass_cycles;    // cycles of the current pass
  int refinements;    // residual passes
  int fallback;       // DI-CYC cycles after an empty DI-SOP cycle
  int state;          // BState
  int cyc_mode;       // the next cycle selects every |F| > 0
};

struct BatchArgs {
  const di_graph* g;
  int kp;              // columns (8 .. 256, power of two)
  int ke;              // working width: columns >= ke are idle (8 .. kp,
                       // power of two); the cycle and residual kernels
                       // look at columns [0, ke) only
  int prec;            // kF64 or kF32
  double d;
  int method;          // DI_SOP or DI_CYC
  int max_cycles;
  double tol_rel;      // refined solve: inner stop relative to r_start (< 0: none)
  hipStream_t stream;
};

// Device buffers of one batch shape, pooled per graph.
struct BatchWs {
  int kp = 0;
  int prec = kF64;
  bool refine_bufs = false;
  void* F = nullptr;           // [n][kp] fluid
  void* H = nullptr;           // [n][kp] history
  void* sent = nullptr;        // [n][kp] amount per link of each sender
  unsigned long long* front_bits = nullptr;  // node-level frontier
  double* Bd = nullptr;        // [n][kp] right-hand sides (refined solves)
  double* X64 = nullptr;       // [n][kp] FP64 solution (refined solves)
  double* Y64 = nullptr;       // [n][kp] d X / out (refined solves)
  double* rec = nullptr;       // [nrec][kp] sums of |F| per block
  int64_t nrec_cap = 0;
  unsigned long long* rec_ops = nullptr;  // [select grid][kp + 1]
  unsigned int* rec_sel = nullptr;        // [select grid][kp + 1]
  double* rec_e = nullptr;                // [select grid][kp]
  double* segv = nullptr;      // [n_segs][kp] heavy-row segment sums
  BCtl* bctl = nullptr;        // kp + 1 entries
  BCtl* host_bctl = nullptr;   // pinned copy
  std::vector<hipEvent_t> events;
};

void free_batch_ws(BatchWs* ws);

int bselect_grid(int64_t n);
int bheavy_grid(const di_graph* g);
int brecords_grid(int64_t n);

// F, H (and Bd, X64 when given) from the caller's k x n right-hand sides
// (B_in == nullptr: b_uniform everywhere); columns >= k are zero.
hipError_t launch_bload(const BatchArgs& a, BatchWs* ws, const double* B_in, int k,
                        double b_uniform);
// per-block sums of |F| per column: rec[0, brecords_grid)
hipError_t launch_brecords(const BatchArgs& a, BatchWs* ws);
// one cycle: selection, pull, heavy rows, per-column reduction
hipError_t launch_bcycle(const BatchArgs& a, BatchWs* ws, hipEvent_t ev0, hipEvent_t ev1);
// per-column reduction of the records of a load (want = kBFresh) or of a
// residual pass (want = kBInner): those columns start a pass; nrec records
hipError_t launch_bfirst(const BatchArgs& a, BatchWs* ws, int nrec, int want);
// residual pass for the columns in state kBInner: X += H, H = 0, y, and
// F = R = B + P.X - X with the records of |R|; returns the record count
hipError_t launch_brefine(const BatchArgs& a, BatchWs* ws, int* nrec);
// X_out (k x n) = H (+ X64 when refined)
hipError_t launch_bstore(const BatchArgs& a, BatchWs* ws, double* X_out, int k, bool refined);

// Starting columns of a running batch (device arrays): flag[KP] marks the
// columns to clear (b_uni[c]: their uniform right-hand side value, 0 for
// seed lists); entry j < ncols starts column col[j] with value val[j] at
// seeds[off[j] .. off[j+1]) and tolerance tol[j].
struct ColInit {
  int ncols;
  const int* flag;
  const double* b_uni;
  const int* col;
  const int64_t* off;
  const int32_t* seeds;
  const double* val;
  const double* tol;
};
hipError_t launch_bcol_init(const BatchArgs& a, BatchWs* ws, const ColInit& ci);
// X_out (n doubles, device) = column c of H (+ X64 when refined)
hipError_t launch_bcol_out(const BatchArgs& a, BatchWs* ws, int c, bool refined, double* X_out);
// x[idx[q]] = v for q < count, on stream (indices in range: the caller checks).
hipError_t launch_scatter_value(hipStream_t stream, double* x, const int32_t* idx, int64_t count,
                                double v);
// allocation and pooling of batch workspaces (di_batch.cpp)
di_status batch_ws_create(const di_graph* g, int kp, int prec, bool refine, BatchWs** out);
size_t batch_ws_bytes(const di_graph* g, int kp, int prec, bool refine);

}  // namespace di
