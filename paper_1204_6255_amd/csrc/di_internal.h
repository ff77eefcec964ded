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
constexpr int kSelectBlock = 256;     // threads per select block
constexpr int kSelectPerThread = 4;   // consecutive nodes per select thread
constexpr int kSelectNodes = kSelectBlock * kSelectPerThread;
constexpr int kPushBlock = 256;       // threads per push block
constexpr int kPushTile = 1024;       // frontier links per push tile
constexpr int kReduceBlock = 256;     // threads per reduction block
constexpr int kMaxParts = 256;        // reduction blocks (partial sums)
constexpr int kMaxPushGrid = 4096;    // push blocks (grid-stride over tiles)

// Per-node word: out-degree (self-loop included) in bits 0..30, self-loop
// flag in bit 31.
constexpr uint32_t kLoopBit = 0x80000000u;
constexpr uint32_t kOutMask = 0x7fffffffu;

// Frontier counter: selected nodes with out-links in bits 0..30, their
// links (self-loops excluded) in bits 31..63. One 64-bit atomic reserves
// both ranges, so link offsets grow with frontier positions.
constexpr int kPackShift = 31;
constexpr uint64_t kPackNodeMask = (1ull << kPackShift) - 1;

// Device control block of one solve. Three rotating slots keep the counters
// of cycles c-1, c and c+1 apart (slot c % 3).
struct Ctl {
  double e;               // fluid absorbed by dangling nodes (atomics)
  double e_snap;          // e at the start of the current cycle
  double final_r;         // sum |F| at the stop test that ended the solve
  double paper_err;       // last sum F / (1 - d - d e)
  double r_last;          // r of the last diffusion cycle
  double r_first;         // r of the first cycle
  unsigned long long packed[3];  // frontier counter per slot
  unsigned int sel[3];           // diffused nodes (dangling ones too) per slot
  int cycles;             // cycles run
  int fallback;           // DI-CYC cycles run after an empty DI-SOP cycle
  int done;               // 0 running, 1 converged, 2 stopped at max_cycles,
                          // 3 non-finite fluid
  int cur;                // index of the current cycle (-1 before the first)
  unsigned long long edges_total;  // link operations so far
  unsigned long long front_total;  // frontier entries so far
  unsigned long long sel_total;    // diffused nodes so far
};

enum Prec { kF64 = 0, kF32 = 1 };

// Buffers of one solve; pooled per graph so repeated solves do not allocate.
struct Workspace {
  int prec = kF64;
  int64_t n = 0;
  void* F = nullptr;           // fluid, n values of the fluid type
  void* H = nullptr;           // history, n values
  int64_t* fr_start = nullptr; // frontier: first link offset of each entry
  int64_t* fr_base = nullptr;  // frontier: CSR offset of the node's links
  void* fr_s = nullptr;        // frontier: amount sent along each link
  int32_t* tile_first = nullptr;  // frontier entry holding link b*kPushTile
  double* part_abs = nullptr;  // per-block sum |F|
  double* part_sum = nullptr;  // per-block sum F
  Ctl* ctl = nullptr;
  Ctl* host_ctl = nullptr;     // pinned copy for the stop check
  double* X64 = nullptr;       // FP64 solution (refinement)
  double* R64 = nullptr;       // FP64 residual / scratch (refinement)
  std::vector<hipEvent_t> events;
};

}  // namespace di

struct di_graph {
  int64_t n = 0;
  int64_t L = 0;           // links, self-loops included
  int64_t Lp = 0;          // links pushed by a diffusion (self-loops removed)
  int64_t n_dangling = 0;
  int64_t n_loops = 0;
  int64_t max_out = 0;
  int device = 0;
  bool has_csc = false;
  // out-links (columns of P): CSR without self-loops
  int64_t* row_ptr = nullptr;  // n + 1
  int32_t* col = nullptr;      // Lp
  uint32_t* info = nullptr;    // n: out-degree | self-loop bit
  // in-links (rows of P), self-loops kept
  int64_t* csc_ptr = nullptr;  // n + 1
  int32_t* csc_idx = nullptr;  // L
  std::mutex mu;
  std::vector<di::Workspace*> pool;
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

// ---- kernel launchers (di_kernels.hip) ------------------------------------
struct CycleArgs {
  const di_graph* g;
  Workspace* ws;
  double d;
  double tol;
  int method;      // DI_SOP or DI_CYC
  int stop;        // DI_STOP_RESID or DI_STOP_PAPER
  int max_cycles;  // the stop test of cycle max_cycles ends the solve
  int nparts;      // reduction blocks
  int push_grid;   // push blocks
  hipStream_t stream;
};

// The device keeps the cycle index (Ctl::cur), so every cycle is the same
// three launches: reduce, select, push.
hipError_t launch_reset_ctl(const CycleArgs& a);
template <typename T>
hipError_t launch_init(const CycleArgs& a, const double* B, double b_uniform);
template <typename T>
hipError_t launch_reduce(const CycleArgs& a);
template <typename T>
hipError_t launch_select(const CycleArgs& a);
template <typename T>
hipError_t launch_push(const CycleArgs& a);
template <typename T>
hipError_t launch_h_to_x(const CycleArgs& a, double* X);

int reduce_parts(int64_t n);
int push_grid(int64_t Lp);

}  // namespace di
