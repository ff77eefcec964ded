// The residual entry point for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops): the same FP64
// residual pass as di_residual_dev, with its scratch buffers carved out of a
// fixed device array instead of the graph's pooled workspace.
//
// `scratch` is a file-scope device array; every GPU the library runs on
// holds its own copy until the process ends. Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in
// symbol): the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress and used from then on.

#include <mutex>
#include <string>

#include "di_internal.h"

namespace di {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (looked up on first use
// with the device current).
di_status scratch_ptr(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("di_residual_dev_noalloc: device index " + std::to_string(dev) + " out of range");
    return DI_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(err));
      (void)hipGetLastError();
      return DI_E_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return DI_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

di_status residual_noalloc(const di_graph* gc, const double* B_dev, double d, const double* X_dev,
                           double* R_dev, double* l1_out, void* stream_v) {
  if (!gc || !X_dev || !(d > 0.0 && d < 1.0)) {
    set_error("di_residual_dev_noalloc: invalid argument");
    return DI_E_INVAL;
  }
  di_graph* g = const_cast<di_graph*>(gc);
  const int grid = pull_grid(g);
  const size_t n = (size_t)g->n;
  // layout: y, the segment sums, the records (grid + 1), |R|_1, and R when
  // the caller passes none
  const size_t off_seg = align256(n * sizeof(double));
  const size_t off_part =
      off_seg + align256((size_t)std::max<int64_t>(g->n_segs, 1) * sizeof(double));
  const size_t off_l1 = off_part + align256(((size_t)grid + 1) * sizeof(Part));
  const size_t off_r = off_l1 + 256;
  const size_t need = R_dev ? off_r : off_r + n * sizeof(double);
  if (need > kScratchBytes) {
    set_error("di_residual_dev_noalloc: the graph needs " + std::to_string(need) +
              " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
              " bytes available (n = " + std::to_string(n) + (R_dev ? "" : ", R in scratch") + ")");
    return DI_E_INVAL;
  }
  int prev = -1;
  DI_HIP(hipGetDevice(&prev));
  if (prev != g->device) DI_HIP(hipSetDevice(g->device));
  struct Restore {
    int prev, dev;
    ~Restore() {
      if (prev != dev) (void)hipSetDevice(prev);
    }
  } restore{prev, g->device};
  unsigned char* base = nullptr;
  DI_TRY(scratch_ptr(g->device, &base));
  Workspace ws;  // borrowed pointers only: nothing here is allocated or freed
  ws.Y64 = (double*)base;
  ws.seg_val = (double*)(base + off_seg);
  ws.blk_part = (Part*)(base + off_part);
  double* l1_dev = (double*)(base + off_l1);
  double* R = R_dev ? R_dev : (double*)(base + off_r);
  CycleArgs a{};
  a.g = g;
  a.ws = &ws;
  a.d = d;
  a.direction = kPull;
  a.stream = (hipStream_t)stream_v;
  DI_HIP(launch_refine<double>(a, const_cast<double*>(X_dev), (double*)nullptr, B_dev,
                               (1.0 - d) / (double)g->n, R));
  // |R|_1 from the pass's records in the order di_residual_dev sums them
  // (its pabs, the record's first field, at l1_dev)
  DI_HIP(launch_sum_parts(a, grid + 1, (Part*)l1_dev));
  double l1 = 0.0;
  DI_HIP(hipMemcpyAsync(&l1, l1_dev, sizeof(double), hipMemcpyDeviceToHost, a.stream));
  DI_HIP(hipStreamSynchronize(a.stream));
  if (l1_out) *l1_out = l1;
  return DI_OK;
}

}  // namespace
}  // namespace di

extern "C" di_status di_residual_dev_noalloc(const di_graph* g, const double* B_dev, double d,
                                             const double* X_dev, double* R_dev, double* l1,
                                             void* stream) {
  try {
    return di::residual_noalloc(g, B_dev, d, X_dev, R_dev, l1, stream);
  } catch (...) {
    di::set_error("di_residual_dev_noalloc: unexpected exception");
    return DI_E_INVAL;
  }
}
