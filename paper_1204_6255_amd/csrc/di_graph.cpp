// libdi host side: errors, device check, graph validation and upload.
//
// The graph input is the origin-sorted link list of Section 2.1. P is
// implied by it (Section 1): column j of P holds d/out_j at every link
// j -> i, out_j counting all links of j (self-loop included, Section 2.4).

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "di_internal.h"

namespace di {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

di_status check_device(int* device_out) {
  int count = 0;
  hipError_t err = hipGetDeviceCount(&count);
  if (err != hipSuccess || count <= 0) {
    set_error(std::string("no HIP device available (") +
              (err != hipSuccess ? hipGetErrorString(err) : "0 devices") +
              "); libdi has no CPU fallback");
    (void)hipGetLastError();
    return DI_E_DEVICE;
  }
  int dev = 0;
  DI_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  DI_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("libdi is built for gfx950, the current device is ") + prop.gcnArchName);
    return DI_E_DEVICE;
  }
  if (device_out) *device_out = dev;
  return DI_OK;
}

void free_workspace(Workspace* ws);

}  // namespace di

namespace {

void free_graph_device(di_graph* g) {
  (void)hipFree(g->row_ptr);
  (void)hipFree(g->col);
  (void)hipFree(g->info);
  (void)hipFree(g->csc_ptr);
  (void)hipFree(g->csc_idx);
  g->row_ptr = nullptr;
  g->col = nullptr;
  g->info = nullptr;
  g->csc_ptr = nullptr;
  g->csc_idx = nullptr;
}

template <typename V>
di_status upload(V** dst, const std::vector<V>& src) {
  const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(V);
  hipError_t err = hipMalloc((void**)dst, bytes);
  if (err != hipSuccess) {
    *dst = nullptr;
    di::set_error(std::string("hipMalloc of ") + std::to_string(bytes) +
                  " bytes: " + hipGetErrorString(err));
    (void)hipGetLastError();
    return err == hipErrorOutOfMemory ? DI_E_NOMEM : DI_E_DEVICE;
  }
  if (!src.empty()) DI_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
  return DI_OK;
}

}  // namespace

extern "C" {

const char* di_last_error(void) { return di::g_error.c_str(); }

int32_t di_version(void) { return (1 << 16) | 0; }

void di_opts_default(di_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = DI_SOP;
  o->precision = DI_FP64;
  o->stop = DI_STOP_RESID;
  o->max_cycles = 100000;
  o->flags = 0;
  o->inner_tol = 1e-5;
  o->stream = nullptr;
}

di_status di_graph_create(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                          uint32_t flags, di_graph** out) {
  try {
    if (!out) {
      di::set_error("di_graph_create: out is NULL");
      return DI_E_INVAL;
    }
    *out = nullptr;
    if (n <= 0 || n > 0x7fffffffLL) {
      di::set_error("di_graph_create: n must be in [1, 2^31 - 1]");
      return DI_E_INVAL;
    }
    if (m < 0 || m >= (1LL << 33)) {
      di::set_error("di_graph_create: m must be in [0, 2^33)");
      return DI_E_INVAL;
    }
    if (m > 0 && (!src || !dst)) {
      di::set_error("di_graph_create: src or dst is NULL");
      return DI_E_INVAL;
    }
    // validation, in one pass, before any device work
    for (int64_t e = 0; e < m; ++e) {
      const int64_t a = src[e], b = dst[e];
      if (a < 0 || a >= n || b < 0 || b >= n) {
        di::set_error("di_graph_create: link " + std::to_string(e) + " (" + std::to_string(a) +
                      " -> " + std::to_string(b) + ") has an id outside [0, n)");
        return DI_E_RANGE;
      }
      if (e > 0) {
        const int64_t pa = src[e - 1], pb = dst[e - 1];
        if (a < pa || (a == pa && b < pb)) {
          di::set_error("di_graph_create: links are not sorted by (origin, destination) at link " +
                        std::to_string(e));
          return DI_E_UNSORTED;
        }
        if (a == pa && b == pb) {
          di::set_error("di_graph_create: link " + std::to_string(a) + " -> " + std::to_string(b) +
                        " is listed twice");
          return DI_E_DUP;
        }
      }
    }
    int dev = 0;
    di_status st = di::check_device(&dev);
    if (st != DI_OK) return st;

    // host build: out-link lists without self-loops, per-node words, CSC
    std::vector<int64_t> row_ptr((size_t)n + 1, 0);
    std::vector<uint32_t> info((size_t)n, 0);
    int64_t n_loops = 0;
    for (int64_t e = 0; e < m; ++e) {
      const int32_t a = src[e];
      info[a] += 1;
      if (a == dst[e]) {
        info[a] |= di::kLoopBit;
        ++n_loops;
      } else {
        row_ptr[a + 1] += 1;
      }
    }
    int64_t n_dangling = 0, max_out = 0;
    for (int64_t i = 0; i < n; ++i) {
      row_ptr[i + 1] += row_ptr[i];
      const int64_t o = info[i] & di::kOutMask;
      n_dangling += o == 0;
      max_out = std::max(max_out, o);
    }
    const int64_t Lp = row_ptr[n];
    std::vector<int32_t> col((size_t)Lp);
    {
      int64_t q = 0;
      for (int64_t e = 0; e < m; ++e)
        if (src[e] != dst[e]) col[q++] = dst[e];
    }
    di_graph* g = new di_graph;
    g->n = n;
    g->L = m;
    g->Lp = Lp;
    g->n_dangling = n_dangling;
    g->n_loops = n_loops;
    g->max_out = max_out;
    g->device = dev;
    st = upload(&g->row_ptr, row_ptr);
    if (st == DI_OK) st = upload(&g->col, col);
    if (st == DI_OK) st = upload(&g->info, info);
    std::vector<int64_t>().swap(row_ptr);
    std::vector<int32_t>().swap(col);
    if (st == DI_OK && (flags & DI_BUILD_CSC)) {
      std::vector<int64_t> cptr((size_t)n + 1, 0);
      for (int64_t e = 0; e < m; ++e) cptr[dst[e] + 1] += 1;
      for (int64_t i = 0; i < n; ++i) cptr[i + 1] += cptr[i];
      std::vector<int32_t> cidx((size_t)m);
      std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
      for (int64_t e = 0; e < m; ++e) cidx[fill[dst[e]]++] = src[e];
      st = upload(&g->csc_ptr, cptr);
      if (st == DI_OK) st = upload(&g->csc_idx, cidx);
      g->has_csc = st == DI_OK;
    }
    if (st != DI_OK) {
      free_graph_device(g);
      delete g;
      return st;
    }
    *out = g;
    return DI_OK;
  } catch (const std::bad_alloc&) {
    di::set_error("di_graph_create: host allocation failed");
    return DI_E_NOMEM;
  } catch (...) {
    di::set_error("di_graph_create: unexpected exception");
    return DI_E_INVAL;
  }
}

void di_graph_destroy(di_graph* g) {
  if (!g) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != g->device) (void)hipSetDevice(g->device);
  {
    std::lock_guard<std::mutex> lock(g->mu);
    for (di::Workspace* ws : g->pool) di::free_workspace(ws);
    g->pool.clear();
  }
  free_graph_device(g);
  if (cur != g->device) (void)hipSetDevice(cur);
  delete g;
}

di_status di_graph_info(const di_graph* g, int64_t* n, int64_t* m, int64_t* n_dangling,
                        int64_t* n_loops) {
  if (!g) {
    di::set_error("di_graph_info: graph is NULL");
    return DI_E_INVAL;
  }
  if (n) *n = g->n;
  if (m) *m = g->L;
  if (n_dangling) *n_dangling = g->n_dangling;
  if (n_loops) *n_loops = g->n_loops;
  return DI_OK;
}

}  // extern "C"
