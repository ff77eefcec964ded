// libdi solve driver: workspace pool, the cycle loop and the stop check.
//
// The host queues whole cycles (reduce, select, push) in chunks; the device
// keeps the cycle index and the stop flag, and every kernel returns at once
// after the stop, so a chunk may run past convergence at the cost of empty
// launches. After each chunk the host reads the control block (a pinned
// copy) and sizes the next chunk from the observed contraction of r.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "di_internal.h"

namespace di {

void free_workspace(Workspace* ws) {
  if (!ws) return;
  (void)hipFree(ws->F);
  (void)hipFree(ws->H);
  (void)hipFree(ws->fr_start);
  (void)hipFree(ws->fr_base);
  (void)hipFree(ws->fr_s);
  (void)hipFree(ws->tile_first);
  (void)hipFree(ws->part_abs);
  (void)hipFree(ws->part_sum);
  (void)hipFree(ws->ctl);
  (void)hipFree(ws->X64);
  (void)hipFree(ws->R64);
  if (ws->host_ctl) (void)hipHostFree(ws->host_ctl);
  for (hipEvent_t e : ws->events) (void)hipEventDestroy(e);
  delete ws;
}

namespace {

di_status dmalloc(void** p, size_t bytes) {
  hipError_t err = hipMalloc(p, bytes ? bytes : 1);
  if (err != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(err));
    return err == hipErrorOutOfMemory ? DI_E_NOMEM : DI_E_DEVICE;
  }
  return DI_OK;
}

di_status alloc_workspace(const di_graph* g, int prec, Workspace** out) {
  Workspace* ws = new (std::nothrow) Workspace;
  if (!ws) return DI_E_NOMEM;
  ws->prec = prec;
  ws->n = g->n;
  const size_t n = (size_t)g->n;
  const size_t s = prec == kF64 ? sizeof(double) : sizeof(float);
  const size_t tiles = (size_t)((g->Lp + kPushTile - 1) / kPushTile) + 2;
  di_status st = DI_OK;
  if (st == DI_OK) st = dmalloc(&ws->F, n * s);
  if (st == DI_OK) st = dmalloc(&ws->H, n * s);
  if (st == DI_OK) st = dmalloc((void**)&ws->fr_start, n * sizeof(int64_t));
  if (st == DI_OK) st = dmalloc((void**)&ws->fr_base, n * sizeof(int64_t));
  if (st == DI_OK) st = dmalloc(&ws->fr_s, n * s);
  if (st == DI_OK) st = dmalloc((void**)&ws->tile_first, tiles * sizeof(int32_t));
  if (st == DI_OK) st = dmalloc((void**)&ws->part_abs, kMaxParts * sizeof(double));
  if (st == DI_OK) st = dmalloc((void**)&ws->part_sum, kMaxParts * sizeof(double));
  if (st == DI_OK) st = dmalloc((void**)&ws->ctl, sizeof(Ctl));
  if (st == DI_OK) st = dmalloc((void**)&ws->R64, n * sizeof(double));
  if (st == DI_OK) {
    hipError_t err = hipHostMalloc((void**)&ws->host_ctl, sizeof(Ctl), hipHostMallocDefault);
    if (err != hipSuccess) {
      ws->host_ctl = nullptr;
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(err));
      st = DI_E_NOMEM;
    }
  }
  if (st != DI_OK) {
    free_workspace(ws);
    return st;
  }
  *out = ws;
  return DI_OK;
}

Workspace* acquire(di_graph* g, int prec, di_status* st) {
  {
    std::lock_guard<std::mutex> lock(g->mu);
    for (size_t k = 0; k < g->pool.size(); ++k) {
      if (g->pool[k]->prec == prec) {
        Workspace* ws = g->pool[k];
        g->pool.erase(g->pool.begin() + (long)k);
        *st = DI_OK;
        return ws;
      }
    }
  }
  Workspace* ws = nullptr;
  *st = alloc_workspace(g, prec, &ws);
  return ws;
}

void release(di_graph* g, Workspace* ws) {
  std::lock_guard<std::mutex> lock(g->mu);
  g->pool.push_back(ws);
}

struct PoolGuard {
  di_graph* g;
  Workspace* ws;
  ~PoolGuard() {
    if (ws) release(g, ws);
  }
};

di_status ensure_events(Workspace* ws, size_t count) {
  while (ws->events.size() < count) {
    hipEvent_t e;
    DI_HIP(hipEventCreate(&e));
    ws->events.push_back(e);
  }
  return DI_OK;
}

// Runs cycles until the device reports a stop. Fills the timing fields of
// *st and leaves the final control block in ws->host_ctl.
template <typename T>
di_status run_cycles(const CycleArgs& a, bool timing, double* seconds, double* push_seconds,
                     int* push_launches) {
  Workspace* ws = a.ws;
  hipEvent_t ev_begin, ev_end;
  DI_TRY(ensure_events(ws, 2));
  ev_begin = ws->events[0];
  ev_end = ws->events[1];
  DI_HIP(hipEventRecord(ev_begin, a.stream));
  int launched = 0;
  int chunk = 8;
  for (;;) {
    const int todo = std::min(chunk, a.max_cycles + 1 - launched);
    if (timing) DI_TRY(ensure_events(ws, 2 + 2 * (size_t)(launched + todo)));
    for (int q = 0; q < todo; ++q) {
      DI_HIP(launch_reduce<T>(a));
      DI_HIP(launch_select<T>(a));
      if (timing) DI_HIP(hipEventRecord(ws->events[2 + 2 * (size_t)launched], a.stream));
      DI_HIP(launch_push<T>(a));
      if (timing) DI_HIP(hipEventRecord(ws->events[3 + 2 * (size_t)launched], a.stream));
      ++launched;
    }
    DI_HIP(hipEventRecord(ev_end, a.stream));
    DI_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, a.stream));
    DI_HIP(hipStreamSynchronize(a.stream));
    const Ctl& h = *ws->host_ctl;
    if (h.done) break;
    if (launched > a.max_cycles) {
      set_error("internal: the device did not stop after max_cycles");
      return DI_E_DEVICE;
    }
    // size the next chunk from the contraction of r per cycle so far
    int next = 16;
    if (a.stop == DI_STOP_RESID && h.cycles >= 2 && h.r_first > 0.0 && h.r_last > 0.0 &&
        h.r_last < h.r_first) {
      const double rate = std::log(h.r_last / h.r_first) / (double)(h.cycles - 1);
      const double need = std::log(a.tol / h.r_last) / rate;  // cycles still needed
      if (std::isfinite(need)) next = (int)std::ceil(need) + 1;
    }
    chunk = std::max(2, std::min(next, 64));
  }
  float ms = 0.f;
  DI_HIP(hipEventElapsedTime(&ms, ev_begin, ev_end));
  *seconds = ms * 1e-3;
  *push_seconds = 0.0;
  *push_launches = 0;
  if (timing) {
    const int real = std::min(ws->host_ctl->cycles, launched);
    for (int c = 0; c < real; ++c) {
      float pm = 0.f;
      DI_HIP(hipEventElapsedTime(&pm, ws->events[2 + 2 * (size_t)c], ws->events[3 + 2 * (size_t)c]));
      *push_seconds += pm * 1e-3;
    }
    *push_launches = real;
  }
  return DI_OK;
}

template <typename T>
void fill_stats(const di_graph* g, const Workspace* ws, double d, int precision_bytes, di_stats* st) {
  const Ctl& h = *ws->host_ctl;
  st->cycles = h.cycles;
  st->fallback_cycles = h.fallback;
  st->edges_pushed = (int64_t)h.edges_total;
  st->nb_iter = g->L > 0 ? (double)h.edges_total / (double)g->L : 0.0;
  st->resid_l1 = h.final_r;
  st->err_bound = h.final_r / (1.0 - d);
  st->paper_err = h.paper_err;
  st->e = h.e;
  // algorithmic bytes (s = bytes per fluid value):
  //   push:   per link 4 (index) + 2s (atomic read-modify-write);
  //           per frontier entry 8 + 8 + s (entry read into LDS);
  //   reduce: N s per cycle; select: N (s + 4) per cycle, 3s per diffused
  //           node (F write, H read and write), 8 + 8 + 8 + s per frontier
  //           entry (offset read, entry write).
  const double s = precision_bytes;
  const double push = (double)h.edges_total * (4.0 + 2.0 * s) + (double)h.front_total * (16.0 + s);
  const double per_cycle = (double)g->n * (2.0 * s + 4.0);
  st->push_bytes = push;
  st->bytes_moved = push + (double)h.cycles * per_cycle + (double)h.sel_total * 3.0 * s +
                    (double)h.front_total * (24.0 + s);
}

di_status status_from_done(int done) {
  if (done == 1) return DI_OK;
  if (done == 2) {
    set_error("max_cycles reached before the tolerance");
    return DI_E_NOCONV;
  }
  set_error("the fluid became non-finite (non-finite B?)");
  return DI_E_INVAL;
}

di_status check_common(const di_graph* g, double d, double tol, const di_opts& o) {
  if (!g) {
    set_error("graph is NULL");
    return DI_E_INVAL;
  }
  if (!(d > 0.0 && d < 1.0)) {
    set_error("d must lie in (0, 1)");
    return DI_E_INVAL;
  }
  if (o.stop == DI_STOP_RESID ? !(tol > 0.0) : !(tol >= 0.0)) {
    set_error("tol must be > 0 (>= 0 with DI_STOP_PAPER)");
    return DI_E_INVAL;
  }
  if (o.method != DI_SOP && o.method != DI_CYC) {
    set_error("unknown method");
    return DI_E_INVAL;
  }
  if (o.stop != DI_STOP_RESID && o.stop != DI_STOP_PAPER) {
    set_error("unknown stop rule");
    return DI_E_INVAL;
  }
  if (o.precision != DI_FP64 && o.precision != DI_FP32) {
    set_error("precision not supported by this entry point");
    return DI_E_INVAL;
  }
  return DI_OK;
}

struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename T>
di_status solve_t(di_graph* g, const double* B_dev, double d, double tol, const di_opts& o,
                  double* X_dev, di_stats* st, Workspace* ws, hipStream_t stream) {
  CycleArgs a{};
  a.g = g;
  a.ws = ws;
  a.d = d;
  a.tol = tol;
  a.method = o.method;
  a.stop = o.stop;
  a.max_cycles = o.max_cycles > 0 ? o.max_cycles : 100000;
  a.nparts = reduce_parts(g->n);
  a.push_grid = push_grid(g->Lp);
  a.stream = stream;
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(launch_init<T>(a, B_dev, (1.0 - d) / (double)g->n));
  double secs = 0.0, push_secs = 0.0;
  int push_launches = 0;
  di_status rs = run_cycles<T>(a, (o.flags & DI_FLAG_KERNEL_TIMING) != 0, &secs, &push_secs,
                               &push_launches);
  if (rs != DI_OK) return rs;
  DI_HIP(launch_h_to_x<T>(a, X_dev));
  DI_HIP(hipStreamSynchronize(stream));
  di_stats tmp;
  std::memset(&tmp, 0, sizeof(tmp));
  fill_stats<T>(g, ws, d, (int)sizeof(T), &tmp);
  tmp.seconds = secs;
  tmp.push_seconds = push_secs;
  tmp.push_launches = push_launches;
  if (st) *st = tmp;
  return status_from_done(ws->host_ctl->done);
}

di_status solve_any(const di_graph* gc, const double* B, bool B_on_host, double d, double tol,
                    const di_opts* opts, double* X, bool X_on_host, di_stats* st) {
  di_opts o;
  di_opts_default(&o);
  if (opts) o = *opts;
  di_status cs = check_common(gc, d, tol, o);
  if (cs != DI_OK) return cs;
  if (!X) {
    set_error("X is NULL");
    return DI_E_INVAL;
  }
  di_graph* g = const_cast<di_graph*>(gc);
  if (B && B_on_host) {
    for (int64_t i = 0; i < g->n; ++i)
      if (!std::isfinite(B[i])) {
        set_error("B[" + std::to_string(i) + "] is not finite");
        return DI_E_INVAL;
      }
  }
  DeviceScope scope(g->device);
  const int prec = o.precision == DI_FP64 ? kF64 : kF32;
  di_status ast = DI_OK;
  Workspace* ws = acquire(g, prec, &ast);
  if (ast != DI_OK) return ast;
  PoolGuard guard{g, ws};
  hipStream_t stream = (hipStream_t)o.stream;
  const size_t nbytes = (size_t)g->n * sizeof(double);
  const double* B_dev = B;
  if (B && B_on_host) {
    DI_HIP(hipMemcpyAsync(ws->R64, B, nbytes, hipMemcpyHostToDevice, stream));
    B_dev = ws->R64;
  }
  double* X_dev = X;
  if (X_on_host) {
    if (!ws->X64) {
      di_status s2 = dmalloc((void**)&ws->X64, nbytes);
      if (s2 != DI_OK) return s2;
    }
    X_dev = ws->X64;
  }
  di_status rs = prec == kF64 ? solve_t<double>(g, B_dev, d, tol, o, X_dev, st, ws, stream)
                              : solve_t<float>(g, B_dev, d, tol, o, X_dev, st, ws, stream);
  if (rs != DI_OK && rs != DI_E_NOCONV) return rs;
  if (X_on_host) DI_HIP(hipMemcpy(X, X_dev, nbytes, hipMemcpyDeviceToHost));
  return rs;
}

}  // namespace
}  // namespace di

extern "C" {

di_status di_solve(const di_graph* g, const double* B, double d, double tol, const di_opts* opts,
                   double* X, di_stats* stats) {
  try {
    return di::solve_any(g, B, true, d, tol, opts, X, true, stats);
  } catch (const std::bad_alloc&) {
    di::set_error("host allocation failed");
    return DI_E_NOMEM;
  } catch (...) {
    di::set_error("unexpected exception");
    return DI_E_INVAL;
  }
}

di_status di_solve_dev(const di_graph* g, const double* B_dev, double d, double tol,
                       const di_opts* opts, double* X_dev, di_stats* stats) {
  try {
    return di::solve_any(g, B_dev, false, d, tol, opts, X_dev, false, stats);
  } catch (const std::bad_alloc&) {
    di::set_error("host allocation failed");
    return DI_E_NOMEM;
  } catch (...) {
    di::set_error("unexpected exception");
    return DI_E_INVAL;
  }
}

di_status di_cycles_dev(const di_graph* gc, double d, int32_t method, double* F_dev,
                        double* H_dev, int32_t cycles, double* e_inout, void* stream_v,
                        di_stats* stats) {
  try {
    if (!gc || !F_dev || !H_dev || cycles < 0 || !(d > 0.0 && d < 1.0) ||
        (method != DI_SOP && method != DI_CYC)) {
      di::set_error("di_cycles_dev: invalid argument");
      return DI_E_INVAL;
    }
    di_graph* g = const_cast<di_graph*>(gc);
    di::DeviceScope scope(g->device);
    di_status ast = DI_OK;
    di::Workspace* ws = di::acquire(g, di::kF64, &ast);
    if (ast != DI_OK) return ast;
    di::PoolGuard guard{g, ws};
    // run on the caller's state: borrow the workspace with F and H swapped
    di::Workspace view = *ws;
    view.F = F_dev;
    view.H = H_dev;
    hipStream_t stream = (hipStream_t)stream_v;
    di::CycleArgs a{};
    a.g = g;
    a.ws = &view;
    a.d = d;
    a.tol = -1.0;  // never stops early
    a.method = method;
    a.stop = DI_STOP_RESID;
    a.max_cycles = cycles;
    a.nparts = di::reduce_parts(g->n);
    a.push_grid = di::push_grid(g->Lp);
    a.stream = stream;
    DI_HIP(di::launch_reset_ctl(a));
    if (e_inout)
      DI_HIP(hipMemcpyAsync(&ws->ctl->e, e_inout, sizeof(double), hipMemcpyHostToDevice, stream));
    double secs = 0.0, ps = 0.0;
    int pl = 0;
    di_status rs = di::run_cycles<double>(a, false, &secs, &ps, &pl);
    ws->events = view.events;  // keep events created while borrowing
    if (rs != DI_OK) return rs;
    const di::Ctl& h = *ws->host_ctl;
    if (h.done == 3) return di::status_from_done(3);
    if (e_inout) *e_inout = h.e;
    if (stats) {
      di_stats tmp;
      std::memset(&tmp, 0, sizeof(tmp));
      di::fill_stats<double>(g, ws, d, 8, &tmp);
      tmp.seconds = secs;
      *stats = tmp;
    }
    return DI_OK;
  } catch (const std::bad_alloc&) {
    di::set_error("host allocation failed");
    return DI_E_NOMEM;
  } catch (...) {
    di::set_error("unexpected exception");
    return DI_E_INVAL;
  }
}

}  // extern "C"
