// libdi batched solves: k right-hand sides of one graph diffused together
// (personalized PageRank batches). Workspace pool per (graph, shape), the
// cycle loop with per-column stop states, and the residual passes of
// refined (FP32 + FP64) solves.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "di_batch.h"

namespace di {

void free_batch_ws(BatchWs* ws) {
  if (!ws) return;
  void* ptrs[] = {ws->F,   ws->H,       ws->sent,    ws->front_bits, ws->Bd,
                  ws->X64, ws->Y64,     ws->rec,     ws->rec_ops,    ws->rec_sel,
                  ws->rec_e, ws->segv,  ws->bctl};
  for (void* p : ptrs) (void)hipFree(p);
  if (ws->host_bctl) (void)hipHostFree(ws->host_bctl);
  for (hipEvent_t e : ws->events) (void)hipEventDestroy(e);
  delete ws;
}

namespace {

di_status bmalloc(void** p, size_t bytes) {
  hipError_t err = hipMalloc(p, bytes ? bytes : 1);
  if (err != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(err));
    return err == hipErrorOutOfMemory ? DI_E_NOMEM : DI_E_DEVICE;
  }
  return DI_OK;
}

int64_t nrec_needed(const di_graph* g) {
  return std::max<int64_t>(brecords_grid(g->n), (int64_t)pull_grid(g) + bheavy_grid(g));
}

di_status alloc_batch(const di_graph* g, int kp, int prec, bool refine, BatchWs** out) {
  BatchWs* ws = new (std::nothrow) BatchWs;
  if (!ws) return DI_E_NOMEM;
  ws->kp = kp;
  ws->prec = prec;
  const size_t n = (size_t)g->n, K = (size_t)kp;
  const size_t s = prec == kF64 ? sizeof(double) : sizeof(float);
  const size_t sgrid = (size_t)bselect_grid(g->n);
  ws->nrec_cap = nrec_needed(g);
  di_status st = DI_OK;
  if (st == DI_OK) st = bmalloc(&ws->F, n * K * s);
  if (st == DI_OK) st = bmalloc(&ws->H, n * K * s);
  if (st == DI_OK) st = bmalloc(&ws->sent, n * K * s);
  if (st == DI_OK) st = bmalloc((void**)&ws->front_bits, ((n + 63) / 64) * 8);
  if (st == DI_OK) st = bmalloc((void**)&ws->rec, (size_t)ws->nrec_cap * K * sizeof(double));
  if (st == DI_OK) st = bmalloc((void**)&ws->rec_ops, sgrid * (K + 1) * 8);
  if (st == DI_OK) st = bmalloc((void**)&ws->rec_sel, sgrid * (K + 1) * 4);
  if (st == DI_OK) st = bmalloc((void**)&ws->rec_e, sgrid * K * 8);
  if (st == DI_OK)
    st = bmalloc((void**)&ws->segv, (size_t)std::max<int64_t>(g->n_segs, 1) * K * sizeof(double));
  if (st == DI_OK) st = bmalloc((void**)&ws->bctl, (K + 1) * sizeof(BCtl));
  if (st == DI_OK) {
    hipError_t err = hipHostMalloc((void**)&ws->host_bctl, (K + 1) * sizeof(BCtl),
                                   hipHostMallocDefault);
    if (err != hipSuccess) {
      ws->host_bctl = nullptr;
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(err));
      st = DI_E_NOMEM;
    }
  }
  if (st == DI_OK && refine) {
    st = bmalloc((void**)&ws->Bd, n * K * 8);
    if (st == DI_OK) st = bmalloc((void**)&ws->X64, n * K * 8);
    if (st == DI_OK) st = bmalloc((void**)&ws->Y64, n * K * 8);
    // columns not being refined are read (never used) by the residual pull
    if (st == DI_OK && hipMemset(ws->Y64, 0, n * K * 8) != hipSuccess) st = DI_E_DEVICE;
    ws->refine_bufs = st == DI_OK;
  }
  if (st != DI_OK) {
    free_batch_ws(ws);
    return st;
  }
  *out = ws;
  return DI_OK;
}

}  // namespace

di_status batch_ws_create(const di_graph* g, int kp, int prec, bool refine, BatchWs** out) {
  return alloc_batch(g, kp, prec, refine, out);
}

size_t batch_ws_bytes(const di_graph* g, int kp, int prec, bool refine) {
  const size_t n = (size_t)g->n, K = (size_t)kp;
  const size_t s = prec == kF64 ? 8 : 4;
  const size_t sgrid = (size_t)bselect_grid(g->n);
  size_t b = 3 * n * K * s + ((n + 63) / 64) * 8 + (size_t)nrec_needed(g) * K * 8 +
             sgrid * (K + 1) * 12 + sgrid * K * 8 + (size_t)std::max<int64_t>(g->n_segs, 1) * K * 8 +
             (K + 1) * sizeof(BCtl);
  if (refine) b += 3 * n * K * 8;
  return b;
}

namespace {

BatchWs* acquire_batch(di_graph* g, int kp, int prec, bool refine, di_status* st) {
  {
    std::lock_guard<std::mutex> lock(g->mu);
    for (size_t q = 0; q < g->bpool.size(); ++q) {
      BatchWs* ws = g->bpool[q];
      if (ws->kp == kp && ws->prec == prec && (!refine || ws->refine_bufs)) {
        g->bpool.erase(g->bpool.begin() + (long)q);
        *st = DI_OK;
        return ws;
      }
    }
  }
  BatchWs* ws = nullptr;
  *st = alloc_batch(g, kp, prec, refine, &ws);
  return ws;
}

void release_batch(di_graph* g, BatchWs* ws) {
  std::lock_guard<std::mutex> lock(g->mu);
  g->bpool.push_back(ws);
}

struct BatchGuard {
  di_graph* g;
  BatchWs* ws;
  ~BatchGuard() {
    if (ws) release_batch(g, ws);
  }
};

di_status ensure_bevents(BatchWs* ws, size_t count) {
  while (ws->events.size() < count) {
    hipEvent_t e;
    DI_HIP(hipEventCreate(&e));
    ws->events.push_back(e);
  }
  return DI_OK;
}

int kp_for(int k) {
  int kp = 8;
  while (kp < k) kp <<= 1;
  return kp;
}

struct DeviceScopeB {
  int prev = -1;
  explicit DeviceScopeB(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceScopeB() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool column_active(int state) { return state == kBRun || state == kBInner || state == kBFresh; }

// One launch group of at most kBatchMaxKP columns: B_dev (k x n device, or
// NULL), X_dev (k x n device).
di_status batch_group(di_graph* g, int k, const double* B_dev, double d, const double* tol,
                      const di_opts& o, double* X_dev, di_stats* stats, hipStream_t stream) {
  const bool refine = o.precision == DI_FP32_REFINE;
  const int prec = o.precision == DI_FP64 ? kF64 : kF32;
  const int kp = kp_for(k);
  di_status ast = DI_OK;
  BatchWs* ws = acquire_batch(g, kp, prec, refine, &ast);
  if (ast != DI_OK) return ast;
  BatchGuard guard{g, ws};
  BatchArgs a{};
  a.g = g;
  a.kp = kp;
  a.ke = kp;
  a.prec = prec;
  a.d = d;
  a.method = o.method;
  a.max_cycles = o.max_cycles > 0 ? o.max_cycles : 100000;
  a.tol_rel = refine ? (o.inner_tol > 0.0 ? o.inner_tol : 1e-5) : -1.0;
  a.stream = stream;
  const bool timing = (o.flags & DI_FLAG_KERNEL_TIMING) != 0;
  DI_TRY(ensure_bevents(ws, 2));
  // control blocks: columns < k start fresh, the others idle
  for (int c = 0; c <= kp; ++c) {
    BCtl b;
    std::memset(&b, 0, sizeof(b));
    b.state = c < k ? kBFresh : kBIdle;
    b.tol = c < k ? tol[c] : 0.0;
    ws->host_bctl[c] = b;
  }
  DI_HIP(hipEventRecord(ws->events[0], stream));
  DI_HIP(hipMemcpyAsync(ws->bctl, ws->host_bctl, (size_t)(kp + 1) * sizeof(BCtl),
                        hipMemcpyHostToDevice, stream));
  DI_HIP(launch_bload(a, ws, B_dev, k, (1.0 - d) / (double)g->n));
  DI_HIP(launch_brecords(a, ws));
  DI_HIP(launch_bfirst(a, ws, brecords_grid(g->n), kBFresh));
  double move_seconds = 0.0;
  int move_launches = 0, queued = 0;
  const int guard_cycles = a.max_cycles + 8;
  for (;;) {
    DI_HIP(hipMemcpyAsync(ws->host_bctl, ws->bctl, (size_t)(kp + 1) * sizeof(BCtl),
                          hipMemcpyDeviceToHost, stream));
    DI_HIP(hipStreamSynchronize(stream));
    bool inner = false, active = false;
    int need = 2;
    for (int c = 0; c < k; ++c) {
      const BCtl& b = ws->host_bctl[c];
      inner |= b.state == kBInner;
      active |= column_active(b.state);
      if (b.state == kBRun) {
        // cycles still needed from this column's contraction so far
        int nc = 16;
        const double target = refine ? std::max(kInnerStop * b.tol, a.tol_rel * b.r_start) : b.tol;
        if (b.pass_cycles >= 1 && b.r > 0.0 && b.r < b.r_start && target > 0.0) {
          const double rate = std::log(b.r / b.r_start) / (double)b.pass_cycles;
          const double est = std::log(target / b.r) / rate;
          if (std::isfinite(est)) nc = (int)std::ceil(est) + 1;
        }
        need = std::max(need, nc);
      }
    }
    if (inner) {  // residual pass for the columns whose FP32 pass ended
      int nrec = 0;
      DI_HIP(launch_brefine(a, ws, &nrec));
      DI_HIP(launch_bfirst(a, ws, nrec, kBInner));
      continue;
    }
    if (!active) break;
    if (queued > 2 * guard_cycles + 64 * (kBMaxRefinements + 2)) {
      set_error("internal: batched columns did not stop");
      return DI_E_DEVICE;
    }
    const int chunk = std::max(2, std::min(need, 64));
    if (timing) DI_TRY(ensure_bevents(ws, 2 + 2 * (size_t)chunk));
    for (int q = 0; q < chunk; ++q) {
      hipEvent_t e0 = timing ? ws->events[2 + 2 * (size_t)q] : nullptr;
      hipEvent_t e1 = timing ? ws->events[3 + 2 * (size_t)q] : nullptr;
      DI_HIP(launch_bcycle(a, ws, e0, e1));
    }
    queued += chunk;
    if (timing) {
      DI_HIP(hipStreamSynchronize(stream));
      for (int q = 0; q < chunk; ++q) {
        float ms = 0.f;
        DI_HIP(hipEventElapsedTime(&ms, ws->events[2 + 2 * (size_t)q],
                                   ws->events[3 + 2 * (size_t)q]));
        move_seconds += ms * 1e-3;
      }
      move_launches += chunk;
    }
  }
  DI_HIP(launch_bstore(a, ws, X_dev, k, refine));
  DI_HIP(hipEventRecord(ws->events[1], stream));
  DI_HIP(hipEventSynchronize(ws->events[1]));
  float ms = 0.f;
  DI_HIP(hipEventElapsedTime(&ms, ws->events[0], ws->events[1]));
  // statistics: per column, and the batch's node-level totals
  const BCtl& tot = ws->host_bctl[kp];
  const double s = prec == kF64 ? 8.0 : 4.0, N = (double)g->n, K = (double)kp;
  const double C = (double)tot.cycles;
  // select: F row read, node word, bitmap; claims (F, H rows) and sent rows
  // of the frontier; pull: in-link ids and offsets, bitmap, the senders'
  // rows per gathered link, F rows read and written
  double sel_claims = 0.0;
  for (int c = 0; c < k; ++c) sel_claims += (double)ws->host_bctl[c].sel_total;
  const double select_b = C * N * (K * s + 4.0 + 0.125) + sel_claims * 3.0 * s +
                          (double)tot.sel_total * K * s;
  const double pull_b = C * ((double)g->Lp * 4.0 + N * 8.0 + N * 0.125) +
                        (double)tot.edges * K * s + C * N * K * s * 2.0;
  int refinements_max = 0;
  for (int c = 0; c < k; ++c) refinements_max = std::max(refinements_max, ws->host_bctl[c].refinements);
  const double refine_b =
      (double)refinements_max * ((double)g->Lp * (4.0 + K * 8.0) + N * K * (8.0 * 5 + 2.0 * s));
  di_status result = DI_OK;
  for (int c = 0; c < k; ++c) {
    const BCtl& b = ws->host_bctl[c];
    if (b.state == kBNonFinite) {
      set_error("column " + std::to_string(c) + ": the fluid became non-finite");
      result = DI_E_INVAL;
    } else if (b.state != kBConv && result == DI_OK) {
      set_error("column " + std::to_string(c) + ": max_cycles reached before the tolerance");
      result = DI_E_NOCONV;
    }
    if (stats) {
      di_stats& t = stats[c];
      std::memset(&t, 0, sizeof(t));
      t.cycles = b.cycles;
      t.fallback_cycles = b.fallback;
      t.refinements = b.refinements;
      t.move_launches = move_launches;
      t.edges_pushed = (int64_t)b.edges;
      t.nb_iter = g->L > 0 ? (double)b.edges / (double)g->L : 0.0;
      t.resid_l1 = b.final_r;
      t.err_bound = b.final_r / (1.0 - d);
      t.e = b.e;
      t.seconds = ms * 1e-3;
      t.move_seconds = move_seconds;
      t.bytes_moved = select_b + pull_b + refine_b;
      t.move_bytes = move_launches > 0 ? pull_b : 0.0;
      t.seconds_to_1e9 = -1.0;  // not recorded for batched columns
    }
  }
  return result;
}

di_status check_batch(const di_graph* g, int32_t k, double d, const double* tol, const di_opts& o) {
  if (!g) {
    set_error("graph is NULL");
    return DI_E_INVAL;
  }
  if (k < 1) {
    set_error("k must be >= 1");
    return DI_E_INVAL;
  }
  if (!tol) {
    set_error("tol is NULL");
    return DI_E_INVAL;
  }
  for (int c = 0; c < k; ++c)
    if (!(tol[c] > 0.0)) {
      set_error("tol[" + std::to_string(c) + "] must be > 0");
      return DI_E_INVAL;
    }
  if (!(d > 0.0 && d < 1.0)) {
    set_error("d must lie in (0, 1)");
    return DI_E_INVAL;
  }
  if (o.method != DI_SOP && o.method != DI_CYC) {
    set_error("batched solves run DI_SOP or DI_CYC");
    return DI_E_INVAL;
  }
  if (o.stop != DI_STOP_RESID) {
    set_error("batched solves stop on the residual only (DI_STOP_RESID)");
    return DI_E_INVAL;
  }
  if (o.precision != DI_FP64 && o.precision != DI_FP32 && o.precision != DI_FP32_REFINE) {
    set_error("unknown precision");
    return DI_E_INVAL;
  }
  if (o.kernel == DI_KERNEL_PUSH || o.kernel == DI_KERNEL_WINDOW) {
    set_error("batched solves move the fluid by the pull kernel only");
    return DI_E_INVAL;
  }
  return DI_OK;
}

di_status batch_any(const di_graph* gc, int32_t k, const double* B, bool on_host, double d,
                    const double* tol, const di_opts* opts, double* X, di_stats* stats) {
  di_opts o;
  di_opts_default(&o);
  if (opts) o = *opts;
  DI_TRY(check_batch(gc, k, d, tol, o));
  if (!X) {
    set_error("X is NULL");
    return DI_E_INVAL;
  }
  di_graph* g = const_cast<di_graph*>(gc);
  const size_t n = (size_t)g->n;
  if (B && on_host) {
    for (size_t q = 0; q < (size_t)k * n; ++q)
      if (!std::isfinite(B[q])) {
        set_error("B[" + std::to_string(q / n) + "][" + std::to_string(q % n) + "] is not finite");
        return DI_E_INVAL;
      }
  }
  DeviceScopeB scope(g->device);
  hipStream_t stream = (hipStream_t)o.stream;
  di_status result = DI_OK;
  for (int c0 = 0; c0 < k; c0 += kBatchMaxKP) {
    const int kk = std::min(k - c0, kBatchMaxKP);
    const size_t bytes = (size_t)kk * n * sizeof(double);
    double* Bg = nullptr;
    double* Xg = nullptr;
    struct Free {
      void* p;
      ~Free() {
        if (p) (void)hipFree(p);
      }
    } fb{nullptr}, fx{nullptr};
    const double* B_dev = B ? B + (size_t)c0 * n : nullptr;
    double* X_dev = X + (size_t)c0 * n;
    if (on_host) {
      if (B) {
        DI_TRY(bmalloc((void**)&Bg, bytes));
        fb.p = Bg;
        DI_HIP(hipMemcpyAsync(Bg, B_dev, bytes, hipMemcpyHostToDevice, stream));
        B_dev = Bg;
      }
      DI_TRY(bmalloc((void**)&Xg, bytes));
      fx.p = Xg;
      X_dev = Xg;
    }
    di_status rs = batch_group(g, kk, B_dev, d, tol + c0, o, X_dev, stats ? stats + c0 : nullptr,
                               stream);
    if (rs != DI_OK && rs != DI_E_NOCONV) return rs;
    if (on_host) DI_HIP(hipMemcpy(X + (size_t)c0 * n, Xg, bytes, hipMemcpyDeviceToHost));
    if (rs != DI_OK) result = rs;
  }
  return result;
}

template <typename Fn>
di_status guarded_b(Fn&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DI_E_NOMEM;
  } catch (...) {
    set_error("unexpected exception");
    return DI_E_INVAL;
  }
}

}  // namespace
}  // namespace di

extern "C" {

di_status di_solve_batch(const di_graph* g, int32_t k, const double* B, double d, const double* tol,
                         const di_opts* opts, double* X, di_stats* stats) {
  return di::guarded_b([&] { return di::batch_any(g, k, B, true, d, tol, opts, X, stats); });
}

di_status di_solve_batch_dev(const di_graph* g, int32_t k, const double* B_dev, double d,
                             const double* tol, const di_opts* opts, double* X_dev,
                             di_stats* stats) {
  return di::guarded_b([&] { return di::batch_any(g, k, B_dev, false, d, tol, opts, X_dev, stats); });
}

}  // extern "C"
