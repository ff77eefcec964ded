// libdi solve driver: workspace pool, the cycle loop and the stop check.
//
// The host queues whole cycles in chunks; the device keeps the stop flag and
// every kernel returns at once after the stop, so a chunk may run past
// convergence at the cost of empty launches. After each chunk the host reads
// the control block (a pinned copy) and sizes the next chunk from the
// observed contraction of r per cycle.
//
// Also here: the FP32 + FP64 refinement loop, the residual entry point, the
// asynchronous Gauss-Seidel baseline's driver, and a step-driven FP64 solve
// that the serving worker advances a chunk at a time.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>

#include "di_internal.h"

namespace di {

void free_workspace(Workspace* ws) {
  if (!ws) return;
  void* ptrs[] = {ws->F,         ws->H,         ws->sent,     ws->front_bits,
                  ws->fr_lstart, ws->fr_base,   ws->fr_s,     ws->tile_stat,
                  ws->blk_part,  ws->seg_val,   ws->ctl,      ws->X64,      ws->B64,
                  ws->Y64,       ws->trace,     ws->hret,     ws->hacc,
                  ws->wA,        ws->whalo,     ws->whub,     ws->wrec,     ws->wflag};
  for (void* p : ptrs) (void)hipFree(p);
  if (ws->host_ctl) (void)hipHostFree(ws->host_ctl);
  if (ws->host_flag) (void)hipHostFree(ws->host_flag);
  if (ws->host_part) (void)hipHostFree(ws->host_part);
  for (hipEvent_t e : ws->events) (void)hipEventDestroy(e);
  if (ws->copied) (void)hipEventDestroy(ws->copied);
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
  const size_t n = (size_t)g->n;
  const size_t s = prec == kF64 ? sizeof(double) : sizeof(float);
  const size_t ntiles =
      (size_t)std::max(select_stat_records(g->n, kPull), select_stat_records(g->n, kPush));
  // one record per pull/reduce block, plus the heavy-row record of a
  // residual pass
  const size_t nparts = (size_t)std::max(kPullMaxGrid, kReduceGrid) + 1;
  di_status st = DI_OK;
  if (st == DI_OK) st = dmalloc(&ws->F, n * s);
  if (st == DI_OK) st = dmalloc(&ws->H, n * s);
  if (st == DI_OK) st = dmalloc(&ws->sent, n * s);
  if (st == DI_OK) st = dmalloc((void**)&ws->front_bits, ((n + 63) / 64) * sizeof(unsigned long long));
  if (st == DI_OK) st = dmalloc((void**)&ws->tile_stat, ntiles * sizeof(SelStat));
  if (st == DI_OK) st = dmalloc((void**)&ws->blk_part, nparts * sizeof(Part));
  if (st == DI_OK)
    st = dmalloc((void**)&ws->seg_val, (size_t)std::max<int64_t>(g->n_segs, 1) * sizeof(double));
  const size_t nh = (size_t)std::max<int64_t>(g->n_heavy, 1);
  if (st == DI_OK) st = dmalloc(&ws->hret, 2 * nh * s);
  if (st == DI_OK) st = dmalloc((void**)&ws->hacc, 2 * nh * sizeof(double));
  if (st == DI_OK) st = dmalloc((void**)&ws->ctl, 2 * sizeof(Ctl));
  if (st == DI_OK) {
    // coherent (fine-grained) pinned memory: the selection kernels store the
    // control block straight into it
    hipError_t err = hipHostMalloc((void**)&ws->host_ctl, 2 * sizeof(Ctl), hipHostMallocCoherent);
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

// Push buffers are allocated on first use (pull solves never need them).
di_status ensure_push_buffers(const di_graph* g, Workspace* ws) {
  if (ws->fr_lstart) return DI_OK;
  const size_t slots = (size_t)select_tiles(g->n, kPush) * kSelectTilePush;
  const size_t s = ws->prec == kF64 ? sizeof(double) : sizeof(float);
  DI_TRY(dmalloc((void**)&ws->fr_base, slots * sizeof(int64_t)));
  DI_TRY(dmalloc(&ws->fr_s, slots * s));
  DI_TRY(dmalloc((void**)&ws->fr_lstart, slots * sizeof(int64_t)));
  return DI_OK;
}

// Window-push buffers, allocated on first use: far accumulators, halos, hub
// partials and records, two copies each, and the sign flag.
di_status ensure_window_buffers(const di_graph* g, Workspace* ws) {
  if (ws->wA) return DI_OK;
  const size_t s = ws->prec == kF64 ? sizeof(double) : sizeof(float);
  // sized for every configuration: the smallest tile (most halos), the
  // largest grid and hub count
  DI_TRY(dmalloc(&ws->whalo, 2 * (size_t)std::max<int64_t>(g->n_wtiles[0], 1) * 2 * kWinHalo * s));
  DI_TRY(dmalloc(&ws->whub, 2 * (size_t)win_hub_rows(g->n_wtiles[0]) * kWinHubMax * s));
  DI_TRY(dmalloc((void**)&ws->wrec, 2 * (size_t)kWinMaxGrid * sizeof(Part)));
  DI_TRY(dmalloc((void**)&ws->wflag, sizeof(int)));
  if (!ws->host_flag) {
    hipError_t err = hipHostMalloc((void**)&ws->host_flag, sizeof(int), hipHostMallocDefault);
    if (err != hipSuccess) {
      ws->host_flag = nullptr;
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(err));
      return DI_E_NOMEM;
    }
  }
  DI_TRY(dmalloc(&ws->wA, 2 * (size_t)win_stride(g->n) * s));  // last: marks the set complete
  return DI_OK;
}

// Bytes of the window-push buffers of a workspace of precision prec.
size_t window_bytes(const di_graph* g, int prec) {
  const size_t s = prec == kF64 ? sizeof(double) : sizeof(float);
  return 2 * (size_t)std::max<int64_t>(g->n_wtiles[0], 1) * 2 * kWinHalo * s +
         2 * (size_t)win_hub_rows(g->n_wtiles[0]) * kWinHubMax * s +
         2 * (size_t)kWinMaxGrid * sizeof(Part) + sizeof(int) + 2 * (size_t)win_stride(g->n) * s;
}

// Pinned host copy of the per-block records, allocated on first use.
di_status ensure_host_part(Workspace* ws) {
  if (!ws->host_part) {
    hipError_t err = hipHostMalloc((void**)&ws->host_part, sizeof(Part), hipHostMallocCoherent);
    if (err != hipSuccess) {
      ws->host_part = nullptr;
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(err));
      return DI_E_NOMEM;
    }
  }
  return DI_OK;
}

// Residual-pass buffers, allocated on first use.
di_status ensure_refine_buffers(const di_graph* g, Workspace* ws) {
  if (!ws->Y64) DI_TRY(dmalloc((void**)&ws->Y64, (size_t)g->n * sizeof(double)));
  return ensure_host_part(ws);
}

// sum |R| (and sum R) of the records [0, count) of a residual pass, in
// k_sum_parts' fixed order: residual_queue sums them on the device into
// host_part[0]; residual_wait waits for the stream and reads the sums.
di_status residual_queue(const CycleArgs& a, int count) {
  DI_HIP(launch_sum_parts(a, count, a.ws->host_part));
  return DI_OK;
}
di_status residual_wait(const CycleArgs& a, double* l1, double* sum) {
  DI_HIP(hipStreamSynchronize(a.stream));
  *l1 = a.ws->host_part[0].pabs;
  if (sum) *sum = a.ws->host_part[0].psum;
  return DI_OK;
}
di_status residual_norm(const CycleArgs& a, int count, double* l1, double* sum) {
  DI_TRY(residual_queue(a, count));
  return residual_wait(a, l1, sum);
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

// Timing events: events[0] and [1] bracket a solve, the others time single
// launches. None carries a system-scope fence (a cache write-back and
// invalidation that held the stream for about 10 us on this device, or
// landed inside the timed launch): the host reads only their timestamps.
// The control block has its own event, `copied`, which keeps the fence.
di_status ensure_events(Workspace* ws, size_t count) {
  while (ws->events.size() < count) {
    hipEvent_t e;
    DI_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    ws->events.push_back(e);
  }
  return DI_OK;
}

// The control block that the selection of cycle `sel` decided (copy
// (sel + 1) & 1), once an event after that selection has completed: the
// pinned copy its kernel stored, or, should that copy not be the new one
// (seq other than sel + 1), the device's copy.
di_status read_ctl(const CycleArgs& a, int sel, Ctl* out) {
  Workspace* ws = a.ws;
  const int k = (sel + 1) & 1;
  *out = ws->host_ctl[k];
  if (out->seq == (unsigned long long)(sel + 1)) return DI_OK;
  DI_HIP(hipMemcpyAsync(out, ws->ctl + k, sizeof(Ctl), hipMemcpyDeviceToHost, a.stream));
  DI_HIP(hipStreamSynchronize(a.stream));
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

struct RunTimes {
  double seconds = 0.0;       // first queued kernel to the end of the last
  double move_seconds = 0.0;  // summed pull/push kernel time (timing flag)
  int move_launches = 0;
  Ctl state{};                // the final control block
  // device wall clock at the first run's first selection and at the first
  // selection (of any run) with an FP64 residual <= 1e-9
  unsigned long long t_start = 0, t_1e9 = 0;
};

// Rate of the device wall clock (wall_clock64), in Hz; 0 if unknown.
double wall_clock_hz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0.0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0.0;
  }
  return (double)khz * 1e3;
}

// The cycles to queue next, after the read-back of the state h at
// selection last_sel: from the contraction of r per cycle so far, the
// cycles still needed to reach the target, within [2, 64] (the first chunk
// keeps its size).
int next_chunk(const CycleArgs& a, const Ctl& h, int last_sel, int chunk) {
  if (last_sel == 0) return chunk;
  int next = 16;
  const double target = a.tol_rel >= 0.0 ? std::max(a.tol_in, a.tol_rel * h.r_start) : a.tol;
  if (a.stop == DI_STOP_RESID && h.cycles >= 1 && h.r_first > 0.0 && h.r > 0.0 &&
      h.r < h.r_first && target > 0.0) {
    const double rate = std::log(h.r / h.r_first) / (double)h.cycles;
    const double need = std::log(target / h.r) / rate;
    if (std::isfinite(need)) next = (int)std::ceil(need) + 1;
  }
  return std::max(2, std::min(next, 64));
}

// Queues cycles until the device reports a stop: the selection of cycle 0,
// then (move c, selection c + 1) pairs in chunks. The newest control copy
// after selection c is copy (c + 1) & 1; it is left in rt->state.
// ev_begin was recorded before the start kernels.
// Each read-back of the control block is followed by kLookahead more queued
// cycles, so the device works while the host waits for the copy and queues
// the next chunk. Once the device has stopped, their launches return at once.
constexpr int kLookahead = 1;
template <typename T>
di_status run_cycles(const CycleArgs& a, bool timing, hipEvent_t ev_begin, RunTimes* rt) {
  Workspace* ws = a.ws;
  DI_TRY(ensure_events(ws, 2));
  if (!ws->copied) DI_HIP(hipEventCreateWithFlags(&ws->copied, hipEventDisableTiming));
  hipEvent_t ev_end = ws->events[1];
  int last_sel = 0;  // selections queued after the first
  const bool window = a.direction == kWindow;
  // timing events: pull/push direction, pair c brackets the move of cycle c;
  // window push, pair c brackets the launch of cycle c
  auto events_of = [&](int c, hipEvent_t* e0, hipEvent_t* e1) -> di_status {
    *e0 = *e1 = nullptr;
    if (!timing) return DI_OK;
    DI_TRY(ensure_events(ws, 4 + 2 * (size_t)c));
    *e0 = ws->events[2 + 2 * (size_t)c];
    *e1 = ws->events[3 + 2 * (size_t)c];
    return DI_OK;
  };
  auto queue_cycle = [&]() -> di_status {
    const int c = last_sel;
    hipEvent_t e0, e1;
    if (window) {
      DI_TRY(events_of(c + 1, &e0, &e1));
      DI_HIP(launch_wcycle<T>(a, c + 1, e0, e1));
    } else {
      DI_TRY(events_of(c, &e0, &e1));
      DI_HIP(launch_move<T>(a, c, e0, e1));
      DI_HIP(launch_select<T>(a, c + 1, 0));
    }
    last_sel = c + 1;
    return DI_OK;
  };
  if (window) {
    hipEvent_t e0, e1;
    DI_TRY(events_of(0, &e0, &e1));
    DI_HIP(launch_wcycle<T>(a, 0, e0, e1));
  } else {
    DI_HIP(launch_select<T>(a, 0, 1));
  }
  int chunk = 8;
  int at = 0;  // the selection the last read-back follows
  for (;;) {
    at = last_sel;
    // the selection kernels also store the control block into host_ctl:
    // once this event completes, host_ctl holds selection `at`'s copy
    DI_HIP(hipEventRecord(ev_end, a.stream));
    DI_HIP(hipEventRecord(ws->copied, a.stream));
    for (int q = 0; q < kLookahead && last_sel < a.max_cycles; ++q) DI_TRY(queue_cycle());
    DI_HIP(hipEventSynchronize(ws->copied));
    Ctl h;
    DI_TRY(read_ctl(a, at, &h));
    rt->state = h;
    if (h.done) break;
    if (at >= a.max_cycles) {
      set_error("internal: the device did not stop after max_cycles");
      return DI_E_DEVICE;
    }
    chunk = next_chunk(a, h, at, chunk);
    // the cycles queued behind the read-back count toward the chunk
    const int todo = std::min(chunk - (last_sel - at), a.max_cycles - last_sel);
    for (int q = 0; q < todo; ++q) DI_TRY(queue_cycle());
  }
  if (rt->t_start == 0) rt->t_start = rt->state.t_start;
  if (rt->t_1e9 == 0) rt->t_1e9 = rt->state.t_1e9;
  float ms = 0.f;
  DI_HIP(hipEventElapsedTime(&ms, ev_begin, ev_end));
  rt->seconds = ms * 1e-3;
  if (timing) {
    // the launches that moved fluid: cycles 0 .. cycles - 1
    const int real = std::min(rt->state.cycles, window ? last_sel + 1 : last_sel);
    for (int c = 0; c < real; ++c) {
      float pm = 0.f;
      DI_HIP(hipEventElapsedTime(&pm, ws->events[2 + 2 * (size_t)c], ws->events[3 + 2 * (size_t)c]));
      rt->move_seconds += pm * 1e-3;
    }
    rt->move_launches += real;
  }
  return DI_OK;
}

// Algorithmic bytes: what the method itself moves (s = bytes per fluid
// value), whatever the kernel reads besides:
//   per cycle, the selection: N (s + 4) (F and the node word read);
//   per diffused node: 8 + 4s (its link offset, F claimed, H read and
//     written);
//   per link moved: 4 + 2s (the link id and the read-modify-write of the
//     destination's fluid);
//   per residual pass (refinement): Lp 12 (in-link id, y of the sender) +
//     N (56 + 3s) (X, H, node word, y, B, in-link offsets, R).
// move_bytes covers the timed launches that move the fluid: the links moved
// for the pull and the push, the whole cycle for the window push (which
// selects and moves in one launch).
void fill_stats(const di_graph* g, const Ctl& h, double d, int s_bytes, int direction,
                const RunTimes& rt, int refinements, di_stats* st) {
  st->cycles = h.cycles;
  st->fallback_cycles = h.fallback;
  st->edges_pushed = (int64_t)h.edges_total;
  st->nb_iter = g->L > 0 ? (double)h.edges_total / (double)g->L : 0.0;
  st->resid_l1 = h.final_r;
  st->err_bound = h.final_r / (1.0 - d);
  st->paper_err = h.paper_err;
  st->e = h.e;
  const double s = s_bytes, N = (double)g->n, C = (double)h.cycles;
  const double links = (double)h.edges_total * (4.0 + 2.0 * s);
  const double select = C * N * (s + 4.0) + (double)h.sel_total * (8.0 + 4.0 * s);
  const double refine = (double)refinements * ((double)g->Lp * 12.0 + N * (56.0 + 3.0 * s));
  const double move = direction == kWindow ? links + select : links;
  st->refinements = refinements;
  st->move_bytes = rt.move_launches > 0 ? move : 0.0;
  st->bytes_moved = links + select + refine;
  st->seconds = rt.seconds;
  st->move_seconds = rt.move_seconds;
  st->move_launches = rt.move_launches;
  const double hz = rt.t_1e9 != 0 ? wall_clock_hz() : 0.0;
  st->seconds_to_1e9 = (hz > 0.0 && rt.t_1e9 >= rt.t_start)
                           ? (double)(rt.t_1e9 - rt.t_start) / hz
                           : -1.0;
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
  if (o.method != DI_SOP && o.method != DI_CYC && o.method != DI_PI && o.method != DI_GS_ASYNC) {
    set_error("unknown method");
    return DI_E_INVAL;
  }
  if (o.method == DI_GS_ASYNC && (o.precision != DI_FP64 || o.stop != DI_STOP_RESID ||
                                  o.kernel == DI_KERNEL_PUSH || o.kernel == DI_KERNEL_WINDOW)) {
    set_error("DI_GS_ASYNC runs in FP64 with the pull and stops on the residual");
    return DI_E_INVAL;
  }
  if (o.stop != DI_STOP_RESID && o.stop != DI_STOP_PAPER) {
    set_error("unknown stop rule");
    return DI_E_INVAL;
  }
  if (o.precision != DI_FP64 && o.precision != DI_FP32 && o.precision != DI_FP32_REFINE) {
    set_error("unknown precision");
    return DI_E_INVAL;
  }
  if (o.precision == DI_FP32_REFINE && o.stop != DI_STOP_RESID) {
    set_error("DI_FP32_REFINE stops on the residual only (DI_STOP_RESID)");
    return DI_E_INVAL;
  }
  if (o.kernel < DI_KERNEL_AUTO || o.kernel > DI_KERNEL_WINDOW) {
    set_error("unknown kernel direction");
    return DI_E_INVAL;
  }
  return DI_OK;
}

int direction_of(const di_opts& o) {
  if (o.kernel == DI_KERNEL_PUSH) return kPush;
  if (o.kernel == DI_KERNEL_WINDOW) return kWindow;
  return kPull;
}

// ---- window configuration and its tuner ------------------------------------

// The default window configuration: 2048-node tiles, up to 256 active hubs,
// the largest grid (a smaller tile when the graph needs it).
WinCfg default_window_cfg(const di_graph* g) {
  WinCfg c;
  c.shape = 1;
  if (!g->window_ok[c.shape])
    for (int sh = 0; sh < kWinShapes; ++sh)
      if (g->window_ok[sh]) c.shape = sh;
  c.hubs = (int)std::min<int64_t>(kWinHubMax, g->n_hubs);
  c.grid_cap = kWinMaxGrid;
  return c;
}

// The graph's window configuration: the tuned one, else the default.
WinCfg window_cfg(const di_graph* gc) {
  di_graph* g = const_cast<di_graph*>(gc);
  std::lock_guard<std::mutex> lock(g->mu);
  return g->win_tuned ? g->win_cfg : default_window_cfg(g);
}

bool window_usable(const di_graph* g) {
  for (int sh = 0; sh < kWinShapes; ++sh)
    if (g->window_ok[sh]) return true;
  return false;
}

// Configurations already tuned in this process, by graph shape.
using TuneKey = std::tuple<int64_t, int64_t, int64_t, int64_t>;
struct TuneEntry {
  WinCfg cfg;
  bool use_pull;
  double us_default, us_tuned, pull_us;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry>& tune_cache() {
  static std::map<TuneKey, TuneEntry> m;
  return m;
}

// The tuner's timed run: the solve from the PageRank right-hand side until
// the residual has fallen four decades (at most kTuneMaxCycles cycles), with
// the solve's own cycle loop and read-backs. A whole run, not its first few
// cycles, since the cycles differ along a solve (the first ones diffuse
// most of the nodes) and the two-round cycle gains more in the later ones.
constexpr double kTuneCut = 1e-4;
constexpr int kTuneMaxCycles = 400;
// a candidate replaces the best so far only when at least 2% faster (runs
// of one configuration differ by about 1%), so that near ties keep the
// earlier, more common configuration
constexpr double kTuneGain = 0.98;

// A candidate's time for one tenfold cut of the residual: us over the
// decades r fell.
double per_decade(double us, double r_before, double r_after) {
  if (r_after > 0.0 && r_before > r_after) return us / std::log10(r_before / r_after);
  return us;
}

CycleArgs tune_args(di_graph* g, Workspace* ws, hipStream_t stream, double d, int direction) {
  CycleArgs a{};
  a.g = g;
  a.ws = ws;
  a.d = d;
  a.tol = (1.0 - d) * kTuneCut;  // Σ|B| = 1 - d at the start
  a.tol_in = a.tol;
  a.tol_rel = -1.0;
  a.method = DI_SOP;
  a.stop = DI_STOP_RESID;
  a.max_cycles = kTuneMaxCycles;
  a.direction = direction;
  a.stream = stream;
  a.first_parts = part_count(a) + 1;
  return a;
}

// One window configuration's time per tenfold cut of the residual over the
// tuner's timed run. Leaves the workspace's state undefined.
template <typename T>
di_status time_window_cfg(di_graph* g, Workspace* ws, hipStream_t stream, double d,
                          const WinCfg& c, double* us) {
  CycleArgs a = tune_args(g, ws, stream, d, kWindow);
  a.wcfg = c;
  DI_TRY(ensure_events(ws, 2));
  // one untimed cycle first: a kernel's first launch in the process also
  // loads its code
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(launch_wstart<T>(a, nullptr, (1.0 - d) / (double)g->n));
  DI_HIP(launch_wcycle<T>(a, 0, nullptr, nullptr));
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(hipEventRecord(ws->events[0], stream));
  DI_HIP(launch_wstart<T>(a, nullptr, (1.0 - d) / (double)g->n));
  RunTimes rt;
  DI_TRY(run_cycles<T>(a, false, ws->events[0], &rt));
  *us = per_decade(1e6 * rt.seconds, rt.state.r_first, rt.state.r);
  return DI_OK;
}

// The same for the select + pull pair.
template <typename T>
di_status time_pull(di_graph* g, Workspace* ws, hipStream_t stream, double d, double* us) {
  CycleArgs a = tune_args(g, ws, stream, d, kPull);
  DI_TRY(ensure_events(ws, 2));
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(launch_start<T>(a, nullptr, (1.0 - d) / (double)g->n));
  DI_HIP(launch_select<T>(a, 0, 1));
  DI_HIP(launch_move<T>(a, 0, nullptr, nullptr));
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(hipEventRecord(ws->events[0], stream));
  DI_HIP(launch_start<T>(a, nullptr, (1.0 - d) / (double)g->n));
  RunTimes rt;
  DI_TRY(run_cycles<T>(a, false, ws->events[0], &rt));
  *us = per_decade(1e6 * rt.seconds, rt.state.r_first, rt.state.r);
  return DI_OK;
}

// Picks the graph's window configuration by timing candidates, greedily:
// the tile shapes at the default hub count, then the hub counts at the best
// shape, then smaller grids, with one and with two rounds a cycle; and
// whether the select + pull pair is faster still (small graphs, where each
// launch's own latency dominates). Candidates compare by time per tenfold
// cut of the residual. Or takes the choice made for a graph of the same
// shape (n, L, largest in- and out-degree) earlier in the process.
template <typename T>
di_status tune_window(di_graph* g, Workspace* ws, hipStream_t stream, double d) {
  {
    std::lock_guard<std::mutex> lock(g->mu);
    if (g->win_tuned) return DI_OK;
  }
  const TuneKey key{g->n, g->L, g->max_in, g->max_out};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      std::lock_guard<std::mutex> lock2(g->mu);
      g->win_cfg = it->second.cfg;
      g->win_use_pull = it->second.use_pull;
      g->win_us_default = it->second.us_default;
      g->win_us_tuned = it->second.us_tuned;
      g->pull_us = it->second.pull_us;
      g->win_tuned = true;
      return DI_OK;
    }
  }
  const WinCfg def = default_window_cfg(g);
  double def_us = 0.0;
  DI_TRY(time_window_cfg<T>(g, ws, stream, d, def, &def_us));
  WinCfg best = def;
  double best_us = def_us;
  // a greedy search from a timed start: the tile shapes, then the hub
  // counts at the best shape, then smaller grids
  auto search = [&](const WinCfg& start, double start_us) -> di_status {
    WinCfg local = start;
    double local_us = start_us;
    auto consider = [&](const WinCfg& c) -> di_status {
      double us = 0.0;
      DI_TRY(time_window_cfg<T>(g, ws, stream, d, c, &us));
      if (us < kTuneGain * local_us) {
        local_us = us;
        local = c;
      }
      return DI_OK;
    };
    auto shapes = [&]() -> di_status {
      const WinCfg from = local;
      for (int sh = 0; sh < kWinShapes; ++sh)
        if (sh != from.shape && g->window_ok[sh]) {
          WinCfg c = from;
          c.shape = sh;
          DI_TRY(consider(c));
        }
      return DI_OK;
    };
    DI_TRY(shapes());
    const WinCfg shaped = local;
    for (int h : {0, 64, 128, 256, 512, 1024}) {
      const int hh = (int)std::min<int64_t>(h, g->n_hubs);
      if (hh == shaped.hubs) continue;
      WinCfg c = shaped;
      c.hubs = hh;
      DI_TRY(consider(c));
    }
    // the shapes once more if the hub count changed
    if (local.hubs != shaped.hubs) DI_TRY(shapes());
    const WinCfg hubbed = local;
    for (int cap : {256, 512})
      if (cap < g->n_wtiles[hubbed.shape]) {
        WinCfg c = hubbed;
        c.grid_cap = cap;
        DI_TRY(consider(c));
      }
    if (local_us < kTuneGain * best_us) {
      best_us = local_us;
      best = local;
    }
    return DI_OK;
  };
  // with the default rounds a cycle, then with the other number
  DI_TRY(search(def, def_us));
  WinCfg other = def;
  other.rounds = 3 - def.rounds;
  double other_us = 0.0;
  DI_TRY(time_window_cfg<T>(g, ws, stream, d, other, &other_us));
  DI_TRY(search(other, other_us));
  double pull_us = 0.0;
  DI_TRY(time_pull<T>(g, ws, stream, d, &pull_us));
  const bool use_pull = pull_us < best_us;
  {
    std::lock_guard<std::mutex> lock(g->mu);
    g->win_cfg = best;
    g->win_use_pull = use_pull;
    g->win_us_default = def_us;
    g->win_us_tuned = best_us;
    g->pull_us = pull_us;
    g->win_tuned = true;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache()[key] = TuneEntry{best, use_pull, def_us, best_us, pull_us};
  return DI_OK;
}

}  // namespace

di_status tune_window_f64(di_graph* g, double d) {
  if (!window_usable(g)) return DI_OK;
  {
    std::lock_guard<std::mutex> lock(g->mu);
    if (g->win_tuned) return DI_OK;
  }
  di_status st = DI_OK;
  Workspace* ws = acquire(g, kF64, &st);
  if (st != DI_OK) return st;
  hipStream_t stream = nullptr;
  hipError_t err = hipStreamCreate(&stream);
  if (err != hipSuccess) {
    release(g, ws);
    set_error(std::string("hipStreamCreate: ") + hipGetErrorString(err));
    return DI_E_DEVICE;
  }
  st = ensure_window_buffers(g, ws);
  if (st == DI_OK) st = tune_window<double>(g, ws, stream, d);
  (void)hipStreamSynchronize(stream);
  (void)hipStreamDestroy(stream);
  release(g, ws);
  return st;
}

namespace {

constexpr int kMaxRefinements = 100;

// Adds the counters of one run (control block h) to the totals.
void add_run(Ctl* tot, const Ctl& h) {
  tot->cycles += h.cycles;
  tot->fallback += h.fallback;
  tot->edges_total += h.edges_total;
  tot->front_total += h.front_total;
  tot->sel_total += h.sel_total;
  tot->e += h.e;
}

// Asynchronous Gauss-Seidel: sweeps queued in chunks (sized from the
// contraction of sum |dx| per sweep), the control block read back after
// each chunk. At the stop the FP64 residual of x is computed exactly; when
// rounding leaves it above tol, sweeping goes on.
di_status gs_solve(di_graph* g, const double* B_dev, double d, double tol, const di_opts& o,
                   double* X_dev, di_stats* st, Workspace* ws, hipStream_t stream) {
  CycleArgs a{};
  a.g = g;
  a.ws = ws;
  a.d = d;
  a.tol = tol;
  a.tol_in = tol;
  a.tol_rel = -1.0;
  a.method = o.method;
  a.stop = DI_STOP_RESID;
  a.max_cycles = o.max_cycles > 0 ? o.max_cycles : 100000;
  a.direction = kPull;
  a.stream = stream;
  a.first_parts = part_count(a) + 1;
  const double bu = (1.0 - d) / (double)g->n;
  DI_TRY(ensure_events(ws, 2));
  DI_TRY(ensure_refine_buffers(g, ws));
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(hipEventRecord(ws->events[0], stream));
  DI_HIP(launch_gs_init(a, B_dev, bu));
  int queued = 0, chunk = 8, checks = 0;
  double resid = 0.0;
  Ctl h{};
  for (;;) {
    const int todo = std::max(1, std::min(chunk, a.max_cycles - queued));
    for (int q = 0; q < todo; ++q) DI_HIP(launch_gs_sweep(a, B_dev, bu));
    queued += todo;
    DI_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    DI_HIP(hipStreamSynchronize(stream));
    h = ws->host_ctl[0];
    if (h.done == 3) break;
    if (h.done == 1 || h.done == 2) {
      DI_HIP(launch_refine<double>(a, (double*)ws->H, (double*)nullptr, B_dev, bu,
                                   (double*)ws->sent));
      DI_TRY(residual_norm(a, pull_grid(g) + 1, &resid, nullptr));
      if (h.done == 1 && resid > tol && checks < 8) {
        ++checks;  // the bound holds in exact arithmetic: sweep on
        ws->host_ctl[0].done = 0;
        DI_HIP(hipMemcpyAsync(ws->ctl, ws->host_ctl, sizeof(Ctl), hipMemcpyHostToDevice, stream));
        chunk = 2;
        continue;
      }
      break;
    }
    if (queued >= a.max_cycles) {
      set_error("internal: the device did not stop after max_cycles");
      return DI_E_DEVICE;
    }
    chunk = 16;
    if (h.cycles >= 2 && h.r > 0.0 && h.r < h.r_first) {
      const double rate = std::log(h.r / h.r_first) / (double)(h.cycles - 1);
      const double need = std::log(tol / (d * h.r)) / rate;
      if (std::isfinite(need)) chunk = std::max(2, std::min((int)std::ceil(need) + 1, 64));
    }
  }
  DI_HIP(hipMemcpyAsync(X_dev, ws->H, (size_t)g->n * sizeof(double), hipMemcpyDeviceToDevice,
                        stream));
  DI_HIP(hipEventRecord(ws->events[1], stream));
  DI_HIP(hipEventSynchronize(ws->events[1]));
  float ms = 0.f;
  DI_HIP(hipEventElapsedTime(&ms, ws->events[0], ws->events[1]));
  di_stats t;
  std::memset(&t, 0, sizeof(t));
  t.cycles = h.cycles;
  t.edges_pushed = (int64_t)h.edges_total;
  t.nb_iter = g->L > 0 ? (double)h.edges_total / (double)g->L : 0.0;
  t.resid_l1 = h.done == 3 ? h.final_r : resid;
  t.err_bound = t.resid_l1 / (1.0 - d);
  t.seconds = ms * 1e-3;
  // per sweep: in-link ids and y gathers, and per row its offsets, x read
  // and written, y written, B and the node word; plus the residual passes
  const double N = (double)g->n, Lp = (double)g->Lp;
  t.bytes_moved = (double)h.cycles * (Lp * 12.0 + N * 44.0) + (double)(checks + 1) * (Lp * 12.0 + N * 80.0);
  t.seconds_to_1e9 = -1.0;  // GS sweeps are not cycles of a residual
  if (st) *st = t;
  if (h.done == 3) {
    set_error("the iterate became non-finite (non-finite B?)");
    return DI_E_INVAL;
  }
  if (h.done == 2 || resid > tol) {
    set_error("max_cycles reached before the tolerance");
    return DI_E_NOCONV;
  }
  return DI_OK;
}

template <typename T>
di_status solve_t(di_graph* g, const double* B_dev, double d, double tol, const di_opts& o,
                  double* X_dev, di_stats* st, Workspace* ws, hipStream_t stream, int trace_cap,
                  bool signed_B) {
  CycleArgs a{};
  a.g = g;
  a.ws = ws;
  a.d = d;
  a.tol = tol;
  a.tol_in = tol;
  a.tol_rel = -1.0;
  a.method = o.method;
  a.stop = o.stop;
  a.max_cycles = o.max_cycles > 0 ? o.max_cycles : 100000;
  a.direction = direction_of(o);
  a.stream = stream;
  a.first_parts = part_count(a) + 1;
  a.trace = trace_cap > 0 ? ws->trace : nullptr;
  a.trace_cap = trace_cap;
  const bool timing = (o.flags & DI_FLAG_KERNEL_TIMING) != 0;
  const double b_uniform = (1.0 - d) / (double)g->n;
  const bool window = a.direction == kWindow;
  if (window) a.wcfg = window_cfg(g);
  if (window && !g->window_ok[a.wcfg.shape]) {
    set_error("the window push needs every tile of the graph to hold fewer than 2^31 links");
    return DI_E_INVAL;
  }
  if (a.direction == kPush) DI_TRY(ensure_push_buffers(g, ws));
  if (window) {
    DI_TRY(ensure_window_buffers(g, ws));
    DI_TRY(ensure_refine_buffers(g, ws));
    a.folded = signed_B ? 1 : 0;
  }
  DI_TRY(ensure_events(ws, 2));
  DI_HIP(launch_reset_ctl(a));
  DI_HIP(hipEventRecord(ws->events[0], stream));
  if (window) DI_HIP(launch_wstart<T>(a, B_dev, b_uniform));
  else DI_HIP(launch_start<T>(a, B_dev, b_uniform));
  RunTimes rt;
  di_stats tmp;
  std::memset(&tmp, 0, sizeof(tmp));
  // window push: once a run has stopped at cycle c, its fluid (parity c & 1)
  // is gathered into F (and its exact residual summed, when `sum`)
  auto window_finish = [&](const Ctl& h, bool sum) -> di_status {
    DI_HIP(launch_wfinal<T>(a, h.cycles & 1, (!a.folded && h.cycles > 0) ? 1 : 0));
    return sum ? residual_queue(a, win_grid(g, a.wcfg)) : DI_OK;
  };
  auto elapsed = [&](double* sec) -> di_status {
    DI_HIP(hipEventRecord(ws->events[1], stream));
    DI_HIP(hipEventSynchronize(ws->events[1]));
    float ms = 0.f;
    DI_HIP(hipEventElapsedTime(&ms, ws->events[0], ws->events[1]));
    *sec = ms * 1e-3;
    return DI_OK;
  };
  const int max_cycles = a.max_cycles;
  if (o.precision != DI_FP32_REFINE) {
    if (!window) {
      DI_TRY(run_cycles<T>(a, timing, ws->events[0], &rt));
      DI_HIP(launch_h_to_x<T>(a, X_dev));
      DI_HIP(hipStreamSynchronize(stream));
      fill_stats(g, rt.state, d, (int)sizeof(T), a.direction, rt, 0, &tmp);
      if (st) *st = tmp;
      return status_from_done(rt.state.done);
    }
    Ctl tot{};
    int restarts = 0;
    for (;;) {
      a.max_cycles = max_cycles - tot.cycles;
      a.trace = trace_cap > tot.cycles ? ws->trace + tot.cycles : nullptr;
      a.trace_cap = std::max(0, trace_cap - tot.cycles);
      DI_TRY(run_cycles<T>(a, timing, ws->events[0], &rt));
      const Ctl h = rt.state;
      add_run(&tot, h);
      tot.done = h.done;
      tot.paper_err = h.paper_err;
      if (h.done == 3) return status_from_done(3);
      DI_TRY(window_finish(h, true));
      // X from the history while the host waits for the residual (a
      // restart below writes it again)
      DI_HIP(launch_h_to_x<T>(a, X_dev));
      double r_exact = 0.0;
      DI_TRY(residual_wait(a, &r_exact, nullptr));
      tot.final_r = r_exact;
      // the stop compared the kept-plus-pushed sum with tol; should rounding
      // leave the exact residual above tol, the solve goes on from the
      // gathered fluid (first selection on the exact records)
      if (h.done == 1 && a.stop == DI_STOP_RESID && r_exact > tol && restarts < 4 &&
          tot.cycles < max_cycles) {
        ++restarts;
        a.first_parts = win_grid(g, a.wcfg);
        DI_HIP(launch_reset_ctl(a));
        continue;
      }
      break;
    }
    DI_TRY(elapsed(&rt.seconds));
    fill_stats(g, tot, d, (int)sizeof(T), a.direction, rt, 0, &tmp);
    if (st) *st = tmp;
    return status_from_done(tot.done);
  }
  // FP32 passes with FP64 residual passes between them: X accumulates the
  // passes' histories; each pass solves for the correction of X. A signed
  // right-hand side is not gathered after every cycle either (below).
  a.folded = 0;
  DI_TRY(ensure_refine_buffers(g, ws));
  DI_HIP(hipMemsetAsync(X_dev, 0, (size_t)g->n * sizeof(double), stream));
  a.tol_in = kInnerStop * tol;
  a.tol_rel = o.inner_tol > 0.0 ? o.inner_tol : 1e-5;
  Ctl tot{};
  int refinements = 0;
  di_status result = DI_OK;
  for (;;) {
    a.max_cycles = max_cycles - tot.cycles;
    // the passes' cycles are numbered one after another in the trace
    a.trace = trace_cap > tot.cycles ? ws->trace + tot.cycles : nullptr;
    a.trace_cap = std::max(0, trace_cap - tot.cycles);
    DI_TRY(run_cycles<T>(a, timing, ws->events[0], &rt));
    const Ctl h = rt.state;
    add_run(&tot, h);
    if (h.done == 1) {  // the FP64 residual of X is within tol
      tot.final_r = h.final_r;
      break;
    }
    if (h.done == 3) return status_from_done(3);
    if (window) DI_TRY(window_finish(h, false));  // clears the far accumulators
    // inner stop or max_cycles: fold H into X and recompute the residual
    DI_HIP(launch_refine<T>(a, X_dev, (T*)ws->H, B_dev, b_uniform, (T*)ws->F));
    ++refinements;
    a.first_parts = pull_grid(g) + 1;
    // the residual is a signed fluid; an FP32 pass does not gather it after
    // every cycle: its stop is an inner one, taken on the records' bound of
    // sum |F| (|kept| + |pushed|), and the FP64 residual pass decides
    a.folded = 0;
    if (h.done == 2 || refinements >= kMaxRefinements) {
      DI_TRY(residual_norm(a, a.first_parts, &tot.final_r, nullptr));
      result = tot.final_r <= tol ? DI_OK : DI_E_NOCONV;
      if (result != DI_OK)
        set_error(h.done == 2 ? "max_cycles reached before the tolerance"
                              : "refinement stalled above the tolerance");
      break;
    }
    DI_HIP(launch_reset_ctl(a));
  }
  DI_TRY(elapsed(&rt.seconds));
  fill_stats(g, tot, d, (int)sizeof(T), a.direction, rt, refinements, &tmp);
  if (st) *st = tmp;
  return result;
}

di_status solve_any(const di_graph* gc, const double* B, bool B_on_host, double d, double tol,
                    const di_opts* opts, double* X, bool X_on_host, di_stats* st,
                    di_cycle_rec* trace = nullptr, int trace_cap = 0, int32_t* trace_count = nullptr) {
  di_opts o;
  di_opts_default(&o);
  if (opts) o = *opts;
  DI_TRY(check_common(gc, d, tol, o));
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
  const int prec = o.precision == DI_FP64 ? kF64 : kF32;  // FP32 and FP32 + FP64 refinement
  di_status ast = DI_OK;
  Workspace* ws = acquire(g, prec, &ast);
  if (ast != DI_OK) return ast;
  PoolGuard guard{g, ws};
  hipStream_t stream = (hipStream_t)o.stream;
  const size_t nbytes = (size_t)g->n * sizeof(double);
  const double* B_dev = B;
  if (B && B_on_host) {
    if (!ws->B64) DI_TRY(dmalloc((void**)&ws->B64, nbytes));
    DI_HIP(hipMemcpyAsync(ws->B64, B, nbytes, hipMemcpyHostToDevice, stream));
    B_dev = ws->B64;
  }
  double* X_dev = X;
  if (X_on_host) {
    if (!ws->X64) DI_TRY(dmalloc((void**)&ws->X64, nbytes));
    X_dev = ws->X64;
  }
  // DI_KERNEL_AUTO: DI-SOP moves a small share of the links each cycle, so it
  // takes the window push (tuned on the graph's first such solve); DI-CYC and
  // the power iteration move nearly every link every cycle and take the pull
  if (o.kernel == DI_KERNEL_AUTO && o.method != DI_GS_ASYNC) {
    o.kernel = DI_KERNEL_PULL;
    if (o.method == DI_SOP && window_usable(g)) {
      o.kernel = DI_KERNEL_WINDOW;
      if (!(o.flags & DI_FLAG_NO_TUNE)) {
        DI_TRY(ensure_window_buffers(g, ws));
        DI_TRY(prec == kF64 ? tune_window<double>(g, ws, stream, d)
                            : tune_window<float>(g, ws, stream, d));
        std::lock_guard<std::mutex> lock(g->mu);
        if (g->win_use_pull) o.kernel = DI_KERNEL_PULL;
      }
    }
  }
  if (trace_cap > ws->trace_cap) {
    if (ws->trace) (void)hipFree(ws->trace);
    ws->trace = nullptr;
    ws->trace_cap = 0;
    DI_TRY(dmalloc((void**)&ws->trace, (size_t)trace_cap * sizeof(di_cycle_rec)));
    ws->trace_cap = trace_cap;
  }
  // the window push sums the next r from kept and pushed amounts, which is
  // exact only for a fluid that stays >= 0: find out whether B has a
  // negative entry
  bool signed_B = false;
  if (B && o.method != DI_GS_ASYNC && direction_of(o) == kWindow) {
    if (B_on_host) {
      for (int64_t i = 0; i < g->n && !signed_B; ++i) signed_B = B[i] < 0.0;
    } else {
      DI_TRY(ensure_window_buffers(g, ws));
      DI_HIP(launch_any_negative(B_dev, g->n, ws->wflag, stream));
      DI_HIP(hipMemcpyAsync(ws->host_flag, ws->wflag, sizeof(int), hipMemcpyDeviceToHost, stream));
      DI_HIP(hipStreamSynchronize(stream));
      signed_B = *ws->host_flag != 0;
    }
  }
  di_stats local;
  if (!st) st = &local;
  di_status rs =
      o.method == DI_GS_ASYNC
          ? gs_solve(g, B_dev, d, tol, o, X_dev, st, ws, stream)
          : (prec == kF64 ? solve_t<double>(g, B_dev, d, tol, o, X_dev, st, ws, stream, trace_cap,
                                            signed_B)
                          : solve_t<float>(g, B_dev, d, tol, o, X_dev, st, ws, stream, trace_cap,
                                           signed_B));
  if (trace_count && (rs == DI_OK || rs == DI_E_NOCONV)) {
    const int written = std::min(trace_cap, (int)st->cycles);
    if (written > 0)
      DI_HIP(hipMemcpy(trace, ws->trace, (size_t)written * sizeof(di_cycle_rec),
                       hipMemcpyDeviceToHost));
    *trace_count = written;
  }
  if (rs != DI_OK && rs != DI_E_NOCONV) return rs;
  if (X_on_host) DI_HIP(hipMemcpy(X, X_dev, nbytes, hipMemcpyDeviceToHost));
  return rs;
}

template <typename Fn>
di_status guarded(Fn&& body) {
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

di_status cycles_dev(const di_graph* gc, double d, int32_t method, double* F_dev, double* H_dev,
                     int32_t cycles, double* e_inout, void* stream_v, di_stats* stats) {
  if (!gc || !F_dev || !H_dev || cycles < 0 || !(d > 0.0 && d < 1.0) ||
      (method != DI_SOP && method != DI_CYC && method != DI_PI)) {
    set_error("di_cycles_dev: invalid argument");
    return DI_E_INVAL;
  }
  di_graph* g = const_cast<di_graph*>(gc);
  DeviceScope scope(g->device);
  di_status ast = DI_OK;
  Workspace* ws = acquire(g, kF64, &ast);
  if (ast != DI_OK) return ast;
  PoolGuard guard{g, ws};
  // run on the caller's state: the workspace with F and H swapped in
  struct Swap {
    Workspace* ws;
    void* F;
    void* H;
    ~Swap() {
      ws->F = F;
      ws->H = H;
    }
  } swap{ws, ws->F, ws->H};
  ws->F = F_dev;
  ws->H = H_dev;
  hipStream_t stream = (hipStream_t)stream_v;
  CycleArgs a{};
  a.g = g;
  a.ws = ws;
  a.d = d;
  a.tol = -1.0;  // no stop test: exactly `cycles` cycles
  a.tol_in = -1.0;
  a.tol_rel = -1.0;
  a.method = method;
  a.stop = DI_STOP_RESID;
  a.max_cycles = cycles;
  a.direction = kPull;
  a.stream = stream;
  a.first_parts = part_count(a) + 1;
  DI_TRY(ensure_events(ws, 2));
  DI_HIP(launch_reset_ctl(a));
  if (e_inout)
    DI_HIP(hipMemcpyAsync(&ws->ctl->e, e_inout, sizeof(double), hipMemcpyHostToDevice, stream));
  DI_HIP(hipEventRecord(ws->events[0], stream));
  DI_HIP(launch_start_state<double>(a));
  RunTimes rt;
  DI_TRY(run_cycles<double>(a, false, ws->events[0], &rt));
  const Ctl& h = rt.state;
  if (h.done == 3) return status_from_done(3);
  if (e_inout) *e_inout = h.e;
  if (stats) {
    di_stats tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    fill_stats(g, h, d, 8, a.direction, rt, 0, &tmp);
    *stats = tmp;
  }
  return DI_OK;
}

di_status residual_dev(const di_graph* gc, const double* B_dev, double d, const double* X_dev,
                       double* R_dev, double* l1_out, void* stream_v) {
  if (!gc || !X_dev || !(d > 0.0 && d < 1.0)) {
    set_error("di_residual_dev: invalid argument");
    return DI_E_INVAL;
  }
  di_graph* g = const_cast<di_graph*>(gc);
  DeviceScope scope(g->device);
  di_status ast = DI_OK;
  Workspace* ws = acquire(g, kF64, &ast);
  if (ast != DI_OK) return ast;
  PoolGuard guard{g, ws};
  DI_TRY(ensure_refine_buffers(g, ws));
  CycleArgs a{};
  a.g = g;
  a.ws = ws;
  a.d = d;
  a.direction = kPull;
  a.stream = (hipStream_t)stream_v;
  double* R = R_dev ? R_dev : (double*)ws->F;
  DI_HIP(launch_refine<double>(a, const_cast<double*>(X_dev), (double*)nullptr, B_dev,
                               (1.0 - d) / (double)g->n, R));
  double l1 = 0.0;
  DI_TRY(residual_norm(a, pull_grid(g) + 1, &l1, nullptr));
  if (l1_out) *l1_out = l1;
  return DI_OK;
}

}  // namespace

// ---- step-driven FP64 solve -------------------------------------------------

size_t workspace_bytes(const di_graph* g, int prec) {
  const size_t n = (size_t)g->n;
  const size_t s = prec == kF64 ? sizeof(double) : sizeof(float);
  const size_t ntiles =
      (size_t)std::max(select_stat_records(g->n, kPull), select_stat_records(g->n, kPush));
  const size_t nparts = (size_t)std::max(kPullMaxGrid, kReduceGrid) + 1;
  const size_t nh = (size_t)std::max<int64_t>(g->n_heavy, 1);
  return 3 * n * s + ((n + 63) / 64) * sizeof(unsigned long long) + ntiles * sizeof(SelStat) +
         nparts * sizeof(Part) + (size_t)std::max<int64_t>(g->n_segs, 1) * sizeof(double) +
         2 * nh * (s + sizeof(double)) + 2 * sizeof(Ctl);
}

size_t solo_run_bytes(const di_graph* g) {
  return workspace_bytes(g, kF64) + (window_usable(g) ? window_bytes(g, kF64) : 0);
}

di_status solo_create(di_graph* g, SoloRun** out) {
  SoloRun* r = new (std::nothrow) SoloRun;
  if (!r) return DI_E_NOMEM;
  r->g = g;
  di_status st = alloc_workspace(g, kF64, &r->ws);
  if (st == DI_OK && window_usable(g)) st = ensure_window_buffers(g, r->ws);
  if (st == DI_OK) st = ensure_host_part(r->ws);
  if (st != DI_OK) {
    free_workspace(r->ws);
    delete r;
    return st;
  }
  *out = r;
  return DI_OK;
}

void solo_destroy(SoloRun* r) {
  if (!r) return;
  free_workspace(r->ws);
  delete r;
}

// The first selection of a run and the read-back of its control block.
di_status solo_first(SoloRun* r) {
  CycleArgs& a = r->a;
  r->last_sel = 0;
  r->chunk = 8;
  // (the selection also stores the control block into host_ctl, which the
  // caller reads once the stream's work so far has completed)
  if (r->window) DI_HIP(launch_wcycle<double>(a, 0, nullptr, nullptr));
  else DI_HIP(launch_select<double>(a, 0, 1));
  return DI_OK;
}

di_status solo_start(SoloRun* r, const double* B_dev, double b_uniform, double d, double tol,
                     int method, int max_cycles, bool allow_window, hipStream_t stream) {
  CycleArgs& a = r->a;
  a = CycleArgs{};
  a.g = r->g;
  a.ws = r->ws;
  a.d = d;
  a.tol = tol;
  a.tol_in = tol;
  a.tol_rel = -1.0;
  a.method = method;
  a.stop = DI_STOP_RESID;
  a.max_cycles = max_cycles;
  {
    std::lock_guard<std::mutex> lock(r->g->mu);
    r->window = allow_window && method == DI_SOP && r->ws->wA != nullptr && !r->g->win_use_pull;
  }
  a.direction = r->window ? kWindow : kPull;
  if (r->window) a.wcfg = window_cfg(r->g);
  a.stream = stream;
  a.first_parts = part_count(a) + 1;
  r->tot = Ctl{};
  r->restarts = 0;
  r->max_cycles = max_cycles;
  DI_HIP(launch_reset_ctl(a));
  if (r->window) DI_HIP(launch_wstart<double>(a, B_dev, b_uniform));
  else DI_HIP(launch_start<double>(a, B_dev, b_uniform));
  return solo_first(r);
}

di_status solo_next(SoloRun* r, int* done) {
  CycleArgs& a = r->a;
  Ctl h;
  DI_TRY(read_ctl(a, r->last_sel, &h));
  *done = h.done;
  if (h.done) return DI_OK;
  if (r->last_sel >= a.max_cycles) {
    set_error("internal: the device did not stop after max_cycles");
    return DI_E_DEVICE;
  }
  r->chunk = next_chunk(a, h, r->last_sel, r->chunk);
  const int todo = std::max(1, std::min(r->chunk, a.max_cycles - r->last_sel));
  for (int q = 0; q < todo; ++q) {
    const int c = r->last_sel;
    if (r->window) {
      DI_HIP(launch_wcycle<double>(a, c + 1, nullptr, nullptr));
    } else {
      DI_HIP(launch_move<double>(a, c, nullptr, nullptr));
      DI_HIP(launch_select<double>(a, c + 1, 0));
    }
    r->last_sel = c + 1;
  }
  return DI_OK;
}

di_status solo_finish(SoloRun* r, double* X_dev, di_stats* st, bool* again) {
  CycleArgs& a = r->a;
  Ctl h;
  DI_TRY(read_ctl(a, r->last_sel, &h));
  *again = false;
  Ctl tot = r->tot;
  add_run(&tot, h);
  tot.done = h.done;
  tot.final_r = h.final_r;
  if (r->window && h.done != 3) {
    // the whole fluid into F, and its exact residual
    DI_HIP(launch_wfinal<double>(a, h.cycles & 1, h.cycles > 0 ? 1 : 0));
    double r_exact = 0.0;
    DI_TRY(residual_norm(a, win_grid(r->g, a.wcfg), &r_exact, nullptr));
    tot.final_r = r_exact;
    if (h.done == 1 && r_exact > a.tol && r->restarts < 4 && tot.cycles < r->max_cycles) {
      r->tot = tot;
      r->restarts += 1;
      a.max_cycles = r->max_cycles - tot.cycles;
      a.first_parts = win_grid(r->g, a.wcfg);
      DI_HIP(launch_reset_ctl(a));
      DI_TRY(solo_first(r));
      *again = true;
      return DI_OK;
    }
  }
  DI_HIP(launch_h_to_x<double>(a, X_dev));
  RunTimes rt;
  std::memset(st, 0, sizeof(*st));
  fill_stats(r->g, tot, a.d, (int)sizeof(double), a.direction, rt, 0, st);
  return tot.done == 1 ? DI_OK : (tot.done == 2 ? DI_E_NOCONV : DI_E_INVAL);
}

}  // namespace di

extern "C" {

di_status di_solve(const di_graph* g, const double* B, double d, double tol, const di_opts* opts,
                   double* X, di_stats* stats) {
  return di::guarded([&] { return di::solve_any(g, B, true, d, tol, opts, X, true, stats); });
}

di_status di_solve_dev(const di_graph* g, const double* B_dev, double d, double tol,
                       const di_opts* opts, double* X_dev, di_stats* stats) {
  return di::guarded(
      [&] { return di::solve_any(g, B_dev, false, d, tol, opts, X_dev, false, stats); });
}

di_status di_solve_trace_dev(const di_graph* g, const double* B_dev, double d, double tol,
                             const di_opts* opts, double* X_dev, di_stats* stats,
                             di_cycle_rec* trace, int32_t capacity, int32_t* count) {
  return di::guarded([&] {
    if (count) *count = 0;
    if (capacity < 0 || (capacity > 0 && !trace) || !count) {
      di::set_error("trace needs capacity >= 0, a trace array when capacity > 0, and count");
      return DI_E_INVAL;
    }
    if (opts && opts->method == DI_GS_ASYNC) {
      di::set_error("DI_GS_ASYNC has no cycles to trace");
      return DI_E_INVAL;
    }
    return di::solve_any(g, B_dev, false, d, tol, opts, X_dev, false, stats, trace, capacity,
                         count);
  });
}

di_status di_cycles_dev(const di_graph* g, double d, int32_t method, double* F_dev, double* H_dev,
                        int32_t cycles, double* e_inout, void* stream, di_stats* stats) {
  return di::guarded(
      [&] { return di::cycles_dev(g, d, method, F_dev, H_dev, cycles, e_inout, stream, stats); });
}

di_status di_residual_dev(const di_graph* g, const double* B_dev, double d, const double* X_dev,
                          double* R_dev, double* l1, void* stream) {
  return di::guarded([&] { return di::residual_dev(g, B_dev, d, X_dev, R_dev, l1, stream); });
}

di_status di_graph_tuning(const di_graph* gc, int32_t* kernel, int32_t* tile, int32_t* hubs,
                          int32_t* grid, int32_t* rounds, int32_t* tuned, double* us_default,
                          double* us_tuned, double* us_pull) {
  if (!gc) {
    di::set_error("di_graph_tuning: graph is NULL");
    return DI_E_INVAL;
  }
  di_graph* g = const_cast<di_graph*>(gc);
  const di::WinCfg c = di::window_cfg(g);
  std::lock_guard<std::mutex> lock(g->mu);
  if (kernel) *kernel = g->win_tuned && g->win_use_pull ? DI_KERNEL_PULL : DI_KERNEL_WINDOW;
  if (tile) *tile = di::kWinTileOf[c.shape];
  if (hubs) *hubs = c.hubs;
  if (grid) *grid = di::win_grid(g, c);
  if (rounds) *rounds = c.rounds;
  if (tuned) *tuned = g->win_tuned ? 1 : 0;
  if (us_default) *us_default = g->win_us_default;
  if (us_tuned) *us_tuned = g->win_us_tuned;
  if (us_pull) *us_pull = g->pull_us;
  return DI_OK;
}

di_status di_graph_set_window(di_graph* g, int32_t tile, int32_t hubs, int32_t grid_cap,
                              int32_t rounds) {
  if (!g) {
    di::set_error("di_graph_set_window: graph is NULL");
    return DI_E_INVAL;
  }
  int shape = -1;
  for (int sh = 0; sh < di::kWinShapes; ++sh)
    if (di::kWinTileOf[sh] == tile) shape = sh;
  if (shape < 0 || !g->window_ok[shape]) {
    di::set_error("di_graph_set_window: tile must be 1024, 2048 or 4096 and allowed by the graph");
    return DI_E_INVAL;
  }
  if (hubs < 0 || hubs > std::min<int64_t>(g->n_hubs, di::kWinHubMax) || grid_cap < 1 ||
      grid_cap > di::kWinMaxGrid || rounds < 1 || rounds > 2) {
    di::set_error("di_graph_set_window: hubs, grid_cap or rounds out of range");
    return DI_E_INVAL;
  }
  std::lock_guard<std::mutex> lock(g->mu);
  g->win_cfg.shape = shape;
  g->win_cfg.hubs = hubs;
  g->win_cfg.grid_cap = grid_cap;
  g->win_cfg.rounds = rounds;
  g->win_use_pull = false;
  g->win_us_default = g->win_us_tuned = g->pull_us = 0.0;
  g->win_tuned = true;
  return DI_OK;
}

}  // extern "C"
