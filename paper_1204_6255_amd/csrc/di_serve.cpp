// libdi serving loop: personalized PageRank requests on resident graphs,
// continuously batched.
//
// A graph with work holds one or more column sets: batch workspaces of KP
// columns (di_batch.h), each with its own HIP stream, so the kernels of
// different sets and graphs overlap on the device. A graph has one open set
// whose width follows its demand (a power of two from 8 to k_max); when the
// demand outgrows it or shrinks well below it, a new open set of the right
// width takes the new requests and the old one drains. Requests take the
// lowest free column, and a set's kernels look only at the power-of-two
// prefix of columns that covers the occupied ones. A worker thread moves every set on its own: when the work queued for a
// set has finished, it reads out the columns that finished (which frees
// them), starts waiting requests in free columns (the other columns keep
// their state: the columns of a batch are independent solves), and queues
// the residual passes its columns are waiting for, the next chunk of cycles
// and the read-back of the column states. A new set is allocated when a
// graph's requests find no free column and the HBM budget allows it; idle
// sets are released to make room; a request that cannot be placed waits (an
// admission stall).
//
// While a graph has few requests (running or waiting, at most kSoloDemand)
// they run in solo slots instead, up to kSoloPerGraph per graph: the single
// right-hand side path in FP64 (for DI-SOP the graph's tuned window push),
// each on its own stream and queued a chunk at a time like a set. A set of
// eight columns costs a whole batched cycle per cycle of any one of them, so
// a request at light load finishes there many times later than alone; the
// column sets are for heavy load, where they give more solves per second.
// Requests that find every solo slot busy wait for one, unless the demand
// outgrows kSoloDemand.
//
// Each request records when its start was queued and when the worker saw it
// stop, so its latency splits into waiting, running and reading out.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "di_batch.h"

namespace di {
namespace {

constexpr int kMaxSetsPerGraph = 64;
constexpr int kSoloPerGraph = 4;
constexpr int kSoloDemand = 2 * kSoloPerGraph;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket;
  std::vector<int32_t> seeds;  // sorted, unique; empty = uniform B
  double d;
  double tol;
  double t_submit;
};

struct Result {
  di_status status = DI_PENDING;
  std::vector<double> X;
  di_stats stats{};
};

struct Lane {
  uint64_t ticket = 0;  // 0: free
  double t_submit = 0.0;
  double t_start = 0.0;  // its start queued
};

// The latency split of a finished request (t_seen: the worker saw it stop;
// t_out: its X is on the host).
void set_times(di_stats* t, const Lane& ln, double t_seen, double t_out) {
  t->queue_seconds = ln.t_start - ln.t_submit;
  t->run_seconds = t_seen - ln.t_start;
  t->readout_seconds = t_out - t_seen;
  t->seconds = t_out - ln.t_submit;  // latency: submission to completion
  t->seconds_to_1e9 = -1.0;          // not recorded for served requests
}

struct GraphSlot;

// A solo slot of a graph: one request on the single right-hand side path.
// `claimed` changes under the server mutex; the rest is the worker's.
struct Solo {
  SoloRun* run = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;     // end of the queued work
  double* out_dev = nullptr;   // the right-hand side, then X (n doubles)
  int32_t* d_seeds = nullptr;  // the running request's seeds
  size_t seeds_cap = 0;
  std::vector<int32_t> seeds;  // their host copy, kept until the run ends
  size_t bytes = 0;            // counted in the budget while the slot exists
  bool ready = false;          // run, stream, event and out_dev exist
  bool claimed = false;        // a request is placed here (started or not)
  bool launched = false;
  Lane lane;                   // the running request
};

// One batch workspace of a graph. `active` and `d` change under the server
// mutex; the rest is the worker's.
struct ColumnSet {
  GraphSlot* owner = nullptr;
  int kp = 8;                 // columns of this set
  BatchWs* ws = nullptr;
  size_t bytes = 0;
  double d = 0.85;
  std::vector<Lane> lanes;
  int active = 0;
  double* out_dev = nullptr;  // one column read out (n doubles)
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;    // end of the set's queued work
  bool launched = false;
  bool ready = false;         // workspace, stream and event exist
  bool draining = false;      // takes no new requests; freed once idle
};

struct GraphSlot {
  const di_graph* g = nullptr;
  int32_t id = 0;
  std::deque<Request> pending;
  std::vector<ColumnSet*> sets;
  std::vector<Solo*> solos;
  bool stalled = false;  // counted once per stall episode
};

}  // namespace
}  // namespace di

struct di_server {
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  size_t budget = 0;
  size_t in_use = 0;
  int kp = 8;
  di_opts opts{};
  int device = 0;
  std::map<int32_t, di::GraphSlot*> graphs;
  std::unordered_map<uint64_t, di::Result> results;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, stalls = 0, solo_requests = 0;
  double busy_seconds = 0.0;
  std::string worker_error;
  std::thread worker;
  // device staging for starting columns (used by one set at a time)
  int* d_flag = nullptr;
  double* d_buni = nullptr;
  int* d_col = nullptr;
  int64_t* d_off = nullptr;
  double* d_val = nullptr;
  double* d_tol = nullptr;
  int32_t* d_seeds = nullptr;
  size_t seeds_cap = 0;
};

namespace di {
namespace {

bool refine_of(const di_server* s) { return s->opts.precision == DI_FP32_REFINE; }
int prec_of(const di_server* s) { return s->opts.precision == DI_FP64 ? kF64 : kF32; }

// The working width of a set: its occupied columns are the lowest ones
// (requests take the lowest free column), so the cycle kernels only look
// at the power of two that covers the highest occupied column.
int pow2_at_least(int k) {
  int p = 8;
  while (p < k) p <<= 1;
  return p;
}

int working_width(const ColumnSet* cs) {
  int hi = 0;
  for (int c = 0; c < (int)cs->lanes.size(); ++c)
    if (cs->lanes[(size_t)c].ticket != 0) hi = c + 1;
  return std::min(pow2_at_least(hi), cs->kp);
}

BatchArgs args_of(const di_server* s, const ColumnSet* cs) {
  BatchArgs a{};
  a.g = cs->owner->g;
  a.kp = cs->kp;
  a.ke = working_width(cs);
  a.prec = prec_of(s);
  a.d = cs->d;
  a.method = s->opts.method;
  a.max_cycles = s->opts.max_cycles > 0 ? s->opts.max_cycles : 100000;
  a.tol_rel = refine_of(s) ? (s->opts.inner_tol > 0.0 ? s->opts.inner_tol : 1e-5) : -1.0;
  a.stream = cs->stream;
  return a;
}

size_t set_bytes(const di_server* s, const di_graph* g, int kp) {
  return batch_ws_bytes(g, kp, prec_of(s), refine_of(s)) + (size_t)g->n * sizeof(double);
}

bool set_idle(const ColumnSet* cs) { return cs->active == 0 && !cs->launched; }

size_t solo_bytes(const di_graph* g) {
  return solo_run_bytes(g) + (size_t)g->n * sizeof(double);
}

bool solo_idle(const Solo* so) { return so->ready && !so->claimed && !so->launched; }

// What reserve_bytes takes out of the books for the caller to free outside
// the lock.
struct Freed {
  std::vector<ColumnSet*> sets;
  std::vector<Solo*> solos;
};

// Under s->mu: reserves `need` bytes for gs, taking idle sets and idle solo
// slots of graphs without waiting requests out of the books. True when the
// bytes are reserved.
bool reserve_bytes(di_server* s, GraphSlot* gs, size_t need, Freed* freed) {
  if (s->in_use + need > s->budget) {
    for (auto& kv : s->graphs) {
      GraphSlot* o = kv.second;
      if (o == gs || !o->pending.empty()) continue;
      for (size_t q = 0; q < o->sets.size() && s->in_use + need > s->budget;) {
        ColumnSet* cs = o->sets[q];
        if (cs->ready && set_idle(cs)) {
          s->in_use -= cs->bytes;
          freed->sets.push_back(cs);
          o->sets.erase(o->sets.begin() + (long)q);
        } else {
          ++q;
        }
      }
      for (size_t q = 0; q < o->solos.size() && s->in_use + need > s->budget;) {
        Solo* so = o->solos[q];
        if (solo_idle(so)) {
          s->in_use -= so->bytes;
          freed->solos.push_back(so);
          o->solos.erase(o->solos.begin() + (long)q);
        } else {
          ++q;
        }
      }
      if (s->in_use + need <= s->budget) break;
    }
  }
  if (s->in_use + need > s->budget) return false;
  s->in_use += need;
  return true;
}

void destroy_solo(Solo* so) {
  if (so->stream) (void)hipStreamSynchronize(so->stream);
  solo_destroy(so->run);
  if (so->out_dev) (void)hipFree(so->out_dev);
  if (so->d_seeds) (void)hipFree(so->d_seeds);
  if (so->ev) (void)hipEventDestroy(so->ev);
  if (so->stream) (void)hipStreamDestroy(so->stream);
  delete so;
}

void destroy_set(ColumnSet* cs) {
  if (cs->stream) (void)hipStreamSynchronize(cs->stream);
  if (cs->ws) free_batch_ws(cs->ws);
  if (cs->out_dev) (void)hipFree(cs->out_dev);
  if (cs->ev) (void)hipEventDestroy(cs->ev);
  if (cs->stream) (void)hipStreamDestroy(cs->stream);
  delete cs;
}

di_status create_set_ws(di_server* s, ColumnSet* cs) {
  const di_graph* g = cs->owner->g;
  DI_HIP(hipStreamCreate(&cs->stream));
  DI_HIP(hipEventCreateWithFlags(&cs->ev, hipEventDisableTiming));
  DI_TRY(batch_ws_create(g, cs->kp, prec_of(s), refine_of(s), &cs->ws));
  hipError_t err = hipMalloc((void**)&cs->out_dev, (size_t)g->n * sizeof(double));
  if (err != hipSuccess) {
    cs->out_dev = nullptr;
    set_error(std::string("hipMalloc: ") + hipGetErrorString(err));
    return DI_E_NOMEM;
  }
  for (int c = 0; c <= cs->kp; ++c) {
    BCtl b;
    std::memset(&b, 0, sizeof(b));
    b.state = kBIdle;
    cs->ws->host_bctl[c] = b;
  }
  DI_HIP(hipMemcpyAsync(cs->ws->bctl, cs->ws->host_bctl, (size_t)(cs->kp + 1) * sizeof(BCtl),
                        hipMemcpyHostToDevice, cs->stream));
  cs->lanes.assign((size_t)cs->kp, Lane{});
  cs->ready = true;
  return DI_OK;
}

di_status ensure_seed_staging(di_server* s, size_t count) {
  if (count <= s->seeds_cap) return DI_OK;
  if (s->d_seeds) (void)hipFree(s->d_seeds);
  s->d_seeds = nullptr;
  const size_t cap = std::max<size_t>(count, 4096);
  hipError_t err = hipMalloc((void**)&s->d_seeds, cap * sizeof(int32_t));
  if (err != hipSuccess) {
    s->seeds_cap = 0;
    set_error(std::string("hipMalloc: ") + hipGetErrorString(err));
    return DI_E_NOMEM;
  }
  s->seeds_cap = cap;
  return DI_OK;
}

// Starts the requests in the lowest free columns of cs.
di_status start_requests(di_server* s, ColumnSet* cs, std::vector<Request>& reqs) {
  const BatchArgs a = args_of(s, cs);
  const int kp = cs->kp;
  std::vector<int> flag((size_t)kp, 0), col;
  std::vector<double> buni((size_t)kp, 0.0), val, tol;
  std::vector<int64_t> off{0};
  std::vector<int32_t> seeds;
  int c = 0;
  const double t_start = now_s();
  for (Request& r : reqs) {
    while (cs->lanes[(size_t)c].ticket != 0) ++c;
    cs->lanes[(size_t)c] = Lane{r.ticket, r.t_submit, t_start};
    flag[(size_t)c] = 1;
    col.push_back(c);
    const double v = r.seeds.empty() ? (1.0 - r.d) / (double)a.g->n
                                     : (1.0 - r.d) / (double)r.seeds.size();
    if (r.seeds.empty()) buni[(size_t)c] = v;
    val.push_back(v);
    tol.push_back(r.tol);
    seeds.insert(seeds.end(), r.seeds.begin(), r.seeds.end());
    off.push_back((int64_t)seeds.size());
  }
  DI_TRY(ensure_seed_staging(s, seeds.size()));
  const int nc = (int)col.size();
  hipStream_t st = cs->stream;
  DI_HIP(hipMemcpyAsync(s->d_flag, flag.data(), (size_t)kp * sizeof(int), hipMemcpyHostToDevice, st));
  DI_HIP(hipMemcpyAsync(s->d_buni, buni.data(), (size_t)kp * sizeof(double), hipMemcpyHostToDevice, st));
  DI_HIP(hipMemcpyAsync(s->d_col, col.data(), (size_t)nc * sizeof(int), hipMemcpyHostToDevice, st));
  DI_HIP(hipMemcpyAsync(s->d_off, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  DI_HIP(hipMemcpyAsync(s->d_val, val.data(), (size_t)nc * sizeof(double), hipMemcpyHostToDevice, st));
  DI_HIP(hipMemcpyAsync(s->d_tol, tol.data(), (size_t)nc * sizeof(double), hipMemcpyHostToDevice, st));
  if (!seeds.empty())
    DI_HIP(hipMemcpyAsync(s->d_seeds, seeds.data(), seeds.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
  ColInit ci{nc, s->d_flag, s->d_buni, s->d_col, s->d_off, s->d_seeds, s->d_val, s->d_tol};
  DI_HIP(launch_bcol_init(a, cs->ws, ci));
  // the host copies are pageable and the staging is shared: wait
  DI_HIP(hipStreamSynchronize(st));
  return DI_OK;
}

// Reads out cs's finished columns and completes their tickets.
di_status finish_columns(di_server* s, ColumnSet* cs) {
  const BatchArgs a = args_of(s, cs);
  BatchWs* ws = cs->ws;
  const di_graph* g = a.g;
  const double t_seen = now_s();
  for (int c = 0; c < cs->kp; ++c) {
    Lane& ln = cs->lanes[(size_t)c];
    const BCtl& b = ws->host_bctl[c];
    if (ln.ticket == 0 || !(b.state == kBConv || b.state == kBMaxCyc || b.state == kBNonFinite))
      continue;
    Result res;
    res.status = b.state == kBConv ? DI_OK : (b.state == kBMaxCyc ? DI_E_NOCONV : DI_E_INVAL);
    res.X.resize((size_t)g->n);
    DI_HIP(launch_bcol_out(a, ws, c, refine_of(s), cs->out_dev));
    DI_HIP(hipMemcpyAsync(res.X.data(), cs->out_dev, (size_t)g->n * sizeof(double),
                          hipMemcpyDeviceToHost, cs->stream));
    // the column is free again
    BCtl idle = b;
    idle.state = kBIdle;
    ws->host_bctl[c] = idle;
    DI_HIP(hipMemcpyAsync(ws->bctl + c, &ws->host_bctl[c], sizeof(BCtl), hipMemcpyHostToDevice,
                          cs->stream));
    DI_HIP(hipStreamSynchronize(cs->stream));
    di_stats& t = res.stats;
    std::memset(&t, 0, sizeof(t));
    t.cycles = b.cycles;
    t.fallback_cycles = b.fallback;
    t.refinements = b.refinements;
    t.edges_pushed = (int64_t)b.edges;
    t.nb_iter = g->L > 0 ? (double)b.edges / (double)g->L : 0.0;
    t.resid_l1 = b.final_r;
    t.err_bound = b.final_r / (1.0 - cs->d);
    t.e = b.e;
    set_times(&t, ln, t_seen, now_s());
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->results[ln.ticket] = std::move(res);
      s->completed += 1;
      cs->active -= 1;
    }
    ln = Lane{};
  }
  return DI_OK;
}

di_status create_solo(GraphSlot* gs, Solo* so) {
  const di_graph* g = gs->g;
  DI_HIP(hipStreamCreate(&so->stream));
  DI_HIP(hipEventCreateWithFlags(&so->ev, hipEventDisableTiming));
  DI_TRY(solo_create(const_cast<di_graph*>(g), &so->run));
  hipError_t err = hipMalloc((void**)&so->out_dev, (size_t)g->n * sizeof(double));
  if (err != hipSuccess) {
    so->out_dev = nullptr;
    set_error(std::string("hipMalloc: ") + hipGetErrorString(err));
    return DI_E_NOMEM;
  }
  so->ready = true;
  return DI_OK;
}

// Starts request r in solo slot so: B on the device (the seed values
// scattered into zeros, or uniform), the start state and the first
// selection, then the slot's event. Nothing here waits for the device: the
// slot keeps the seeds (its own device copy and the host copy the transfer
// reads) until the run ends.
di_status start_solo(di_server* s, GraphSlot* gs, Solo* so, Request& r) {
  const di_graph* g = gs->g;
  const double* B = nullptr;
  const double bu = (1.0 - r.d) / (double)g->n;
  so->seeds = std::move(r.seeds);
  if (!so->seeds.empty()) {
    if (so->seeds.size() > so->seeds_cap) {
      if (so->d_seeds) (void)hipFree(so->d_seeds);
      so->d_seeds = nullptr;
      so->seeds_cap = 0;
      const size_t cap = std::max<size_t>(so->seeds.size(), 1024);
      hipError_t err = hipMalloc((void**)&so->d_seeds, cap * sizeof(int32_t));
      if (err != hipSuccess) {
        so->d_seeds = nullptr;
        set_error(std::string("hipMalloc: ") + hipGetErrorString(err));
        return DI_E_NOMEM;
      }
      so->seeds_cap = cap;
    }
    DI_HIP(hipMemsetAsync(so->out_dev, 0, (size_t)g->n * sizeof(double), so->stream));
    DI_HIP(hipMemcpyAsync(so->d_seeds, so->seeds.data(), so->seeds.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, so->stream));
    DI_HIP(launch_scatter_value(so->stream, so->out_dev, so->d_seeds, (int64_t)so->seeds.size(),
                                (1.0 - r.d) / (double)so->seeds.size()));
    B = so->out_dev;
  }
  const int max_cycles = s->opts.max_cycles > 0 ? s->opts.max_cycles : 100000;
  DI_TRY(solo_start(so->run, B, bu, r.d, r.tol, s->opts.method, max_cycles,
                    s->opts.kernel != DI_KERNEL_PULL, so->stream));
  DI_HIP(hipEventRecord(so->ev, so->stream));
  so->lane = Lane{r.ticket, r.t_submit, now_s()};
  so->launched = true;
  return DI_OK;
}

// After solo slot so's queued work finished: the next chunk, or the result.
di_status step_solo(di_server* s, GraphSlot* gs, Solo* so) {
  int done = 0;
  DI_TRY(solo_next(so->run, &done));
  if (done == 0) {
    DI_HIP(hipEventRecord(so->ev, so->stream));
    so->launched = true;
    return DI_OK;
  }
  const double t_seen = now_s();
  const di_graph* g = gs->g;
  Result res;
  bool again = false;
  res.status = solo_finish(so->run, so->out_dev, &res.stats, &again);
  if (again) {
    // rounding left the exact residual above tol: the run goes on
    DI_HIP(hipEventRecord(so->ev, so->stream));
    so->launched = true;
    return DI_OK;
  }
  res.X.resize((size_t)g->n);
  DI_HIP(hipMemcpyAsync(res.X.data(), so->out_dev, (size_t)g->n * sizeof(double),
                        hipMemcpyDeviceToHost, so->stream));
  DI_HIP(hipStreamSynchronize(so->stream));
  set_times(&res.stats, so->lane, t_seen, now_s());
  so->seeds.clear();
  std::lock_guard<std::mutex> lk(s->mu);
  s->results[so->lane.ticket] = std::move(res);
  s->completed += 1;
  so->lane = Lane{};
  so->claimed = false;
  return DI_OK;
}

// Queues cs's next work on its stream: the residual passes of the columns
// whose FP32 pass ended (states from the last read-back), a chunk of
// cycles, and the read-back of the column states.
di_status launch_set(di_server* s, ColumnSet* cs) {
  const BatchArgs a = args_of(s, cs);
  BatchWs* ws = cs->ws;
  const int kp = cs->kp;
  bool inner = false;
  int need = 2;
  for (int c = 0; c < kp; ++c) {
    const BCtl& b = ws->host_bctl[c];
    inner |= b.state == kBInner;
    // a column just started has no read-back state yet
    if (cs->lanes[(size_t)c].ticket != 0 && b.state == kBIdle) need = std::max(need, 16);
    if (b.state != kBRun) continue;
    int nc = 16;
    const double target = a.tol_rel >= 0.0 ? std::max(kInnerStop * b.tol, a.tol_rel * b.r_start) : b.tol;
    if (b.pass_cycles >= 1 && b.r > 0.0 && b.r < b.r_start && target > 0.0) {
      const double rate = std::log(b.r / b.r_start) / (double)b.pass_cycles;
      const double est = std::log(target / b.r) / rate;
      if (std::isfinite(est)) nc = (int)std::ceil(est) + 1;
    }
    need = std::max(need, nc);
  }
  if (inner) {
    int nrec = 0;
    DI_HIP(launch_brefine(a, ws, &nrec));
    DI_HIP(launch_bfirst(a, ws, nrec, kBInner));
  }
  // short chunks keep new requests waiting little; the kernels of columns
  // that are not running return at once
  const int chunk = std::max(2, std::min(need, 16));
  for (int q = 0; q < chunk; ++q) DI_HIP(launch_bcycle(a, ws, nullptr, nullptr));
  DI_HIP(hipMemcpyAsync(ws->host_bctl, ws->bctl, (size_t)(kp + 1) * sizeof(BCtl),
                        hipMemcpyDeviceToHost, cs->stream));
  DI_HIP(hipEventRecord(cs->ev, cs->stream));
  cs->launched = true;
  return DI_OK;
}

void fail_all(di_server* s, di_status st, const std::string& msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->worker_error = msg;
  for (auto& kv : s->graphs) {
    GraphSlot* gs = kv.second;
    for (ColumnSet* cs : gs->sets) {
      for (Lane& ln : cs->lanes)
        if (ln.ticket) {
          s->results[ln.ticket].status = st;
          ln = Lane{};
        }
      cs->active = 0;
    }
    for (Solo* so : gs->solos) {
      if (so->lane.ticket) {
        s->results[so->lane.ticket].status = st;
        so->lane = Lane{};
      }
      so->claimed = false;
    }
    for (Request& r : gs->pending) s->results[r.ticket].status = st;
    gs->pending.clear();
  }
}

bool graph_busy(const GraphSlot* gs) {
  if (!gs->pending.empty()) return true;
  for (const Solo* so : gs->solos)
    if (so->claimed || so->launched) return true;
  for (const ColumnSet* cs : gs->sets)
    if (cs->launched || cs->active > 0) return true;
  return false;
}

struct Placement {
  ColumnSet* cs;
  std::vector<Request> reqs;
};

struct SoloStart {
  Solo* so;  // not yet `ready` when just reserved: the worker creates it
  Request req;
};

// Under s->mu: places waiting requests of gs.
// While the graph's demand (requests running or waiting) is at most
// kSoloDemand, requests take free solo slots, reserving new ones up to
// kSoloPerGraph as the budget allows (*solo_starts; the worker creates the
// new ones), and the rest wait for a slot. Otherwise they go to column sets.
// A graph has at most one open set (the others drain: they take no new
// requests and are freed once idle). The open set's width follows the
// demand (as a power of two from 8 to k_max): when the demand outgrows it,
// or falls to a quarter of it, a new open set of the demanded width is
// reserved (*fresh, not yet created) and the old one drains. Requests join
// an open set between its chunks of cycles (not while its work is queued).
// A set takes requests of its own d; an idle open set takes the d of the
// next request. Idle sets and slots of other graphs released to make room
// go to *freed.
void place_requests(di_server* s, GraphSlot* gs, std::vector<Placement>* out,
                    ColumnSet** fresh, Freed* freed, std::vector<SoloStart>* solo_starts) {
  *fresh = nullptr;
  if (gs->pending.empty()) return;
  ColumnSet* open = nullptr;
  int demand = (int)gs->pending.size();
  for (ColumnSet* cs : gs->sets) {
    demand += cs->active;
    if (!cs->draining) open = cs;
  }
  for (const Solo* so : gs->solos) demand += so->claimed ? 1 : 0;
  if (demand <= kSoloDemand && !(s->opts.flags & DI_FLAG_SERVE_NO_SOLO)) {
    for (Solo* so : gs->solos) {
      if (gs->pending.empty()) break;
      if (so->claimed) continue;
      so->claimed = true;
      solo_starts->push_back(SoloStart{so, std::move(gs->pending.front())});
      gs->pending.pop_front();
    }
    while (!gs->pending.empty() && (int)gs->solos.size() < kSoloPerGraph &&
           reserve_bytes(s, gs, solo_bytes(gs->g), freed)) {
      Solo* so = new Solo;
      so->bytes = solo_bytes(gs->g);
      so->claimed = true;
      gs->solos.push_back(so);
      solo_starts->push_back(SoloStart{so, std::move(gs->pending.front())});
      gs->pending.pop_front();
    }
    if (!gs->solos.empty()) {
      gs->stalled = false;
      return;  // the rest wait for a slot
    }
  }
  const int want = std::min(pow2_at_least(demand), s->kp);
  if (open && open->ready && open->active == 0) open->d = gs->pending.front().d;
  const bool resize = !open || want > open->kp || want * 4 <= open->kp;
  if (open && open->ready && !open->launched) {
    Placement p{open, {}};
    while (open->active + (int)p.reqs.size() < open->kp && !gs->pending.empty() &&
           gs->pending.front().d == open->d && !resize) {
      p.reqs.push_back(std::move(gs->pending.front()));
      gs->pending.pop_front();
    }
    if (!p.reqs.empty()) {
      open->active += (int)p.reqs.size();  // columns taken (started by the worker)
      out->push_back(std::move(p));
    }
  }
  if (gs->pending.empty()) {
    gs->stalled = false;
    return;
  }
  if (!resize && open) return;  // the open set is full or busy: wait for it
  if ((int)gs->sets.size() >= kMaxSetsPerGraph) return;
  if (!reserve_bytes(s, gs, set_bytes(s, gs->g, want), freed)) {
    if (!gs->stalled) {
      s->stalls += 1;
      gs->stalled = true;
    }
    return;
  }
  gs->stalled = false;
  if (open) open->draining = true;
  ColumnSet* cs = new ColumnSet;
  cs->owner = gs;
  cs->kp = want;
  cs->bytes = set_bytes(s, gs->g, want);
  cs->d = gs->pending.front().d;
  Placement p{cs, {}};
  while ((int)p.reqs.size() < want && !gs->pending.empty() && gs->pending.front().d == cs->d) {
    p.reqs.push_back(std::move(gs->pending.front()));
    gs->pending.pop_front();
  }
  cs->active = (int)p.reqs.size();
  gs->sets.push_back(cs);
  *fresh = cs;
  out->push_back(std::move(p));
}

// Under s->mu: takes gs's idle draining sets out of the books; the caller
// frees them.
void retire_drained(di_server* s, GraphSlot* gs, std::vector<ColumnSet*>* to_free) {
  for (size_t q = 0; q < gs->sets.size();) {
    ColumnSet* cs = gs->sets[q];
    if (cs->draining && cs->ready && set_idle(cs)) {
      s->in_use -= cs->bytes;
      to_free->push_back(cs);
      gs->sets.erase(gs->sets.begin() + (long)q);
    } else {
      ++q;
    }
  }
}

// The worker: sets progress independently. A set whose queued work has
// finished (its event) is collected and relaunched at once, with the
// requests that arrived meanwhile started in its free columns; the loop
// naps briefly only when no set could move.
void worker_loop(di_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<GraphSlot*> work;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] {
        if (s->stop) return true;
        for (auto& kv : s->graphs)
          if (graph_busy(kv.second)) return true;
        return false;
      });
      if (s->stop) return;
      for (auto& kv : s->graphs)
        if (graph_busy(kv.second)) work.push_back(kv.second);
    }
    const double t0 = now_s();
    di_status st = DI_OK;
    bool progressed = false;
    for (GraphSlot* gs : work) {
      // collect the sets whose work has finished
      std::vector<ColumnSet*> sets;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        sets = gs->sets;
      }
      for (ColumnSet* cs : sets) {
        if (!cs->launched) continue;
        const hipError_t q = hipEventQuery(cs->ev);
        if (q == hipErrorNotReady) {
          (void)hipGetLastError();  // not an error: keep it out of later checks
          continue;
        }
        cs->launched = false;
        if (q != hipSuccess) {
          set_error(std::string("serving worker: ") + hipGetErrorString(q));
          st = DI_E_DEVICE;
          break;
        }
        st = finish_columns(s, cs);
        if (st != DI_OK) break;
        progressed = true;
      }
      if (st != DI_OK) break;
      // the solo slots (only the worker creates, launches and frees them)
      std::vector<Solo*> solos;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        solos = gs->solos;
      }
      for (Solo* so : solos) {
        if (!so->launched) continue;
        const hipError_t q = hipEventQuery(so->ev);
        if (q == hipErrorNotReady) {
          (void)hipGetLastError();
          continue;
        }
        so->launched = false;
        if (q != hipSuccess) {
          set_error(std::string("serving worker: ") + hipGetErrorString(q));
          st = DI_E_DEVICE;
          break;
        }
        st = step_solo(s, gs, so);
        if (st != DI_OK) break;
        progressed = true;
      }
      if (st != DI_OK) break;
      // place waiting requests
      std::vector<Placement> places;
      ColumnSet* fresh = nullptr;
      std::vector<ColumnSet*> to_free;
      Freed freed;
      std::vector<SoloStart> solo_starts;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        retire_drained(s, gs, &to_free);
        place_requests(s, gs, &places, &fresh, &freed, &solo_starts);
        s->solo_requests += (int64_t)solo_starts.size();
        sets = gs->sets;
      }
      for (ColumnSet* cs : to_free) destroy_set(cs);
      for (ColumnSet* cs : freed.sets) destroy_set(cs);
      for (Solo* so : freed.solos) destroy_solo(so);
      for (SoloStart& ss : solo_starts) {
        if (st != DI_OK) break;
        if (!ss.so->ready) st = create_solo(gs, ss.so);
        if (st == DI_OK) st = start_solo(s, gs, ss.so, ss.req);
        progressed = true;
      }
      if (st == DI_OK && fresh) st = create_set_ws(s, fresh);
      for (size_t q = 0; st == DI_OK && q < places.size(); ++q)
        st = start_requests(s, places[q].cs, places[q].reqs);
      // queue the next work of every set with columns in use
      for (ColumnSet* cs : sets) {
        if (st != DI_OK) break;
        if (!cs->ready || cs->launched || cs->active == 0) continue;
        st = launch_set(s, cs);
        progressed = true;
      }
      if (st != DI_OK) {
        // placed requests may not hold a column or the solo slot yet
        std::lock_guard<std::mutex> lk(s->mu);
        for (Placement& p : places)
          for (Request& r : p.reqs) s->results[r.ticket].status = st;
        for (SoloStart& ss : solo_starts) s->results[ss.req.ticket].status = st;
        break;
      }
    }
    if (st != DI_OK) {
      // drain what was queued before failing the requests
      std::lock_guard<std::mutex> lk(s->mu);
      for (auto& kv : s->graphs) {
        for (ColumnSet* cs : kv.second->sets)
          if (cs->launched) {
            (void)hipEventSynchronize(cs->ev);
            cs->launched = false;
          }
        for (Solo* so : kv.second->solos)
          if (so->launched) {
            (void)hipEventSynchronize(so->ev);
            so->launched = false;
          }
      }
    }
    if (st != DI_OK) fail_all(s, st, "serving worker: " + std::string(di_last_error()));
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    std::lock_guard<std::mutex> lk(s->mu);
    s->busy_seconds += now_s() - t0;
  }
}

template <typename Fn>
di_status guarded_s(Fn&& body) {
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

di_status serve_create(size_t budget, int32_t k_max, const di_opts* opts, di_server** out) {
  if (!out) {
    set_error("di_serve_create: out is NULL");
    return DI_E_INVAL;
  }
  *out = nullptr;
  if (k_max < 1 || k_max > kBatchMaxKP) {
    set_error("k_max must lie in [1, 256]");
    return DI_E_INVAL;
  }
  di_opts o;
  di_opts_default(&o);
  if (opts) o = *opts;
  if (!opts) o.precision = DI_FP32_REFINE;
  if (o.method != DI_SOP && o.method != DI_CYC) {
    set_error("serving runs DI_SOP or DI_CYC");
    return DI_E_INVAL;
  }
  if (o.precision != DI_FP64 && o.precision != DI_FP32 && o.precision != DI_FP32_REFINE) {
    set_error("unknown precision");
    return DI_E_INVAL;
  }
  if (o.stop != DI_STOP_RESID || o.kernel == DI_KERNEL_PUSH || o.kernel == DI_KERNEL_WINDOW) {
    set_error("serving stops on the residual and moves fluid by the pull kernel only");
    return DI_E_INVAL;
  }
  int dev = 0;
  DI_TRY(check_device(&dev));
  di_server* s = new (std::nothrow) di_server;
  if (!s) return DI_E_NOMEM;
  s->budget = budget;
  int kp = 8;
  while (kp < k_max) kp <<= 1;
  s->kp = kp;
  s->opts = o;
  s->device = dev;
  hipError_t err = hipMalloc((void**)&s->d_flag, (size_t)kp * sizeof(int));
  if (err == hipSuccess) err = hipMalloc((void**)&s->d_buni, (size_t)kp * sizeof(double));
  if (err == hipSuccess) err = hipMalloc((void**)&s->d_col, (size_t)kp * sizeof(int));
  if (err == hipSuccess) err = hipMalloc((void**)&s->d_off, (size_t)(kp + 1) * sizeof(int64_t));
  if (err == hipSuccess) err = hipMalloc((void**)&s->d_val, (size_t)kp * sizeof(double));
  if (err == hipSuccess) err = hipMalloc((void**)&s->d_tol, (size_t)kp * sizeof(double));
  if (err != hipSuccess) {
    set_error(std::string("di_serve_create: ") + hipGetErrorString(err));
    di_serve_destroy(s);
    return DI_E_DEVICE;
  }
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return DI_OK;
}

}  // namespace
}  // namespace di

extern "C" {

di_status di_serve_create(size_t hbm_budget_bytes, int32_t k_max, const di_opts* opts,
                          di_server** out) {
  return di::guarded_s([&] { return di::serve_create(hbm_budget_bytes, k_max, opts, out); });
}

di_status di_serve_add_graph(di_server* s, const di_graph* g, int32_t graph_id) {
  return di::guarded_s([&]() -> di_status {
    if (!s || !g) {
      di::set_error("di_serve_add_graph: NULL argument");
      return DI_E_INVAL;
    }
    if (di::set_bytes(s, g, 8) > s->budget) {
      di::set_error("one column set of the graph exceeds the HBM budget");
      return DI_E_NOMEM;
    }
    // the solo slots' window push, tuned once for the graph
    const di_opts& o = s->opts;
    if (o.method == DI_SOP && o.kernel != DI_KERNEL_PULL &&
        !(o.flags & (DI_FLAG_NO_TUNE | DI_FLAG_SERVE_NO_SOLO))) {
      int cur = 0;
      if (hipGetDevice(&cur) != hipSuccess) cur = s->device;
      if (cur != s->device) (void)hipSetDevice(s->device);
      const di_status ts = di::tune_window_f64(const_cast<di_graph*>(g), 0.85);
      if (cur != s->device) (void)hipSetDevice(cur);
      if (ts != DI_OK) return ts;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->graphs.count(graph_id)) {
      di::set_error("graph_id already registered");
      return DI_E_INVAL;
    }
    di::GraphSlot* gs = new di::GraphSlot;
    gs->g = g;
    gs->id = graph_id;
    s->graphs[graph_id] = gs;
    return DI_OK;
  });
}

di_status di_serve_submit(di_server* s, int32_t graph_id, int32_t nseeds, const int32_t* seeds,
                          double d, double tol, uint64_t* ticket) {
  return di::guarded_s([&]() -> di_status {
    if (!s || !ticket || nseeds < 0 || (nseeds > 0 && !seeds)) {
      di::set_error("di_serve_submit: invalid argument");
      return DI_E_INVAL;
    }
    if (!(d > 0.0 && d < 1.0) || !(tol > 0.0)) {
      di::set_error("d must lie in (0, 1) and tol must be > 0");
      return DI_E_INVAL;
    }
    di::Request r;
    r.seeds.assign(seeds, seeds + nseeds);
    std::sort(r.seeds.begin(), r.seeds.end());
    r.seeds.erase(std::unique(r.seeds.begin(), r.seeds.end()), r.seeds.end());
    r.d = d;
    r.tol = tol;
    r.t_submit = di::now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->graphs.find(graph_id);
    if (it == s->graphs.end()) {
      di::set_error("unknown graph_id");
      return DI_E_NOTFOUND;
    }
    if (!s->worker_error.empty()) {
      di::set_error(s->worker_error);
      return DI_E_DEVICE;
    }
    const int64_t n = it->second->g->n;
    if (!r.seeds.empty() && (r.seeds.front() < 0 || r.seeds.back() >= n)) {
      di::set_error("seed id outside [0, n)");
      return DI_E_RANGE;
    }
    r.ticket = s->next_ticket++;
    *ticket = r.ticket;
    s->results[r.ticket].status = DI_PENDING;
    it->second->pending.push_back(std::move(r));
    s->submitted += 1;
    s->cv.notify_all();
    return DI_OK;
  });
}

di_status di_serve_poll(di_server* s, uint64_t ticket, double* X, di_stats* stats) {
  return di::guarded_s([&]() -> di_status {
    if (!s) {
      di::set_error("di_serve_poll: server is NULL");
      return DI_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) {
      di::set_error("unknown ticket (never issued, or already collected)");
      return DI_E_NOTFOUND;
    }
    di::Result& r = it->second;
    if (r.status == DI_PENDING) return DI_PENDING;
    const di_status st = r.status;
    if (X && !r.X.empty()) std::memcpy(X, r.X.data(), r.X.size() * sizeof(double));
    if (stats) *stats = r.stats;
    if (st != DI_OK) di::set_error(st == DI_E_NOCONV ? "max_cycles reached before the tolerance"
                                                    : "the request failed: " + s->worker_error);
    s->results.erase(it);
    return st;
  });
}

di_status di_serve_info(di_server* s, di_serve_stats* out) {
  if (!s || !out) {
    di::set_error("di_serve_info: NULL argument");
    return DI_E_INVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->admission_stalls = s->stalls;
  int64_t active = 0, pending = 0;
  for (auto& kv : s->graphs) {
    for (const di::ColumnSet* cs : kv.second->sets) active += cs->active;
    for (const di::Solo* so : kv.second->solos) active += so->claimed ? 1 : 0;
    pending += (int64_t)kv.second->pending.size();
  }
  out->active = active;
  out->pending = pending;
  out->bytes_in_use = (int64_t)s->in_use;
  out->busy_seconds = s->busy_seconds;
  out->solo_requests = s->solo_requests;
  return DI_OK;
}

void di_serve_destroy(di_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != s->device) (void)hipSetDevice(s->device);
  for (auto& kv : s->graphs) {
    for (di::ColumnSet* cs : kv.second->sets) di::destroy_set(cs);
    for (di::Solo* so : kv.second->solos) di::destroy_solo(so);
    delete kv.second;
  }
  void* ptrs[] = {s->d_flag, s->d_buni, s->d_col, s->d_off, s->d_val, s->d_tol, s->d_seeds};
  for (void* p : ptrs) (void)hipFree(p);
  if (cur != s->device) (void)hipSetDevice(cur);
  delete s;
}

}  // extern "C"
