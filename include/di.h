/*
 * di.h -- C ABI of the MI355X D-iteration library (libdi.so).
 *
 * The library solves the PageRank-type linear system of Section 1 of
 * "Revisiting the D-iteration method: runtime comparison" (Hong, Burnside,
 * Raoult, 2012):
 *
 *     X = P.X + B,   P[i][j] = d / out_j for every link j -> i,
 *
 * where out_j counts every link leaving j (a self-loop included) and a
 * dangling node (out_j = 0) has a zero column (Section 2.4). Its hot path is
 * the DI-SOP fluid diffusion of Sections 2.3 and 2.5.5: a fluid vector F
 * starts at B and a history H at 0; each cycle computes r = sum_i |F_i| and
 * diffuses every node with |F_i| > 0 and |F_i| >= (r/L)*out_i (L = number
 * of links): H_i += transit, F_i = 0, and transit*d/out_i goes to every
 * out-neighbour j != i, where transit = F_i, or F_i*out_i/(out_i - d) for a
 * node with a self-loop (Section 2.5.4). H converges to X, and
 * F = B - (I - P).H holds after every cycle, so sum_i |F_i| is exactly the
 * L1 residual |B + P.H - H|_1.
 *
 * On the GPU a cycle is frontier-synchronous: the selected set and the
 * diffused amounts are fixed from F at the start of the cycle, and fluid
 * that arrives during the cycle waits for the next one. Any diffusion order
 * converges to the same X; only the trajectory differs from the paper's
 * sequential sweep.
 *
 * Conventions for every call:
 *   - Returns a di_status; nothing throws or aborts across the ABI. On a
 *     status other than DI_OK / DI_PENDING, di_last_error() returns a
 *     message for the calling thread.
 *   - Input arrays are read during the call and never kept; the caller
 *     keeps ownership. Handles belong to the library until *_destroy.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device allocations (e.g. torch tensors on cuda:0) on the device that
 *     was current when the graph was created.
 *   - Node ids are int32 in [0, n); n < 2^31; links m < 2^33.
 *   - There is no CPU fallback: without a usable gfx950 device, calls that
 *     compute return DI_E_DEVICE.
 */
#ifndef DI_H
#define DI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum di_status {
  DI_OK = 0,
  DI_PENDING = 1,      /* the request is still running (di_serve_poll) */
  DI_E_INVAL = -1,     /* bad argument (null pointer, d outside (0,1), ...) */
  DI_E_UNSORTED = -2,  /* links not sorted by (origin, destination) */
  DI_E_DUP = -3,       /* the same link listed twice */
  DI_E_RANGE = -4,     /* node id outside [0, n) */
  DI_E_NOMEM = -5,     /* host or device allocation failed */
  DI_E_NOCONV = -6,    /* max_cycles reached before the tolerance */
  DI_E_DEVICE = -7,    /* no usable GPU, or a HIP call failed */
  DI_E_BUSY = -8,      /* (reserved) */
  DI_E_NOTFOUND = -9   /* unknown graph id or ticket (serving) */
} di_status;

/* di_opts.method: which nodes each (frontier-synchronous) cycle diffuses.
 *   DI_SOP: F_i >= (r/L)*out_i with r = sum|F| at the cycle's start
 *           (Section 2.5.5);
 *   DI_CYC: every node with F_i != 0 (Section 2.5.4);
 *   DI_PI:  every node, fluid or not. The history after c cycles is then the
 *           power iteration's c-th iterate from zero, sum_{k<c} P^k B, and
 *           sum|F| = |P^c B|_1 its residual: the unnormalized power (Jacobi)
 *           iteration of Sections 2.5.1-2.5.2 with its cost (every link
 *           moves every cycle). Single right-hand side only.
 *   DI_GS_ASYNC: not a D-iteration: the Gauss-Seidel baseline of Section
 *           2.5.3 as an asynchronous GPU relaxation. x starts at B; each
 *           sweep updates every row in place, x_i = (B_i + sum over in-links
 *           j != i of d x_j / out_j) / (1 - d/out_i if i has a self-loop),
 *           from whatever x_j is visible (so results vary in the last bits
 *           from run to run). It stops when d * sum|x_new - x_old| <= tol,
 *           which bounds the residual, and reports the exact FP64 residual.
 *           di_solve / di_solve_dev only, FP64, DI_STOP_RESID, pull. A
 *           "cycle" in di_stats is a sweep. */
enum { DI_SOP = 0, DI_CYC = 1, DI_PI = 2, DI_GS_ASYNC = 3 };
/* di_opts.precision */
enum { DI_FP64 = 0, DI_FP32_REFINE = 1, DI_FP32 = 2 };
/* di_opts.stop */
enum { DI_STOP_RESID = 0, DI_STOP_PAPER = 1 };
/* di_opts.flags */
#define DI_FLAG_KERNEL_TIMING 1u /* time every pull/push launch with HIP events */
#define DI_FLAG_SERVE_NO_SOLO 2u /* serving: a lone request also runs in a column set */
#define DI_FLAG_NO_TUNE 4u       /* DI_KERNEL_AUTO: the default window configuration,
                                    without timing candidates on a first solve */

/* di_opts.kernel: how a cycle moves the claimed fluid along the links */
enum {
  DI_KERNEL_AUTO = 0, /* the library's choice: for DI_SOP the faster of the
                         window push (tuned) and the pull on this graph (see
                         di_graph_tuning); DI_KERNEL_PULL for DI_CYC and
                         DI_PI, whose cycles move nearly every link */
  DI_KERNEL_PULL = 1, /* every node sums what its in-links send (CSC);
                         no atomics, bit-reproducible */
  DI_KERNEL_PUSH = 2, /* every diffused node adds to its out-neighbours
                         (CSR) with device-scope float atomics */
  DI_KERNEL_WINDOW = 3 /* one launch per cycle selects and pushes a tile of
                         nodes: links within 512 ids into an LDS window, the
                         far links into LDS hub rows or device-scope atomics;
                         reads only the links it moves. For DI_SOP it runs
                         two rounds a cycle over each tile by default (see
                         di_graph_tuning): the second diffuses, against the
                         cycle's r, what the first moved inside the tile, so
                         its cycles are not the pull's. Atomic order varies,
                         so results agree with the oracle to rounding */
};

typedef struct di_graph di_graph;

typedef struct di_opts {
  int32_t method;     /* DI_SOP (default), DI_CYC, DI_PI or DI_GS_ASYNC (see above) */
  int32_t precision;  /* DI_FP64 (default), DI_FP32_REFINE, DI_FP32 */
  int32_t stop;       /* DI_STOP_RESID (default): stop when sum|F| <= tol;
                         DI_STOP_PAPER: stop after a cycle when
                         sum F / (1 - d - d*e) <= tol, e = fluid absorbed by
                         dangling nodes (the paper's rule, target 1/N) */
  int32_t max_cycles; /* <= 0: 100000 */
  uint32_t flags;     /* DI_FLAG_* */
  int32_t kernel;     /* DI_KERNEL_* (default DI_KERNEL_AUTO) */
  double inner_tol;   /* DI_FP32_REFINE: relative residual reduction asked
                         of each FP32 pass (<= 0: 1e-5). A refined solve
                         runs FP32 DI-SOP cycles until sum|F| <=
                         max(0.9 tol, inner_tol * r_start), then folds H
                         into an FP64 X and recomputes the fluid as the
                         FP64 residual B + P.X - X; it stops when that
                         residual is <= tol. DI_STOP_RESID only. */
  void* stream;       /* hipStream_t for the *_dev calls; NULL = the
                         default (null) stream */
} di_opts;

typedef struct di_stats {
  int32_t cycles;           /* diffusion cycles run */
  int32_t fallback_cycles;  /* DI-CYC cycles run after a DI-SOP cycle that
                               selected nothing (rounding at a tie) */
  int32_t refinements;      /* FP64 residual passes (DI_FP32_REFINE) */
  int32_t move_launches;    /* pull/push launches timed (DI_FLAG_KERNEL_TIMING) */
  int64_t edges_pushed;     /* link operations: pushes along links j != i */
  double nb_iter;           /* edges_pushed / L: cost in units of one
                               matrix-vector product */
  double resid_l1;          /* final |B + P.X - X|_1 (sum |F|, or the FP64
                               residual pass in DI_FP32_REFINE) */
  double err_bound;         /* resid_l1 / (1 - d) >= |X - X_exact|_1 */
  double paper_err;         /* last sum F / (1 - d - d*e) */
  double e;                 /* fluid absorbed by dangling nodes */
  double seconds;           /* device time of the solve (first cycle to
                               stop), excluding host<->device copies */
  double move_seconds;      /* summed time of the pull/push kernel that moves
                               the fluid (with DI_FLAG_KERNEL_TIMING) */
  double bytes_moved;       /* algorithmic bytes of the whole solve */
  double move_bytes;        /* algorithmic bytes of those pull/push launches */
  double seconds_to_1e9;    /* device time from the first cycle to the first
                               cycle start with an L1 residual <= 1e-9 (an
                               FP64 one: with DI_FP32_REFINE, a residual
                               pass), by the device wall clock; -1 when the
                               solve never got there (or for batched and
                               served solves, which do not record it) */
  /* served requests only (0 otherwise); seconds is then their latency, the
     sum of the three and the worker's bookkeeping: */
  double queue_seconds;     /* submission to the queueing of its start */
  double run_seconds;       /* start queued to the worker seeing it stop */
  double readout_seconds;   /* X gathered and copied to the host */
} di_stats;

/* One cycle of a traced solve (di_solve_trace_dev). */
typedef struct di_cycle_rec {
  double r;          /* sum |F| at the cycle's start: the r its selection used
                        (Section 2.5.5) */
  int64_t links;     /* link operations of the cycle */
  int32_t selected;  /* nodes diffused */
  int32_t senders;   /* diffused nodes with links to move */
} di_cycle_rec;

/* Fills *opts with the defaults listed in di_opts. */
void di_opts_default(di_opts* opts);

/* Builds a graph from its link list, origin src[e] -> destination dst[e],
 * e in [0, m), sorted by (origin, destination) as in the input format of
 * Section 2.1. Self-loops are allowed (p_ii = d/out_i). The link list is
 * validated on the host before any device work:
 *   DI_E_INVAL if n < 0, m < 0 or an array is NULL while m > 0,
 *   DI_E_RANGE if an id is outside [0, n),
 *   DI_E_UNSORTED if the list is not sorted by (origin, destination),
 *   DI_E_DUP if a link appears twice.
 * flags must be 0 (reserved).
 * On success the device holds the out-link lists (CSR, self-loops removed,
 * int64 offsets + int32 ids), the in-link lists (CSC, self-loops removed),
 * a per-node word with out_i and the self-loop bit, and the pull work
 * items (runs of rows with at most 2048 in-links; longer in-link lists are
 * split). Arrays are host memory; they are copied. */
di_status di_graph_create(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                          uint32_t flags, di_graph** out);

/* What DI_KERNEL_AUTO runs for DI_SOP on a graph, and the window-push
 * configuration (also used by DI_KERNEL_WINDOW): *kernel DI_KERNEL_WINDOW or
 * DI_KERNEL_PULL; *tile nodes per tile (1024, 2048 or 4096), *hubs active
 * hub rows (far links into the nodes with the most far in-links, summed per
 * block in LDS; at most 1024), *grid the largest number of blocks, *rounds
 * the DI-SOP diffusion rounds per cycle over each tile (2: a second round
 * diffuses, against the same r, the fluid the first round moved inside the
 * tile; 1: the frontier-synchronous cycle). *tuned is 1 once the tuner has
 * picked them and 0 for the defaults (2048-node tiles, 1024 hub rows, two
 * rounds). The tuner runs on the graph's first DI_KERNEL_AUTO DI-SOP solve
 * (unless DI_FLAG_NO_TUNE): per candidate (the three tile shapes, then hub
 * counts, then smaller grids, each with one and with two rounds, then the
 * select + pull pair) it times a solve from the PageRank right-hand side
 * until the residual has fallen four decades (at most 400 cycles), divides
 * by the decades it fell, and keeps the fastest (a candidate replaces the
 * best so far only when 2% faster); a graph of the same n, L
 * and largest in- and out-degree reuses the process's earlier choice.
 * *us_default, *us_tuned and *us_pull receive those times (microseconds per
 * tenfold cut of the residual) of the default window configuration, of the
 * best one and of the pull (0 before tuning). Any output pointer may be
 * NULL. */
di_status di_graph_tuning(const di_graph* g, int32_t* kernel, int32_t* tile, int32_t* hubs,
                          int32_t* grid, int32_t* rounds, int32_t* tuned, double* us_default,
                          double* us_tuned, double* us_pull);

/* Sets the graph's window-push configuration instead of tuning it: tile
 * nodes per tile (1024, 2048 or 4096, a shape the graph allows), hubs active
 * hub rows (0 to the graph's ranked hubs, at most 1024), grid_cap the largest
 * number of blocks (1 to 1024), rounds 1 or 2 (as in di_graph_tuning).
 * DI_KERNEL_AUTO then runs DI-SOP with this window configuration (no
 * tuning, no pull), as does DI_KERNEL_WINDOW. For profiling, reproducible
 * timing and the frontier-synchronous cycle (rounds 1). DI_E_INVAL for a
 * value outside those ranges, with nothing changed. Not to be called while
 * a solve on the graph runs. */
di_status di_graph_set_window(di_graph* g, int32_t tile, int32_t hubs, int32_t grid_cap,
                              int32_t rounds);

/* Frees the graph and its device memory. NULL is ignored. */
void di_graph_destroy(di_graph* g);

/* n, links L, dangling nodes and self-loops of a graph (any pointer may be
 * NULL). */
di_status di_graph_info(const di_graph* g, int64_t* n, int64_t* m, int64_t* n_dangling,
                        int64_t* n_loops);

/* Solves X = P.X + B by DI-SOP until |B + P.X - X|_1 <= tol.
 * B: n doubles (host), all finite; NULL means the PageRank right-hand side
 *    B = (1-d)/n for every node.
 * X: n doubles (host), caller-allocated, receives the solution (H).
 * d in (0, 1); tol > 0 (tol >= 0 with DI_STOP_PAPER).
 * opts may be NULL (defaults); stats may be NULL.
 * Returns DI_E_NOCONV (X and stats still filled) after max_cycles. */
di_status di_solve(const di_graph* g, const double* B, double d, double tol, const di_opts* opts,
                   double* X, di_stats* stats);

/* As di_solve with B and X in device memory (n doubles each); the work is
 * queued on opts->stream and the call returns once it has finished. */
di_status di_solve_dev(const di_graph* g, const double* B_dev, double d, double tol,
                       const di_opts* opts, double* X_dev, di_stats* stats);

/* di_solve_dev with a per-cycle trace: record c of trace[0, capacity) (host,
 * caller-allocated) describes cycle c of the solve (DI_FP32_REFINE numbers
 * the cycles of its passes one after another). *count (host, required)
 * receives the number of records written, min(cycles, capacity); it is 0
 * when the call fails other than with DI_E_NOCONV. capacity 0 writes none
 * (trace may then be NULL). The records pass through a device buffer of
 * capacity records that the graph's pooled workspace keeps.
 * DI-SOP, DI-CYC and PI; DI_E_INVAL for DI_GS_ASYNC (its sweeps are not
 * cycles), a negative capacity, a NULL trace with capacity > 0 or a NULL
 * count. Otherwise as di_solve_dev. */
di_status di_solve_trace_dev(const di_graph* g, const double* B_dev, double d, double tol,
                             const di_opts* opts, double* X_dev, di_stats* stats,
                             di_cycle_rec* trace, int32_t capacity, int32_t* count);

/* Runs exactly `cycles` frontier-synchronous FP64 cycles of DI-SOP
 * (method DI_SOP) or DI-CYC (DI_CYC) on the state (F, H) in place, with no
 * stop test. F and H are device arrays of n doubles. Because
 * F = B - (I - P).H is preserved, (F, H) is an exact checkpoint of a solve:
 * calling this again resumes it. *e_inout (host, may be NULL) is the
 * absorbed-fluid total, updated. */
di_status di_cycles_dev(const di_graph* g, double d, int32_t method, double* F_dev,
                        double* H_dev, int32_t cycles, double* e_inout, void* stream,
                        di_stats* stats);

/* Solves k systems X_c = P.X_c + B_c (c < k) on one graph together, e.g.
 * a batch of personalized PageRank vectors: every cycle applies the DI-SOP
 * rule of Section 2.5.5 to each column with that column's own
 * r = sum_i |F_ic| (and claims, diffuses and counts per column), and one
 * set of launches moves all columns; a column stops when its residual is
 * within its tolerance while the others go on.
 *   B: k x n doubles (host), right-hand side c at B + c*n, all finite;
 *      NULL means (1-d)/n in every column.
 *   tol: k doubles (host), each > 0: column c stops when
 *      |B_c + P.X_c - X_c|_1 <= tol[c].
 *   X: k x n doubles (host), caller-allocated; column c at X + c*n.
 *   opts: method DI_SOP or DI_CYC; precision DI_FP64, DI_FP32, or
 *      DI_FP32_REFINE (FP32 fluid with FP64 residual passes, as di_opts
 *      describes, per column); stop DI_STOP_RESID only; kernel AUTO or
 *      PULL; max_cycles counts each column's cycles.
 *   stats: NULL or k entries; entry c describes column c, except seconds,
 *      move_seconds, bytes_moved and move_bytes, which cover the batch.
 * Columns run in launch groups of at most 256. A group of k columns holds
 * 3 arrays of n*KP fluid values (KP = k rounded up to a power of two,
 * at least 8), plus 3 arrays of n*KP doubles with DI_FP32_REFINE.
 * Returns DI_E_NOCONV (X and stats still filled) when a column reached
 * max_cycles, DI_E_INVAL when a column's fluid became non-finite. */
di_status di_solve_batch(const di_graph* g, int32_t k, const double* B, double d,
                         const double* tol, const di_opts* opts, double* X, di_stats* stats);

/* As di_solve_batch with B and X in device memory (k x n doubles each; B may
 * be NULL); tol and stats stay on the host. Work is queued on opts->stream
 * and the call returns once it has finished. */
di_status di_solve_batch_dev(const di_graph* g, int32_t k, const double* B_dev, double d,
                             const double* tol, const di_opts* opts, double* X_dev,
                             di_stats* stats);

/* ---- serving ------------------------------------------------------------
 * A server answers personalized PageRank requests (one right-hand side
 * B = (1-d)/|S| on a seed set S, or the uniform (1-d)/n) on resident graphs
 * with continuous batching. Each request is its own DI-SOP (or DI-CYC) solve
 * of Sections 2.5.4-2.5.5 and finishes when its own residual is within its
 * tolerance, as in di_solve_batch.
 * - A worker thread keeps, per graph with work, column sets: batches of KP
 *   columns (a power of two from 8 to k_max rounded up), each on its own
 *   HIP stream. One set per graph is open; its width follows the graph's
 *   demand (columns in use plus requests waiting), and a set that no longer
 *   fits the demand drains and is freed once idle. Waiting requests start in
 *   free columns as they free up.
 * - While a graph has few requests (running or waiting: at most twice its
 *   solo slots) they take solo slots instead, up to four per graph: the
 *   single right-hand side path in FP64 (whatever the server's precision;
 *   for DI-SOP the graph's tuned window push), which finishes a request
 *   several times sooner than a column set; the others wait for a free
 *   slot. Past that demand, new requests go to column sets, which give more
 *   solves per second. DI_FLAG_SERVE_NO_SOLO in opts.flags turns solo slots
 *   off.
 * - Sets and solo slots are allocated when the HBM budget allows them; idle
 *   ones of other graphs are released to make room; a request that cannot be
 *   placed waits (an admission stall). Requests with another d wait until
 *   their graph's open set is idle.
 * Every di_serve_* call is thread-safe. */
typedef struct di_server di_server;

typedef struct di_serve_stats {
  int64_t submitted;        /* requests accepted */
  int64_t completed;        /* requests finished (collected or not) */
  int64_t admission_stalls; /* times a graph's requests found no HBM room */
  int64_t active;           /* columns and solo slots in use now */
  int64_t pending;          /* requests waiting for a column */
  int64_t bytes_in_use;     /* device bytes held by column sets and solo slots */
  double busy_seconds;      /* worker time spent on work */
  int64_t solo_requests;    /* requests started in solo slots */
} di_serve_stats;

/* Creates a server that may hold up to hbm_budget_bytes of column sets and
 * solo slots, with k_max in [1, 256] columns per set. opts (may be NULL:
 * DI-SOP, DI_FP32_REFINE) gives method, precision (of the column sets),
 * max_cycles, inner_tol and flags (DI_FLAG_SERVE_NO_SOLO); stop must be
 * DI_STOP_RESID and kernel AUTO or PULL. The device current at the call is
 * used. */
di_status di_serve_create(size_t hbm_budget_bytes, int32_t k_max, const di_opts* opts,
                          di_server** out);

/* Registers graph g under graph_id (unique). g must outlive the server.
 * DI_E_NOMEM if the graph's batch alone exceeds the budget. For a DI-SOP
 * server without DI_FLAG_NO_TUNE the graph's window push is tuned here (as
 * on a first DI_KERNEL_AUTO solve; the call waits for it), so that its solo
 * slots run the tuned configuration. */
di_status di_serve_add_graph(di_server* s, const di_graph* g, int32_t graph_id);

/* Queues a request: seeds (host, nseeds ids in [0, n), duplicates ignored;
 * nseeds = 0 means the uniform right-hand side), d in (0, 1), tol > 0.
 * *ticket receives its ticket. DI_E_NOTFOUND for an unknown graph_id,
 * DI_E_RANGE for a seed outside [0, n). */
di_status di_serve_submit(di_server* s, int32_t graph_id, int32_t nseeds, const int32_t* seeds,
                          double d, double tol, uint64_t* ticket);

/* DI_PENDING while the request runs. Once it has finished: copies X (host,
 * n doubles; may be NULL) and stats (may be NULL; seconds = time from
 * submission to completion), forgets the ticket and returns the request's
 * status (DI_OK, DI_E_NOCONV with X filled, ...). DI_E_NOTFOUND for a
 * ticket never issued or already collected. */
di_status di_serve_poll(di_server* s, uint64_t ticket, double* X, di_stats* stats);

/* Counters of the server. */
di_status di_serve_info(di_server* s, di_serve_stats* out);

/* Stops the worker (running requests are dropped) and frees the server.
 * NULL is ignored. */
void di_serve_destroy(di_server* s);

/* The FP64 residual R = B + P.X - X of an approximate solution X, and
 * |R|_1 (the refinement step of DI_FP32_REFINE, which recomputes the fluid
 * of Sections 2.5.4-2.5.5 as F = B - (I - P).X). B_dev: n doubles on the
 * device, or NULL for the PageRank right-hand side (1-d)/n. X_dev: n
 * doubles on the device (read only). R_dev: n doubles on the device, or NULL when only the
 * norm is wanted. *l1 (host, may be NULL) receives |R|_1, summed in FP64.
 * Work is queued on `stream` (NULL = the null stream); the call returns
 * once it has finished. */
di_status di_residual_dev(const di_graph* g, const double* B_dev, double d, const double* X_dev,
                          double* R_dev, double* l1, void* stream);

/* di_residual_dev for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops and harnesses that forbid hipMalloc):
 * the same pass, arguments and result (|R|_1 bit for bit), with its scratch
 * (y = d X / out, the heavy-row segment sums, the per-block records and,
 * when R_dev is NULL, R itself) taken from a fixed 128 MiB device array that
 * each GPU holds from the first call until the process ends. The call
 * allocates no device memory.
 * Limit: 8 n + 8 (heavy-row segments) + about 82 KB of records, plus 8 n
 * when R_dev is NULL, must fit in 128 MiB (n up to about 16.7M with R_dev,
 * 8.3M without); a larger graph returns DI_E_INVAL before any device work.
 * Every call on one GPU uses that GPU's array: calls that overlap on the
 * same GPU (other host threads, or other streams before this call returns)
 * race on it and must be serialized by the caller. */
di_status di_residual_dev_noalloc(const di_graph* g, const double* B_dev, double d,
                                  const double* X_dev, double* R_dev, double* l1, void* stream);

/* Message describing the calling thread's last failure ("" if none). */
const char* di_last_error(void);

/* ABI version: (major << 16) | minor. */
int32_t di_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DI_H */
