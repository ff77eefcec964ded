/*
 * Plain FP64 CPU oracle for the iterations compared in "Revisiting the
 * D-iteration method: runtime comparison" (Hong, Burnside, Raoult, 2012).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it. It shares no code with the GPU path.
 *
 * The problem (Section 1): X = P.X + B, where for every link j -> i,
 * P[i][j] = d / out_j (out_j counts every link leaving j, a self-loop
 * included, Section 2.4); a column j with out_j = 0 (dangling node) is zero.
 * The iterators of Section 2.1 are kept as two adjacency lists:
 *   l_out[i] = out-links of i (column i of P),
 *   l_in[i]  = in-links of i  (row i of P).
 *
 * Style: double everywhere, one thread, nodes visited in ascending order,
 * no blocking or reordering beyond what each method states. Built with
 * -ffp-contract=off so every a*b+c rounds twice, as written.
 *
 * Readings where the paper is silent or inconsistent (the same readings are
 * listed in the design notes):
 *   - r of DI-SOP is computed once per cycle, at its start (Section 2.3 says
 *     "per cycle").
 *   - DI-SOP selects i when |F_i| > 0 and |F_i| >= (r/L)*out_i; the paper's
 *     strict ">" can select nothing at an exact tie (the chain 0->1 stalls),
 *     and a cycle that still selects nothing is followed by one DI-CYC cycle
 *     (counted as a fallback).
 *   - A dangling node has threshold 0 (r/L*0), so any fluid it holds is
 *     absorbed; when L = 0 this avoids r/L = inf.
 *   - Fluid may be signed (a residual used as a right-hand side): the
 *     predicates and r use |F_i|; for B >= 0 this is the paper's rule.
 *   - The dangling branch of DI-CYC is "if out_i == 0 then e += transit else
 *     push" (the printed braces do not balance).
 *   - PI and PI' swap x_old and x_new at the end of each iteration, start
 *     with error = +infinity, and both stop at error <= target (the printed
 *     PI' threshold target*(1-d)/d contradicts the equal PI / PI' iteration
 *     counts of every table).
 *   - GS starts from x = B (equal to (1-d)/N for the PageRank B).
 *   - "nb iter" = link operations / L; a self-loop is not a link operation
 *     of the D-iteration push (it is folded into the transit formula).
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_DUP (-3)
#define ORC_E_RANGE (-4)
#define ORC_E_NOMEM (-5)
#define ORC_E_NOCONV (-6)

typedef struct orc_graph {
  int64_t n;
  int64_t L;           /* links (non-null entries of P) */
  int64_t *out_ptr;    /* l_out[i] = out_idx[out_ptr[i] .. out_ptr[i+1]) */
  int32_t *out_idx;
  int64_t *in_ptr;     /* l_in[i] = in_idx[in_ptr[i] .. in_ptr[i+1]) */
  int32_t *in_idx;
  int32_t *out;        /* out-degree, self-loop included */
  uint8_t *loop;       /* 1 if the link i -> i exists */
} orc_graph;

typedef struct orc_stats {
  int64_t cycles;          /* DI cycles, PI iterations or GS sweeps */
  int64_t link_ops;        /* links traversed by the iteration */
  int64_t fallback_cycles; /* DI-CYC cycles run after an empty DI-SOP cycle */
  double nb_iter;          /* link_ops / L */
  double resid_l1;         /* ||B + P.X - X||_1 of the result (DI: ||F||_1) */
  double paper_err;        /* last value of the paper's error estimator */
  double e;                /* fluid absorbed by dangling nodes (DI), or
                              sum of x over dangling nodes (GS) */
  double seconds;          /* wall time of the iteration loop */
} orc_stats;

static double now_seconds(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

void orc_graph_free(orc_graph *g) {
  if (!g) return;
  free(g->out_ptr);
  free(g->out_idx);
  free(g->in_ptr);
  free(g->in_idx);
  free(g->out);
  free(g->loop);
  free(g);
}

/* Builds both iterator sets from a link list (origin src[e] -> destination
 * dst[e]). Lists keep the input order inside l_out and ascending origin
 * inside l_in when the input is sorted by origin. Duplicate links are
 * rejected (P would not be a 0/d-out matrix). */
int orc_graph_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    orc_graph **out_g) {
  if (!out_g || n < 0 || m < 0 || (m > 0 && (!src || !dst))) return ORC_E_INVAL;
  *out_g = NULL;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORC_E_RANGE;
  orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
  if (!g) return ORC_E_NOMEM;
  g->n = n;
  g->L = m;
  size_t nn = (size_t)n + 1;
  g->out_ptr = (int64_t *)calloc(nn, sizeof(int64_t));
  g->in_ptr = (int64_t *)calloc(nn, sizeof(int64_t));
  g->out_idx = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  g->in_idx = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  g->out = (int32_t *)calloc(nn, sizeof(int32_t));
  g->loop = (uint8_t *)calloc(nn, 1);
  int64_t *fill = (int64_t *)malloc(nn * sizeof(int64_t));
  if (!g->out_ptr || !g->in_ptr || !g->out_idx || !g->in_idx || !g->out || !g->loop || !fill) {
    free(fill);
    orc_graph_free(g);
    return ORC_E_NOMEM;
  }
  for (int64_t e = 0; e < m; ++e) {
    g->out_ptr[src[e] + 1]++;
    g->in_ptr[dst[e] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) {
    g->out_ptr[i + 1] += g->out_ptr[i];
    g->in_ptr[i + 1] += g->in_ptr[i];
    g->out[i] = (int32_t)(g->out_ptr[i + 1] - g->out_ptr[i]);
  }
  memcpy(fill, g->out_ptr, (size_t)n * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) g->out_idx[fill[src[e]]++] = dst[e];
  memcpy(fill, g->in_ptr, (size_t)n * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) g->in_idx[fill[dst[e]]++] = src[e];
  free(fill);
  /* self-loops, and duplicates: a repeated destination inside one out-list
   * (adjacent when the list is ascending, else found by comparing all pairs) */
  for (int64_t i = 0; i < n; ++i) {
    int ascending = 1;
    for (int64_t a = g->out_ptr[i]; a < g->out_ptr[i + 1]; ++a) {
      if (g->out_idx[a] == i) g->loop[i] = 1;
      if (a > g->out_ptr[i] && g->out_idx[a] <= g->out_idx[a - 1]) ascending = 0;
    }
    if (ascending) continue;
    for (int64_t a = g->out_ptr[i]; a < g->out_ptr[i + 1]; ++a)
      for (int64_t b = a + 1; b < g->out_ptr[i + 1]; ++b)
        if (g->out_idx[b] == g->out_idx[a]) {
          orc_graph_free(g);
          return ORC_E_DUP;
        }
  }
  *out_g = g;
  return ORC_OK;
}

int64_t orc_graph_n(const orc_graph *g) { return g ? g->n : -1; }
int64_t orc_graph_links(const orc_graph *g) { return g ? g->L : -1; }

/* R = B + P.X - X (the residual of the linear system, its plain
 * definition: R_i = B_i + sum_{j in l_in[i]} d*X_j/out_j - X_i).
 * Returns ||R||_1; R may be NULL. */
double orc_residual(const orc_graph *g, const double *B, double d, const double *X, double *R) {
  double l1 = 0.0;
  for (int64_t i = 0; i < g->n; ++i) {
    double acc = B[i];
    for (int64_t q = g->in_ptr[i]; q < g->in_ptr[i + 1]; ++q) {
      int32_t j = g->in_idx[q];
      acc += d * X[j] / g->out[j];
    }
    acc -= X[i];
    if (R) R[i] = acc;
    l1 += fabs(acc);
  }
  return l1;
}

/* y = P.x (row by row). */
void orc_apply_p(const orc_graph *g, double d, const double *x, double *y) {
  for (int64_t i = 0; i < g->n; ++i) {
    double acc = 0.0;
    for (int64_t q = g->in_ptr[i]; q < g->in_ptr[i + 1]; ++q) {
      int32_t j = g->in_idx[q];
      acc += d * x[j] / g->out[j];
    }
    y[i] = acc;
  }
}

static double l1_norm(const double *v, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += fabs(v[i]);
  return s;
}

/* ---------------------------------------------------------------------
 * D-iteration (Sections 2.3, 2.5.4, 2.5.5).
 *
 * Diffusing node i (Section 2.5.4):
 *   transit = F_i, or F_i*out_i/(out_i - d) when i has a self-loop
 *             (the self-loop's share is summed as a geometric series);
 *   H_i += transit; F_i = 0;
 *   out_i == 0: e += transit (the fluid leaves the system);
 *   else: every out-link i -> j with j != i receives transit*d/out_i.
 * ------------------------------------------------------------------- */

static void di_diffuse(const orc_graph *g, double d, int64_t i, double f, double *F, double *H,
                       double *e, int64_t *link_ops) {
  double transit;
  if (g->loop[i]) transit = f * g->out[i] / (g->out[i] - d);
  else transit = f;
  H[i] += transit;
  if (g->out[i] == 0) {
    *e += transit;
    return;
  }
  double sent = transit * d / g->out[i];
  for (int64_t q = g->out_ptr[i]; q < g->out_ptr[i + 1]; ++q) {
    int32_t j = g->out_idx[q];
    if (j != i) {
      F[j] += sent;
      ++*link_ops;
    }
  }
}

/* di_diffuse for schedule 2: the amount sent along i -> j reaches F_j at
 * once when |i - j| <= reach and j lies in i's tile of `tile` ids, and
 * next_F_j (the next cycle's) otherwise. */
static void di_diffuse_routed(const orc_graph *g, double d, int64_t i, double f, double *F,
                              double *next_F, int64_t tile, int64_t reach, double *H, double *e,
                              int64_t *link_ops) {
  double transit;
  if (g->loop[i]) transit = f * g->out[i] / (g->out[i] - d);
  else transit = f;
  H[i] += transit;
  if (g->out[i] == 0) {
    *e += transit;
    return;
  }
  double sent = transit * d / g->out[i];
  for (int64_t q = g->out_ptr[i]; q < g->out_ptr[i + 1]; ++q) {
    int32_t j = g->out_idx[q];
    if (j == i) continue;
    if (j - i <= reach && i - j <= reach && j / tile == i / tile) F[j] += sent;
    else next_F[j] += sent;
    ++*link_ops;
  }
}

/* Selection predicate. variant 0: DI-SOP, 1: DI-CYC. r is the cycle's
 * r_{n'} = sum_i |F_i|. */
static int di_selected(const orc_graph *g, int variant, double r, int64_t i, double f) {
  double a = fabs(f);
  if (!(a > 0.0)) return 0;
  if (variant == 1) return 1;
  double thr = g->out[i] == 0 ? 0.0 : r / g->L * g->out[i];
  return a >= thr;
}

/* One cycle over all nodes. schedule 0: the paper's sequential cycle (node i
 * sees fluid pushed by nodes diffused earlier in the same cycle); schedule 1:
 * frontier-synchronous cycle (the selected set and the claimed amounts come
 * from the fluid at the start of the cycle; fluid pushed during the cycle
 * waits for the next one) -- a labelled variant, not the paper's schedule.
 * r_{n'} = sum |F| at the start of the cycle is returned in *r_out.
 * selected (nullable) receives 1 for each diffused node. claim is scratch of
 * n doubles for schedule 1. Returns the number of diffused nodes. */
int64_t orc_di_cycle(const orc_graph *g, double d, int variant, int schedule, double *F, double *H,
                     double *e, int64_t *link_ops, uint8_t *selected, double *claim, double *r_out) {
  const int64_t n = g->n;
  double r = l1_norm(F, n);
  if (r_out) *r_out = r;
  int64_t count = 0;
  if (selected) memset(selected, 0, (size_t)n);
  if (schedule == 0) {
    for (int64_t i = 0; i < n; ++i) {
      if (!di_selected(g, variant, r, i, F[i])) continue;
      double f = F[i];
      F[i] = 0.0;
      di_diffuse(g, d, i, f, F, H, e, link_ops);
      if (selected) selected[i] = 1;
      ++count;
    }
  } else {
    for (int64_t i = 0; i < n; ++i) {
      claim[i] = 0.0;
      if (di_selected(g, variant, r, i, F[i])) {
        claim[i] = F[i];
        if (selected) selected[i] = 1;
        ++count;
      }
    }
    for (int64_t i = 0; i < n; ++i)
      if (claim[i] != 0.0) F[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      if (claim[i] != 0.0) di_diffuse(g, d, i, claim[i], F, H, e, link_ops);
  }
  return count;
}

/* One cycle of any schedule. Schedules 0 and 1 as orc_di_cycle (tile,
 * reach and rounds unused). Schedule 2, "tiled": the frontier-synchronous
 * cycle run in `rounds` rounds over contiguous tiles of `tile` node ids -- a
 * labelled variant, not the paper's schedule. Each round selects, against
 * the r of the cycle's start, from every node's current fluid, claims the
 * selected nodes and diffuses them; what a node sends along a link i -> j
 * with |i - j| <= reach and j in i's tile reaches F_j at once (so a later
 * round of the same cycle sees it, as node i's successors see it in the
 * paper's sequential cycle), what it sends along any other link waits for
 * the next cycle. DI-CYC (and a fallback cycle) runs one round. next_F is
 * scratch of n doubles for schedule 2. The count is of diffusions (a node
 * diffused in two rounds counts twice); selected marks the nodes diffused
 * at least once. */
int64_t orc_di_cycle2(const orc_graph *g, double d, int variant, int schedule, int64_t tile,
                      int64_t reach, int rounds, double *F, double *H, double *e,
                      int64_t *link_ops, uint8_t *selected, double *claim, double *next_F,
                      double *r_out) {
  if (schedule != 2)
    return orc_di_cycle(g, d, variant, schedule, F, H, e, link_ops, selected, claim, r_out);
  const int64_t n = g->n;
  double r = l1_norm(F, n);
  if (r_out) *r_out = r;
  int64_t count = 0;
  if (selected) memset(selected, 0, (size_t)n);
  for (int64_t i = 0; i < n; ++i) next_F[i] = 0.0;
  const int nr = variant == 0 ? rounds : 1;
  for (int k = 0; k < nr; ++k) {
    for (int64_t i = 0; i < n; ++i) {
      claim[i] = 0.0;
      if (di_selected(g, variant, r, i, F[i])) {
        claim[i] = F[i];
        if (selected) selected[i] = 1;
        ++count;
      }
    }
    for (int64_t i = 0; i < n; ++i)
      if (claim[i] != 0.0) F[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      if (claim[i] != 0.0)
        di_diffuse_routed(g, d, i, claim[i], F, next_F, tile, reach, H, e, link_ops);
  }
  for (int64_t i = 0; i < n; ++i) F[i] += next_F[i];
  return count;
}

/* Full D-iteration solve from F = B, H = 0, e = 0.
 * variant: 0 DI-SOP, 1 DI-CYC. schedule: 0 sequential, 1 sync-frontier, 2
 * tiled (tile, reach, rounds as in orc_di_cycle2; orc_diter takes 0 or 1).
 * stop 0 ("resid"): stop at the start of a cycle when sum|F| <= tol
 *   (sum|F| = ||B + P.H - H||_1 exactly, since F = B - (I-P).H);
 * stop 1 ("paper"): after each cycle, stop when
 *   sum F / (1 - d - d*e) <= tol (Section 2.5.4 with target 1/N).
 * H receives X; F (nullable) the remaining fluid. */
int orc_diter2(const orc_graph *g, const double *B, double d, int variant, int schedule,
               int64_t tile, int64_t reach, int rounds, int stop, double tol, int64_t max_cycles,
               double *H, double *F_out, orc_stats *st) {
  if (!g || !B || !H || !(d > 0.0 && d < 1.0) || !(tol >= 0.0) || variant < 0 || variant > 1 ||
      schedule < 0 || schedule > 2 || (schedule == 2 && (tile < 1 || reach < 0 || rounds < 1)))
    return ORC_E_INVAL;
  const int64_t n = g->n;
  const size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
  double *F = (double *)malloc(bytes);
  double *claim = schedule ? (double *)malloc(bytes) : NULL;
  double *next_F = schedule == 2 ? (double *)malloc(bytes) : NULL;
  if (!F || (schedule && !claim) || (schedule == 2 && !next_F)) {
    free(F);
    free(claim);
    free(next_F);
    return ORC_E_NOMEM;
  }
  for (int64_t i = 0; i < n; ++i) {
    F[i] = B[i];
    H[i] = 0.0;
  }
  orc_stats s;
  memset(&s, 0, sizeof(s));
  s.paper_err = INFINITY;
  double e = 0.0;
  int rc = ORC_OK;
  double t0 = now_seconds();
  for (;;) {
    if (stop == 0) {
      double r = l1_norm(F, n);
      s.resid_l1 = r;
      if (r <= tol) break;
    }
    if (s.cycles >= max_cycles) {
      rc = ORC_E_NOCONV;
      break;
    }
    double r_used = 0.0;
    int64_t cnt = orc_di_cycle2(g, d, variant, schedule, tile, reach, rounds, F, H, &e, &s.link_ops,
                                NULL, claim, next_F, &r_used);
    ++s.cycles;
    if (cnt == 0 && r_used > 0.0 && variant == 0) {
      orc_di_cycle2(g, d, 1, schedule, tile, reach, rounds, F, H, &e, &s.link_ops, NULL, claim,
                    next_F, NULL);
      ++s.fallback_cycles;
    }
    if (stop == 1) {
      double sum = 0.0;
      for (int64_t i = 0; i < n; ++i) sum += F[i];
      s.paper_err = sum / (1.0 - d - d * e);
      if (s.paper_err <= tol) break;
    }
  }
  s.seconds = now_seconds() - t0;
  s.resid_l1 = l1_norm(F, n);
  s.e = e;
  s.nb_iter = g->L > 0 ? (double)s.link_ops / (double)g->L : 0.0;
  if (F_out) memcpy(F_out, F, (size_t)n * sizeof(double));
  if (st) *st = s;
  free(F);
  free(claim);
  free(next_F);
  return rc;
}

int orc_diter(const orc_graph *g, const double *B, double d, int variant, int schedule, int stop,
              double tol, int64_t max_cycles, double *H, double *F_out, orc_stats *st) {
  if (schedule < 0 || schedule > 1) return ORC_E_INVAL;
  return orc_diter2(g, B, d, variant, schedule, 1, 0, 1, stop, tol, max_cycles, H, F_out, st);
}

/* ---------------------------------------------------------------------
 * Power iteration (Sections 2.5.1 and 2.5.2): the normalized PageRank
 * vector. x starts at 1/N; each iteration
 *   x_new_i = (1-d)/N + sum_{j in l_in[i]} d*x_old_j/out_j  (PI, by rows)
 *   or the same sum scattered along l_out (PI', by columns);
 *   x_new += (1 - sum x_new)/N;  error = d/(1-d) * ||x_new - x_old||_1.
 * Stops when error <= target. Its fixed point is X/||X||_1.
 * ------------------------------------------------------------------- */
int orc_pi(const orc_graph *g, double d, int by_columns, double target, int64_t max_iter,
           double *x, orc_stats *st) {
  if (!g || !x || !(d > 0.0 && d < 1.0) || g->n <= 0) return ORC_E_INVAL;
  const int64_t n = g->n;
  double *x_old = (double *)malloc((size_t)n * sizeof(double));
  double *x_new = (double *)malloc((size_t)n * sizeof(double));
  if (!x_old || !x_new) {
    free(x_old);
    free(x_new);
    return ORC_E_NOMEM;
  }
  for (int64_t i = 0; i < n; ++i) x_old[i] = 1.0 / n;
  orc_stats s;
  memset(&s, 0, sizeof(s));
  double error = INFINITY;
  int rc = ORC_OK;
  double t0 = now_seconds();
  while (error > target) {
    if (s.cycles >= max_iter) {
      rc = ORC_E_NOCONV;
      break;
    }
    for (int64_t i = 0; i < n; ++i) x_new[i] = (1 - d) / n;
    if (!by_columns) {
      for (int64_t i = 0; i < n; ++i)
        for (int64_t q = g->in_ptr[i]; q < g->in_ptr[i + 1]; ++q) {
          int32_t j = g->in_idx[q];
          x_new[i] += d * x_old[j] / g->out[j];
        }
    } else {
      for (int64_t i = 0; i < n; ++i) {
        if (g->out[i] == 0) continue;
        double transit = d * x_old[i] / g->out[i];
        for (int64_t q = g->out_ptr[i]; q < g->out_ptr[i + 1]; ++q) x_new[g->out_idx[q]] += transit;
      }
    }
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) sum += x_new[i];
    for (int64_t i = 0; i < n; ++i) x_new[i] += (1.0 - sum) / n;
    error = 0.0;
    for (int64_t i = 0; i < n; ++i) error += fabs(x_new[i] - x_old[i]);
    error *= d / (1 - d);
    double *tmp = x_old;
    x_old = x_new;
    x_new = tmp;
    ++s.cycles;
    s.link_ops += g->L;
  }
  s.seconds = now_seconds() - t0;
  s.paper_err = error;
  s.nb_iter = (double)s.cycles;
  memcpy(x, x_old, (size_t)n * sizeof(double));
  if (st) *st = s;
  free(x_old);
  free(x_new);
  return rc;
}

/* Power iteration on the unnormalized system (Jacobi iteration, which the
 * paper states PI is equivalent to): x = B, then x <- B + P.x. Each step
 * first measures the residual ||B + P.x - x||_1 of the current x and stops
 * when it is <= tol, so the returned x carries that residual. */
int orc_jacobi(const orc_graph *g, const double *B, double d, double tol, int64_t max_iter,
               double *x, orc_stats *st) {
  if (!g || !B || !x || !(d > 0.0 && d < 1.0)) return ORC_E_INVAL;
  const int64_t n = g->n;
  double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!y) return ORC_E_NOMEM;
  memcpy(x, B, (size_t)n * sizeof(double));
  orc_stats s;
  memset(&s, 0, sizeof(s));
  int rc = ORC_OK;
  double t0 = now_seconds();
  for (;;) {
    orc_apply_p(g, d, x, y);
    double res = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      y[i] += B[i];
      res += fabs(y[i] - x[i]);
    }
    s.link_ops += g->L;
    s.resid_l1 = res;
    if (res <= tol) break;
    if (s.cycles >= max_iter) {
      rc = ORC_E_NOCONV;
      break;
    }
    memcpy(x, y, (size_t)n * sizeof(double));
    ++s.cycles;
  }
  s.seconds = now_seconds() - t0;
  s.nb_iter = g->L > 0 ? (double)s.link_ops / (double)g->L : 0.0;
  if (st) *st = s;
  free(y);
  return rc;
}

/* ---------------------------------------------------------------------
 * Gauss-Seidel, cyclic sweep in ascending order (Section 2.5.3):
 *   x_i <- (B_i + sum_{j in l_in[i], j != i} d*x_j/out_j) / (1 - d/out_i [i has a loop])
 * using the newest x_j. stop 1 ("paper"): error = d * sum(x_i - previous)
 * / (1 - d - d*e) with e = sum of x over dangling nodes, against tol;
 * stop 0 ("resid"): ||B + P.x - x||_1 <= tol after a sweep.
 * ------------------------------------------------------------------- */
int orc_gs(const orc_graph *g, const double *B, double d, int stop, double tol, int64_t max_sweeps,
           double *x, orc_stats *st) {
  if (!g || !B || !x || !(d > 0.0 && d < 1.0)) return ORC_E_INVAL;
  const int64_t n = g->n;
  for (int64_t i = 0; i < n; ++i) x[i] = B[i];
  orc_stats s;
  memset(&s, 0, sizeof(s));
  int rc = ORC_OK;
  double t0 = now_seconds();
  for (;;) {
    if (stop == 0) {
      s.resid_l1 = orc_residual(g, B, d, x, NULL);
      if (s.resid_l1 <= tol) break;
    }
    if (s.cycles >= max_sweeps) {
      rc = ORC_E_NOCONV;
      break;
    }
    double error = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double previous = x[i];
      double xi = B[i];
      double diag = 1.0;
      for (int64_t q = g->in_ptr[i]; q < g->in_ptr[i + 1]; ++q) {
        int32_t j = g->in_idx[q];
        if (j != i) xi += d * x[j] / g->out[j];
        else diag -= d / g->out[i];
      }
      x[i] = xi / diag;
      error += x[i] - previous;
    }
    ++s.cycles;
    s.link_ops += g->L;
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i)
      if (g->out[i] == 0) e += x[i];
    s.e = e;
    s.paper_err = error * d / (1 - d - d * e);
    if (stop == 1 && s.paper_err <= tol) break;
  }
  s.seconds = now_seconds() - t0;
  if (stop == 1) s.resid_l1 = orc_residual(g, B, d, x, NULL);
  s.nb_iter = (double)s.cycles;
  if (st) *st = s;
  return rc;
}
