// HIP kernels of batched D-iteration: KP right-hand sides diffused together
// on one graph (personalized PageRank batches).
//
// Each column is an independent DI-SOP solve (Sections 2.3 and 2.5.5) with
// its own r = sum_i |F_ic|, tolerance and pass state; the columns share the
// graph and the launches. A cycle is three launches:
//   select  per (node, column): the DI-SOP rule against the column's r;
//           claim (H += transit, F = 0); the node's amounts per link go to
//           sent[node][*] (0 in the columns that did not select it), and the
//           node's bit in the frontier bitmap is set when any column sends.
//   pull    per work item (the single-RHS pull items: rows with at most
//           2048 in-links, or a segment of a longer row): the item's in-link
//           ids, filtered by the bitmap, are staged in LDS; the lane groups
//           of the block take equal shares of the links and add the senders'
//           rows of KP values; rows cut by a share boundary are finished in
//           a fixed order. Per-block sums of |F| per column are written.
//   reduce  one block per column: completes the rows split into segments
//           (the segment sums in order), then the stop test and the next
//           state.
// Lanes whose columns are all idle load and store nothing, and the serving
// loop fills the lowest free columns first, so a batch with few running
// columns touches few cache lines per node.
// The residual pass of a refined solve (FP64: R = B + P.X - X) runs through
// the same pull and heavy kernels with y = d X / out as the senders' rows,
// for the columns waiting for it.
//
// Lane layouts (per kernel; the memory layout is shared): the pull gives a
// lane 8 consecutive columns (one 32-byte gather in FP32; 4 at 256 columns)
// so each lane group walks a short share of an item's links and narrow
// batches get many shares with their gathers in flight together; the
// selection keeps one column per lane up to 64 columns.

#include <algorithm>
#include <type_traits>

#include "di_batch.h"

namespace di {
namespace {

// Lane layouts: a group of G = KP / V lanes holds one node's KP values, V
// consecutive columns per lane; a wave holds P = 64 / G groups. The memory
// layout ([n][KP]) is the same for every kernel; the lane layout is each
// kernel's own choice.
template <int KP, int V_>
struct LayV {
  static constexpr int V = V_;
  static constexpr int G = KP / V;
  static constexpr int P = 64 / G;
  static constexpr int NW = kBBlock / 64;
  static constexpr int NG = NW * P;
  static_assert(KP % V == 0 && G >= 1 && G <= 64, "lane layout");
};
// selection: one column per lane up to 64 columns (per-column work stays
// spread over lanes)
template <int KP>
using LaySel = LayV<KP, (KP <= 64 ? 1 : KP / 64)>;
// pull: 8 columns per lane (one 32-byte gather in FP32), so each lane group
// walks a short share of an item's links; 4 at 256 columns
template <int KP>
using Lay = LayV<KP, (KP >= 256 ? 4 : 8)>;

__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return (double)x; }

template <typename S, int V>
struct alignas(sizeof(S) * V) Pack {
  S v[V];
};

template <typename S, int V>
__device__ inline Pack<S, V> ld(const S* p) {
  return *reinterpret_cast<const Pack<S, V>*>(p);
}
template <typename S, int V>
__device__ inline void st(S* p, const Pack<S, V>& x) {
  *reinterpret_cast<Pack<S, V>*>(p) = x;
}
template <typename S, int V>
__device__ inline Pack<S, V> zero_pack() {
  Pack<S, V> x;
#pragma unroll
  for (int v = 0; v < V; ++v) x.v[v] = (S)0;
  return x;
}

// Sum over the P lanes of a wave that hold the same columns.
template <int G, typename A>
__device__ inline A group_fold(A x) {
#pragma unroll
  for (int off = 32; off >= G; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <typename A>
__device__ inline A wave_sum(A v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum, valid in every thread (fixed order). lds: kBBlock / 64 values.
template <typename A>
__device__ A block_sum_all(A v, A* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  A t = 0;
#pragma unroll
  for (int w = 0; w < kBBlock / 64; ++w) t += lds[w];
  __syncthreads();
  return t;
}

// Sum of v[q * stride] for q in [q0, q1), added in order; the loads are
// issued eight at a time so a long run does not wait on each one.
__device__ inline double ordered_sum(const double* __restrict__ v, int64_t q0, int64_t q1,
                                     int64_t stride) {
  double acc = 0.0;
  int64_t q = q0;
  for (; q + 8 <= q1; q += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = v[(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += t[u];
  }
  for (; q < q1; ++q) acc += v[q * stride];
  return acc;
}

// Per-column block totals of acc (each thread holds columns gl*V + v),
// written to out[0, KW). lds: (kBBlock / 64) * KW values. Fixed order.
template <typename Ly, int KW, typename A>
__device__ inline void col_sum_store(A (&acc)[Ly::V], A* lds, A* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < Ly::V; ++v) acc[v] = group_fold<Ly::G>(acc[v]);
  if (lane < Ly::G) {
#pragma unroll
    for (int v = 0; v < Ly::V; ++v) lds[wave * KW + lane * Ly::V + v] = acc[v];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < KW; c += kBBlock) {
    A s = 0;
#pragma unroll
    for (int w = 0; w < Ly::NW; ++w) s += lds[w * KW + c];
    out[c] = s;
  }
  __syncthreads();
}

// ---- load / records / store ---------------------------------------------

// Tile transposition of the caller's k x n right-hand sides into [n][KP]:
// F = B (rounded to T), H = 0, and Bd = B, X64 = 0 when given. A block moves
// 32 nodes x 64 columns through LDS.
template <typename T, int KP>
__global__ __launch_bounds__(kBBlock) void k_bload(const double* __restrict__ B_in, int k,
                                                   int64_t n, double b_uniform, T* __restrict__ F,
                                                   T* __restrict__ H, double* __restrict__ Bd,
                                                   double* __restrict__ X64) {
  __shared__ double tile[64][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 64;
  for (int e = threadIdx.x; e < 64 * 32; e += kBBlock) {
    const int cl = e >> 5, il = e & 31;
    const int64_t i = i0 + il;
    const int c = c0 + cl;
    double b = 0.0;
    if (c < k && i < n) b = B_in ? B_in[(int64_t)c * n + i] : b_uniform;
    tile[cl][il] = b;
  }
  __syncthreads();
  const int cw = KP - c0 < 64 ? KP - c0 : 64;
  for (int e = threadIdx.x; e < 32 * 64; e += kBBlock) {
    const int il = e >> 6, cl = e & 63;
    const int64_t i = i0 + il;
    if (i < n && cl < cw) {
      const int64_t q = i * KP + c0 + cl;
      const double b = tile[cl][il];
      F[q] = (T)b;
      H[q] = (T)0;
      if (Bd) Bd[q] = b;
      if (X64) X64[q] = 0.0;
    }
  }
}

// X_out[c][i] = H[i][c] (+ X64[i][c]) for c < k; the reverse tile move.
template <typename T, int KP>
__global__ __launch_bounds__(kBBlock) void k_bstore(const T* __restrict__ H,
                                                    const double* __restrict__ X64,
                                                    double* __restrict__ X_out, int k, int64_t n) {
  __shared__ double tile[64][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 64;
  const int cw = KP - c0 < 64 ? KP - c0 : 64;
  for (int e = threadIdx.x; e < 32 * 64; e += kBBlock) {
    const int il = e >> 6, cl = e & 63;
    const int64_t i = i0 + il;
    double x = 0.0;
    if (i < n && cl < cw) {
      const int64_t q = i * KP + c0 + cl;
      x = to_d(H[q]);
      if (X64) x += X64[q];
    }
    tile[cl][il] = x;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 32; e += kBBlock) {
    const int cl = e >> 5, il = e & 31;
    const int64_t i = i0 + il;
    const int c = c0 + cl;
    if (c < k && i < n) X_out[(int64_t)c * n + i] = tile[cl][il];
  }
}

// rec[block][c] = sum of |F[i][c]| over the block's nodes.
template <typename T, int KP>
__global__ __launch_bounds__(kBBlock) void k_brecords(const T* __restrict__ F, int64_t n,
                                                      double* __restrict__ rec) {
  using Ly = Lay<KP>;
  __shared__ double lds[Ly::NW * KP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / Ly::G, gl = lane % Ly::G;
  double acc[Ly::V];
#pragma unroll
  for (int v = 0; v < Ly::V; ++v) acc[v] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * Ly::NG;
  for (int64_t i = (int64_t)blockIdx.x * Ly::NG + wave * Ly::P + grp; i < n; i += stride) {
    const Pack<T, Ly::V> f = ld<T, Ly::V>(F + i * KP + gl * Ly::V);
#pragma unroll
    for (int v = 0; v < Ly::V; ++v) acc[v] += fabs(to_d(f.v[v]));
  }
  col_sum_store<Ly, KP>(acc, lds, rec + (int64_t)blockIdx.x * KP);
}

// ---- selection ----------------------------------------------------------

// Waves take 64-node words of the frontier bitmap; a wave covers its word
// in 64 / P passes of P nodes. Per-column counters go to the block's
// records (rec_ops / rec_sel / rec_e row blockIdx.x); column KP of rec_ops
// and rec_sel holds the node-level frontier (links gathered, nodes).
// Only columns [0, KE) are looked at (the others are idle); rows are KP
// values apart.
template <typename T, int KP, int KE>
__global__ __launch_bounds__(kBBlock) void k_bselect(
    T* __restrict__ F, T* __restrict__ H, T* __restrict__ sent,
    unsigned long long* __restrict__ front_bits, const uint32_t* __restrict__ info, int64_t n,
    int64_t L, double d, const BCtl* __restrict__ bctl, unsigned long long* __restrict__ rec_ops,
    unsigned int* __restrict__ rec_sel, double* __restrict__ rec_e) {
  using Ly = LaySel<KE>;
  constexpr int G = Ly::G, P = Ly::P, V = Ly::V;
  __shared__ double s_rl[KE];
  __shared__ int s_flag[KE];
  __shared__ unsigned long long s_u64[Ly::NW * KE];
  __shared__ unsigned int s_u32[Ly::NW * KE];
  __shared__ double s_f64[Ly::NW * KE];
  __shared__ unsigned long long s_n64[Ly::NW];
  __shared__ unsigned int s_n32[Ly::NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane / G, gl = lane % G;
  int any = 0;
  for (int c = tid; c < KE; c += kBBlock) {
    const int state = bctl[c].state;
    const int run = state == kBRun ? 1 : 0;
    s_flag[c] = run | (bctl[c].cyc_mode ? 2 : 0);
    s_rl[c] = bctl[c].r / (double)L;
    any |= run;
  }
  if (!__syncthreads_or(any)) return;
  double rl[V];
  bool run[V], cyc[V];
  unsigned long long ops[V];
  unsigned int sel[V];
  double eab[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = gl * V + v;
    rl[v] = s_rl[c];
    run[v] = (s_flag[c] & 1) != 0;
    cyc[v] = (s_flag[c] & 2) != 0;
    ops[v] = 0;
    sel[v] = 0;
    eab[v] = 0.0;
  }
  unsigned long long fops = 0;
  unsigned int fnodes = 0;
  bool lane_run = false;  // a lane whose columns are all idle loads nothing
#pragma unroll
  for (int v = 0; v < V; ++v) lane_run |= run[v];
  const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << (G & 63)) - 1ull);
  constexpr int NT = 64 / P;          // passes per 64-node word
  constexpr int NB = NT < 4 ? NT : 4;  // passes whose loads are issued together
  const int64_t words = (n + 63) / 64;
  for (int64_t w = (int64_t)blockIdx.x * Ly::NW + wave; w < words;
       w += (int64_t)gridDim.x * Ly::NW) {
    unsigned long long word = 0;
    for (int t0 = 0; t0 < NT; t0 += NB) {
      uint32_t wis[NB];
      Pack<T, V> fs[NB], hs[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int64_t i = w * 64 + (t0 + u) * P + grp;
        wis[u] = i < n ? info[i] : 0u;
        fs[u] = (i < n && lane_run) ? ld<T, V>(F + i * KP + gl * V) : zero_pack<T, V>();
        // narrow batches load H with F (one round of loads instead of a
        // dependent one); wide ones load it only where a column selects
        if constexpr (KE <= 32)
          hs[u] = (i < n && lane_run) ? ld<T, V>(H + i * KP + gl * V) : zero_pack<T, V>();
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int t = t0 + u;
        const int64_t i = w * 64 + t * P + grp;
        bool lane_front = false;
        int np = 0;
        Pack<T, V> sv = zero_pack<T, V>();
        if (i < n) {
          const uint32_t wi = wis[u];
          const int out = (int)(wi & kOutMask);
          const bool loop = (wi & kLoopBit) != 0;
          np = out - (loop ? 1 : 0);
          Pack<T, V> f = fs[u];
          double tr[V];
          bool any_sel = false;
#pragma unroll
          for (int v = 0; v < V; ++v) {
            tr[v] = 0.0;
            const double fv = to_d(f.v[v]);
            const double a = fabs(fv);
            const double thr = (cyc[v] || out == 0) ? 0.0 : rl[v] * (double)out;
            if (run[v] && a > 0.0 && a >= thr) {
              tr[v] = loop ? fv * (double)out / ((double)out - d) : fv;
              f.v[v] = (T)0;
              any_sel = true;
              ++sel[v];
              if (out == 0) {
                eab[v] += tr[v];
              } else if (np > 0) {
                sv.v[v] = (T)(tr[v] * d / (double)out);
                ops[v] += (unsigned long long)np;
                lane_front = true;
              }
            }
          }
          if (any_sel) {
            st<T, V>(F + i * KP + gl * V, f);
            T* Hi = H + i * KP + gl * V;
            Pack<T, V> h;
            if constexpr (KE <= 32) h = hs[u];
            else h = ld<T, V>(Hi);
#pragma unroll
            for (int v = 0; v < V; ++v)
              if (tr[v] != 0.0) h.v[v] = (T)(to_d(h.v[v]) + tr[v]);
            st<T, V>(Hi, h);
          }
        }
        const unsigned long long b = __ballot(lane_front);
        const bool front = ((b >> (grp * G)) & gmask) != 0;
        if (front) {
          // the pull reads the sender rows of running columns only
          if (lane_run) st<T, V>(sent + i * KP + gl * V, sv);
          if (gl == 0) {
            fops += (unsigned long long)np;
            ++fnodes;
          }
        }
        if constexpr (G == 1) {
          word |= b;  // one node per lane: the ballot is the word
        } else {
#pragma unroll
          for (int g2 = 0; g2 < P; ++g2)
            if ((b >> (g2 * G)) & gmask) word |= 1ull << (t * P + g2);
        }
      }
    }
    if (lane == 0) front_bits[w] = word;
  }
  unsigned long long* ro = rec_ops + (int64_t)blockIdx.x * (KP + 1);
  unsigned int* rs = rec_sel + (int64_t)blockIdx.x * (KP + 1);
  col_sum_store<Ly, KE>(ops, s_u64, ro);
  col_sum_store<Ly, KE>(sel, s_u32, rs);
  col_sum_store<Ly, KE>(eab, s_f64, rec_e + (int64_t)blockIdx.x * KP);
  fops = wave_sum(fops);
  fnodes = wave_sum(fnodes);
  if (lane == 0) {
    s_n64[wave] = fops;
    s_n32[wave] = fnodes;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long a = 0;
    unsigned int b = 0;
    for (int q = 0; q < Ly::NW; ++q) {
      a += s_n64[q];
      b += s_n32[q];
    }
    ro[KP] = a;
    rs[KP] = b;
  }
}

// ---- pull (fluid, MODE 0) and residual pass (MODE 1) -----------------------

template <typename T, int KP, int MODE>
struct PullIo {
  T* F;                    // fluid (MODE 1: receives R)
  const T* sent;           // MODE 0 senders' rows
  const unsigned long long* front_bits;
  const double* Y;         // MODE 1 senders' rows (d X / out)
  const double* X;         // MODE 1
  const double* Bd;        // MODE 1
  const uint32_t* info;
};

// Finishes row `row` with its in-link sum acc (this lane's V columns).
// MODE 0: F += acc; MODE 1: F = R = B - X + (self-loop ? y : 0) + acc for
// the masked columns. rsum += |F| (or |R|) per column.
template <typename T, int KP, int KE, int MODE>
__device__ inline void row_epilogue(const PullIo<T, KP, MODE>& io, int64_t row, int gl,
                                    const double (&acc)[Lay<KE>::V], const bool (&mask)[Lay<KE>::V],
                                    double (&rsum)[Lay<KE>::V]) {
  constexpr int V = Lay<KE>::V;
  T* Fr = io.F + row * KP + gl * V;
  if (MODE == 0) {
    bool anym = false;
#pragma unroll
    for (int v = 0; v < V; ++v) anym |= mask[v];
    if (!anym) return;  // idle columns: no arrivals, no record needed
    Pack<T, V> f = ld<T, V>(Fr);
    bool ch = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (acc[v] != 0.0) {
        f.v[v] = (T)(to_d(f.v[v]) + acc[v]);
        ch = true;
      }
      rsum[v] += fabs(to_d(f.v[v]));
    }
    if (ch) st<T, V>(Fr, f);
  } else {
    bool anym = false;
#pragma unroll
    for (int v = 0; v < V; ++v) anym |= mask[v];
    if (!anym) return;
    const bool self = (io.info[row] & kLoopBit) != 0;
    const int64_t q = row * KP + gl * V;
    const Pack<double, V> x = ld<double, V>(io.X + q);
    const Pack<double, V> b = ld<double, V>(io.Bd + q);
    Pack<double, V> y = zero_pack<double, V>();
    if (self) y = ld<double, V>(io.Y + q);
    Pack<T, V> f = ld<T, V>(Fr);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (mask[v]) {
        const double r = b.v[v] - x.v[v] + y.v[v] + acc[v];
        f.v[v] = (T)r;
        rsum[v] += fabs(r);
      }
    }
    st<T, V>(Fr, f);
  }
}

// MODE 0 also adds the selection's node-level counters (column KP of
// rec_ops / rec_sel, nsel rows) to entry KP of the control blocks (block 0),
// once the selection is known to have run. Columns [0, KE) only.
template <typename T, int KP, int KE, int MODE>
__global__ __launch_bounds__(kBBlock) void k_bpull(
    PullIo<T, KP, MODE> io, const int64_t* __restrict__ csc_ptr,
    const int32_t* __restrict__ csc_idx, const int64_t* __restrict__ it_r0,
    const int64_t* __restrict__ it_r1, const int64_t* __restrict__ it_l0,
    const int64_t* __restrict__ it_l1, const int32_t* __restrict__ it_seg, int64_t n_items,
    double* __restrict__ segv, double* __restrict__ rec, BCtl* __restrict__ bctl,
    const unsigned long long* __restrict__ rec_ops, const unsigned int* __restrict__ rec_sel,
    int nsel) {
  using Ly = Lay<KE>;
  constexpr int G = Ly::G, P = Ly::P, V = Ly::V, NG = Ly::NG;
  constexpr int U = 4;
  using SrcT = typename std::conditional<MODE == 0, T, double>::type;
  __shared__ int32_t s_idx[kPullChunk];
  __shared__ int32_t s_ptr[kPullMaxRows + 1];
  __shared__ double s_part[NG * 2 * KE];
  __shared__ double s_rec[Ly::NW * KE];
  __shared__ unsigned long long s_cnt[Ly::NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane / G, gl = lane % G;
  const int gid = wave * P + grp;
  const SrcT* src_rows;
  if constexpr (MODE == 0) src_rows = io.sent;
  else src_rows = io.Y;
  // columns this pass works on: MODE 0 the running ones (any), MODE 1 the
  // ones waiting for a residual pass
  bool mask[V];
  int any = 0;
  for (int c = tid; c < KE; c += kBBlock)
    any |= bctl[c].state == (MODE == 0 ? kBRun : kBInner) ? 1 : 0;
  if (!__syncthreads_or(any)) return;
  if (MODE == 0 && blockIdx.x == 0) {
    unsigned long long na = 0, nb = 0;
    for (int q = tid; q < nsel; q += kBBlock) {
      na += rec_ops[(int64_t)q * (KP + 1) + KP];
      nb += rec_sel[(int64_t)q * (KP + 1) + KP];
    }
    na = block_sum_all(na, s_cnt);
    nb = block_sum_all(nb, s_cnt);
    if (tid == 0) {
      bctl[KP].cycles += 1;
      bctl[KP].edges += na;
      bctl[KP].sel_total += nb;
    }
  }
  bool lane_on = false;  // the lane has a column this pass works on
#pragma unroll
  for (int v = 0; v < V; ++v) {
    mask[v] = bctl[gl * V + v].state == (MODE == 0 ? kBRun : kBInner);
    lane_on |= mask[v];
  }
  double rsum[V];
#pragma unroll
  for (int v = 0; v < V; ++v) rsum[v] = 0.0;
  // XCD-aware item order (see the single-RHS pull)
  int64_t it_begin = blockIdx.x, it_end = n_items, it_step = gridDim.x;
  if (gridDim.x % kXcds == 0) {
    const int64_t x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
    it_begin = n_items * x / kXcds + blockIdx.x / kXcds;
    it_end = n_items * (x + 1) / kXcds;
    it_step = per;
  }
  for (int64_t it = it_begin; it < it_end; it += it_step) {
    const int64_t l0 = it_l0[it], l1 = it_l1[it], r0 = it_r0[it], r1 = it_r1[it];
    const int seg = it_seg[it];
    const int nl = (int)(l1 - l0), nrows = (int)(r1 - r0);
    for (int p = tid; p < nl; p += kBBlock) {
      const int32_t src = csc_idx[l0 + p];
      bool ok = true;
      if (MODE == 0) ok = ((io.front_bits[src >> 6] >> (src & 63)) & 1ull) != 0;
      s_idx[p] = ok ? src : -1;
    }
    if (seg < 0)
      for (int r = tid; r <= nrows; r += kBBlock) s_ptr[r] = (int)(csc_ptr[r0 + r] - l0);
    __syncthreads();
    // this group's share of the links
    const int q0 = (int)((int64_t)nl * gid / NG), q1 = (int)((int64_t)nl * (gid + 1) / NG);
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    int first_row = -1, cur = -1;
    if (q0 < q1) {
      int end = nl;
      if (seg < 0) {  // the row holding link q0
        int lo = 0, hi = nrows - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_ptr[mid] <= q0) lo = mid;
          else hi = mid - 1;
        }
        cur = first_row = lo;
        end = s_ptr[cur + 1];
      }
      for (int q = q0; q < q1; q += U) {
        Pack<SrcT, V> val[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int src = q + u < q1 ? s_idx[q + u] : -1;
          val[u] = (src >= 0 && lane_on) ? ld<SrcT, V>(src_rows + (int64_t)src * KP + gl * V)
                                         : zero_pack<SrcT, V>();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int qq = q + u;
          if (qq < q1) {
            if (qq >= end) {  // seg < 0 only: row `cur` ends inside the share
              if (s_ptr[cur] >= q0) row_epilogue<T, KP, KE, MODE>(io, r0 + cur, gl, acc, mask, rsum);
              else {
#pragma unroll
                for (int v = 0; v < V; ++v) s_part[(gid * 2) * KE + gl * V + v] = acc[v];
              }
#pragma unroll
              for (int v = 0; v < V; ++v) acc[v] = 0.0;
              do {
                ++cur;
              } while (s_ptr[cur + 1] <= qq);
              end = s_ptr[cur + 1];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] += to_d(val[u].v[v]);
          }
        }
      }
      // the share's last row: finished here when it lies inside the share
      if (seg < 0 && s_ptr[cur] >= q0 && s_ptr[cur + 1] <= q1) {
        row_epilogue<T, KP, KE, MODE>(io, r0 + cur, gl, acc, mask, rsum);
      } else {
        const int slot = (seg >= 0 || cur == first_row) ? 0 : 1;
#pragma unroll
        for (int v = 0; v < V; ++v) s_part[(gid * 2 + slot) * KE + gl * V + v] = acc[v];
      }
    }
    __syncthreads();
    if (seg >= 0) {
      // a segment of a heavy row: the shares' sums in order
      for (int c = tid; c < KE; c += kBBlock) {
        double s = 0.0;
        for (int g2 = 0; g2 < NG; ++g2) {
          const int qa = (int)((int64_t)nl * g2 / NG), qb = (int)((int64_t)nl * (g2 + 1) / NG);
          if (qa < qb) s += s_part[(g2 * 2) * KE + c];
        }
        segv[(int64_t)seg * KP + c] = s;
      }
    } else {
      // a row cut by share boundaries is finished by the share it starts in
      if (q0 < q1 && s_ptr[cur] >= q0 && s_ptr[cur + 1] > q1) {
        double tot[V];
        const int slot = cur == first_row ? 0 : 1;
#pragma unroll
        for (int v = 0; v < V; ++v) tot[v] = s_part[(gid * 2 + slot) * KE + gl * V + v];
        for (int g2 = gid + 1; g2 < NG; ++g2) {
          const int qa = (int)((int64_t)nl * g2 / NG), qb = (int)((int64_t)nl * (g2 + 1) / NG);
          if (qa >= s_ptr[cur + 1]) break;
          if (qa < qb) {
#pragma unroll
            for (int v = 0; v < V; ++v) tot[v] += s_part[(g2 * 2) * KE + gl * V + v];
          }
        }
        row_epilogue<T, KP, KE, MODE>(io, r0 + cur, gl, tot, mask, rsum);
      }
      // rows without in-links
      double zero[V];
#pragma unroll
      for (int v = 0; v < V; ++v) zero[v] = 0.0;
      for (int r = gid; r < nrows; r += NG)
        if (s_ptr[r] == s_ptr[r + 1]) row_epilogue<T, KP, KE, MODE>(io, r0 + r, gl, zero, mask, rsum);
    }
    __syncthreads();
  }
  col_sum_store<Ly, KE>(rsum, s_rec, rec + (int64_t)blockIdx.x * KP);
}

// Heavy rows: F += (MODE 1: F = R with) the sum of the row's segment sums,
// in segment order. Block b handles heavy rows b*HPB + hs (strided); its
// per-column sums of |F| go to rec[rec_base + b].
template <typename T, int KP, int KE, int MODE>
__global__ __launch_bounds__(kBBlock) void k_bheavy(
    PullIo<T, KP, MODE> io, const int32_t* __restrict__ heavy_row,
    const int64_t* __restrict__ heavy_seg, int64_t n_heavy, const double* __restrict__ segv,
    double* __restrict__ rec, int rec_base, const BCtl* __restrict__ bctl) {
  constexpr int HPB = kBBlock / KE;
  __shared__ double s_sum[kBBlock];
  const int c = threadIdx.x % KE, hs = threadIdx.x / KE;
  const int want = MODE == 0 ? kBRun : kBInner;
  const bool m = bctl[c].state == want;
  double rsum = 0.0;
  for (int64_t h = (int64_t)blockIdx.x * HPB + hs; h < n_heavy; h += (int64_t)gridDim.x * HPB) {
    const int64_t row = heavy_row[h];
    const double acc = ordered_sum(segv + c, heavy_seg[h], heavy_seg[h + 1], KP);
    const int64_t qi = row * KP + c;
    if (MODE == 0) {
      double f = to_d(io.F[qi]);
      if (acc != 0.0) {
        const T nv = (T)(f + acc);
        io.F[qi] = nv;
        f = to_d(nv);
      }
      rsum += fabs(f);
    } else if (m) {
      const bool self = (io.info[row] & kLoopBit) != 0;
      const double r = io.Bd[qi] - io.X[qi] + (self ? io.Y[qi] : 0.0) + acc;
      io.F[qi] = (T)r;
      rsum += fabs(r);
    }
  }
  s_sum[threadIdx.x] = rsum;
  __syncthreads();
  if (threadIdx.x < KE) {
    double t = 0.0;
    for (int q = 0; q < HPB; ++q) t += s_sum[q * KE + threadIdx.x];
    rec[(int64_t)(rec_base + blockIdx.x) * KP + threadIdx.x] = t;
  }
}

// ---- residual pass: fold H into X and the senders' rows ------------------

template <typename T, int KP, int KE>
__global__ __launch_bounds__(kBBlock) void k_brefine_y(double* __restrict__ X64,
                                                       T* __restrict__ H, double* __restrict__ Y,
                                                       const uint32_t* __restrict__ info,
                                                       int64_t n, double d,
                                                       const BCtl* __restrict__ bctl) {
  using Ly = Lay<KE>;
  constexpr int V = Ly::V;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / Ly::G, gl = lane % Ly::G;
  bool mask[V];
  bool anym = false;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    mask[v] = bctl[gl * V + v].state == kBInner;
    anym |= mask[v];
  }
  if (!anym) return;  // per lane: the lane's columns need nothing
  const int64_t stride = (int64_t)gridDim.x * Ly::NG;
  for (int64_t i = (int64_t)blockIdx.x * Ly::NG + wave * Ly::P + grp; i < n; i += stride) {
    const int out = (int)(info[i] & kOutMask);
    const int64_t q = i * KP + gl * V;
    Pack<double, V> x = ld<double, V>(X64 + q);
    Pack<T, V> h = ld<T, V>(H + q);
    Pack<double, V> y = ld<double, V>(Y + q);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (mask[v]) {
        x.v[v] += to_d(h.v[v]);
        h.v[v] = (T)0;
        y.v[v] = out > 0 ? d * x.v[v] / (double)out : 0.0;
      }
    }
    st<double, V>(X64 + q, x);
    st<T, V>(H + q, h);
    st<double, V>(Y + q, y);
  }
}

// ---- per-column reduction and stop test -----------------------------------

// Block c: column c. FIRST (after a load or a residual pass): columns in
// state `want` (kBFresh or kBInner) take r = the records' sum as the start
// of a pass (converged if r <= tol). CYCLE: running columns fold the
// cycle's records and selection counters.
// CYCLE also completes the column's heavy rows (F += the segment sums, in
// segment order) and adds their |F| to the sum.
template <typename T, int KP, bool FIRST>
__global__ __launch_bounds__(kBBlock) void k_breduce(
    BCtl* __restrict__ bctl, const double* __restrict__ rec, int nrec,
    const unsigned long long* __restrict__ rec_ops, const unsigned int* __restrict__ rec_sel,
    const double* __restrict__ rec_e, int nsel, int method, int max_cycles, double tol_rel,
    int want, T* __restrict__ F, const int32_t* __restrict__ heavy_row,
    const int64_t* __restrict__ heavy_seg, int64_t n_heavy, const double* __restrict__ segv) {
  __shared__ double s_d[kBBlock / 64];
  __shared__ unsigned long long s_u[kBBlock / 64];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int state = bctl[c].state;
  const bool mine = FIRST ? state == want : state == kBRun;
  if (!mine) return;
  double r = 0.0;
  for (int q0 = tid; q0 < nrec; q0 += 8 * kBBlock) {  // 8 loads in flight, same order
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * kBBlock;
      t[u] = q < nrec ? rec[(int64_t)q * KP + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) r += t[u];
  }
  if (!FIRST) {
    for (int64_t h = tid; h < n_heavy; h += kBBlock) {
      const int64_t qi = (int64_t)heavy_row[h] * KP + c;
      const double acc = ordered_sum(segv + c, heavy_seg[h], heavy_seg[h + 1], KP);
      double f = to_d(F[qi]);
      if (acc != 0.0) {
        const T nv = (T)(f + acc);
        F[qi] = nv;
        f = to_d(nv);
      }
      r += fabs(f);
    }
  }
  r = block_sum_all(r, s_d);
  unsigned long long ops = 0, sel = 0;
  double e = 0.0;
  if (!FIRST) {
    for (int q = tid; q < nsel; q += kBBlock) {
      ops += rec_ops[(int64_t)q * (KP + 1) + c];
      sel += rec_sel[(int64_t)q * (KP + 1) + c];
      e += rec_e[(int64_t)q * KP + c];
    }
    ops = block_sum_all(ops, s_u);
    sel = block_sum_all(sel, s_u);
    e = block_sum_all(e, s_d);
  }
  if (tid != 0) return;
  BCtl b = bctl[c];
  if (FIRST) {
    if (state == kBInner) b.refinements += 1;
    b.r = r;
    b.r_start = r;
    b.pass_cycles = 0;
    b.cyc_mode = method == DI_CYC ? 1 : 0;
    if (!isfinite(r)) {
      b.state = kBNonFinite;
      b.final_r = r;
    } else if (r <= b.tol) {
      b.state = kBConv;
      b.final_r = r;
    } else if (b.cycles >= max_cycles || b.refinements >= kBMaxRefinements) {
      b.state = kBMaxCyc;
      b.final_r = r;
    } else {
      b.state = kBRun;
    }
  } else {
    b.cycles += 1;
    b.pass_cycles += 1;
    b.edges += ops;
    b.sel_total += sel;
    b.e += e;
    const bool empty = sel == 0 && r > 0.0;
    b.cyc_mode = (method == DI_CYC || empty) ? 1 : 0;
    if (method != DI_CYC && empty) b.fallback += 1;
    b.r = r;
    if (!isfinite(r)) {
      b.state = kBNonFinite;
      b.final_r = r;
    } else if (tol_rel >= 0.0) {
      // refined solve: the FP32 pass ends; convergence is decided on the
      // FP64 residual of the next pass
      if (r <= fmax(kInnerStop * b.tol, tol_rel * b.r_start)) {
        b.state = kBInner;
        b.final_r = r;
      } else if (b.cycles >= max_cycles) {
        b.state = kBInner;  // folded into X by a last residual pass
        b.final_r = r;
      }
    } else if (r <= b.tol) {
      b.state = kBConv;
      b.final_r = r;
    } else if (b.cycles >= max_cycles) {
      b.state = kBMaxCyc;
      b.final_r = r;
    }
  }
  bctl[c] = b;
}

// ---- serving: columns started and read out one by one -------------------

// Clears the columns with flag[c] != 0 in every row: F = B, Bd = B (B = 0,
// or b_uni[c] for a column whose right-hand side is uniform), H = 0,
// X64 = 0.
template <typename T, int KP>
__global__ __launch_bounds__(kBBlock) void k_bcol_clear(T* __restrict__ F, T* __restrict__ H,
                                                        double* __restrict__ Bd,
                                                        double* __restrict__ X64, int64_t n,
                                                        const int* __restrict__ flag,
                                                        const double* __restrict__ b_uni) {
  using Ly = Lay<KP>;
  constexpr int V = Ly::V;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / Ly::G, gl = lane % Ly::G;
  bool m[V];
  double bu[V];
  bool any = false;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    m[v] = flag[gl * V + v] != 0;
    bu[v] = m[v] ? b_uni[gl * V + v] : 0.0;
    any |= m[v];
  }
  if (!any) return;
  const int64_t stride = (int64_t)gridDim.x * Ly::NG;
  for (int64_t i = (int64_t)blockIdx.x * Ly::NG + wave * Ly::P + grp; i < n; i += stride) {
    const int64_t q = i * KP + gl * V;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (m[v]) {
        F[q + v] = (T)bu[v];
        H[q + v] = (T)0;
        if (Bd) Bd[q + v] = bu[v];
        if (X64) X64[q + v] = 0.0;
      }
    }
  }
}

// x[idx[q]] = v for q < count (a personalized right-hand side for a solve
// that runs alone).
__global__ __launch_bounds__(256) void k_scatter_value(double* __restrict__ x,
                                                       const int32_t* __restrict__ idx,
                                                       int64_t count, double v) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * blockDim.x)
    x[idx[q]] = v;
}

// Block j starts column col[j]: B = val[j] at its seeds
// seeds[off[j] .. off[j+1]) (or the uniform value written by k_bcol_clear
// when the list is empty), r = sum |F| in FP64, and a fresh control block
// (running, or converged when r <= tol[j]).
template <typename T, int KP>
__global__ __launch_bounds__(kBBlock) void k_bcol_seed(
    T* __restrict__ F, double* __restrict__ Bd, BCtl* __restrict__ bctl, int64_t n,
    const int* __restrict__ col, const int64_t* __restrict__ off, const int32_t* __restrict__ seeds,
    const double* __restrict__ val, const double* __restrict__ tol, int method) {
  __shared__ double lds[kBBlock / 64];
  const int j = blockIdx.x, c = col[j];
  const int64_t s0 = off[j], s1 = off[j + 1];
  double r = 0.0;
  if (s1 > s0) {
    const T v = (T)val[j];
    for (int64_t q = s0 + threadIdx.x; q < s1; q += kBBlock) {
      const int64_t i = seeds[q];
      F[i * KP + c] = v;
      if (Bd) Bd[i * KP + c] = val[j];
      r += fabs(to_d(v));
    }
  }
  r = block_sum_all(r, lds);
  if (threadIdx.x == 0) {
    if (s1 == s0) r = (double)n * fabs(to_d((T)val[j]));
    BCtl b;
    b.r = r;
    b.r_start = r;
    b.final_r = r;
    b.tol = tol[j];
    b.e = 0.0;
    b.edges = 0;
    b.sel_total = 0;
    b.cycles = 0;
    b.pass_cycles = 0;
    b.refinements = 0;
    b.fallback = 0;
    b.cyc_mode = method == DI_CYC ? 1 : 0;
    b.state = !isfinite(r) ? kBNonFinite : (r <= b.tol ? kBConv : kBRun);
    bctl[c] = b;
  }
}

// X_out[i] = H[i][c] (+ X64[i][c]): one column read out.
template <typename T, int KP>
__global__ void k_bcol_out(const T* __restrict__ H, const double* __restrict__ X64, int c,
                           int64_t n, double* __restrict__ X_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double x = to_d(H[i * KP + c]);
    if (X64) x += X64[i * KP + c];
    X_out[i] = x;
  }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T, int KP>
PullIo<T, KP, 0> fluid_io(const BatchArgs& a, BatchWs* ws) {
  PullIo<T, KP, 0> io;
  io.F = (T*)ws->F;
  io.sent = (const T*)ws->sent;
  io.front_bits = ws->front_bits;
  io.Y = nullptr;
  io.X = nullptr;
  io.Bd = nullptr;
  io.info = a.g->info;
  return io;
}

template <typename T, int KP>
PullIo<T, KP, 1> residual_io(const BatchArgs& a, BatchWs* ws) {
  PullIo<T, KP, 1> io;
  io.F = (T*)ws->F;
  io.sent = nullptr;
  io.front_bits = nullptr;
  io.Y = ws->Y64;
  io.X = ws->X64;
  io.Bd = ws->Bd;
  io.info = a.g->info;
  return io;
}

template <typename T, int KP>
hipError_t bload_t(const BatchArgs& a, BatchWs* ws, const double* B_in, int k, double bu) {
  const dim3 grid((unsigned)ceil_div(a.g->n, 32), (unsigned)ceil_div(KP, 64));
  hipLaunchKernelGGL((k_bload<T, KP>), grid, dim3(kBBlock), 0, a.stream, B_in, k, a.g->n, bu,
                     (T*)ws->F, (T*)ws->H, ws->Bd, ws->X64);
  return hipGetLastError();
}

template <typename T, int KP>
hipError_t brecords_t(const BatchArgs& a, BatchWs* ws) {
  hipLaunchKernelGGL((k_brecords<T, KP>), dim3(brecords_grid(a.g->n)), dim3(kBBlock), 0, a.stream,
                     (const T*)ws->F, a.g->n, ws->rec);
  return hipGetLastError();
}

template <typename T, int KP, int KE>
hipError_t bcycle_t(const BatchArgs& a, BatchWs* ws, hipEvent_t ev0, hipEvent_t ev1) {
  const di_graph* g = a.g;
  const int sgrid = bselect_grid(g->n);
  hipLaunchKernelGGL((k_bselect<T, KP, KE>), dim3(sgrid), dim3(kBBlock), 0, a.stream, (T*)ws->F,
                     (T*)ws->H, (T*)ws->sent, ws->front_bits, g->info, g->n, g->L, a.d,
                     (const BCtl*)ws->bctl, ws->rec_ops, ws->rec_sel, ws->rec_e);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (ev0 && (err = hipEventRecord(ev0, a.stream)) != hipSuccess) return err;
  const int pgrid = pull_grid(g);
  hipLaunchKernelGGL((k_bpull<T, KP, KE, 0>), dim3(pgrid), dim3(kBBlock), 0, a.stream,
                     fluid_io<T, KP>(a, ws), g->csc_ptr, g->csc_idx, g->it_r0, g->it_r1, g->it_l0,
                     g->it_l1, g->it_seg, g->n_items, ws->segv, ws->rec, ws->bctl,
                     (const unsigned long long*)ws->rec_ops, (const unsigned int*)ws->rec_sel,
                     sgrid);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (ev1 && (err = hipEventRecord(ev1, a.stream)) != hipSuccess) return err;
  hipLaunchKernelGGL((k_breduce<T, KP, false>), dim3(KE), dim3(kBBlock), 0, a.stream, ws->bctl,
                     (const double*)ws->rec, pgrid, (const unsigned long long*)ws->rec_ops,
                     (const unsigned int*)ws->rec_sel, (const double*)ws->rec_e, sgrid, a.method,
                     a.max_cycles, a.tol_rel, (int)kBRun, (T*)ws->F, g->heavy_row, g->heavy_seg,
                     g->n_heavy, (const double*)ws->segv);
  return hipGetLastError();
}

template <typename T, int KP>
hipError_t bfirst_t(const BatchArgs& a, BatchWs* ws, int nrec, int want) {
  hipLaunchKernelGGL((k_breduce<T, KP, true>), dim3(a.ke), dim3(kBBlock), 0, a.stream, ws->bctl,
                     (const double*)ws->rec, nrec, (const unsigned long long*)nullptr,
                     (const unsigned int*)nullptr, (const double*)nullptr, 0, a.method,
                     a.max_cycles, a.tol_rel, want, (T*)nullptr, (const int32_t*)nullptr,
                     (const int64_t*)nullptr, (int64_t)0, (const double*)nullptr);
  return hipGetLastError();
}

template <typename T, int KP, int KE>
hipError_t brefine_t(const BatchArgs& a, BatchWs* ws, int* nrec) {
  const di_graph* g = a.g;
  using Ly = Lay<KE>;
  const int ygrid = (int)std::min<int64_t>(ceil_div(g->n, Ly::NG), 8192);
  hipLaunchKernelGGL((k_brefine_y<T, KP, KE>), dim3(ygrid), dim3(kBBlock), 0, a.stream, ws->X64,
                     (T*)ws->H, ws->Y64, g->info, g->n, a.d, (const BCtl*)ws->bctl);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int pgrid = pull_grid(g);
  hipLaunchKernelGGL((k_bpull<T, KP, KE, 1>), dim3(pgrid), dim3(kBBlock), 0, a.stream,
                     residual_io<T, KP>(a, ws), g->csc_ptr, g->csc_idx, g->it_r0, g->it_r1,
                     g->it_l0, g->it_l1, g->it_seg, g->n_items, ws->segv, ws->rec, ws->bctl,
                     (const unsigned long long*)nullptr, (const unsigned int*)nullptr, 0);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const int hgrid = bheavy_grid(g);
  if (hgrid > 0) {
    hipLaunchKernelGGL((k_bheavy<T, KP, KE, 1>), dim3(hgrid), dim3(kBBlock), 0, a.stream,
                       residual_io<T, KP>(a, ws), g->heavy_row, g->heavy_seg, g->n_heavy,
                       (const double*)ws->segv, ws->rec, pgrid, (const BCtl*)ws->bctl);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  *nrec = pgrid + hgrid;
  return hipSuccess;
}

template <typename T, int KP>
hipError_t bstore_t(const BatchArgs& a, BatchWs* ws, double* X_out, int k, bool refined) {
  const dim3 grid((unsigned)ceil_div(a.g->n, 32), (unsigned)ceil_div(KP, 64));
  hipLaunchKernelGGL((k_bstore<T, KP>), grid, dim3(kBBlock), 0, a.stream, (const T*)ws->H,
                     refined ? (const double*)ws->X64 : (const double*)nullptr, X_out, k, a.g->n);
  return hipGetLastError();
}

template <typename T, int KP>
hipError_t bcol_init_t(const BatchArgs& a, BatchWs* ws, const ColInit& ci) {
  using Ly = Lay<KP>;
  const int grid = (int)std::min<int64_t>(ceil_div(a.g->n, Ly::NG), 4096);
  hipLaunchKernelGGL((k_bcol_clear<T, KP>), dim3(grid), dim3(kBBlock), 0, a.stream, (T*)ws->F,
                     (T*)ws->H, ws->Bd, ws->X64, a.g->n, ci.flag, ci.b_uni);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_bcol_seed<T, KP>), dim3(ci.ncols), dim3(kBBlock), 0, a.stream, (T*)ws->F,
                     ws->Bd, ws->bctl, a.g->n, ci.col, ci.off, ci.seeds, ci.val, ci.tol, a.method);
  return hipGetLastError();
}

template <typename T, int KP>
hipError_t bcol_out_t(const BatchArgs& a, BatchWs* ws, int c, bool refined, double* X_out) {
  hipLaunchKernelGGL((k_bcol_out<T, KP>), dim3((unsigned)std::min<int64_t>(ceil_div(a.g->n, 256), 4096)),
                     dim3(256), 0, a.stream, (const T*)ws->H,
                     refined ? (const double*)ws->X64 : (const double*)nullptr, c, a.g->n, X_out);
  return hipGetLastError();
}

// Calls f.template operator()<T, KP, KE>() for a working width KE <= KP.
template <typename T, int KP, typename Fn>
hipError_t dispatch_ke(int ke, Fn&& f) {
  switch (ke) {
    case 8:
      if constexpr (KP >= 8) return f.template operator()<T, KP, 8>();
      break;
    case 16:
      if constexpr (KP >= 16) return f.template operator()<T, KP, 16>();
      break;
    case 32:
      if constexpr (KP >= 32) return f.template operator()<T, KP, 32>();
      break;
    case 64:
      if constexpr (KP >= 64) return f.template operator()<T, KP, 64>();
      break;
    case 128:
      if constexpr (KP >= 128) return f.template operator()<T, KP, 128>();
      break;
    case 256:
      if constexpr (KP >= 256) return f.template operator()<T, KP, 256>();
      break;
  }
  return hipErrorInvalidValue;
}

// Calls f.template operator()<T, KP>() for the batch's shape.
template <typename Fn>
hipError_t dispatch(const BatchArgs& a, Fn&& f) {
  if (a.prec == kF64) {
    switch (a.kp) {
      case 8: return f.template operator()<double, 8>();
      case 16: return f.template operator()<double, 16>();
      case 32: return f.template operator()<double, 32>();
      case 64: return f.template operator()<double, 64>();
      case 128: return f.template operator()<double, 128>();
      case 256: return f.template operator()<double, 256>();
    }
  } else {
    switch (a.kp) {
      case 8: return f.template operator()<float, 8>();
      case 16: return f.template operator()<float, 16>();
      case 32: return f.template operator()<float, 32>();
      case 64: return f.template operator()<float, 64>();
      case 128: return f.template operator()<float, 128>();
      case 256: return f.template operator()<float, 256>();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

int bselect_grid(int64_t n) {
  const int64_t words = ceil_div(n, 64);
  const int64_t g = ceil_div(words, kBBlock / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kBSelectMaxGrid));
}

int bheavy_grid(const di_graph* g) {
  return (int)std::min<int64_t>(g->n_heavy, kBHeavyMaxGrid);
}

int brecords_grid(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 64), 1024));
}

hipError_t launch_bload(const BatchArgs& a, BatchWs* ws, const double* B_in, int k,
                        double b_uniform) {
  return dispatch(a, [&]<typename T, int KP>() { return bload_t<T, KP>(a, ws, B_in, k, b_uniform); });
}

hipError_t launch_brecords(const BatchArgs& a, BatchWs* ws) {
  return dispatch(a, [&]<typename T, int KP>() { return brecords_t<T, KP>(a, ws); });
}

hipError_t launch_bcycle(const BatchArgs& a, BatchWs* ws, hipEvent_t ev0, hipEvent_t ev1) {
  return dispatch(a, [&]<typename T, int KP>() {
    return dispatch_ke<T, KP>(a.ke, [&]<typename T2, int KP2, int KE>() {
      return bcycle_t<T2, KP2, KE>(a, ws, ev0, ev1);
    });
  });
}

hipError_t launch_bfirst(const BatchArgs& a, BatchWs* ws, int nrec, int want) {
  return dispatch(a, [&]<typename T, int KP>() { return bfirst_t<T, KP>(a, ws, nrec, want); });
}

hipError_t launch_brefine(const BatchArgs& a, BatchWs* ws, int* nrec) {
  return dispatch(a, [&]<typename T, int KP>() {
    return dispatch_ke<T, KP>(a.ke, [&]<typename T2, int KP2, int KE>() {
      return brefine_t<T2, KP2, KE>(a, ws, nrec);
    });
  });
}

hipError_t launch_bcol_init(const BatchArgs& a, BatchWs* ws, const ColInit& ci) {
  return dispatch(a, [&]<typename T, int KP>() { return bcol_init_t<T, KP>(a, ws, ci); });
}

hipError_t launch_bcol_out(const BatchArgs& a, BatchWs* ws, int c, bool refined, double* X_out) {
  return dispatch(a, [&]<typename T, int KP>() { return bcol_out_t<T, KP>(a, ws, c, refined, X_out); });
}

hipError_t launch_bstore(const BatchArgs& a, BatchWs* ws, double* X_out, int k, bool refined) {
  return dispatch(a,
                  [&]<typename T, int KP>() { return bstore_t<T, KP>(a, ws, X_out, k, refined); });
}

hipError_t launch_scatter_value(hipStream_t stream, double* x, const int32_t* idx, int64_t count,
                                double v) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_value, dim3((unsigned)std::min<int64_t>(ceil_div(count, 256), 1024)),
                     dim3(256), 0, stream, x, idx, count, v);
  return hipGetLastError();
}

}  // namespace di
