// Window-push D-iteration cycle on gfx950: one launch per cycle, whose work
// follows the diffused links.
//
// A cycle of DI-SOP (Sections 2.3 and 2.5.5) selects, against r = sum_i |F_i|
// of the fluid at the cycle's start, every node with |F_i| >= (r/L) out_i,
// claims it (Section 2.5.4: H_i += transit, the fluid leaves F_i, a dangling
// node absorbs it) and pushes transit * d / out_i along each out-link j != i.
// Here one block owns a tile of consecutive node ids and does all
// of that for its tile in one launch:
//   - the fluid of node i at the cycle's start is F_i (what the node kept,
//     plus what its own tile pushed to it) + the far accumulator A_i (far
//     links, device-scope atomics) + what the neighbouring tiles left in
//     their halos (near links across a tile boundary) + for a hub row what
//     the blocks of the previous launch sent it (far links into the hubs);
//   - near links (|i - j| <= kWinHalo) are added into the tile's LDS window
//     [a - kWinHalo, a + tile + kWinHalo) with LDS atomics; the window's
//     middle goes straight to F, its two halos to the neighbours' next cycle;
//   - far links into one of the graph's hub rows (the nodes with the most
//     far in-links) are added into per-block LDS accumulators, whose nonzero
//     values each block writes once per launch into a table by hub and
//     block; the hub's tile sums its row there at the next cycle's start and
//     clears it. Other far links are device-scope atomics into the far
//     accumulator of the next cycle.
// So the links a cycle reads are the links it moves (plus each sender's row
// offset), and every state array has two copies by cycle parity: cycle c
// reads copy c & 1 and pushes into copy (c + 1) & 1, so no block reads what
// another block of the same launch writes.
//
// r of the next cycle: for a fluid that stays >= 0 (B >= 0), sum_i F_i after
// the cycle equals what the nodes kept plus what the senders pushed, which
// every block sums for its own nodes and senders; so the next launch folds
// the per-block records and needs no pass over F. A signed fluid (an FP64
// residual as right-hand side) runs a fold pass after every cycle instead,
// which gathers each node's fluid into F and sums |F| exactly. The fold also
// runs once after the stop, to leave the whole fluid in F and measure the
// final residual exactly.
//
// The summation order of the LDS and device atomics varies from run to run,
// so results agree with the pull direction to rounding, not bit for bit.

#include "di_device.h"
#include <hip/hip_ext.h>

namespace di {
namespace {

using namespace dev;

constexpr int W = kWinHalo;
constexpr int KMAX = kWinHubMax;
constexpr int kHubBatch = 8;  // hub-partial loads in flight per lane
constexpr int kUnroll = 4;  // links in flight per thread in the push

__device__ inline void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_add(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Graph and fluid arrays of one launch (state arrays already offset to the
// launch's parity).
template <typename T>
struct WinState {
  const uint32_t* wp_info;  // node words with the ranked-hub bit
  const int64_t* row_ptr;
  const int32_t* wp_col;
  const int32_t* hub_rank_node;  // node of each hub rank
  const int32_t* hub_id_node;    // ranked hubs by ascending id ...
  const int32_t* hub_id_rank;    // ... and their ranks
  const int32_t* hub_tile;       // each tile's range of hub_id_*
  int64_t n, L, ntiles;
  int K;                         // active hubs: ranks below K
  T* F;
  T* H;
  T* A_cur;           // far accumulator read (and cleared) this cycle
  T* A_next;          // far accumulator this cycle pushes into
  const T* halo_cur;  // per tile: left halo, then right halo (W values each)
  T* halo_next;
  // hub partials, by hub rank then block ([r][b], row stride hub_gs): what
  // block b of the last launch sent hub r (read and cleared by the hub's
  // tile), and those this launch writes (its nonzero ones only: every entry
  // is zero between uses)
  T* hub_cur;
  T* hub_next;
  int64_t hub_gs;
  int rounds;  // diffusion rounds per cycle over each tile (DI-SOP), 1 or 2
  Ctl* ctl_host;  // pinned host copies of the control block (or null)
};

// The tile's ranked hubs: their ids ascending (s_hnode) and, when `add`,
// what the last launch's G blocks sent the active ones (rank below K) in
// their LDS accumulators (s_hadd; 0 for the others, whose far links went to
// the far accumulator), each summed over the blocks in one order; with
// `clear` the nonzero partials read are cleared. Returns the number of
// ranked hubs in the tile.
template <typename T, int BLOCK>
__device__ inline int tile_hubs(const WinState<T>& S, int64_t tile, int G, bool add, bool clear,
                                int32_t* s_hnode, T* s_hadd) {
  constexpr int NW = BLOCK / 64;
  const int h0 = S.hub_tile[tile], h1 = S.hub_tile[tile + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < h1 - h0; k += NW) {
    const int r = S.hub_id_rank[h0 + k];
    const int node = S.hub_id_node[h0 + k];
    double acc = 0.0;
    if (add && r < S.K) {
      // kHubBatch loads of the row in flight per lane, then their sum (in
      // ascending block order per lane)
      T* row = S.hub_cur + (int64_t)r * S.hub_gs;
      for (int b0 = 0; b0 < G; b0 += 64 * kHubBatch) {
        T v[kHubBatch];
#pragma unroll
        for (int j = 0; j < kHubBatch; ++j) {
          const int b = b0 + 64 * j + lane;
          v[j] = b < G ? row[b] : (T)0;
        }
#pragma unroll
        for (int j = 0; j < kHubBatch; ++j)
          if (v[j] != (T)0) {
            acc += to_d(v[j]);
            if (clear) row[b0 + 64 * j + lane] = (T)0;
          }
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      s_hnode[k] = node;
      s_hadd[k] = (T)acc;
    }
  }
  return h1 - h0;
}

// Puts back the hub sums tile_hubs read (and cleared) for a launch that
// then found the solve stopped: each active hub's sum into its first
// partial, which the final fold then adds as the sum itself.
template <typename T, int BLOCK>
__device__ inline void restore_tile_hubs(const WinState<T>& S, int64_t tile, const T* s_hadd) {
  const int h0 = S.hub_tile[tile], h1 = S.hub_tile[tile + 1];
  for (int k = threadIdx.x; k < h1 - h0; k += BLOCK) {
    const int r = S.hub_id_rank[h0 + k];
    if (r < S.K) S.hub_cur[(int64_t)r * S.hub_gs] = s_hadd[k];
  }
}

// Fluid of node i (position li in its tile) at the cycle's start: kept +
// far accumulator + halos + hub partials, added in this order. The far
// accumulator is cleared as it is read.
template <typename T, int TILE>
__device__ inline T start_value(const WinState<T>& S, T f, int64_t i, int64_t tile, int li,
                                uint32_t wn, const int32_t* s_hnode, const T* s_hadd, int nh) {
  const T av = S.A_cur[i];
  if (av != (T)0) {
    f = f + av;
    S.A_cur[i] = (T)0;
  }
  if (li < W && tile > 0) f = f + S.halo_cur[(tile - 1) * 2 * W + W + li];
  if (li >= TILE - W && tile + 1 < S.ntiles)
    f = f + S.halo_cur[(tile + 1) * 2 * W + (li - (TILE - W))];
  if (wn & kHubBit) {
    int lo = 0, hi = nh - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_hnode[mid] < i) lo = mid + 1;
      else hi = mid;
    }
    f = f + s_hadd[lo];
  }
  return f;
}

// One link i -> code of a push: links into an active hub (code = -1 - r,
// r < K) into the block's hub accumulators, near links (|code - i| <= W)
// into the window, other far links into the next far accumulator.
template <typename T>
__device__ inline void push_link(const WinState<T>& S, int32_t code, int64_t i, int64_t win0, T s,
                                 T* s_win, T* s_hub) {
  if (code < 0) {
    const int r = -1 - code;
    if (r < S.K) lds_add(&s_hub[r], s);
    else atomic_add(&S.A_next[S.hub_rank_node[r]], s);
  } else if (code - i <= W && i - code <= W) {
    lds_add(&s_win[code - win0], s);
  } else {
    atomic_add(&S.A_next[code], s);
  }
}

// Four consecutive values of a node array, as one vector access when all
// four nodes exist (i0 is a multiple of 4 and every node array starts on a
// 256-byte boundary).
template <typename V>
struct alignas(4 * sizeof(V)) Quad {
  V v[4];
};
template <typename V>
__device__ inline void load4(const V* p, int64_t i0, int64_t n, V (&out)[4]) {
  if (i0 + 4 <= n) {
    const Quad<V> q = *reinterpret_cast<const Quad<V>*>(p + i0);
#pragma unroll
    for (int m = 0; m < 4; ++m) out[m] = q.v[m];
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) out[m] = i0 + m < n ? p[i0 + m] : (V)0;
  }
}
template <typename V>
__device__ inline void store4(V* p, int64_t i0, int64_t n, const V (&val)[4]) {
  if (i0 + 4 <= n) {
    Quad<V> q;
#pragma unroll
    for (int m = 0; m < 4; ++m) q.v[m] = val[m];
    *reinterpret_cast<Quad<V>*>(p + i0) = q;
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (i0 + m < n) p[i0 + m] = val[m];
  }
}

// Inclusive sums over the lanes of a wave (lane l: lanes 0..l), two at once.
__device__ inline void wave_scan2(int& x, int& y) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(x, o, 64), v = __shfl_up(y, o, 64);
    if (lane >= o) {
      x += u;
      y += v;
    }
  }
}

// One cycle: the stop test on the last cycle's records, then select, claim
// and push every tile of the block (grid-stride). Thread tid holds the four
// consecutive nodes a + 4 tid .. a + 4 tid + 3 of tile a. The first tile's
// loads that the selection needs (and its hub rows' sums) are issued before
// the stop test, which they do not depend on; nothing is written before
// it. first: the records
// are the start records and F is the whole fluid; folded: F is the whole
// fluid (a fold pass ran after the last cycle).
// Waves per SIMD: as many as the block's LDS lets a compute unit hold, at
// most four (at most 128 VGPRs): two 512-thread blocks or one 1024-thread
// block; three 256-thread blocks in FP64 (up to 168 VGPRs), four in FP32.
template <typename T, int BLOCK>
constexpr int win_waves() {
  return (sizeof(T) == 8 && BLOCK == 256) ? 3 : 4;
}
template <typename T, int BLOCK, int ROUNDS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(win_waves<T, BLOCK>())))
void k_wcycle(
    WinState<T> S, const Part* __restrict__ rec_in, int nrec_in, Part* __restrict__ rec_out,
    Ctl* __restrict__ ctl, int parity, int first, int folded, double d, double tol,
    double tol_in, double tol_rel, int method, int stop, int max_cycles,
    di_cycle_rec* __restrict__ trace, int trace_cap) {
  constexpr int TILE = 4 * BLOCK;  // four nodes per thread
  constexpr int WIN = TILE + 2 * W;
  static_assert(W <= TILE, "a near link lands in the tile or a neighbour");
  static_assert(W % 4 == 0, "halo in whole quads");
  constexpr int NW = BLOCK / 64;
  __shared__ T s_win[WIN];
  __shared__ T s_hub[KMAX];
  __shared__ T s_hadd[KMAX];
  __shared__ int32_t s_hnode[KMAX];
  __shared__ Part s_part[NW];
  // per node of the tile (node order): position of its first moved link
  // among the tile's moved links, offset of its first link from the tile's
  // first link, and the amount it sends along each link
  __shared__ int32_t s_off[TILE];
  __shared__ int32_t s_rel[TILE];
  __shared__ T s_snd[TILE];
  __shared__ int s_wtot[2 * NW];
  __shared__ double s_r;
  __shared__ int s_done, s_cyc;
  __shared__ Ctl s_ctl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = gridDim.x;
  const int nhub = S.K;
  const bool add = !first && !folded;
  const int l0 = 4 * tid;  // the thread's first node in the tile

  // a tile's loads: kept fluid, far accumulator, node words, the halo
  // values of the tile's first and last W nodes, the tile's first link (the
  // history hv is loaded later, at the top of the tile's work)
  T raw[4], av[4], hv[4], hl[4], hr[4];
  uint32_t w[4];
  int64_t ebase = 0;
  int nh = 0;
  auto load_tile = [&](int64_t tile) {
    const int64_t i0 = tile * TILE + l0;
    load4(S.F, i0, S.n, raw);
    load4(S.wp_info, i0, S.n, w);
    ebase = S.row_ptr[tile * TILE];
#pragma unroll
    for (int m = 0; m < 4; ++m) av[m] = hl[m] = hr[m] = (T)0;
    if (add) {
      load4(S.A_cur, i0, S.n, av);
      if (l0 < W && tile > 0) load4(S.halo_cur, (tile - 1) * 2 * W + W + l0, INT64_MAX, hl);
      if (l0 >= TILE - W && tile + 1 < S.ntiles)
        load4(S.halo_cur, (tile + 1) * 2 * W + (l0 - (TILE - W)), INT64_MAX, hr);
    }
    for (int q = tid; q < WIN; q += BLOCK) s_win[q] = (T)0;
    nh = tile_hubs<T, BLOCK>(S, tile, G, add, true, s_hnode, s_hadd);
  };

  // the last cycle's records, folded in one order by every block (the
  // first BLOCK of them loaded before the tile, so that the two overlap)
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  Part rp = v;
  if (tid < nrec_in) rp = rec_in[tid];
  int64_t tile = blockIdx.x;
  load_tile(tile);
  // the control block, fetched by the last wave behind its tile loads
  if (tid == BLOCK - 64) s_ctl = ctl[parity];
  for (int k = tid; k < nhub; k += BLOCK) s_hub[k] = (T)0;
  part_add(v, rp);
  for (int p = tid + BLOCK; p < nrec_in; p += BLOCK) part_add(v, rec_in[p]);
  v = block_sum_part_w0<NW>(v, s_part, blockIdx.x == 0);
  if (tid == 0) {
    Ctl c = next_ctl(s_ctl, v, first, d, tol, tol_in, tol_rel, method, stop, max_cycles);
    c.seq = s_ctl.seq + 1;
    if (blockIdx.x == 0) {
      ctl[parity ^ 1] = c;
      if (S.ctl_host) store_ctl_host(&S.ctl_host[parity ^ 1], c);
      if (trace && !first && !s_ctl.done && c.cycles - 1 < trace_cap)
        trace[c.cycles - 1] = di_cycle_rec{c.r_last, (int64_t)v.ops, (int32_t)v.sel,
                                           (int32_t)v.nfront};
    }
    s_done = c.done;
    s_cyc = c.cyc_mode;
    s_r = c.r;
  }
  __syncthreads();
  if (s_done) {
    // the first tile's hub partials were read and cleared before the
    // decision; the final fold still needs them
    if (add) restore_tile_hubs<T, BLOCK>(S, tile, s_hadd);
    return;
  }
  // 0: the DI-SOP threshold; 1: every node holding fluid (DI-CYC); 2: every
  // node (the power iteration's cost)
  const int mode = s_cyc;
  const double rl = s_r / (double)S.L;

  // |kept| + |pushed|: the fluid the next cycle starts with when it stays
  // nonnegative, a bound of its sum |F| otherwise; the absorbed fluid
  double my_r = 0.0, my_e = 0.0;
  unsigned long long my_ops = 0;
  unsigned int my_sel = 0, my_front = 0;
  // a second round of the cycle over each tile (DI-SOP's threshold only)
  const bool two = ROUNDS == 2 && mode == 0;

  // push, parallel over the tile's moved links: thread tid moves links
  // base + tid, base + tid + BLOCK, ..., kUnroll at a time. A link's sender
  // is the last node whose first moved link is at or before it (that node
  // has links): a search of fixed depth over the positions, the kUnroll
  // searches side by side, then the kUnroll link loads in flight together.
  auto push_pass = [&](int64_t a, int64_t win0, int total) {
    for (int q0 = tid; q0 < total; q0 += kUnroll * BLOCK) {
      int lo[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) lo[u] = 0;
#pragma unroll
      for (int step = TILE / 2; step > 0; step >>= 1) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (s_off[lo[u] + step] <= q0 + u * BLOCK) lo[u] += step;
      }
      int32_t code[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int q = q0 + u * BLOCK;
        code[u] = q < total ? S.wp_col[ebase + s_rel[lo[u]] + (q - s_off[lo[u]])] : 0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (q0 + u * BLOCK < total)
          push_link<T>(S, code[u], a + lo[u], win0, s_snd[lo[u]], s_win, s_hub);
    }
  };

  for (;;) {
    const int64_t a = tile * TILE;
    const int64_t i0 = a + l0;
    const int64_t win0 = a - W;
    // the history, needed only once the tile's nodes are selected: loaded
    // after the stop decision, so that the loads the decision and the
    // selection wait for go out alone
    load4(S.H, i0, S.n, hv);
    // fluid at the cycle's start: kept + far accumulator + halos + hubs
    T fv[4], keep[4], snd[4];
    double t[4];
    int deg[4], np[4];
    bool sel[4];
    bool any_a = false, any_sel = false;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int64_t i = i0 + m;
      fv[m] = raw[m];
      if (add && i < S.n) {
        if (av[m] != (T)0) {
          fv[m] = fv[m] + av[m];
          any_a = true;
        }
        if (l0 < W && tile > 0) fv[m] = fv[m] + hl[m];
        if (l0 >= TILE - W && tile + 1 < S.ntiles) fv[m] = fv[m] + hr[m];
        if (w[m] & kHubBit) {
          int lo = 0, hi = nh - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_hnode[mid] < i) lo = mid + 1;
            else hi = mid;
          }
          fv[m] = fv[m] + s_hadd[lo];
        }
      }
      const double f = to_d(fv[m]);
      const int out = (int)(w[m] & kOutMask);
      const bool loop = (w[m] & kLoopBit) != 0;
      deg[m] = out - (loop ? 1 : 0);
      const double af = fabs(f);
      const double thr = (mode != 0 || out == 0) ? 0.0 : rl * (double)out;
      sel[m] = i < S.n && (mode == 2 || (af > 0.0 && af >= thr));
      np[m] = 0;
      t[m] = 0.0;
      snd[m] = (T)0;
      keep[m] = fv[m];
      if (sel[m]) {
        any_sel = true;
        t[m] = loop ? f * (double)out / ((double)out - d) : f;
        keep[m] = (T)0;
        hv[m] = (T)(to_d(hv[m]) + t[m]);
        ++my_sel;
        if (out == 0) {
          my_e += t[m];
        } else if (deg[m] > 0) {
          np[m] = deg[m];
          snd[m] = (T)(t[m] * d / (double)out);
          my_ops += (unsigned long long)np[m];
          ++my_front;
          my_r += fabs(to_d(snd[m])) * (double)np[m];
        }
      }
      my_r += fabs(to_d(keep[m]));
    }
    // the far accumulator entries read are cleared; the history of the
    // diffused nodes
    if (any_a) {
      const T zero[4] = {(T)0, (T)0, (T)0, (T)0};
      store4(S.A_cur, i0, S.n, zero);
    }
    if (any_sel) store4(S.H, i0, S.n, hv);
    // the kept fluid starts the tile's part of the window, which the near
    // pushes then add to (the window was cleared before the last barrier)
#pragma unroll
    for (int m = 0; m < 4; ++m) s_win[W + l0 + m] = keep[m];
    // block scans of the link counts (node order): every node's first link
    // relative to the tile's first link, and each sender's position among
    // the tile's moved links
    int dsum = 0, nsum = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      dsum += deg[m];
      nsum += np[m];
    }
    int dinc = dsum, ninc = nsum;
    wave_scan2(dinc, ninc);
    if (lane == 63) {
      s_wtot[wave] = dinc;
      s_wtot[NW + wave] = ninc;
    }
    __syncthreads();
    int dpos = dinc - dsum, npos = ninc - nsum, total = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int x = s_wtot[q], y = s_wtot[NW + q];
      if (q < wave) {
        dpos += x;
        npos += y;
      }
      total += y;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      s_off[l0 + m] = npos;
      s_rel[l0 + m] = dpos;
      s_snd[l0 + m] = snd[m];
      dpos += deg[m];
      npos += np[m];
    }
    __syncthreads();
    push_pass(a, win0, total);
    if constexpr (ROUNDS == 2) if (two) {
      // second round: every node of the tile against the same threshold,
      // with its fluid now (kept + what the first round moved to it inside
      // the tile); what it moves waits for the next cycle like every other
      // push. The first round counted its kept and pushed fluid whole;
      // a node that diffuses again takes |f| out of that count and puts
      // back what it pushes, so that the record still sums to the fluid
      // the next cycle starts with (bounds it, for a signed fluid: removing
      // a node's f lowers sum |F| by exactly |f|). The node words and the history
      // (stored by the first round) are read again rather than held
      // through the first push.
      uint32_t w2[4];
      T h2[4];
      load4(S.wp_info, i0, S.n, w2);
      load4(S.H, i0, S.n, h2);
      __syncthreads();
      int nsum2 = 0;
      double t2[4];
      bool sel2[4], any_sel2 = false;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t i = i0 + m;
        const T f2 = s_win[W + l0 + m];
        const double f = to_d(f2);
        const int out = (int)(w2[m] & kOutMask);
        const bool loop = (w2[m] & kLoopBit) != 0;
        const int dg = out - (loop ? 1 : 0);
        // (the threshold from LDS again: not held through the first push)
        const double thr = out == 0 ? 0.0 : s_r / (double)S.L * (double)out;
        const double af = fabs(f);
        np[m] = 0;
        snd[m] = (T)0;
        t2[m] = 0.0;
        sel2[m] = i < S.n && af > 0.0 && af >= thr;
        if (sel2[m]) {
          any_sel2 = true;
          t2[m] = loop ? f * (double)out / ((double)out - d) : f;
          my_r -= af;
          ++my_sel;
          if (out == 0) {
            my_e += t2[m];
          } else if (dg > 0) {
            np[m] = dg;
            snd[m] = (T)(t2[m] * d / (double)out);
            my_ops += (unsigned long long)np[m];
            ++my_front;
            my_r += fabs(to_d(snd[m])) * (double)np[m];
          }
          s_win[W + l0 + m] = (T)0;
        }
        nsum2 += np[m];
      }
      if (any_sel2) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
          if (sel2[m]) h2[m] = (T)(to_d(h2[m]) + t2[m]);
        store4(S.H, i0, S.n, h2);
      }
      int dummy = 0, ninc2 = nsum2;
      wave_scan2(dummy, ninc2);
      if (lane == 63) s_wtot[NW + wave] = ninc2;
      __syncthreads();
      int npos2 = ninc2 - nsum2, total2 = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        const int y = s_wtot[NW + q];
        if (q < wave) npos2 += y;
        total2 += y;
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        s_off[l0 + m] = npos2;
        s_snd[l0 + m] = snd[m];
        npos2 += np[m];
      }
      __syncthreads();
      push_pass(a, win0, total2);
    }
    __syncthreads();
    // kept fluid plus the tile's own near pushes; the halos for the
    // neighbours
    T nv[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) nv[m] = s_win[W + l0 + m];
    store4(S.F, i0, S.n, nv);
    for (int q = tid; q < W; q += BLOCK) {
      S.halo_next[tile * 2 * W + q] = s_win[q];
      S.halo_next[tile * 2 * W + W + q] = s_win[W + TILE + q];
    }
    tile += G;
    if (tile >= S.ntiles) break;
    __syncthreads();  // the window and the hub ids are reused
    load_tile(tile);
    __syncthreads();
  }
  __syncthreads();  // the hub accumulators are complete
  for (int k = tid; k < nhub; k += BLOCK) {
    const T v = s_hub[k];
    if (v != (T)0) S.hub_next[(int64_t)k * S.hub_gs + blockIdx.x] = v;
  }
  Part rec{my_r, my_r, my_e, my_ops, my_sel, my_front};
  rec = block_sum_part_w0<NW>(rec, s_part, true);
  if (tid == 0) rec_out[blockIdx.x] = rec;
}

// Gathers each node's fluid into F (when `add`: kept + far accumulator +
// halos + hub partials, the far accumulator cleared) and writes the exact
// sums of |F| and F of the block's tiles into rec[blockIdx.x] (the other
// fields of the record are kept). Returns at once when ctl says the solve
// has stopped (ctl may be null).
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_wfold(WinState<T> S, Part* __restrict__ rec, int add,
                                                 const Ctl* __restrict__ ctl) {
  constexpr int NW = BLOCK / 64;
  constexpr int M = 4, TILE = 4 * BLOCK;
  __shared__ T s_hadd[KMAX];
  __shared__ int32_t s_hnode[KMAX];
  __shared__ double s_red[NW];
  if (ctl && ctl->done) return;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  double pabs = 0.0, psum = 0.0;
  for (int64_t tile = blockIdx.x; tile < S.ntiles; tile += G) {
    const int64_t a = tile * TILE;
    int nh = 0;
    if (add) nh = tile_hubs<T, BLOCK>(S, tile, G, true, true, s_hnode, s_hadd);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t i = a + tid + (int64_t)m * BLOCK;
      if (i < S.n) {
        const T raw = S.F[i];
        T fv = raw;
        if (add) {
          fv = start_value<T, TILE>(S, fv, i, tile, tid + m * BLOCK, S.wp_info[i], s_hnode, s_hadd,
                                    nh);
          if (fv != raw) S.F[i] = fv;
        }
        pabs += fabs(to_d(fv));
        psum += to_d(fv);
      }
    }
    __syncthreads();
  }
  pabs = block_sum(pabs, s_red);
  psum = block_sum(psum, s_red);
  if (tid == 0) {
    rec[blockIdx.x].pabs = pabs;
    rec[blockIdx.x].psum = psum;
  }
}

// F = B (or the uniform value), H = 0, both far accumulators (stride sa)
// and both copies of the hub partials (nhub entries) 0, and per-block sums
// of |F| and F.
template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_wstart(T* __restrict__ F, T* __restrict__ H,
                                                         T* __restrict__ A2,
                                                         T* __restrict__ hub2, int64_t nhub,
                                                         const double* __restrict__ B,
                                                         double b_uniform, int64_t n, int64_t sa,
                                                         int state, Part* __restrict__ blk_part) {
  __shared__ Part lds[kReduceBlock / 64];
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    T f;
    if (state) {
      f = F[i];
    } else {
      f = B ? (T)B[i] : (T)b_uniform;
      F[i] = f;
      H[i] = (T)0;
    }
    A2[i] = (T)0;
    A2[sa + i] = (T)0;
    v.pabs += fabs(to_d(f));
    v.psum += to_d(f);
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nhub; k += stride)
    hub2[k] = (T)0;
  v = block_sum_part(v, lds);
  if (threadIdx.x == 0) {
    blk_part[blockIdx.x] = v;
    if (blockIdx.x == 0) blk_part[gridDim.x] = Part{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  }
}

__global__ void k_clear_flag(int* flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
}

// Every thread that sees a negative entry stores 1 (all stores agree).
__global__ void k_any_negative(const double* __restrict__ B, int64_t n, int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    if (B[i] < 0.0) *flag = 1;
}

// Entries of the two copies of the hub partials.
int64_t hub_entries(const di_graph* g) { return 2 * win_hub_rows(g->n_wtiles[0]) * KMAX; }

template <typename T>
WinState<T> win_state(const CycleArgs& a, int parity) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  const int sh = a.wcfg.shape;
  const int64_t n = g->n;
  WinState<T> S;
  S.wp_info = g->wp_info;
  S.row_ptr = g->row_ptr;
  S.wp_col = g->wp_col;
  S.hub_rank_node = g->hub_rank_node;
  S.hub_id_node = g->hub_id_node;
  S.hub_id_rank = g->hub_id_rank;
  S.hub_tile = g->hub_tile[sh];
  S.n = n;
  S.L = g->L;
  S.ntiles = g->n_wtiles[sh];
  S.K = a.wcfg.hubs;
  S.F = (T*)ws->F;
  S.H = (T*)ws->H;
  T* A = (T*)ws->wA;
  S.A_cur = A + (int64_t)parity * win_stride(n);
  S.A_next = A + (int64_t)(parity ^ 1) * win_stride(n);
  // halos and hub partials: copies sized for the smallest tile and the
  // largest grid and hub count
  T* halo = (T*)ws->whalo;
  const int64_t hsz = g->n_wtiles[0] * 2 * W;
  S.halo_cur = halo + (int64_t)parity * hsz;
  S.halo_next = halo + (int64_t)(parity ^ 1) * hsz;
  T* hub = (T*)ws->whub;
  const int64_t bsz = win_hub_rows(g->n_wtiles[0]) * KMAX;
  S.hub_cur = hub + (int64_t)parity * bsz;
  S.hub_next = hub + (int64_t)(parity ^ 1) * bsz;
  S.hub_gs = win_hub_rows(g->n_wtiles[0]);
  S.rounds = a.method == DI_SOP ? a.wcfg.rounds : 1;
  S.ctl_host = ws->host_ctl;
  return S;
}

// Launches kernel template K<T, BLOCK> for the configuration's tile shape.
template <template <typename, int> class L, typename T, typename... Args>
hipError_t by_shape(const WinCfg& c, Args&&... args) {
  switch (c.shape) {
    case 0: return L<T, 256>::run(args...);
    case 1: return L<T, 512>::run(args...);
    default: return L<T, 1024>::run(args...);
  }
}

template <typename T, int BLOCK>
struct CycleLaunch {
  static hipError_t run(const CycleArgs& a, int G, hipEvent_t ev0, hipEvent_t ev1,
                        const WinState<T>& S, const Part* rec_in, int nrec_in, Part* rec_out,
                        int parity, int first, int folded) {
    auto kern = S.rounds == 2 ? k_wcycle<T, BLOCK, 2> : k_wcycle<T, BLOCK, 1>;
    if (ev0 || ev1)
      hipExtLaunchKernelGGL(kern, dim3(G), dim3(BLOCK), 0, a.stream, ev0, ev1, 0u, S, rec_in,
                            nrec_in, rec_out, a.ws->ctl, parity, first, folded, a.d, a.tol,
                            a.tol_in, a.tol_rel, a.method, a.stop, a.max_cycles, a.trace,
                            a.trace_cap);
    else
      hipLaunchKernelGGL(kern, dim3(G), dim3(BLOCK), 0, a.stream, S, rec_in, nrec_in, rec_out,
                         a.ws->ctl, parity, first, folded, a.d, a.tol, a.tol_in, a.tol_rel,
                         a.method, a.stop, a.max_cycles, a.trace, a.trace_cap);
    return hipGetLastError();
  }
};

template <typename T, int BLOCK>
struct FoldLaunch {
  static hipError_t run(const CycleArgs& a, int G, const WinState<T>& S, Part* rec, int add,
                        const Ctl* ctl) {
    hipLaunchKernelGGL((k_wfold<T, BLOCK>), dim3(G), dim3(BLOCK), 0, a.stream, S, rec, add, ctl);
    return hipGetLastError();
  }
};

}  // namespace

int win_grid(const di_graph* g, const WinCfg& c) {
  const int64_t t = g->n_wtiles[c.shape] < 1 ? 1 : g->n_wtiles[c.shape];
  const int64_t cap = c.grid_cap < 1 ? 1 : (c.grid_cap > kWinMaxGrid ? kWinMaxGrid : c.grid_cap);
  return (int)(t < cap ? t : cap);
}

template <typename T>
hipError_t launch_wstart(const CycleArgs& a, const double* B, double b_uniform) {
  hipLaunchKernelGGL(k_wstart<T>, dim3(part_count(a)), dim3(kReduceBlock), 0, a.stream,
                     (T*)a.ws->F, (T*)a.ws->H, (T*)a.ws->wA, (T*)a.ws->whub, hub_entries(a.g),
                     B, b_uniform, a.g->n, win_stride(a.g->n), 0, a.ws->blk_part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wstart_state(const CycleArgs& a) {
  hipLaunchKernelGGL(k_wstart<T>, dim3(part_count(a)), dim3(kReduceBlock), 0, a.stream,
                     (T*)a.ws->F, (T*)a.ws->H, (T*)a.ws->wA, (T*)a.ws->whub, hub_entries(a.g),
                     (const double*)nullptr, 0.0, a.g->n, win_stride(a.g->n), 1,
                     a.ws->blk_part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wcycle(const CycleArgs& a, int cycle, hipEvent_t ev0, hipEvent_t ev1) {
  Workspace* ws = a.ws;
  const int G = win_grid(a.g, a.wcfg);
  const int parity = cycle & 1;
  const int first = cycle == 0;
  const WinState<T> S = win_state<T>(a, parity);
  const Part* rec_in = first ? ws->blk_part : ws->wrec + (int64_t)parity * kWinMaxGrid;
  const int nrec_in = first ? a.first_parts : G;
  Part* rec_out = ws->wrec + (int64_t)(parity ^ 1) * kWinMaxGrid;
  const int folded = a.folded ? 1 : 0;
  hipError_t err = by_shape<CycleLaunch, T>(a.wcfg, a, G, ev0, ev1, S, rec_in, nrec_in, rec_out,
                                             parity, first, folded);
  if (err != hipSuccess || !a.folded) return err;
  // a signed fluid: gather it into F and sum |F| before the next selection
  const WinState<T> Sn = win_state<T>(a, parity ^ 1);
  return by_shape<FoldLaunch, T>(a.wcfg, a, G, Sn, rec_out, 1,
                                 (const Ctl*)(ws->ctl + (parity ^ 1)));
}

template <typename T>
hipError_t launch_wfinal(const CycleArgs& a, int parity, int add) {
  const int G = win_grid(a.g, a.wcfg);
  const WinState<T> S = win_state<T>(a, parity);
  return by_shape<FoldLaunch, T>(a.wcfg, a, G, S, a.ws->blk_part, add, (const Ctl*)nullptr);
}

hipError_t launch_any_negative(const double* B, int64_t n, int* flag, hipStream_t stream) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, stream, flag);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  int64_t g = (n + 255) / 256;
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  hipLaunchKernelGGL(k_any_negative, dim3((unsigned)g), dim3(256), 0, stream, B, n, flag);
  return hipGetLastError();
}

template hipError_t launch_wstart<double>(const CycleArgs&, const double*, double);
template hipError_t launch_wstart<float>(const CycleArgs&, const double*, double);
template hipError_t launch_wstart_state<double>(const CycleArgs&);
template hipError_t launch_wstart_state<float>(const CycleArgs&);
template hipError_t launch_wcycle<double>(const CycleArgs&, int, hipEvent_t, hipEvent_t);
template hipError_t launch_wcycle<float>(const CycleArgs&, int, hipEvent_t, hipEvent_t);
template hipError_t launch_wfinal<double>(const CycleArgs&, int, int);
template hipError_t launch_wfinal<float>(const CycleArgs&, int, int);

}  // namespace di
