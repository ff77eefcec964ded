// HIP kernels of one frontier-synchronous D-iteration cycle on gfx950.
//
// Every cycle runs the selection rule of DI-SOP (Sections 2.3 and 2.5.5)
// against r = sum_i |F_i| of the fluid at the start of the cycle, claims the
// selected nodes (Section 2.5.4: H_i += transit, F_i = 0, dangling fluid
// absorbed), and then moves the claimed fluid along the links. Fluid that
// arrives during the cycle waits for the next one, so the selected set and
// the moved amounts depend only on the state at the start of the cycle.
//
// A cycle is two launches:
//   select  every block first sums the per-block records left by the
//           previous move (sum |F|, sum F, and the statistics of the
//           previous selection) in one fixed order, plus |F| of the heavy
//           rows, so all blocks hold the same r bit for bit; thread 0 of
//           each block takes the same stop decision and block 0 writes the
//           next copy of the control block. Then the block selects and
//           claims the nodes of its tiles; in the pull direction each wave
//           leaves one statistics record.
//   move    pull (default): each node sums sent[i] over its in-links (CSC
//           without self-loops, a 16-bit in-link offset per row) whose
//           sender bit is set in the frontier bitmap, staged through LDS in
//           work items of at most kPullChunk links; each block writes one
//           record (sums over its rows and the folded select statistics). A row with more in-links is split into
//           segments whose sums the next selection completes in a fixed
//           order (with more than kHeavyLds such rows, the segments are
//           added to F[row] with FP64 atomics instead).
//           push: each selected node's out-links (CSR) receive
//           transit*d/out_i by device-scope float atomics (one push block
//           per select tile), then a reduction writes the records.
// The selection rule is DI-SOP's, DI-CYC's (every node holding fluid) or
// the power iteration's (every node). Kernels return at once after the stop,
// so the host may queue cycles ahead of the stop test.
//
// Also here: the FP64 residual pass of a refined solve (R = B + P.X - X,
// through the same work items), and the asynchronous Gauss-Seidel baseline
// (an in-place relaxation over the same items).
// Wave and block sums use DPP lane exchanges and readlane (no LDS), always
// in one fixed order.

#include "di_device.h"
#include <hip/hip_ext.h>

namespace di {
namespace {

using namespace dev;


// Adds the tile statistics of tiles [b*k, (b+1)*k) to v, where
// k = ceil(ntiles / gridDim.x): every tile is folded by exactly one block.
__device__ inline void fold_tile_stats(const SelStat* __restrict__ tile_stat, int64_t ntiles,
                                       Part& v) {
  const int64_t k = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t q0 = (int64_t)blockIdx.x * k;
  for (int64_t t = threadIdx.x; t < k; t += blockDim.x) {
    const int64_t q = q0 + t;
    if (q < ntiles) {
      const SelStat st = tile_stat[q];
      v.e += st.e;
      v.ops += st.ops;
      v.sel += st.sel;
      v.nfront += st.nfront;
    }
  }
}

// Both control-block copies cleared, and both copies of the heavy rows'
// atomic segment sums (n2 doubles) set to zero.
__global__ void k_reset_ctl(Ctl* ctl, double* __restrict__ hacc, int64_t n2) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n2;
       q += (int64_t)gridDim.x * blockDim.x)
    hacc[q] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x < 2) {
    Ctl c;
    c.r = 0.0;
    c.psum = 0.0;
    c.e = 0.0;
    c.final_r = 0.0;
    c.paper_err = 0.0;
    c.r_first = 0.0;
    c.r_last = 0.0;
    c.r_start = 0.0;
    c.cycles = 0;
    c.fallback = 0;
    c.done = 0;
    c.cyc_mode = 0;
    c.edges_total = 0;
    c.front_total = 0;
    c.sel_total = 0;
    c.t_start = 0;
    c.t_1e9 = 0;
    c.seq = 0;
    ctl[threadIdx.x] = c;
  }
}

// F = B, H = 0, and per-block sums of |F| and F over all nodes.
template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_start(T* __restrict__ F, T* __restrict__ H,
                                                        const double* __restrict__ B,
                                                        double b_uniform, int64_t n,
                                                        Part* __restrict__ blk_part) {
  __shared__ Part lds[kReduceBlock / 64];
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T f = B ? (T)B[i] : (T)b_uniform;
    F[i] = f;
    H[i] = (T)0;
    v.pabs += fabs(to_d(f));
    v.psum += to_d(f);
  }
  v = block_sum_part(v, lds);
  if (threadIdx.x == 0) {
    blk_part[blockIdx.x] = v;
    // the record after the last one (the heavy-row record of a residual
    // pass) is empty: a first selection sums gridDim.x + 1 records
    if (blockIdx.x == 0) blk_part[gridDim.x] = Part{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  }
}

// Sums of |F| and F per block over all nodes: the start of a caller-held
// state (ctl == nullptr), or the push direction after its push (folding the
// tile statistics).
template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_reduce(const T* __restrict__ F, int64_t n,
                                                         const SelStat* __restrict__ tile_stat,
                                                         int64_t ntiles,
                                                         Part* __restrict__ blk_part,
                                                         const Ctl* __restrict__ ctl) {
  __shared__ Part lds[kReduceBlock / 64];
  if (ctl && ctl->done) return;
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  if (ctl) fold_tile_stats(tile_stat, ntiles, v);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double f = to_d(F[i]);
    v.pabs += fabs(f);
    v.psum += f;
  }
  v = block_sum_part(v, lds);
  if (threadIdx.x == 0) {
    blk_part[blockIdx.x] = v;
    if (!ctl && blockIdx.x == 0) blk_part[gridDim.x] = Part{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  }
}

// Selection and claim. Tile t covers nodes [t*TILE, (t+1)*TILE); thread j of
// the block owns nodes t*TILE + j + m*BLOCK, m < M (coalesced; a wave's 64
// lanes hold 64 consecutive nodes). Blocks loop over tiles.
// PULL: writes sent[i] for the diffused nodes with links, and the frontier
//       bitmap word of each wave (bit set = the node sends this cycle).
// PUSH: writes the tile's frontier (nodes with links to push) at
//       [t*TILE, ...) with tile-local link offsets growing with the entry.
template <typename T, bool PULL, int BLOCK, int M>
__global__ __launch_bounds__(BLOCK) void k_select(
    T* __restrict__ F, T* __restrict__ H, const uint32_t* __restrict__ info,
    const int64_t* __restrict__ row_ptr, int64_t n, int64_t L, T* __restrict__ sent,
    unsigned long long* __restrict__ front_bits, int64_t* __restrict__ fr_lstart,
    int64_t* __restrict__ fr_base, T* __restrict__ fr_s, SelStat* __restrict__ tile_stat,
    const Part* __restrict__ blk_part, int nparts, const int32_t* __restrict__ heavy_row,
    const int32_t* __restrict__ hc_seg0, const int32_t* __restrict__ hc_seg1,
    const int32_t* __restrict__ hc_off, const double* __restrict__ seg_val, int64_t n_heavy,
    int64_t n_hchunks, int heavy_atomic, T* __restrict__ hret, const double* __restrict__ hacc,
    Ctl* __restrict__ ctl, Ctl* __restrict__ ctl_host, int parity, int first, double d,
    double tol, double tol_in, double tol_rel, int method, int stop, int max_cycles,
    di_cycle_rec* __restrict__ trace, int trace_cap) {
  constexpr int TILE = BLOCK * M;
  constexpr int NW = BLOCK / 64;
  constexpr int HPT = PULL ? kHeavyLds / BLOCK : 1;  // heavy rows per thread
  // heavy rows completed here (not first, not heavy_atomic): the chunk sums,
  // the row ids and the completed values
  __shared__ int32_t s_hrow[PULL ? kHeavyLds : 1];
  __shared__ double s_hval[PULL ? kHeavyLds : 1];
  __shared__ double s_hnew[PULL ? kHeavyLds : 1];
  __shared__ Part s_part[NW];
  __shared__ unsigned long long s_ops[NW];
  __shared__ double s_e[NW];
  __shared__ unsigned int s_sel[NW], s_front[NW];
  __shared__ double s_r;
  __shared__ int s_done, s_was_done, s_cyc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ntiles = (n + TILE - 1) / TILE;

  // After a pull the records leave out the heavy rows (the start records
  // cover every row): add their values, completing them with their segment
  // sums in a fixed order (or the sums the pull added atomically). A heavy
  // row's kept fluid is read from the copy of this cycle's parity, which no
  // block of this launch writes: the owner of the row's tile writes the
  // other copy (and F, which no selection reads for a heavy row).
  const bool heavy_here = PULL && !first && !heavy_atomic;
  const T* hret_cur = hret + (int64_t)parity * n_heavy;
  T* hret_next = hret + (int64_t)(parity ^ 1) * n_heavy;
  const double* hacc_cur = hacc + (int64_t)parity * n_heavy;
  // Heavy row `tid` and completion chunk `tid` (slot 0): their graph data is
  // loaded first, so that the loads depending on it (the chunk's segment
  // sums, the row's F) are issued while the node loads are in flight.
  const bool hrow0 = heavy_here && tid < n_heavy;
  const bool hchunk0 = heavy_here && tid < n_hchunks;
  int32_t hr0 = 0, ho0 = 0, ho1 = 0, hq0 = 0, hq1 = 0;
  if (hrow0) {
    hr0 = heavy_row[tid];
    ho0 = hc_off[tid];
    ho1 = hc_off[tid + 1];
  }
  if (hchunk0) {
    hq0 = hc_seg0[tid];
    hq1 = hc_seg1[tid];
  }

  // first round of loads: the first tile's nodes, the records and the
  // control block are independent of one another
  int64_t tile = blockIdx.x;
  double f[M], hv[M];
  uint32_t w[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int64_t i = tile * TILE + tid + (int64_t)m * BLOCK;
    const bool in = tile < ntiles && i < n;
    f[m] = in ? to_d(F[i]) : 0.0;
    hv[m] = in ? to_d(H[i]) : 0.0;
    w[m] = in ? info[i] : 0u;
  }
  Ctl c0;
  if (tid == 0) c0 = ctl[parity];
  double sv[kHeavyChunkSegs], fh0 = 0.0;
#pragma unroll
  for (int u = 0; u < kHeavyChunkSegs; ++u)
    sv[u] = hchunk0 && hq0 + u < hq1 ? seg_val[hq0 + u] : 0.0;
  if (hrow0) fh0 = to_d(hret_cur[tid]);
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  for (int p = tid; p < nparts; p += BLOCK) part_add(v, blk_part[p]);
  if (heavy_here) {
    // chunk sums (slot 0 from the registers), then each row's chunks in order
    if (hchunk0) {
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kHeavyChunkSegs; ++u)
        if (hq0 + u < hq1) acc += sv[u];
      s_hval[tid] = acc;
    }
    for (int64_t k = tid + BLOCK; k < n_hchunks; k += BLOCK) {
      const int64_t q0 = hc_seg0[k], q1 = hc_seg1[k];
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kHeavyChunkSegs; ++u)
        if (q0 + u < q1) acc += seg_val[q0 + u];
      s_hval[k] = acc;
    }
    int32_t hr[HPT];
    double hf[HPT];
    hr[0] = hr0;
    hf[0] = fh0;
#pragma unroll
    for (int k = 1; k < HPT; ++k) {
      const int64_t h = tid + (int64_t)k * BLOCK;
      hr[k] = h < n_heavy ? heavy_row[h] : 0;
      hf[k] = h < n_heavy ? to_d(hret_cur[h]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int64_t h = tid + (int64_t)k * BLOCK;
      if (h < n_heavy) {
        const int64_t q0 = k == 0 ? ho0 : hc_off[h], q1 = k == 0 ? ho1 : hc_off[h + 1];
        double acc = 0.0;
        for (int64_t q = q0; q < q1; ++q) acc += s_hval[q];
        hf[k] = to_d((T)(hf[k] + acc));
        v.pabs += fabs(hf[k]);
        v.psum += hf[k];
        s_hrow[h] = hr[k];
        s_hnew[h] = hf[k];
      }
    }
  } else if (PULL && !first) {
    // heavy_atomic: the pull added the segment sums into hacc
    for (int64_t h = tid; h < n_heavy; h += BLOCK) {
      const double fh = to_d((T)(to_d(hret_cur[h]) + hacc_cur[h]));
      v.pabs += fabs(fh);
      v.psum += fh;
    }
  } else if (PULL && !heavy_atomic) {
    // first selection: heavy rows are read with their tiles; their ids serve
    // the owner's lookup of the row's index
    for (int64_t h = tid; h < n_heavy; h += BLOCK) s_hrow[h] = heavy_row[h];
  }
  v = block_sum_part_w0<NW>(v, s_part, blockIdx.x == 0);
  if (tid == 0) {
    Ctl c = next_ctl(c0, v, first, d, tol, tol_in, tol_rel, method, stop, max_cycles);
    c.seq = c0.seq + 1;
    if (blockIdx.x == 0) {
      ctl[parity ^ 1] = c;
      if (ctl_host) store_ctl_host(&ctl_host[parity ^ 1], c);
      // the cycle just counted: the r its selection used and the statistics
      // of that selection (folded into the records)
      if (trace && !first && !c0.done && c.cycles - 1 < trace_cap)
        trace[c.cycles - 1] = di_cycle_rec{c.r_last, (int64_t)v.ops, (int32_t)v.sel,
                                           (int32_t)v.nfront};
    }
    s_done = c.done;
    s_was_done = c0.done;
    s_cyc = c.cyc_mode;
    s_r = c.r;
  }
  __syncthreads();
  if (s_done) {
    // stopping now: the completed heavy rows still go to F (by the block
    // that owns their tile)
    if (heavy_here && !s_was_done)
      for (int64_t h = tid; h < n_heavy; h += BLOCK) {
        const int32_t row = s_hrow[h];
        if ((row / TILE) % gridDim.x == blockIdx.x) F[row] = (T)s_hnew[h];
      }
    if (PULL && !first && heavy_atomic && !s_was_done)
      for (int64_t h = tid; h < n_heavy; h += BLOCK) {
        const int32_t row = heavy_row[h];
        if ((row / TILE) % gridDim.x == blockIdx.x)
          F[row] = (T)(to_d(hret_cur[h]) + hacc_cur[h]);
      }
    return;
  }
  // 0: the DI-SOP threshold; 1: every node holding fluid (DI-CYC);
  // 2: every node (the power iteration's cost: all links move)
  const int mode = s_cyc;
  const double rl = s_r / (double)L;

  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * TILE + tid;
    if (tile != (int64_t)blockIdx.x) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int64_t i = base + (int64_t)m * BLOCK;
        f[m] = i < n ? to_d(F[i]) : 0.0;
        hv[m] = i < n ? to_d(H[i]) : 0.0;
        w[m] = i < n ? info[i] : 0u;
      }
    }
    int npush[M];
    double snd[M];
    unsigned int my_sel = 0, my_front = 0;
    unsigned long long my_ops = 0;
    double my_e = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      npush[m] = 0;
      snd[m] = 0.0;
      const int64_t i = base + (int64_t)m * BLOCK;
      if (i < n) {
        const int out = (int)(w[m] & kOutMask);
        const bool loop = (w[m] & kLoopBit) != 0;
        // a heavy row: its index by binary search over the ascending ids (in
        // LDS, or in global memory when there are too many for LDS); after a
        // pull its fluid is the completed value
        const bool heavy = PULL && (w[m] & kHeavyBit) != 0;
        int hidx = 0;
        if (heavy) {
          int lo = 0, hi = (int)n_heavy - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((heavy_atomic ? heavy_row[mid] : s_hrow[mid]) < i) lo = mid + 1;
            else hi = mid;
          }
          hidx = lo;
          if (!first)
            f[m] = heavy_atomic ? to_d((T)(to_d(hret_cur[lo]) + hacc_cur[lo])) : s_hnew[lo];
        }
        const double a = fabs(f[m]);
        const double thr = (mode != 0 || out == 0) ? 0.0 : rl * (double)out;
        if (mode == 2 || (a > 0.0 && a >= thr)) {
          const double t = loop ? f[m] * (double)out / ((double)out - d) : f[m];
          H[i] = (T)(hv[m] + t);
          F[i] = (T)0;
          if (heavy) hret_next[hidx] = (T)0;
          ++my_sel;
          if (out == 0) {
            my_e += t;
          } else {
            const int np = out - (loop ? 1 : 0);
            if (np > 0) {
              npush[m] = np;
              snd[m] = t * d / (double)out;
              my_ops += (unsigned long long)np;
              ++my_front;
            }
          }
        } else if (heavy) {
          F[i] = (T)f[m];  // the completed value stays
          hret_next[hidx] = (T)f[m];
        }
        if (PULL && npush[m] > 0) sent[i] = (T)snd[m];
      }
    }
    if (PULL) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const unsigned long long word = __ballot(npush[m] > 0);
        const int64_t first_node = base - lane + (int64_t)m * BLOCK;  // multiple of 64
        if (lane == 0 && first_node < n) front_bits[first_node >> 6] = word;
      }
      // one statistics record per wave (the pull folds them), so the block
      // has no reduction and no barrier behind its stores
      SelStat st;
      st.sel = wave_sum(my_sel);
      st.nfront = wave_sum(my_front);
      st.ops = wave_sum(my_ops);
      st.e = wave_sum(my_e);
      if (lane == 0) tile_stat[tile * NW + wave] = st;
      continue;
    } else {
      // tile-local exclusive scan of (entries, links) over (thread, m) order
      unsigned int cnt_incl = my_front;
      unsigned long long lnk_incl = my_ops;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const unsigned int u = __shfl_up(cnt_incl, off, 64);
        const unsigned long long x = __shfl_up(lnk_incl, off, 64);
        if (lane >= off) {
          cnt_incl += u;
          lnk_incl += x;
        }
      }
      if (lane == 63) {
        s_front[wave] = cnt_incl;
        s_ops[wave] = lnk_incl;
      }
      __syncthreads();
      unsigned int cnt_before = 0;
      unsigned long long lnk_before = 0;
      for (int q = 0; q < wave; ++q) {
        cnt_before += s_front[q];
        lnk_before += s_ops[q];
      }
      __syncthreads();
      unsigned int k = cnt_before + cnt_incl - my_front;
      unsigned long long lo = lnk_before + lnk_incl - my_ops;
      const int64_t fbase = tile * TILE;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (npush[m] > 0) {
          fr_lstart[fbase + k] = (int64_t)lo;
          fr_base[fbase + k] = row_ptr[base + (int64_t)m * BLOCK];
          fr_s[fbase + k] = (T)snd[m];
          ++k;
          lo += (unsigned long long)npush[m];
        }
      }
    }
    // the tile's statistics: wave sums, then wave 0 folds the waves
    my_sel = wave_sum(my_sel);
    my_front = wave_sum(my_front);
    my_ops = wave_sum(my_ops);
    my_e = wave_sum(my_e);
    if (lane == 0) {
      s_sel[wave] = my_sel;
      s_front[wave] = my_front;
      s_ops[wave] = my_ops;
      s_e[wave] = my_e;
    }
    __syncthreads();
    if (wave == 0) {
      SelStat st;
      st.sel = low_lanes_sum<NW>(lane < NW ? s_sel[lane] : 0u);
      st.nfront = low_lanes_sum<NW>(lane < NW ? s_front[lane] : 0u);
      st.ops = low_lanes_sum<NW>(lane < NW ? s_ops[lane] : 0ull);
      st.e = low_lanes_sum<NW>(lane < NW ? s_e[lane] : 0.0);
      if (lane == 0) tile_stat[tile] = st;
    }
    if (tile + gridDim.x < ntiles) __syncthreads();  // LDS reused by the next tile
  }
}

// Pull: F_j += sum of sent[i] over the in-links i -> j (i != j) whose sender
// bit is set. Work items are prepared with the graph: light items (rows
// [r0, r1), at most kPullChunk links) and segments of heavy rows. Each
// thread stages its kPullChunk / kPullBlock links with all index loads,
// then all bitmap loads, then the gathers of the set bits, in flight
// together. Every block writes one Part record: the sums over its light
// rows and the folded tile statistics.
// Eight waves per SIMD (at most 64 VGPRs): the whole pull grid (2048 blocks
// of 4 waves) is resident at once, which measured faster than six waves
// without the register cap, a few spilled registers included.
#ifndef DI_PULL_WAVES_PER_EU
#define DI_PULL_WAVES_PER_EU 8
#endif
template <typename T>
__global__ __launch_bounds__(kPullBlock)
__attribute__((amdgpu_waves_per_eu(DI_PULL_WAVES_PER_EU))) void k_pull(
    T* __restrict__ F, const T* __restrict__ sent,
    const unsigned long long* __restrict__ front_bits, const uint16_t* __restrict__ row_lo,
    const int32_t* __restrict__ csc_idx, const int64_t* __restrict__ it_r0,
    const int64_t* __restrict__ it_r1, const int64_t* __restrict__ it_l0,
    const int64_t* __restrict__ it_l1, const int32_t* __restrict__ it_seg, int64_t n_items,
    double* __restrict__ seg_val, int heavy_atomic, const int32_t* __restrict__ seg_heavy,
    double* __restrict__ hacc_next, double* __restrict__ hacc_clear, int64_t n_heavy,
    const SelStat* __restrict__ tile_stat, int64_t ntiles, Part* __restrict__ blk_part,
    const Ctl* __restrict__ ctl) {
  constexpr int U = kPullChunk / kPullBlock;
  __shared__ double s_val[kPullChunk];
  __shared__ double s_red[kPullBlock / 64];
  __shared__ Part s_part[kPullBlock / 64];
  const int tid = threadIdx.x;
  // XCD-aware order: workgroups are dealt round-robin to the XCDs, so when
  // the grid is a multiple of kXcds, XCD x works through the x-th contiguous
  // eighth of the items and its L2 sees one range of rows and senders
  int64_t it_begin = blockIdx.x, it_end = n_items, it_step = gridDim.x;
  if (gridDim.x % kXcds == 0) {
    const int64_t x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
    const int64_t lo = n_items * x / kXcds, hi = n_items * (x + 1) / kXcds;
    it_begin = lo + blockIdx.x / kXcds;
    it_end = hi;
    it_step = per;
  }
  // the first item's descriptor, read with the control block
  int64_t nl0 = 0, nl1 = 0, nr0 = 0, nr1 = 0;
  int nseg = -1;
  if (it_begin < it_end) {
    nl0 = it_l0[it_begin];
    nl1 = it_l1[it_begin];
    nr0 = it_r0[it_begin];
    nr1 = it_r1[it_begin];
    nseg = it_seg[it_begin];
  }
  double acc_abs = 0.0, acc_sum = 0.0;  // the block's rows: sum |F|, sum F
  if (ctl->done) return;
  // heavy_atomic: the copy the last selection read is cleared for the next
  // pull's additions
  if (heavy_atomic && blockIdx.x == 0)
    for (int64_t h = tid; h < n_heavy; h += kPullBlock) hacc_clear[h] = 0.0;
  for (int64_t it = it_begin; it < it_end; it += it_step) {
    const int64_t l0 = nl0, l1 = nl1, r0 = nr0, r1 = nr1;
    const int seg = nseg;
    const int64_t nx = it + it_step;
    if (nx < it_end) {  // prefetch the next descriptor
      nl0 = it_l0[nx];
      nl1 = it_l1[nx];
      nr0 = it_r0[nx];
      nr1 = it_r1[nx];
      nseg = it_seg[nx];
    }
    const int nl = (int)(l1 - l0);
    // the thread's first row, fetched while the links are in flight
    const int64_t row0 = r0 + tid;
    double f0 = 0.0;
    int a0 = 0, b0 = 0;
    if (seg < 0 && row0 < r1) {
      f0 = to_d(F[row0]);
      a0 = row_lo[row0];
      b0 = row0 + 1 < r1 ? (int)row_lo[row0 + 1] : nl;
    }
    int32_t idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      idx[u] = p < nl ? csc_idx[l0 + p] : 0;
    }
    unsigned long long word[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      word[u] = p < nl ? front_bits[idx[u] >> 6] : 0ull;
    }
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = (word[u] >> (idx[u] & 63)) & 1ull ? to_d(sent[idx[u]]) : 0.0;
    if (seg >= 0) {
      // a segment of a heavy row: its sum is completed by the next
      // selection (or, with too many heavy rows, added atomically to the
      // row's sum of this cycle)
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u];
      acc = block_sum(acc, s_red);
      if (tid == 0) {
        if (!heavy_atomic) seg_val[seg] = acc;
        else if (acc != 0.0) atomic_add(&hacc_next[seg_heavy[seg]], acc);
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      if (p < nl) s_val[p] = v[u];
    }
    __syncthreads();
    // rows r0 + tid + k * kPullBlock; a row with more than kPullLongRow links
    // is summed by its whole wave (strided lanes, then a wave sum)
    const int lane = tid & 63;
    for (int64_t row = row0; row - lane < r1; row += kPullBlock) {
      const bool valid = row < r1;
      double f = 0.0;
      int a = 0, b = 0;
      if (row == row0) {
        f = f0;
        a = a0;
        b = b0;
      } else if (valid) {
        f = to_d(F[row]);
        a = row_lo[row];
        b = row + 1 < r1 ? (int)row_lo[row + 1] : nl;
      }
      const bool longrow = valid && (b - a) > kPullLongRow;
      double acc = 0.0;
      if (valid && !longrow)
        for (int q = a; q < b; ++q) acc += s_val[q];
      unsigned long long mask = __ballot(longrow);
      while (mask) {
        const int src = __ffsll(mask) - 1;
        mask &= mask - 1;
        const int la = read_lane(a, src), lb = read_lane(b, src);
        double part = 0.0;
        for (int q = la + lane; q < lb; q += 64) part += s_val[q];
        part = wave_sum(part);
        if (lane == src) acc = part;
      }
      if (valid) {
        if (acc != 0.0) {
          const T nv = (T)(f + acc);
          F[row] = nv;
          f = to_d(nv);
        }
        acc_abs += fabs(f);
        acc_sum += f;
      }
    }
    __syncthreads();
  }
  Part acc_part{acc_abs, acc_sum, 0.0, 0ull, 0u, 0u};
  fold_tile_stats(tile_stat, ntiles, acc_part);
  acc_part = block_sum_part(acc_part, s_part);
  if (tid == 0) blk_part[blockIdx.x] = acc_part;
}

// Push: block b moves the frontier of select tile b. Entries are staged in
// LDS; each lane finds the entry of its link by binary search on the local
// link offsets and adds the entry's amount to F[col] atomically.
template <typename T>
__global__ __launch_bounds__(kPushBlock) void k_push(T* __restrict__ F,
                                                     const int32_t* __restrict__ col,
                                                     const int64_t* __restrict__ fr_lstart,
                                                     const int64_t* __restrict__ fr_base,
                                                     const T* __restrict__ fr_s,
                                                     const SelStat* __restrict__ tile_stat,
                                                     const Ctl* __restrict__ ctl) {
  __shared__ int64_t s_start[kSelectTilePush];
  __shared__ int64_t s_base[kSelectTilePush];
  __shared__ T s_val[kSelectTilePush];
  if (ctl->done) return;
  const int nf = (int)tile_stat[blockIdx.x].nfront;
  if (nf == 0) return;
  const int64_t E = (int64_t)tile_stat[blockIdx.x].ops;
  const int64_t fbase = (int64_t)blockIdx.x * kSelectTilePush;
  for (int q = threadIdx.x; q < nf; q += blockDim.x) {
    s_start[q] = fr_lstart[fbase + q];
    s_base[q] = fr_base[fbase + q] - fr_lstart[fbase + q];
    s_val[q] = fr_s[fbase + q];
  }
  __syncthreads();
  int lo = 0;
  for (int64_t e = threadIdx.x; e < E; e += blockDim.x) {
    int hi = nf - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_start[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int32_t j = col[s_base[lo] + e];
    atomic_add(&F[j], s_val[lo]);
  }
}

// Sums |F| and F over the records [0, count) in a fixed order (lane l the
// records l, l + 64, ..., then the wave's fixed-order sum) and stores both
// (out->pabs, out->psum) with system-scope stores, so that pinned host
// memory receives them directly. One wave.
__global__ __launch_bounds__(64) void k_sum_parts(const Part* __restrict__ parts, int count,
                                                  Part* __restrict__ out) {
  const int lane = threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int k = lane; k < count; k += 64) {
    s1 += parts[k].pabs;
    s2 += parts[k].psum;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    __hip_atomic_store(&out->pabs, s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&out->psum, s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <typename T>
__global__ void k_h_to_x(const T* __restrict__ H, double* __restrict__ X, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    X[i] = to_d(H[i]);
}

// ---- FP64 residual pass (refinement of an FP32 solve) -----------------
// With the history folded into X, the exact residual R = B + P.X - X is
// recomputed in FP64 and becomes the new fluid: (F, H) = (R, 0) satisfies
// F = R - (I - P).H again, so the next FP32 pass solves for the correction.

// X += H, H = 0 (when H is given); y_j = d X_j / out_j, 0 for dangling j.
template <typename T>
__global__ void k_refine_y(double* __restrict__ X, T* __restrict__ H,
                           const uint32_t* __restrict__ info, double d, int64_t n,
                           double* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double x = X[i];
    if (H) {
      x += to_d(H[i]);
      X[i] = x;
      H[i] = (T)0;
    }
    const int out = (int)(info[i] & kOutMask);
    y[i] = out > 0 ? d * x / (double)out : 0.0;
  }
}

// R_i = B_i - X_i + (self-loop ? y_i : 0) + sum of y_j over the in-links
// j -> i (j != i), over the pull work items (in-link ids staged through
// LDS, ascending within a row). Heavy-row segments leave their sums in
// seg_val for k_refine_heavy. Each block writes one record of its rows'
// sum |R| and sum R.
template <typename T>
// (at most 64 VGPRs, like the pull: eight waves per SIMD keep more of the
// random gathers of y in flight)
__global__ __launch_bounds__(kPullBlock) __attribute__((amdgpu_waves_per_eu(DI_PULL_WAVES_PER_EU)))
void k_refine_r(
    T* __restrict__ R, const double* __restrict__ X, const double* __restrict__ y,
    const double* __restrict__ B, double b_uniform, const uint32_t* __restrict__ info,
    const int64_t* __restrict__ csc_ptr, const int32_t* __restrict__ csc_idx,
    const int64_t* __restrict__ it_r0, const int64_t* __restrict__ it_r1,
    const int64_t* __restrict__ it_l0, const int64_t* __restrict__ it_l1,
    const int32_t* __restrict__ it_seg, int64_t n_items, double* __restrict__ seg_val,
    Part* __restrict__ blk_part) {
  constexpr int U = kPullChunk / kPullBlock;
  __shared__ double s_val[kPullChunk];
  __shared__ double s_red[kPullBlock / 64];
  __shared__ Part s_part[kPullBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63;
  Part acc_part{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int64_t l0 = it_l0[it], l1 = it_l1[it], r0 = it_r0[it], r1 = it_r1[it];
    const int seg = it_seg[it];
    const int nl = (int)(l1 - l0);
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      v[u] = p < nl ? y[csc_idx[l0 + p]] : 0.0;
    }
    if (seg >= 0) {
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u];
      acc = block_sum(acc, s_red);
      if (tid == 0) seg_val[seg] = acc;
      continue;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      if (p < nl) s_val[p] = v[u];
    }
    __syncthreads();
    for (int64_t row = r0 + tid; row - lane < r1; row += kPullBlock) {
      const bool valid = row < r1;
      int a = 0, b = 0;
      if (valid) {
        a = (int)(csc_ptr[row] - l0);
        b = (int)(csc_ptr[row + 1] - l0);
      }
      const bool longrow = valid && (b - a) > kPullLongRow;
      double acc = 0.0;
      if (valid && !longrow)
        for (int q = a; q < b; ++q) acc += s_val[q];
      unsigned long long mask = __ballot(longrow);
      while (mask) {
        const int src = __ffsll(mask) - 1;
        mask &= mask - 1;
        const int la = read_lane(a, src), lb = read_lane(b, src);
        double part = 0.0;
        for (int q = la + lane; q < lb; q += 64) part += s_val[q];
        part = wave_sum(part);
        if (lane == src) acc = part;
      }
      if (valid) {
        const double bi = B ? B[row] : b_uniform;
        const double self = (info[row] & kLoopBit) ? y[row] : 0.0;
        const double r = bi - X[row] + self + acc;
        R[row] = (T)r;
        acc_part.pabs += fabs(r);
        acc_part.psum += r;
      }
    }
    __syncthreads();
  }
  acc_part = block_sum_part(acc_part, s_part);
  if (tid == 0) blk_part[blockIdx.x] = acc_part;
}

// The heavy rows of a residual pass: their segment sums in order. One
// block; writes the record blk_part[slot].
template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_refine_heavy(
    T* __restrict__ R, const double* __restrict__ X, const double* __restrict__ y,
    const double* __restrict__ B, double b_uniform, const uint32_t* __restrict__ info,
    const int32_t* __restrict__ heavy_row, const int64_t* __restrict__ heavy_seg,
    int64_t n_heavy, const double* __restrict__ seg_val, Part* __restrict__ blk_part,
    int slot) {
  __shared__ Part lds[kReduceBlock / 64];
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  for (int64_t h = threadIdx.x; h < n_heavy; h += blockDim.x) {
    const int64_t row = heavy_row[h];
    const double acc = ordered_sum(seg_val, heavy_seg[h], heavy_seg[h + 1], 1);
    const double bi = B ? B[row] : b_uniform;
    const double self = (info[row] & kLoopBit) ? y[row] : 0.0;
    const double r = bi - X[row] + self + acc;
    R[row] = (T)r;
    v.pabs += fabs(r);
    v.psum += r;
  }
  v = block_sum_part(v, lds);
  if (threadIdx.x == 0) blk_part[slot] = v;
}

// ---- asynchronous Gauss-Seidel (the GS baseline's GPU variant) -------------
// Section 2.5.3's sweep updates the rows in order, each from the newest
// values. On the GPU the rows of a sweep update in parallel and in place:
// row i computes x_i = (B_i + sum of y_j over its in-links j != i) /
// (1 - d/out_i if i has a self-loop, else 1), where y_j = d x_j / out_j is
// whatever value of row j is visible at that moment, and writes x_i and
// y_i. Every y_j is written once per sweep, so a read sees its value from
// before the sweep or its final value; the residual after the sweep is then
// R_i = sum over j != i of p_ij (x_j - x_j as read), hence |R|_1 <= d times
// the sum of |x_i(after) - x_i(before)|, which is the stop test. x starts at
// B.

__device__ inline double gs_diag(uint32_t w, double d) {
  const int out = (int)(w & kOutMask);
  return (w & kLoopBit) ? 1.0 - d / (double)out : 1.0;
}

// x = B, y = d x / out (0 for dangling nodes).
__global__ void k_gs_init(double* __restrict__ x, double* __restrict__ y,
                          const uint32_t* __restrict__ info, const double* __restrict__ B,
                          double b_uniform, double d, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double xi = B ? B[i] : b_uniform;
    const int out = (int)(info[i] & kOutMask);
    x[i] = xi;
    y[i] = out > 0 ? d * xi / (double)out : 0.0;
  }
}

// One sweep over the light rows (in place); heavy-row segments leave their
// sums in seg_val. Each block writes one record: sum |dx| and sum dx of its
// rows. y is read and written by every block concurrently: its accesses are
// relaxed device-scope atomics (well defined, and any value a read returns
// is one the bound above allows).
__device__ inline double y_read(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void y_write(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kPullBlock) void k_gs_sweep(
    double* __restrict__ x, double* y, const double* __restrict__ B, double b_uniform,
    double d, const uint32_t* __restrict__ info, const int64_t* __restrict__ csc_ptr,
    const int32_t* __restrict__ csc_idx, const int64_t* __restrict__ it_r0,
    const int64_t* __restrict__ it_r1, const int64_t* __restrict__ it_l0,
    const int64_t* __restrict__ it_l1, const int32_t* __restrict__ it_seg, int64_t n_items,
    double* __restrict__ seg_val, Part* __restrict__ blk_part, const Ctl* __restrict__ ctl) {
  constexpr int U = kPullChunk / kPullBlock;
  __shared__ double s_val[kPullChunk];
  __shared__ double s_red[kPullBlock / 64];
  __shared__ Part s_part[kPullBlock / 64];
  if (ctl->done) return;
  const int tid = threadIdx.x, lane = tid & 63;
  Part acc_part{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int64_t l0 = it_l0[it], l1 = it_l1[it], r0 = it_r0[it], r1 = it_r1[it];
    const int seg = it_seg[it];
    const int nl = (int)(l1 - l0);
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      v[u] = p < nl ? y_read(y + csc_idx[l0 + p]) : 0.0;
    }
    if (seg >= 0) {
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u];
      acc = block_sum(acc, s_red);
      if (tid == 0) seg_val[seg] = acc;
      continue;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      if (p < nl) s_val[p] = v[u];
    }
    __syncthreads();
    for (int64_t row = r0 + tid; row - lane < r1; row += kPullBlock) {
      const bool valid = row < r1;
      int a = 0, b = 0;
      if (valid) {
        a = (int)(csc_ptr[row] - l0);
        b = (int)(csc_ptr[row + 1] - l0);
      }
      const bool longrow = valid && (b - a) > kPullLongRow;
      double acc = 0.0;
      if (valid && !longrow)
        for (int q = a; q < b; ++q) acc += s_val[q];
      unsigned long long mask = __ballot(longrow);
      while (mask) {
        const int src = __ffsll(mask) - 1;
        mask &= mask - 1;
        const int la = read_lane(a, src), lb = read_lane(b, src);
        double part = 0.0;
        for (int q = la + lane; q < lb; q += 64) part += s_val[q];
        part = wave_sum(part);
        if (lane == src) acc = part;
      }
      if (valid) {
        const uint32_t w = info[row];
        const double bi = B ? B[row] : b_uniform;
        const double xo = x[row];
        const double xn = (bi + acc) / gs_diag(w, d);
        const int out = (int)(w & kOutMask);
        x[row] = xn;
        y_write(y + row, out > 0 ? d * xn / (double)out : 0.0);
        acc_part.pabs += fabs(xn - xo);
        acc_part.psum += xn - xo;
      }
    }
    __syncthreads();
  }
  acc_part = block_sum_part(acc_part, s_part);
  if (tid == 0) blk_part[blockIdx.x] = acc_part;
}

// The heavy rows of a sweep, from their segment sums in order. One block;
// writes the record blk_part[slot].
__global__ __launch_bounds__(kReduceBlock) void k_gs_heavy(
    double* __restrict__ x, double* __restrict__ y, const double* __restrict__ B,
    double b_uniform, double d, const uint32_t* __restrict__ info,
    const int32_t* __restrict__ heavy_row, const int64_t* __restrict__ heavy_seg,
    int64_t n_heavy, const double* __restrict__ seg_val, Part* __restrict__ blk_part, int slot,
    const Ctl* __restrict__ ctl) {
  __shared__ Part lds[kReduceBlock / 64];
  if (ctl->done) return;
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  for (int64_t h = threadIdx.x; h < n_heavy; h += blockDim.x) {
    const int64_t row = heavy_row[h];
    const double acc = ordered_sum(seg_val, heavy_seg[h], heavy_seg[h + 1], 1);
    const uint32_t w = info[row];
    const double bi = B ? B[row] : b_uniform;
    const double xo = x[row];
    const double xn = (bi + acc) / gs_diag(w, d);
    const int out = (int)(w & kOutMask);
    x[row] = xn;
    y[row] = out > 0 ? d * xn / (double)out : 0.0;
    v.pabs += fabs(xn - xo);
    v.psum += xn - xo;
  }
  v = block_sum_part(v, lds);
  if (threadIdx.x == 0) blk_part[slot] = v;
}

// The stop test after a sweep: sums the records in order; done = 1 when
// d * sum |dx| <= tol (then |B + P.x - x|_1 <= tol), 2 at max_cycles, 3
// when the sum is not finite.
__global__ __launch_bounds__(kReduceBlock) void k_gs_decide(const Part* __restrict__ blk_part,
                                                            int nparts, double d, double tol,
                                                            int64_t links, int max_cycles,
                                                            Ctl* __restrict__ ctl) {
  __shared__ Part lds[kReduceBlock / 64];
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = ctl->done;
  __syncthreads();
  if (s_done) return;
  Part v{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) part_add(v, blk_part[p]);
  v = block_sum_part(v, lds);
  if (threadIdx.x == 0) {
    Ctl c = *ctl;
    c.cycles += 1;
    c.edges_total += (unsigned long long)links;
    c.r = v.pabs;
    if (c.cycles == 1) c.r_first = v.pabs;
    if (!isfinite(v.pabs)) {
      c.final_r = v.pabs;
      c.done = 3;
    } else if (d * v.pabs <= tol) {
      c.final_r = d * v.pabs;
      c.done = 1;
    } else if (c.cycles >= max_cycles) {
      c.final_r = d * v.pabs;
      c.done = 2;
    }
    *ctl = c;
  }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline unsigned int grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = ceil_div(n, block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned int)g;
}

}  // namespace

int select_tiles(int64_t n, int direction) {
  const int64_t tile = direction == kPull ? kSelectTilePull : kSelectTilePush;
  const int64_t t = ceil_div(n, tile);
  return (int)(t < 1 ? 1 : t);
}

int select_stat_records(int64_t n, int direction) {
  const int t = select_tiles(n, direction);
  return direction == kPull ? t * (kSelectBlockPull / 64) : t;
}

int select_grid(int64_t n, int direction) {
  const int t = select_tiles(n, direction);
  return direction == kPull ? (t < kSelectGridPull ? t : kSelectGridPull) : t;
}

int pull_grid(const di_graph* g) {
  int grid = (int)grid_for(g->n_items, 1, kPullMaxGrid);
  if (grid >= 8 * kXcds) grid -= grid % kXcds;  // XCD-aware order (k_pull)
  return grid;
}

int reduce_grid(int64_t n) { return (int)grid_for(n, kReduceBlock, kReduceGrid); }

int part_count(const CycleArgs& a) {
  return a.direction == kPull ? pull_grid(a.g) : reduce_grid(a.g->n);
}

hipError_t launch_reset_ctl(const CycleArgs& a) {
  const int64_t n2 = a.ws->hacc ? 2 * a.g->n_heavy : 0;
  hipLaunchKernelGGL(k_reset_ctl, dim3(grid_for(n2, 256, 64)), dim3(256), 0, a.stream, a.ws->ctl,
                     a.ws->hacc, n2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_start(const CycleArgs& a, const double* B, double b_uniform) {
  hipLaunchKernelGGL(k_start<T>, dim3(part_count(a)), dim3(kReduceBlock), 0, a.stream,
                     (T*)a.ws->F, (T*)a.ws->H, B, b_uniform, a.g->n, a.ws->blk_part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_start_state(const CycleArgs& a) {
  hipLaunchKernelGGL(k_reduce<T>, dim3(part_count(a)), dim3(kReduceBlock), 0, a.stream,
                     (const T*)a.ws->F, a.g->n, (const SelStat*)a.ws->tile_stat, (int64_t)0,
                     a.ws->blk_part, (const Ctl*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_select(const CycleArgs& a, int cycle, int first) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  const int grid = select_grid(g->n, a.direction);
  const int parity = cycle & 1;
  const int nparts = first ? a.first_parts : part_count(a);
  if (a.direction == kPull) {
    hipLaunchKernelGGL((k_select<T, true, kSelectBlockPull, kSelectPerThreadPull>), dim3(grid),
                       dim3(kSelectBlockPull), 0, a.stream, (T*)ws->F, (T*)ws->H, g->info,
                       g->row_ptr, g->n, g->L, (T*)ws->sent, ws->front_bits, (int64_t*)nullptr,
                       (int64_t*)nullptr, (T*)nullptr, ws->tile_stat, (const Part*)ws->blk_part,
                       nparts, g->heavy_row, g->hc_seg0, g->hc_seg1, g->hc_off,
                       (const double*)ws->seg_val, g->n_heavy, g->n_hchunks, (int)g->heavy_atomic,
                       (T*)ws->hret, (const double*)ws->hacc, ws->ctl, ws->host_ctl, parity, first,
                       a.d, a.tol,
                       a.tol_in, a.tol_rel, a.method, a.stop,
                       a.max_cycles, a.trace, a.trace_cap);
  } else {
    hipLaunchKernelGGL((k_select<T, false, kSelectBlockPush, kSelectPerThreadPush>), dim3(grid),
                       dim3(kSelectBlockPush), 0, a.stream, (T*)ws->F, (T*)ws->H, g->info,
                       g->row_ptr, g->n, g->L, (T*)nullptr, (unsigned long long*)nullptr,
                       ws->fr_lstart, ws->fr_base, (T*)ws->fr_s, ws->tile_stat,
                       (const Part*)ws->blk_part, nparts, (const int32_t*)nullptr,
                       (const int32_t*)nullptr, (const int32_t*)nullptr, (const int32_t*)nullptr,
                       (const double*)nullptr, (int64_t)0, (int64_t)0, 0, (T*)nullptr,
                       (const double*)nullptr, ws->ctl, ws->host_ctl, parity, first,
                       a.d, a.tol, a.tol_in, a.tol_rel, a.method, a.stop, a.max_cycles, a.trace,
                       a.trace_cap);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_move(const CycleArgs& a, int cycle, hipEvent_t ev0, hipEvent_t ev1) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  const Ctl* ctl = ws->ctl + ((cycle + 1) & 1);
  const int64_t ntiles = select_stat_records(g->n, a.direction);
  // Timing events travel in the kernel's own dispatch and take its start and
  // end times (an event recorded beside a launch also times the gap to it).
  const bool timed = ev0 || ev1;
  if (a.direction == kPull) {
    const dim3 grid(pull_grid(g)), block(kPullBlock);
    // the selection of cycle c read hacc copy c & 1; this pull adds into copy
    // (c + 1) & 1 and clears copy c & 1
    double* hacc_next = ws->hacc + (int64_t)((cycle + 1) & 1) * g->n_heavy;
    double* hacc_clear = ws->hacc + (int64_t)(cycle & 1) * g->n_heavy;
    if (timed)
      hipExtLaunchKernelGGL(k_pull<T>, grid, block, 0, a.stream, ev0, ev1, 0u, (T*)ws->F,
                            (const T*)ws->sent, ws->front_bits, g->row_lo, g->csc_idx, g->it_r0,
                            g->it_r1, g->it_l0, g->it_l1, g->it_seg, g->n_items, ws->seg_val,
                            (int)g->heavy_atomic, (const int32_t*)g->seg_heavy, hacc_next,
                            hacc_clear, g->n_heavy, (const SelStat*)ws->tile_stat, ntiles,
                            ws->blk_part, ctl);
    else
      hipLaunchKernelGGL(k_pull<T>, grid, block, 0, a.stream, (T*)ws->F, (const T*)ws->sent,
                         ws->front_bits, g->row_lo, g->csc_idx, g->it_r0, g->it_r1, g->it_l0,
                         g->it_l1, g->it_seg, g->n_items, ws->seg_val, (int)g->heavy_atomic,
                         (const int32_t*)g->seg_heavy, hacc_next, hacc_clear, g->n_heavy,
                         (const SelStat*)ws->tile_stat, ntiles, ws->blk_part, ctl);
    return hipGetLastError();
  }
  const dim3 grid(ntiles), block(kPushBlock);
  if (timed)
    hipExtLaunchKernelGGL(k_push<T>, grid, block, 0, a.stream, ev0, ev1, 0u, (T*)ws->F, g->col,
                          ws->fr_lstart, ws->fr_base, (const T*)ws->fr_s,
                          (const SelStat*)ws->tile_stat, ctl);
  else
    hipLaunchKernelGGL(k_push<T>, grid, block, 0, a.stream, (T*)ws->F, g->col, ws->fr_lstart,
                       ws->fr_base, (const T*)ws->fr_s, (const SelStat*)ws->tile_stat, ctl);
  hipError_t err;
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_reduce<T>, dim3(reduce_grid(g->n)), dim3(kReduceBlock), 0, a.stream,
                     (const T*)ws->F, g->n, (const SelStat*)ws->tile_stat, ntiles, ws->blk_part,
                     ctl);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const CycleArgs& a, int count, Part* out) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, a.stream, (const Part*)a.ws->blk_part,
                     count, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_h_to_x(const CycleArgs& a, double* X) {
  hipLaunchKernelGGL(k_h_to_x<T>, dim3(grid_for(a.g->n, 256, 4096)), dim3(256), 0, a.stream,
                     (const T*)a.ws->H, X, a.g->n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_refine(const CycleArgs& a, double* X, T* H, const double* B, double b_uniform,
                         T* R_out) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  hipLaunchKernelGGL(k_refine_y<T>, dim3(grid_for(g->n, 256, 4096)), dim3(256), 0, a.stream, X, H,
                     g->info, a.d, g->n, ws->Y64);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int grid = pull_grid(g);
  hipLaunchKernelGGL(k_refine_r<T>, dim3(grid), dim3(kPullBlock), 0, a.stream, R_out,
                     (const double*)X, (const double*)ws->Y64, B, b_uniform, g->info, g->csc_ptr,
                     g->csc_idx, g->it_r0, g->it_r1, g->it_l0, g->it_l1, g->it_seg, g->n_items,
                     ws->seg_val, ws->blk_part);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_refine_heavy<T>, dim3(1), dim3(kReduceBlock), 0, a.stream, R_out,
                     (const double*)X, (const double*)ws->Y64, B, b_uniform, g->info,
                     g->heavy_row, g->heavy_seg, g->n_heavy, (const double*)ws->seg_val,
                     ws->blk_part, grid);
  return hipGetLastError();
}

template hipError_t launch_start<double>(const CycleArgs&, const double*, double);
template hipError_t launch_start<float>(const CycleArgs&, const double*, double);
template hipError_t launch_start_state<double>(const CycleArgs&);
template hipError_t launch_start_state<float>(const CycleArgs&);
template hipError_t launch_select<double>(const CycleArgs&, int, int);
template hipError_t launch_select<float>(const CycleArgs&, int, int);
template hipError_t launch_move<double>(const CycleArgs&, int, hipEvent_t, hipEvent_t);
template hipError_t launch_move<float>(const CycleArgs&, int, hipEvent_t, hipEvent_t);
template hipError_t launch_h_to_x<double>(const CycleArgs&, double*);
template hipError_t launch_h_to_x<float>(const CycleArgs&, double*);
hipError_t launch_gs_init(const CycleArgs& a, const double* B, double b_uniform) {
  hipLaunchKernelGGL(k_gs_init, dim3(grid_for(a.g->n, 256, 4096)), dim3(256), 0, a.stream,
                     (double*)a.ws->H, (double*)a.ws->F, a.g->info, B, b_uniform, a.d, a.g->n);
  return hipGetLastError();
}

hipError_t launch_gs_sweep(const CycleArgs& a, const double* B, double b_uniform) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  const int grid = pull_grid(g);
  hipLaunchKernelGGL(k_gs_sweep, dim3(grid), dim3(kPullBlock), 0, a.stream, (double*)ws->H,
                     (double*)ws->F, B, b_uniform, a.d, g->info, g->csc_ptr, g->csc_idx, g->it_r0,
                     g->it_r1, g->it_l0, g->it_l1, g->it_seg, g->n_items, ws->seg_val,
                     ws->blk_part, (const Ctl*)ws->ctl);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_gs_heavy, dim3(1), dim3(kReduceBlock), 0, a.stream, (double*)ws->H,
                     (double*)ws->F, B, b_uniform, a.d, g->info, g->heavy_row, g->heavy_seg,
                     g->n_heavy, (const double*)ws->seg_val, ws->blk_part, grid,
                     (const Ctl*)ws->ctl);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(k_gs_decide, dim3(1), dim3(kReduceBlock), 0, a.stream,
                     (const Part*)ws->blk_part, grid + 1, a.d, a.tol, (int64_t)g->Lp,
                     a.max_cycles, ws->ctl);
  return hipGetLastError();
}

template hipError_t launch_refine<double>(const CycleArgs&, double*, double*, const double*, double,
                                          double*);
template hipError_t launch_refine<float>(const CycleArgs&, double*, float*, const double*, double,
                                         float*);

}  // namespace di
