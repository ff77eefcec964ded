// HIP kernels of one frontier-synchronous D-iteration cycle on gfx950.
//
// Every cycle runs the selection rule of DI-SOP (Sections 2.3 and 2.5.5)
// against r = sum_i |F_i| of the fluid at the start of the cycle, claims the
// selected nodes (Section 2.5.4: H_i += transit, F_i = 0, dangling fluid
// absorbed), and then moves the claimed fluid along the links. Fluid that
// arrives during the cycle waits for the next one, so the selected set and
// the moved amounts depend only on the state at the start of the cycle.
//
// The move has two implementations with identical results:
//   pull  each node sums sent[i] over its in-links (CSC without self-loops),
//         staged through LDS in work items of at most kPullChunk links;
//         in-link lists longer than that are split into segments whose sums
//         the finalize kernel adds. No atomics; the result is deterministic.
//   push  each selected node's out-links (CSR) receive transit*d/out_i by
//         device-scope float atomics; a select block's frontier is pushed
//         by the push block of the same index, link-balanced through LDS.
// A single-block finalize kernel then sums the per-block partials in a fixed
// order into r (the residual |B + P.H - H|_1 = sum |F|), accumulates the
// statistics and runs the stop test. Only it writes the control block while
// cycles run; every kernel returns at once after the stop, so the host may
// queue cycles ahead of the test.

#include "di_internal.h"

namespace di {
namespace {

__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return (double)x; }

__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// Butterfly sum over the 64 lanes of a wave: every lane gets the total, and
// the order of additions is fixed.
template <typename V>
__device__ inline V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum (blockDim.x a multiple of 64, at most 1024); the result is
// valid in thread 0. Fixed order. lds holds blockDim.x / 64 values.
template <typename V>
__device__ V block_sum(V v, V* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  V total = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) total += lds[w];
  __syncthreads();
  return total;
}

__global__ void k_reset_ctl(Ctl* ctl) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->r = 0.0;
    ctl->psum = 0.0;
    ctl->e = 0.0;
    ctl->final_r = 0.0;
    ctl->paper_err = 0.0;
    ctl->r_first = 0.0;
    ctl->r_last = 0.0;
    ctl->cycles = 0;
    ctl->fallback = 0;
    ctl->done = 0;
    ctl->cyc_mode = 0;
    ctl->edges_total = 0;
    ctl->front_total = 0;
    ctl->sel_total = 0;
  }
}

// F = B, H = 0, and per-block partial sums of |F| and F over all nodes.
template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_start(T* __restrict__ F, T* __restrict__ H,
                                                        const double* __restrict__ B,
                                                        double b_uniform, int64_t n,
                                                        double* __restrict__ blk_pabs,
                                                        double* __restrict__ blk_psum) {
  __shared__ double lds[kReduceBlock / 64];
  double pa = 0.0, ps = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T f = B ? (T)B[i] : (T)b_uniform;
    F[i] = f;
    H[i] = (T)0;
    pa += fabs(to_d(f));
    ps += to_d(f);
  }
  pa = block_sum(pa, lds);
  ps = block_sum(ps, lds);
  if (threadIdx.x == 0) {
    blk_pabs[blockIdx.x] = pa;
    blk_psum[blockIdx.x] = ps;
  }
}

// Per-block partial sums of |F| and F (push direction, after the push).
template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_reduce(const T* __restrict__ F, int64_t n,
                                                         double* __restrict__ blk_pabs,
                                                         double* __restrict__ blk_psum,
                                                         const Ctl* __restrict__ ctl) {
  __shared__ double lds[kReduceBlock / 64];
  if (ctl->done) return;
  double pa = 0.0, ps = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double f = to_d(F[i]);
    pa += fabs(f);
    ps += f;
  }
  pa = block_sum(pa, lds);
  ps = block_sum(ps, lds);
  if (threadIdx.x == 0) {
    blk_pabs[blockIdx.x] = pa;
    blk_psum[blockIdx.x] = ps;
  }
}

// Selection and claim. Thread t of block b owns the nodes
// b*kSelectNodes + t + m*kSelectBlock, m < kSelectPerThread (coalesced).
// PULL: writes sent[i] (0 for nodes not diffused) for every node.
// PUSH: writes the block's frontier (nodes with links to push) at
//       [b*kSelectNodes, ...) with block-local link offsets that grow with
//       the entry index.
template <typename T, bool PULL>
__global__ __launch_bounds__(kSelectBlock) void k_select(
    T* __restrict__ F, T* __restrict__ H, const uint32_t* __restrict__ info,
    const int64_t* __restrict__ row_ptr, int64_t n, int64_t L, double d,
    T* __restrict__ sent, int64_t* __restrict__ fr_lstart, int64_t* __restrict__ fr_base,
    T* __restrict__ fr_s, SelStat* __restrict__ blk_stat, const Ctl* __restrict__ ctl) {
  constexpr int M = kSelectPerThread;
  constexpr int NW = kSelectBlock / 64;
  __shared__ unsigned long long s_ops[NW];
  __shared__ double s_e[NW];
  __shared__ unsigned int s_sel[NW], s_front[NW];
  if (ctl->done) return;
  const double r = ctl->r;
  const bool cyc = ctl->cyc_mode != 0;
  const double rl = r / (double)L;

  const int64_t base = (int64_t)blockIdx.x * kSelectNodes + threadIdx.x;
  double f[M];
  uint32_t w[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int64_t i = base + (int64_t)m * kSelectBlock;
    f[m] = i < n ? to_d(F[i]) : 0.0;
    w[m] = i < n ? info[i] : 0u;
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
    const int64_t i = base + (int64_t)m * kSelectBlock;
    if (i < n) {
      const int out = (int)(w[m] & kOutMask);
      const bool loop = (w[m] & kLoopBit) != 0;
      const double a = fabs(f[m]);
      const double thr = (cyc || out == 0) ? 0.0 : rl * (double)out;
      if (a > 0.0 && a >= thr) {
        const double t = loop ? f[m] * (double)out / ((double)out - d) : f[m];
        H[i] = (T)(to_d(H[i]) + t);
        F[i] = (T)0;
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
      }
      if (PULL) sent[i] = (T)snd[m];
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (!PULL) {
    // block-local exclusive scan of (entries, links) over (thread, m) order
    unsigned int cnt_incl = my_front;
    unsigned long long lnk_incl = my_ops;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned int u = __shfl_up(cnt_incl, off, 64);
      const unsigned long long v = __shfl_up(lnk_incl, off, 64);
      if (lane >= off) {
        cnt_incl += u;
        lnk_incl += v;
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
    const int64_t fbase = (int64_t)blockIdx.x * kSelectNodes;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (npush[m] > 0) {
        fr_lstart[fbase + k] = (int64_t)lo;
        fr_base[fbase + k] = row_ptr[base + (int64_t)m * kSelectBlock];
        fr_s[fbase + k] = (T)snd[m];
        ++k;
        lo += (unsigned long long)npush[m];
      }
    }
  }
  // one fused block reduction of the four statistics
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
  if (threadIdx.x == 0) {
    SelStat st;
    st.sel = 0;
    st.nfront = 0;
    st.ops = 0;
    st.e = 0.0;
    for (int q = 0; q < NW; ++q) {
      st.sel += s_sel[q];
      st.nfront += s_front[q];
      st.ops += s_ops[q];
      st.e += s_e[q];
    }
    blk_stat[blockIdx.x] = st;
  }
}

// Pull: F_j += sum of sent[i] over the in-links i -> j (i != j). Work items
// are prepared with the graph: light items (rows [r0, r1), at most
// kPullChunk links) and segments of heavy rows. Each thread stages its
// kPullChunk / kPullBlock links with all index loads, then all gathers, in
// flight together. Per-block partial sums of |F| and F cover the light
// rows; heavy rows are finished by k_finalize.
template <typename T>
__global__ __launch_bounds__(kPullBlock) void k_pull(
    T* __restrict__ F, const T* __restrict__ sent, const int64_t* __restrict__ csc_ptr,
    const int32_t* __restrict__ csc_idx, const int64_t* __restrict__ it_r0,
    const int64_t* __restrict__ it_r1, const int64_t* __restrict__ it_l0,
    const int64_t* __restrict__ it_l1, const int32_t* __restrict__ it_seg, int64_t n_items,
    double* __restrict__ seg_val, double* __restrict__ blk_pabs, double* __restrict__ blk_psum,
    const Ctl* __restrict__ ctl) {
  constexpr int U = kPullChunk / kPullBlock;
  __shared__ double s_val[kPullChunk];
  __shared__ double s_red[kPullBlock / 64];
  if (ctl->done) return;
  const int tid = threadIdx.x;
  double pa = 0.0, ps = 0.0;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int64_t l0 = it_l0[it], l1 = it_l1[it];
    const int seg = it_seg[it];
    const int nl = (int)(l1 - l0);
    const int64_t r0 = it_r0[it], r1 = it_r1[it];
    // the thread's first row, fetched while the links are in flight
    const int64_t row0 = r0 + tid;
    double f0 = 0.0;
    int a0 = 0, b0 = 0;
    if (seg < 0 && row0 < r1) {
      f0 = to_d(F[row0]);
      a0 = (int)(csc_ptr[row0] - l0);
      b0 = (int)(csc_ptr[row0 + 1] - l0);
    }
    int32_t idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      idx[u] = p < nl ? csc_idx[l0 + p] : 0;
    }
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tid + u * kPullBlock;
      v[u] = p < nl ? to_d(sent[idx[u]]) : 0.0;
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
    // rows r0 + tid + k * kPullBlock; a row with more than kPullLongRow links
    // is summed by its whole wave (strided lanes, then a butterfly)
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
        const int la = __shfl(a, src, 64), lb = __shfl(b, src, 64);
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
        pa += fabs(f);
        ps += f;
      }
    }
    __syncthreads();
  }
  pa = block_sum(pa, s_red);
  ps = block_sum(ps, s_red);
  if (tid == 0) {
    blk_pabs[blockIdx.x] = pa;
    blk_psum[blockIdx.x] = ps;
  }
}

// Push: block b moves the frontier of select block b. Entries are staged in
// LDS; each lane finds the entry of its link by binary search on the local
// link offsets and adds the entry's amount to F[col] atomically.
template <typename T>
__global__ __launch_bounds__(kPushBlock) void k_push(T* __restrict__ F,
                                                     const int32_t* __restrict__ col,
                                                     const int64_t* __restrict__ fr_lstart,
                                                     const int64_t* __restrict__ fr_base,
                                                     const T* __restrict__ fr_s,
                                                     const SelStat* __restrict__ blk_stat,
                                                     const Ctl* __restrict__ ctl) {
  __shared__ int64_t s_start[kSelectNodes];
  __shared__ int64_t s_base[kSelectNodes];
  __shared__ T s_val[kSelectNodes];
  if (ctl->done) return;
  const int nf = (int)blk_stat[blockIdx.x].nfront;
  if (nf == 0) return;
  const int64_t E = (int64_t)blk_stat[blockIdx.x].ops;
  const int64_t fbase = (int64_t)blockIdx.x * kSelectNodes;
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

// Single block: finishes heavy rows (pull), sums every partial in a fixed
// order into r = sum |F| and sum F, accumulates the cycle's statistics and
// runs the stop test. start != 0: the test before the first cycle (no
// selection happened; the partials come from k_start / k_reduce).
template <typename T>
__global__ __launch_bounds__(kFinalBlock) void k_finalize(
    T* __restrict__ F, const int32_t* __restrict__ heavy_row, const int64_t* __restrict__ heavy_seg,
    const int64_t* __restrict__ hb_h0, const int64_t* __restrict__ hb_h1, int64_t n_hbatch,
    const double* __restrict__ seg_val, const double* __restrict__ blk_pabs,
    const double* __restrict__ blk_psum, int nparts, const SelStat* __restrict__ blk_stat,
    int nsel, int start, double d, double tol, int method, int stop, int max_cycles,
    Ctl* __restrict__ ctl) {
  __shared__ double s_seg[kFinalSegBatch];
  __shared__ double s_red[kFinalBlock / 64];
  __shared__ unsigned long long s_red64[kFinalBlock / 64];
  if (ctl->done) return;
  const int tid = threadIdx.x;
  double pa = 0.0, ps = 0.0;
  if (!start) {
    for (int64_t b = 0; b < n_hbatch; ++b) {
      const int64_t h0 = hb_h0[b], h1 = hb_h1[b];
      const int64_t s0 = heavy_seg[h0], s1 = heavy_seg[h1];
      const int64_t ns = s1 - s0;
      if (ns > kFinalSegBatch) {
        // one row with many segments: a block-wide sum
        double acc = 0.0;
        for (int64_t s = s0 + tid; s < s1; s += blockDim.x) acc += seg_val[s];
        acc = block_sum(acc, s_red);
        if (tid == 0) {
          const int32_t row = heavy_row[h0];
          double f = to_d(F[row]);
          if (acc != 0.0) {
            const T nv = (T)(f + acc);
            F[row] = nv;
            f = to_d(nv);
          }
          pa += fabs(f);
          ps += f;
        }
        continue;
      }
      for (int64_t q = tid; q < ns; q += blockDim.x) s_seg[q] = seg_val[s0 + q];
      __syncthreads();
      for (int64_t h = h0 + tid; h < h1; h += blockDim.x) {
        const int32_t row = heavy_row[h];
        double acc = 0.0;
        for (int64_t s = heavy_seg[h]; s < heavy_seg[h + 1]; ++s) acc += s_seg[s - s0];
        double f = to_d(F[row]);
        if (acc != 0.0) {
          const T nv = (T)(f + acc);
          F[row] = nv;
          f = to_d(nv);
        }
        pa += fabs(f);
        ps += f;
      }
      __syncthreads();
    }
  }
  for (int p = tid; p < nparts; p += blockDim.x) {
    pa += blk_pabs[p];
    ps += blk_psum[p];
  }
  double e_c = 0.0;
  unsigned long long sel = 0, front = 0, ops = 0;
  if (!start) {
    for (int b = tid; b < nsel; b += blockDim.x) {
      const SelStat st = blk_stat[b];
      sel += st.sel;
      front += st.nfront;
      ops += st.ops;
      e_c += st.e;
    }
  }
  const double r = block_sum(pa, s_red);
  const double psum = block_sum(ps, s_red);
  e_c = block_sum(e_c, s_red);
  sel = block_sum(sel, s_red64);
  front = block_sum(front, s_red64);
  ops = block_sum(ops, s_red64);
  if (tid != 0) return;
  Ctl c = *ctl;
  if (!start) {
    const double r_used = c.r;
    c.cycles += 1;
    if (c.cycles == 1) c.r_first = r_used;
    c.r_last = r_used;
    c.edges_total += ops;
    c.front_total += front;
    c.sel_total += sel;
    c.e += e_c;
    // a DI-SOP cycle that diffused nothing (possible only through rounding
    // at a tie) is followed by one DI-CYC cycle
    const bool empty = sel == 0 && r > 0.0;
    c.cyc_mode = (method == DI_CYC || empty) ? 1 : 0;
    if (method != DI_CYC && empty) c.fallback += 1;
  } else {
    c.cyc_mode = method == DI_CYC ? 1 : 0;
  }
  c.r = r;
  c.psum = psum;
  if (!isfinite(r)) {
    c.final_r = r;
    c.done = 3;
  } else {
    bool stop_now;
    if (stop == DI_STOP_RESID) {
      stop_now = r <= tol;
    } else {
      stop_now = false;
      if (!start) {
        c.paper_err = psum / (1.0 - d - d * c.e);
        stop_now = c.paper_err <= tol;
      }
    }
    if (stop_now) {
      c.final_r = r;
      c.done = 1;
    } else if (c.cycles >= max_cycles) {
      c.final_r = r;
      c.done = 2;
    }
  }
  *ctl = c;
}

template <typename T>
__global__ void k_h_to_x(const T* __restrict__ H, double* __restrict__ X, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    X[i] = to_d(H[i]);
}

inline unsigned int grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned int)g;
}

template <typename T>
hipError_t launch_finalize(const CycleArgs& a, int nparts, int start) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  const bool pull = a.direction == kPull;
  hipLaunchKernelGGL(k_finalize<T>, dim3(1), dim3(kFinalBlock), 0, a.stream, (T*)ws->F,
                     g->heavy_row, g->heavy_seg, g->hb_h0, g->hb_h1,
                     pull ? g->n_hbatch : (int64_t)0, ws->seg_val, ws->blk_pabs, ws->blk_psum,
                     nparts, ws->blk_stat, (int)grid_for(g->n, kSelectNodes, 0x7fffffff), start,
                     a.d, a.tol, a.method, a.stop, a.max_cycles, ws->ctl);
  return hipGetLastError();
}

}  // namespace

int select_grid(int64_t n) { return (int)grid_for(n, kSelectNodes, 0x7fffffff); }

int pull_grid(const di_graph* g) { return (int)grid_for(g->n_items, 1, kPullMaxGrid); }

int reduce_grid(int64_t n) { return (int)grid_for(n, kReduceBlock, kReduceGrid); }

hipError_t launch_reset_ctl(const CycleArgs& a) {
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, a.stream, a.ws->ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_start(const CycleArgs& a, const double* B, double b_uniform) {
  const int grid = reduce_grid(a.g->n);
  hipLaunchKernelGGL(k_start<T>, dim3(grid), dim3(kReduceBlock), 0, a.stream, (T*)a.ws->F,
                     (T*)a.ws->H, B, b_uniform, a.g->n, a.ws->blk_pabs, a.ws->blk_psum);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_finalize<T>(a, grid, 1);
}

template <typename T>
hipError_t launch_start_state(const CycleArgs& a) {
  const int grid = reduce_grid(a.g->n);
  hipLaunchKernelGGL(k_reduce<T>, dim3(grid), dim3(kReduceBlock), 0, a.stream, (const T*)a.ws->F,
                     a.g->n, a.ws->blk_pabs, a.ws->blk_psum, a.ws->ctl);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_finalize<T>(a, grid, 1);
}

template <typename T>
hipError_t launch_cycle(const CycleArgs& a, hipEvent_t ev0, hipEvent_t ev1) {
  const di_graph* g = a.g;
  Workspace* ws = a.ws;
  const int sgrid = select_grid(g->n);
  hipError_t err;
  if (a.direction == kPull) {
    hipLaunchKernelGGL((k_select<T, true>), dim3(sgrid), dim3(kSelectBlock), 0, a.stream,
                       (T*)ws->F, (T*)ws->H, g->info, g->row_ptr, g->n, g->L, a.d, (T*)ws->sent,
                       (int64_t*)nullptr, (int64_t*)nullptr, (T*)nullptr, ws->blk_stat, ws->ctl);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (ev0 && (err = hipEventRecord(ev0, a.stream)) != hipSuccess) return err;
    const int pgrid = pull_grid(g);
    hipLaunchKernelGGL(k_pull<T>, dim3(pgrid), dim3(kPullBlock), 0, a.stream, (T*)ws->F,
                       (const T*)ws->sent, g->csc_ptr, g->csc_idx, g->it_r0, g->it_r1, g->it_l0,
                       g->it_l1, g->it_seg, g->n_items, ws->seg_val, ws->blk_pabs, ws->blk_psum,
                       ws->ctl);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (ev1 && (err = hipEventRecord(ev1, a.stream)) != hipSuccess) return err;
    return launch_finalize<T>(a, pgrid, 0);
  }
  hipLaunchKernelGGL((k_select<T, false>), dim3(sgrid), dim3(kSelectBlock), 0, a.stream,
                     (T*)ws->F, (T*)ws->H, g->info, g->row_ptr, g->n, g->L, a.d, (T*)nullptr,
                     ws->fr_lstart, ws->fr_base, (T*)ws->fr_s, ws->blk_stat, ws->ctl);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (ev0 && (err = hipEventRecord(ev0, a.stream)) != hipSuccess) return err;
  hipLaunchKernelGGL(k_push<T>, dim3(sgrid), dim3(kPushBlock), 0, a.stream, (T*)ws->F, g->col,
                     ws->fr_lstart, ws->fr_base, (const T*)ws->fr_s, ws->blk_stat, ws->ctl);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (ev1 && (err = hipEventRecord(ev1, a.stream)) != hipSuccess) return err;
  const int rgrid = reduce_grid(g->n);
  hipLaunchKernelGGL(k_reduce<T>, dim3(rgrid), dim3(kReduceBlock), 0, a.stream, (const T*)ws->F,
                     g->n, ws->blk_pabs, ws->blk_psum, ws->ctl);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  return launch_finalize<T>(a, rgrid, 0);
}

template <typename T>
hipError_t launch_h_to_x(const CycleArgs& a, double* X) {
  hipLaunchKernelGGL(k_h_to_x<T>, dim3(grid_for(a.g->n, 256, 4096)), dim3(256), 0, a.stream,
                     (const T*)a.ws->H, X, a.g->n);
  return hipGetLastError();
}

template hipError_t launch_start<double>(const CycleArgs&, const double*, double);
template hipError_t launch_start<float>(const CycleArgs&, const double*, double);
template hipError_t launch_start_state<double>(const CycleArgs&);
template hipError_t launch_start_state<float>(const CycleArgs&);
template hipError_t launch_cycle<double>(const CycleArgs&, hipEvent_t, hipEvent_t);
template hipError_t launch_cycle<float>(const CycleArgs&, hipEvent_t, hipEvent_t);
template hipError_t launch_h_to_x<double>(const CycleArgs&, double*);
template hipError_t launch_h_to_x<float>(const CycleArgs&, double*);

}  // namespace di
