// HIP kernels of one frontier-synchronous D-iteration cycle on gfx950.
//
// A cycle is three launches on one stream:
//   k_reduce  r = sum_i |F_i| (and sum_i F_i) as per-block FP64 partials;
//             block 0 advances the device cycle counter and clears the
//             cycle's frontier counters;
//   k_select  every block sums the partials in the same fixed order (so all
//             blocks agree on r bit for bit), runs the stop test, applies
//             the selection rule of DI-SOP (Sections 2.3 and 2.5.5) and, for
//             each selected node, the claim of Section 2.5.4 (H_i += transit,
//             F_i = 0, dangling fluid absorbed); nodes with links to push are
//             compacted into the frontier with a wave64 scan and one 64-bit
//             atomic per block;
//   k_push    edge-balanced push: tile b covers frontier links
//             [b*kPushTile, (b+1)*kPushTile); the tile's frontier entries are
//             staged in LDS, each lane finds its entry by binary search and
//             adds the entry's amount to F[col] with a device-scope float
//             atomic. Index reads are coalesced within each out-link list.
// Every kernel returns at once when the solve is done, so the host can queue
// cycles ahead of the stop test.

#include "di_internal.h"

namespace di {
namespace {

__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return (double)x; }

__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// Butterfly sum over the 64 lanes of a wave; every lane gets the total and
// the order of additions is fixed.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline unsigned int wave_sum_u32(unsigned int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of the first `count` entries of parts (count <= blockDim.x, blockDim.x
// a multiple of 64 and at most 1024) in a fixed order: the same value in
// every block. lds needs blockDim.x / 64 doubles. Called by all threads.
__device__ double block_sum_fixed(const double* parts, int count, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double v = (int)threadIdx.x < count ? parts[threadIdx.x] : 0.0;
  v = wave_sum(v);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double total = 0.0;
  for (int w = 0; w < nw; ++w) total += lds[w];
  __syncthreads();
  return total;
}

// Block sum of a per-thread double; the result is valid in thread 0.
__device__ double block_sum(double v, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double total = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) total += lds[w];
  __syncthreads();
  return total;
}

__global__ void k_reset_ctl(Ctl* ctl) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->e = 0.0;
    ctl->e_snap = 0.0;
    ctl->final_r = 0.0;
    ctl->paper_err = 0.0;
    ctl->r_last = 0.0;
    ctl->r_first = 0.0;
    for (int s = 0; s < 3; ++s) {
      ctl->packed[s] = 0;
      ctl->sel[s] = 0;
    }
    ctl->cycles = 0;
    ctl->fallback = 0;
    ctl->done = 0;
    ctl->cur = -1;
    ctl->edges_total = 0;
    ctl->front_total = 0;
    ctl->sel_total = 0;
  }
}

template <typename T>
__global__ void k_init(T* __restrict__ F, T* __restrict__ H, const double* __restrict__ B,
                       double b_uniform, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    F[i] = B ? (T)B[i] : (T)b_uniform;
    H[i] = (T)0;
  }
}

template <typename T>
__global__ __launch_bounds__(kReduceBlock) void k_reduce(const T* __restrict__ F, int64_t n,
                                                         double* __restrict__ part_abs,
                                                         double* __restrict__ part_sum,
                                                         Ctl* __restrict__ ctl) {
  __shared__ double lds[kReduceBlock / 64];
  if (ctl->done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int c = ctl->cur + 1;
    ctl->cur = c;
    ctl->packed[c % 3] = 0;
    ctl->sel[c % 3] = 0;
    ctl->e_snap = ctl->e;
  }
  double sa = 0.0, ss = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double f = to_d(F[i]);
    sa += fabs(f);
    ss += f;
  }
  sa = block_sum(sa, lds);
  ss = block_sum(ss, lds);
  if (threadIdx.x == 0) {
    part_abs[blockIdx.x] = sa;
    part_sum[blockIdx.x] = ss;
  }
}

template <typename T>
__global__ __launch_bounds__(kSelectBlock) void k_select(
    T* __restrict__ F, T* __restrict__ H, const uint32_t* __restrict__ info,
    const int64_t* __restrict__ row_ptr, int64_t n, int64_t L, double d, double tol, int method,
    int stop, int max_cycles, const double* __restrict__ part_abs,
    const double* __restrict__ part_sum, int nparts, int64_t* __restrict__ fr_start,
    int64_t* __restrict__ fr_base, T* __restrict__ fr_s, int32_t* __restrict__ tile_first,
    Ctl* __restrict__ ctl) {
  __shared__ double s_red[kSelectBlock / 64];
  __shared__ unsigned long long s_scan[kSelectBlock / 64];
  __shared__ unsigned int s_cnt[kSelectBlock / 64];
  __shared__ unsigned long long s_base;
  constexpr int M = kSelectPerThread;

  if (ctl->done) return;
  const int cycle = ctl->cur;
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  const double r = block_sum_fixed(part_abs, nparts, s_red);
  bool stop_now = false;
  if (stop == DI_STOP_RESID) {
    stop_now = r <= tol;
  } else if (cycle > 0) {
    const double psum = block_sum_fixed(part_sum, nparts, s_red);
    const double perr = psum / (1.0 - d - d * ctl->e_snap);
    if (leader) ctl->paper_err = perr;
    stop_now = perr <= tol;
  }
  if (!isfinite(r)) {
    if (leader) {
      ctl->final_r = r;
      ctl->done = 3;
    }
    return;
  }
  if (stop_now || cycle >= max_cycles) {
    if (leader) {
      ctl->final_r = r;
      ctl->done = stop_now ? 1 : 2;
    }
    return;
  }
  bool cyc = method == DI_CYC;
  if (!cyc && cycle > 0 && ctl->sel[(cycle + 2) % 3] == 0) {
    cyc = true;  // the previous cycle selected nothing: one DI-CYC cycle
    if (leader) ctl->fallback += 1;
  }
  if (leader) {
    ctl->cycles = cycle + 1;
    ctl->r_last = r;
    if (cycle == 0) ctl->r_first = r;
  }
  const int slot = cycle % 3;
  const double rl = r / (double)L;

  const int64_t base = (int64_t)blockIdx.x * kSelectNodes + (int64_t)threadIdx.x * M;
  int npush[M];
  double sent[M];
  unsigned long long mine = 0;
  unsigned int my_sel = 0;
  double my_e = 0.0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    npush[m] = 0;
    sent[m] = 0.0;
    const int64_t i = base + m;
    if (i < n) {
      const double f = to_d(F[i]);
      const uint32_t w = info[i];
      const int out = (int)(w & kOutMask);
      const bool loop = (w & kLoopBit) != 0;
      const double a = fabs(f);
      const double thr = (cyc || out == 0) ? 0.0 : rl * (double)out;
      if (a > 0.0 && a >= thr) {
        const double t = loop ? f * (double)out / ((double)out - d) : f;
        H[i] = (T)(to_d(H[i]) + t);
        F[i] = (T)0;
        ++my_sel;
        if (out == 0) {
          my_e += t;
        } else {
          const int np = out - (loop ? 1 : 0);
          if (np > 0) {
            npush[m] = np;
            sent[m] = t * d / (double)out;
            mine += 1ull + ((unsigned long long)np << kPackShift);
          }
        }
      }
    }
  }

  // exclusive scan of the packed (entries, links) counts in node order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) s_scan[wave] = incl;
  const unsigned int wsel = wave_sum_u32(my_sel);
  if (lane == 0) s_cnt[wave] = wsel;
  __syncthreads();
  unsigned long long before = 0, total = 0;
  unsigned int sel_total = 0;
#pragma unroll
  for (int w = 0; w < kSelectBlock / 64; ++w) {
    if (w < wave) before += s_scan[w];
    total += s_scan[w];
    sel_total += s_cnt[w];
  }
  if (threadIdx.x == 0) {
    s_base = total ? atomicAdd(&ctl->packed[slot], total) : 0ull;
    if (sel_total) atomicAdd(&ctl->sel[slot], sel_total);
  }
  __syncthreads();
  unsigned long long pos = s_base + before + incl - mine;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (npush[m] > 0) {
      const int64_t k = (int64_t)(pos & kPackNodeMask);
      const int64_t es = (int64_t)(pos >> kPackShift);
      fr_start[k] = es;
      fr_base[k] = row_ptr[base + m];
      fr_s[k] = (T)sent[m];
      const int64_t b_lo = (es + kPushTile - 1) / kPushTile;
      const int64_t b_hi = (es + npush[m] - 1) / kPushTile;
      for (int64_t b = b_lo; b <= b_hi; ++b) tile_first[b] = (int32_t)k;
      pos += 1ull + ((unsigned long long)npush[m] << kPackShift);
    }
  }
  const double e_blk = block_sum(my_e, s_red);
  if (threadIdx.x == 0 && e_blk != 0.0) atomicAdd(&ctl->e, e_blk);
}

template <typename T>
__global__ __launch_bounds__(kPushBlock) void k_push(T* __restrict__ F,
                                                     const int32_t* __restrict__ col,
                                                     const int64_t* __restrict__ fr_start,
                                                     const int64_t* __restrict__ fr_base,
                                                     const T* __restrict__ fr_s,
                                                     const int32_t* __restrict__ tile_first,
                                                     Ctl* __restrict__ ctl) {
  __shared__ int32_t s_start[kPushTile + 1];
  __shared__ int64_t s_base[kPushTile + 1];
  __shared__ T s_val[kPushTile + 1];
  if (ctl->done) return;
  const int slot = ctl->cur % 3;
  const unsigned long long packed = ctl->packed[slot];
  const int64_t nfront = (int64_t)(packed & kPackNodeMask);
  const int64_t E = (int64_t)(packed >> kPackShift);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->edges_total += (unsigned long long)E;
    ctl->front_total += (unsigned long long)nfront;
    ctl->sel_total += ctl->sel[slot];
  }
  const int64_t ntiles = (E + kPushTile - 1) / kPushTile;
  for (int64_t b = blockIdx.x; b < ntiles; b += gridDim.x) {
    const int64_t t0 = b * kPushTile;
    const int k0 = tile_first[b];
    const int k1 = (b + 1 < ntiles) ? tile_first[b + 1] : (int)(nfront - 1);
    const int cnt = k1 - k0 + 1;
    for (int q = threadIdx.x; q < cnt; q += kPushBlock) {
      const int64_t es = fr_start[k0 + q];
      s_start[q] = (int32_t)(es - t0);
      s_base[q] = fr_base[k0 + q] - es + t0;
      s_val[q] = fr_s[k0 + q];
    }
    __syncthreads();
    const int lim = (int)((E - t0) < kPushTile ? (E - t0) : kPushTile);
    int lo = 0;
    for (int el = threadIdx.x; el < lim; el += kPushBlock) {
      int hi = cnt - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= el) lo = mid;
        else hi = mid - 1;
      }
      const int32_t j = col[s_base[lo] + el];
      atomic_add(&F[j], s_val[lo]);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void k_h_to_x(const T* __restrict__ H, double* __restrict__ X, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    X[i] = to_d(H[i]);
}

inline unsigned int grid_for(int64_t n, int block, unsigned int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned int)g;
}

}  // namespace

int reduce_parts(int64_t n) {
  int64_t p = (n + 8 * kReduceBlock - 1) / (8 * kReduceBlock);
  if (p < 1) p = 1;
  if (p > kMaxParts) p = kMaxParts;
  return (int)p;
}

int push_grid(int64_t Lp) {
  int64_t g = (Lp + kPushTile - 1) / kPushTile;
  if (g < 1) g = 1;
  if (g > kMaxPushGrid) g = kMaxPushGrid;
  return (int)g;
}

hipError_t launch_reset_ctl(const CycleArgs& a) {
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, a.stream, a.ws->ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const CycleArgs& a, const double* B, double b_uniform) {
  hipLaunchKernelGGL(k_init<T>, dim3(grid_for(a.g->n, 256, 4096)), dim3(256), 0, a.stream,
                     (T*)a.ws->F, (T*)a.ws->H, B, b_uniform, a.g->n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const CycleArgs& a) {
  hipLaunchKernelGGL(k_reduce<T>, dim3(a.nparts), dim3(kReduceBlock), 0, a.stream,
                     (const T*)a.ws->F, a.g->n, a.ws->part_abs, a.ws->part_sum, a.ws->ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_select(const CycleArgs& a) {
  const unsigned int grid = grid_for(a.g->n, kSelectNodes, 0x7fffffffu);
  hipLaunchKernelGGL(k_select<T>, dim3(grid), dim3(kSelectBlock), 0, a.stream, (T*)a.ws->F,
                     (T*)a.ws->H, a.g->info, a.g->row_ptr, a.g->n, a.g->L, a.d, a.tol, a.method,
                     a.stop, a.max_cycles, a.ws->part_abs, a.ws->part_sum, a.nparts,
                     a.ws->fr_start, a.ws->fr_base, (T*)a.ws->fr_s, a.ws->tile_first, a.ws->ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_push(const CycleArgs& a) {
  hipLaunchKernelGGL(k_push<T>, dim3(a.push_grid), dim3(kPushBlock), 0, a.stream, (T*)a.ws->F,
                     a.g->col, a.ws->fr_start, a.ws->fr_base, (const T*)a.ws->fr_s,
                     a.ws->tile_first, a.ws->ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_h_to_x(const CycleArgs& a, double* X) {
  hipLaunchKernelGGL(k_h_to_x<T>, dim3(grid_for(a.g->n, 256, 4096)), dim3(256), 0, a.stream,
                     (const T*)a.ws->H, X, a.g->n);
  return hipGetLastError();
}

template hipError_t launch_init<double>(const CycleArgs&, const double*, double);
template hipError_t launch_init<float>(const CycleArgs&, const double*, double);
template hipError_t launch_reduce<double>(const CycleArgs&);
template hipError_t launch_reduce<float>(const CycleArgs&);
template hipError_t launch_select<double>(const CycleArgs&);
template hipError_t launch_select<float>(const CycleArgs&);
template hipError_t launch_push<double>(const CycleArgs&);
template hipError_t launch_push<float>(const CycleArgs&);
template hipError_t launch_h_to_x<double>(const CycleArgs&, double*);
template hipError_t launch_h_to_x<float>(const CycleArgs&, double*);

}  // namespace di
