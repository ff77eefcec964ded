// Device helpers shared by the cycle kernels: lane exchanges and fixed-order
// wave and block sums, record folds, and the stop test with its next
// control-block copy. Device code only; included by the HIP sources.
#pragma once

#include "di_internal.h"

namespace di {
namespace dev {

__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return (double)x; }

__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// A control block into pinned host memory, one 64-bit system-scope store
// per word (written through to the host, not held in the device's caches):
// the host reads it once the launch has completed, with no copy queued
// behind the launch.
static_assert(sizeof(Ctl) % 8 == 0, "the control block in whole 64-bit words");
__device__ inline void store_ctl_host(Ctl* dst, const Ctl& c) {
  const auto* src = reinterpret_cast<const unsigned long long*>(&c);
  auto* out = reinterpret_cast<unsigned long long*>(dst);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(Ctl) / 8); ++k)
    __hip_atomic_store(out + k, src[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Lane exchanges by DPP, an operand modifier of the vector ALU (no LDS
// round trip). Each control used here permutes lanes within groups of 2, 4,
// 8 or 16, so every lane has a source; the whole wave must be active.
template <int CTRL>
__device__ inline uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL, typename V>
__device__ inline V dpp(V v) {
  static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, dpp32<CTRL>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = dpp32<CTRL>((uint32_t)u), hi = dpp32<CTRL>((uint32_t)(u >> 32));
    return __builtin_bit_cast(V, lo | (hi << 32));
  }
}
// The value of lane `src` (uniform across the wave), in every lane.
template <typename V>
__device__ inline V read_lane(V v, int src) {
  static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
    return __builtin_bit_cast(V, lo | (hi << 32));
  }
}
// Sum over each 16-lane row, held by every lane of the row: partners at
// xor 1 and xor 2 (quad permutations), then the mirrored lane in the other
// half of each 8- and 16-lane group. Partners add the same two numbers, so
// they agree exactly; the order of additions is fixed.
template <typename V>
__device__ inline V row_sum16(V v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}
// Sum over the 64 lanes of a wave, the same number in every lane (the four
// row sums added in a fixed order).
template <typename V>
__device__ inline V wave_sum(V v) {
  v = row_sum16(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}
// Sum of lanes [0, NW) of a wave whose other lanes hold zero (NW <= 16), in
// every lane.
template <int NW, typename V>
__device__ inline V low_lanes_sum(V v) {
  static_assert(NW >= 1 && NW <= 16, "at most one row");
  return read_lane(row_sum16(v), 0);
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

__device__ inline void part_add(Part& a, const Part& b) {
  a.pabs += b.pabs;
  a.psum += b.psum;
  a.e += b.e;
  a.ops += b.ops;
  a.sel += b.sel;
  a.nfront += b.nfront;
}

// Block sum of a Part (fixed order); valid in thread 0. lds: blockDim.x/64.
__device__ Part block_sum_part(Part v, Part* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v.pabs = wave_sum(v.pabs);
  v.psum = wave_sum(v.psum);
  v.e = wave_sum(v.e);
  v.ops = wave_sum(v.ops);
  v.sel = wave_sum(v.sel);
  v.nfront = wave_sum(v.nfront);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  Part t{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) part_add(t, lds[w]);
  __syncthreads();
  return t;
}

// Block sum of a Part for a block of NW waves: wave sums, then wave 0 folds
// the NW wave sums (lanes < NW). Fixed order; valid in thread 0. The link and frontier counts are summed only
// when `counts` (they feed the control block, which block 0 writes).
template <int NW>
__device__ Part block_sum_part_w0(Part v, Part* lds, bool counts) {
  static_assert((NW & (NW - 1)) == 0 && NW <= 64, "NW: a power of two <= 64");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v.pabs = wave_sum(v.pabs);
  v.psum = wave_sum(v.psum);
  v.e = wave_sum(v.e);
  v.sel = wave_sum(v.sel);
  if (counts) {
    v.ops = wave_sum(v.ops);
    v.nfront = wave_sum(v.nfront);
  }
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  Part t{0.0, 0.0, 0.0, 0ull, 0u, 0u};
  if (wave == 0) {
    if (lane < NW) t = lds[lane];
    t.pabs = low_lanes_sum<NW>(t.pabs);
    t.psum = low_lanes_sum<NW>(t.psum);
    t.e = low_lanes_sum<NW>(t.e);
    t.sel = low_lanes_sum<NW>(t.sel);
    if (counts) {
      t.ops = low_lanes_sum<NW>(t.ops);
      t.nfront = low_lanes_sum<NW>(t.nfront);
    }
  }
  return t;
}

// The stop test and the next control-block copy, from the sums of the
// records (v) and the current copy (c). first: no cycle has run yet.
// tol_rel >= 0 marks the FP32 pass of a refined solve: only the first
// selection may declare convergence (its r is the FP64 residual of X);
// after a cycle the pass ends (done = 4) once r <= max(tol_in,
// tol_rel * r_start).
__device__ inline Ctl next_ctl(Ctl c, const Part& v, int first, double d, double tol,
                               double tol_in, double tol_rel, int method, int stop,
                               int max_cycles) {
  if (c.done) return c;
  if (!first) {
    const double r_used = c.r;
    c.cycles += 1;
    if (c.cycles == 1) c.r_first = r_used;
    c.r_last = r_used;
    c.edges_total += v.ops;
    c.front_total += v.nfront;
    c.sel_total += v.sel;
    c.e += v.e;
    // a DI-SOP cycle that diffused nothing (possible only through rounding
    // at a tie) is followed by one DI-CYC cycle
    const bool empty = v.sel == 0 && v.pabs > 0.0;
    c.cyc_mode = method == DI_PI ? 2 : ((method == DI_CYC || empty) ? 1 : 0);
    if (method == DI_SOP && empty) c.fallback += 1;
  } else {
    c.cyc_mode = method == DI_PI ? 2 : (method == DI_CYC ? 1 : 0);
  }
  const double r = v.pabs;
  c.r = r;
  c.psum = v.psum;
  if (!isfinite(r)) {
    c.final_r = r;
    c.done = 3;
    return c;
  }
  if (first) {
    c.r_start = r;
    c.t_start = wall_clock64();
  }
  // r is an FP64 residual except inside the FP32 pass of a refined run,
  // where only the first selection's is
  if (c.t_1e9 == 0 && r <= 1e-9 && (tol_rel < 0.0 || first)) c.t_1e9 = wall_clock64();
  bool stop_now;
  if (stop == DI_STOP_RESID) {
    if (tol_rel >= 0.0 && !first) {
      if (r <= fmax(tol_in, tol_rel * c.r_start)) {
        c.final_r = r;
        c.done = 4;
        return c;
      }
      stop_now = false;
    } else {
      stop_now = r <= tol;
    }
  } else {
    stop_now = false;
    if (!first) {
      c.paper_err = v.psum / (1.0 - d - d * c.e);
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
  return c;
}

}  // namespace dev
}  // namespace di
