// Shared device helpers for the CRISP gfx950 kernels.
//
// The whole library is compiled with -ffp-contract=off: every float64
// expression that defines a canonical value (rotation, half distance,
// distance key) is evaluated exactly as written, one rounding per operation.
// Fused multiply-adds appear only where they are spelled out (fmaf in the
// float32 first-pass distance, whose error is bounded separately).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "crisp.h"

namespace crisp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

// Inclusive prefix sum across the 64 lanes.
__device__ __forceinline__ int wave_incl_scan_i32(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    int u = __shfl_up(v, s, kWave);
    if (lane >= s) v += u;
  }
  return v;
}

// The same inclusive prefix sum on DPP lane moves (every lane active): four
// in-row steps (row_shr 1, 2, 4, 8; lanes shifted in from outside the row
// add 0), then lane 15 of rows 0 and 2 is added to rows 1 and 3 (row_bcast
// 15) and lane 31 to rows 2 and 3 (row_bcast 31).
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
  return v;
}

__device__ __forceinline__ unsigned long long lanes_below_mask() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// bfloat16 bits of a finite float32, round to nearest even.
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// Lane l's value of a double (l wave-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), l));
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | lo);
}

// Bits of a non-negative double: monotone as an unsigned integer.
__device__ __forceinline__ unsigned long long dbits(double x) {
  return static_cast<unsigned long long>(__double_as_longlong(x));
}
__device__ __forceinline__ double from_dbits(unsigned long long b) {
  return __longlong_as_double(static_cast<long long>(b));
}

// Block-wide exclusive scan of `n` ints held in LDS (in place); each thread
// scans ceil(n / blockDim) consecutive entries.
// Returns the total.  All threads of the block must call it.
__device__ inline int block_exclusive_scan(int *a, int n, int *tmp /* >= blockDim/64 + 1 ints */) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int b = tid * per;
  int local = 0;
  for (int i = 0; i < per; ++i)
    if (b + i < n) local += a[b + i];
  int incl = wave_incl_scan_i32(local);
  if (lane_id() == kWave - 1) tmp[wave_id()] = incl;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    const int nw = nt / kWave;
    for (int w = 0; w < nw; ++w) {
      int t = tmp[w];
      tmp[w] = run;
      run += t;
    }
    tmp[nw] = run;
  }
  __syncthreads();
  int run = tmp[wave_id()] + incl - local;
  for (int i = 0; i < per; ++i) {
    if (b + i < n) {
      int t = a[b + i];
      a[b + i] = run;
      run += t;
    }
  }
  int total = tmp[nt / kWave];
  __syncthreads();
  return total;
}

// The dispatcher deals consecutive workgroups of a 1-D grid to the eight
// XCDs in turn (workgroup b to XCD b % 8), and each XCD has its own L2.  For a
// grid padded to a multiple of 8, xcd_major(b) gives XCD x the contiguous
// range [x * nb / 8, (x + 1) * nb / 8) of logical blocks, so that neighbouring
// logical blocks (which read overlapping rows) share one L2.  A bijection of
// [0, nb); logical blocks past the real count simply exit.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_pad(int nb) { return (nb + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_major(int b, int nb_padded) {
  return (b % kXcds) * (nb_padded / kXcds) + b / kXcds;
}

// Largest j in [0, n) with a[j] <= v, for non-decreasing a with a[0] <= v.
__device__ __forceinline__ int upper_bound_minus1(const int *a, int n, int v) {
  int lo = 0, hi = n;  // first index with a[idx] > v
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

}  // namespace crisp
