// Index-build kernels (Sections 3, 4.1, 4.2): sample covariance for the
// correlation check, k-means assignment and update per half-codebook, stable
// CSR counting sort, and sign codes.  Row rotation reuses k_rotate_rows.
#pragma once

#include "common.hpp"

namespace crisp {

// Column means of the sampled rows, float64, rows in ascending sample order.
__global__ void k_sample_mean(const float *__restrict__ x, int d, const int64_t *__restrict__ rows, long long s,
                              double *__restrict__ mean) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double acc = 0.0;
  for (long long i = 0; i < s; ++i) acc = acc + static_cast<double>(x[rows[i] * d + j]);
  mean[j] = acc / static_cast<double>(s);
}

// cov[i][j] = sum_s (x_si - mu_i)(x_sj - mu_j) / (S - 1), 64x64 tiles.
__global__ void __launch_bounds__(256) k_covariance(const float *__restrict__ x, int d, const int64_t *__restrict__ rows,
                                                    long long s, const double *__restrict__ mean,
                                                    double *__restrict__ cov) {
  __shared__ double sa[16][65];
  __shared__ double sb[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (long long k0 = 0; k0 < s; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      int kk = e / 64, cc = e % 64;
      long long kr = k0 + kk;
      double va = 0.0, vb = 0.0;
      if (kr < s) {
        const float *row = x + rows[kr] * d;
        va = static_cast<double>(row[i0 + cc]) - mean[i0 + cc];
        vb = static_cast<double>(row[j0 + cc]) - mean[j0 + cc];
      }
      sa[kk][cc] = va;
      sb[kk][cc] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) { a[t] = sa[kk][ty * 4 + t]; b[t] = sb[kk][tx * 4 + t]; }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[p][r] = fma(a[p], b[r], acc[p][r]);
    }
    __syncthreads();
  }
  const double inv = 1.0 / static_cast<double>(s - 1);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      cov[static_cast<long long>(i0 + ty * 4 + p) * d + j0 + tx * 4 + r] = acc[p][r] * inv;
}

// Nearest centroid of one half, lowest index on ties; float64 half distance
// accumulated in ascending coordinate order (unfused).
__global__ void k_assign(const float *__restrict__ x, int d, int col0, int h, const int64_t *__restrict__ rows,
                         long long s, const float *__restrict__ cent, int k, int32_t *__restrict__ label) {
  extern __shared__ float sc[];  // k * h
  for (int i = threadIdx.x; i < k * h; i += blockDim.x) sc[i] = cent[i];
  __syncthreads();
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= s) return;
  long long r = rows ? rows[t] : t;
  const float *a = x + r * d + col0;
  double best = 0.0;
  int arg = 0;
  for (int c = 0; c < k; ++c) {
    const float *cc = sc + c * h;
    double acc = 0.0;
    for (int i = 0; i < h; ++i) {
      double delta = static_cast<double>(a[i]) - static_cast<double>(cc[i]);
      double sq = delta * delta;
      acc = acc + sq;
    }
    if (c == 0 || acc < best) { best = acc; arg = c; }
  }
  label[t] = arg;
}

// Lloyd update: thread per (cluster, coordinate); members ascending.
__global__ void k_update(const float *__restrict__ x, int d, int col0, int h, const int64_t *__restrict__ rows,
                         const int32_t *__restrict__ moff, const int32_t *__restrict__ members, int k,
                         float *__restrict__ cent) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * h) return;
  int c = t / h, i = t % h;
  int a = moff[c], b = moff[c + 1];
  if (b <= a) return;
  // The members' values are loaded 16 at a time (their loads do not depend
  // on the sum) and added in ascending member order, one at a time.
  constexpr int U = 16;
  double acc = 0.0;
  for (int p0 = a; p0 < b; p0 += U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = min(p0 + u, b - 1);  // clamped: every load is issued
      const long long r = rows ? rows[members[p]] : members[p];
      v[u] = x[r * d + col0 + i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (p0 + u < b) acc = acc + static_cast<double>(v[u]);
  }
  cent[t] = static_cast<float>(acc / static_cast<double>(b - a));
}

__global__ void k_combine(const int32_t *__restrict__ l, const int32_t *__restrict__ r, long long n, int k,
                          int32_t *__restrict__ cell) {
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) cell[t] = l[t] * k + r[t];
}

// ---- stable counting sort: per-block cell counts, cell-major scan, then each
// block places its ids in ascending order from its own cursors.
__global__ void k_csr_count(const int32_t *__restrict__ cell_of, long long n, int cells, int blk,
                            int32_t *__restrict__ table /* nblk * cells */) {
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  long long b = t / blk;
  atomicAdd(&table[b * cells + cell_of[t]], 1);
}

// One thread per cell: cursor[b][c] = exclusive prefix over blocks; totals.
__global__ void k_csr_scan_blocks(int32_t *__restrict__ table, int nblk, int cells, int32_t *__restrict__ totals) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  int run = 0;
  for (int b = 0; b < nblk; ++b) {
    int v = table[static_cast<long long>(b) * cells + c];
    table[static_cast<long long>(b) * cells + c] = run;
    run += v;
  }
  totals[c] = run;
}

// Single block: offsets = exclusive scan of totals.
__global__ void k_csr_offsets(const int32_t *__restrict__ totals, int cells, int32_t *__restrict__ offsets) {
  __shared__ int tmp[17];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < cells; c0 += blockDim.x) {
    int c = c0 + threadIdx.x;
    int v = (c < cells) ? totals[c] : 0;
    int incl = wave_incl_scan_i32(v);
    if (lane_id() == kWave - 1) tmp[wave_id()] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int run = 0;
      for (int w = 0; w < static_cast<int>(blockDim.x) / kWave; ++w) { int t = tmp[w]; tmp[w] = run; run += t; }
      tmp[16] = run;
    }
    __syncthreads();
    if (c < cells) offsets[c] = carry + tmp[wave_id()] + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tmp[16];
    __syncthreads();
  }
  if (threadIdx.x == 0) offsets[cells] = carry;
}

__global__ void k_csr_place(const int32_t *__restrict__ cell_of, long long n, int cells, int blk,
                            const int32_t *__restrict__ offsets, int32_t *__restrict__ table,
                            int32_t *__restrict__ ids) {
  long long b = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  long long nblk = (n + blk - 1) / blk;
  if (b >= nblk) return;
  int32_t *cur = table + b * cells;
  long long e = min(n, (b + 1) * blk);
  for (long long t = b * blk; t < e; ++t) {
    int c = cell_of[t];
    int p = offsets[c] + cur[c];
    cur[c] += 1;
    ids[p] = static_cast<int32_t>(t);
  }
}

// Sign codes: one wave per (row, 64-dim word) via ballot, striding over all
// n * D / 64 words (the grid is capped: a dispatch holds < 2^32 threads).
__global__ void k_codes(const float *__restrict__ x, long long n, int d, uint64_t *__restrict__ codes) {
  const int words = d / 64;
  const long long total = n * words;
  const long long step = static_cast<long long>(gridDim.x) * (blockDim.x / kWave);
  for (long long w = static_cast<long long>(blockIdx.x) * (blockDim.x / kWave) + wave_id(); w < total; w += step) {
    const long long r = w / words;
    const int c = static_cast<int>(w % words);
    const unsigned long long b = __ballot(x[r * d + c * 64 + lane_id()] > 0.0f);
    if (lane_id() == 0) codes[w] = b;
  }
}

}  // namespace crisp
