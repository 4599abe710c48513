// Query-path kernels of the CRISP engine (Algorithm 1, Sections 4.3.1-4.3.2).
//
//   k_rotate_rows   (A0) x' = x R, float64 ascending-i accumulation per output
//   k_half_dist     (A1) Dist_1 / Dist_2 for every (query, subspace, half, centroid)
//   k_select_cells  (A2) Multi-Sequence cell set + rank weights per (query, subspace)
//   k_count         (A3/A4) LDS collision counters per (query, id tile),
//                   threshold, ordered compaction, score histogram
//   k_flag / k_tau_eff / k_compact (A4) fallback rule and candidate lists
//   k_hamming_order (A5) Hamming distance + stable counting sort
//   k_rerank        (A6/A7) float32 first pass with a proven band, float64
//                   re-check where the band matters, top-k / patience walk
#pragma once

#include "common.hpp"

namespace crisp {

// ---------------------------------------------------------------------------
// A0: rotation.  64x64 output tile per 256-thread block, 4x4 per thread,
// k staged through LDS 16 at a time.  Every output accumulates its D
// products in ascending k in float64 (products of two float32 are exact in
// float64, so the fused form equals the unfused definition).
// ---------------------------------------------------------------------------
constexpr int kRotBM = 64, kRotBN = 64, kRotBK = 16;

__global__ void __launch_bounds__(256) k_rotate_rows(const float *__restrict__ x, long long rows, int d,
                                                     const float *__restrict__ r, float *__restrict__ out) {
  __shared__ float sa[kRotBK][kRotBM + 1];
  __shared__ float sb[kRotBK][kRotBN];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const long long row0 = static_cast<long long>(blockIdx.y) * kRotBM;
  const int col0 = blockIdx.x * kRotBN;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < d; k0 += kRotBK) {
    // A tile: 64 rows x 16 k; 1024 values, 4 per thread.
    for (int e = threadIdx.x; e < kRotBM * kRotBK; e += 256) {
      int rr = e / kRotBK, kk = e % kRotBK;
      long long gr = row0 + rr;
      sa[kk][rr] = (gr < rows) ? x[gr * d + k0 + kk] : 0.0f;
    }
    for (int e = threadIdx.x; e < kRotBK * kRotBN; e += 256) {
      int kk = e / kRotBN, cc = e % kRotBN;
      sb[kk][cc] = r[static_cast<long long>(k0 + kk) * d + col0 + cc];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kRotBK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = static_cast<double>(sa[kk][ty * 4 + i]);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = static_cast<double>(sb[kk][tx * 4 + j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    long long gr = row0 + ty * 4 + i;
    if (gr < rows) {
#pragma unroll
      for (int j = 0; j < 4; ++j) out[gr * d + col0 + tx * 4 + j] = static_cast<float>(acc[i][j]);
    }
  }
}

__global__ void k_copy_f32(const float *__restrict__ src, float *__restrict__ dst, long long n) {
  long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

template <typename T>
__global__ void k_fill(T *__restrict__ dst, long long n, T v) {
  long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) dst[i] = v;
}

// ---------------------------------------------------------------------------
// A1: half distances, one thread per (query, subspace, half, centroid).
// ---------------------------------------------------------------------------
__global__ void k_half_dist(const float *__restrict__ qrot, int nq, int d, int m, int k, int h,
                            const float *__restrict__ cent, double *__restrict__ out) {
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  long long total = static_cast<long long>(nq) * m * 2 * k;
  if (t >= total) return;
  int c = static_cast<int>(t % k);
  long long r = t / k;
  int s = static_cast<int>(r % 2);
  r /= 2;
  int sub = static_cast<int>(r % m);
  int q = static_cast<int>(r / m);
  const float *qa = qrot + static_cast<long long>(q) * d + sub * 2 * h + s * h;
  const float *ca = cent + ((static_cast<long long>(sub) * 2 + s) * k + c) * h;
  double acc = 0.0;
  for (int i = 0; i < h; ++i) {
    double delta = static_cast<double>(qa[i]) - static_cast<double>(ca[i]);
    double sq = delta * delta;
    acc = acc + sq;
  }
  out[t] = acc;
}

// ---------------------------------------------------------------------------
// A2: cell selection.  One wavefront per (query, subspace).
//
// The heap of Algorithm 1 pops cells in ascending key (cost, i, j) with
// cost = d1s[i] + d2s[j]; since cost is monotone in i and in j the popped
// prefix is exactly {cells with key <= key of the cutoff cell}.  The cutoff
// is the smallest key whose prefix holds >= budget ids.  It is found by
// bisection over the bit patterns of the float64 cost (monotone for
// non-negative values): for a threshold theta each row i of the sorted grid
// contributes the prefix j < n_i(theta) (binary search, cost monotone in j)
// whose size is read from a per-row prefix-size table.  Equal costs are then
// ordered by (i, j).  The k_size-th key (rank weights) is found the same way
// counting cells instead of ids.
// ---------------------------------------------------------------------------
struct SelectShared {
  double d1s[256], d2s[256];
  int o1[256], o2[256];
  int ptab[64 * 65];  // row prefix sizes when K <= 64
  int rowcnt[256];
  int roww[256];
  int misc[8];
};

__device__ __forceinline__ int row_count_le(const SelectShared &S, int k, int i, double th) {
  const double a = S.d1s[i];
  int lo = 0, hi = k;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a + S.d2s[mid] <= th) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(64) k_select_cells(const double *__restrict__ hdist, int m, int k,
                                                     const int32_t *__restrict__ offsets, int budget,
                                                     int ksize, int phi, int32_t *__restrict__ ptab_g,
                                                     int32_t *__restrict__ ncell, int32_t *__restrict__ cells_out,
                                                     int32_t *__restrict__ retrieved) {
  __shared__ SelectShared S;
  const int sub = blockIdx.x, q = blockIdx.y, lane = threadIdx.x;
  const int ncells = k * k;
  const double *h1 = hdist + ((static_cast<long long>(q) * m + sub) * 2) * k;
  const double *h2 = h1 + k;
  // Sort both halves by (distance, index) via ranks.
  for (int c = lane; c < k; c += kWave) {
    double v1 = h1[c], v2 = h2[c];
    int r1 = 0, r2 = 0;
    for (int c2 = 0; c2 < k; ++c2) {
      double u1 = h1[c2], u2 = h2[c2];
      r1 += (u1 < v1) || (u1 == v1 && c2 < c);
      r2 += (u2 < v2) || (u2 == v2 && c2 < c);
    }
    S.d1s[r1] = v1; S.o1[r1] = c;
    S.d2s[r2] = v2; S.o2[r2] = c;
  }
  __syncthreads();
  const int32_t *off = offsets + static_cast<long long>(sub) * (ncells + 1);
  int *P = (k <= 64) ? S.ptab : (ptab_g + (static_cast<long long>(q) * m + sub) * k * (k + 1));
  for (int i = lane; i < k; i += kWave) {
    int base = S.o1[i] * k, acc = 0;
    P[i * (k + 1)] = 0;
    for (int j = 0; j < k; ++j) {
      int c = base + S.o2[j];
      acc += off[c + 1] - off[c];
      P[i * (k + 1) + j + 1] = acc;
    }
  }
  __syncthreads();

  auto size_le = [&](unsigned long long bits) -> int {
    double th = from_dbits(bits);
    int tot = 0;
    for (int i = lane; i < k; i += kWave) tot += P[i * (k + 1) + row_count_le(S, k, i, th)];
    return wave_sum_i32(tot);
  };
  auto count_le = [&](unsigned long long bits) -> int {
    double th = from_dbits(bits);
    int tot = 0;
    for (int i = lane; i < k; i += kWave) tot += row_count_le(S, k, i, th);
    return wave_sum_i32(tot);
  };

  // ---- budget cutoff -------------------------------------------------------
  const unsigned long long top_bits = dbits(S.d1s[k - 1] + S.d2s[k - 1]);
  unsigned long long lo = 0, hi = top_bits;
  while (lo < hi) {
    unsigned long long mid = lo + ((hi - lo) >> 1);
    if (size_le(mid) >= budget) hi = mid; else lo = mid + 1;
  }
  const unsigned long long cstar = hi;
  const int s_lt = (cstar > 0) ? size_le(cstar - 1) : 0;
  // Ties at cost == cstar, walked in (i, j) order.
  int istar = -1, jstar = -1;
  {
    int carry = 0;
    for (int r0 = 0; r0 < k && istar < 0; r0 += kWave) {
      int i = r0 + lane;
      int tlo = 0, thi = 0, tsz = 0;
      if (i < k) {
        thi = row_count_le(S, k, i, from_dbits(cstar));
        tlo = (cstar > 0) ? row_count_le(S, k, i, from_dbits(cstar - 1)) : 0;
        tsz = P[i * (k + 1) + thi] - P[i * (k + 1) + tlo];
      }
      int incl = wave_incl_scan_i32(tsz) + carry;
      unsigned long long hit = __ballot(i < k && s_lt + incl >= budget);
      if (hit) {
        int L = __ffsll(static_cast<long long>(hit)) - 1;
        int excl_L = __shfl(incl - tsz, L, kWave);
        int tlo_L = __shfl(tlo, L, kWave);
        int row = r0 + L;
        int acc = s_lt + excl_L, j = tlo_L;
        for (;; ++j) {
          acc += P[row * (k + 1) + j + 1] - P[row * (k + 1) + j];
          if (acc >= budget) break;
        }
        istar = row;
        jstar = j;
      }
      carry = __shfl(incl, kWave - 1, kWave);
    }
  }
  // Activated cells per row.
  for (int i = lane; i < k; i += kWave) {
    int n;
    if (i < istar) n = row_count_le(S, k, i, from_dbits(cstar));
    else if (i == istar) n = jstar + 1;
    else n = (cstar > 0) ? row_count_le(S, k, i, from_dbits(cstar - 1)) : 0;
    S.rowcnt[i] = n;
  }
  __syncthreads();
  int total = 0, retr = 0;
  for (int i = lane; i < k; i += kWave) {
    total += S.rowcnt[i];
    retr += P[i * (k + 1) + S.rowcnt[i]];
  }
  total = wave_sum_i32(total);
  retr = wave_sum_i32(retr);

  // ---- rank weights (Optimized Mode) ----------------------------------------
  if (phi == 1 && ksize >= total) {
    for (int i = lane; i < k; i += kWave) S.roww[i] = S.rowcnt[i];
  } else if (phi == 1) {
    unsigned long long lo2 = 0, hi2 = top_bits;
    while (lo2 < hi2) {
      unsigned long long mid = lo2 + ((hi2 - lo2) >> 1);
      if (count_le(mid) >= ksize) hi2 = mid; else lo2 = mid + 1;
    }
    const unsigned long long ck = hi2;
    const int c_lt = (ck > 0) ? count_le(ck - 1) : 0;
    int ik = -1, jk = -1;
    int carry = 0;
    for (int r0 = 0; r0 < k && ik < 0; r0 += kWave) {
      int i = r0 + lane;
      int tlo = 0, thi = 0;
      if (i < k) {
        thi = row_count_le(S, k, i, from_dbits(ck));
        tlo = (ck > 0) ? row_count_le(S, k, i, from_dbits(ck - 1)) : 0;
      }
      int tc = thi - tlo;
      int incl = wave_incl_scan_i32(tc) + carry;
      unsigned long long hit = __ballot(i < k && c_lt + incl >= ksize);
      if (hit) {
        int L = __ffsll(static_cast<long long>(hit)) - 1;
        int excl_L = __shfl(incl - tc, L, kWave);
        int tlo_L = __shfl(tlo, L, kWave);
        ik = r0 + L;
        jk = tlo_L + (ksize - c_lt - excl_L) - 1;
      }
      carry = __shfl(incl, kWave - 1, kWave);
    }
    for (int i = lane; i < k; i += kWave) {
      int n;
      if (i < ik) n = row_count_le(S, k, i, from_dbits(ck));
      else if (i == ik) n = jk + 1;
      else n = (ck > 0) ? row_count_le(S, k, i, from_dbits(ck - 1)) : 0;
      S.roww[i] = n;
    }
  } else {
    for (int i = lane; i < k; i += kWave) S.roww[i] = 0;
  }
  __syncthreads();

  // ---- emit (cell | weight << 24), rows in order ----------------------------
  int32_t *dst = cells_out + (static_cast<long long>(q) * m + sub) * ncells;
  int carry = 0;
  for (int r0 = 0; r0 < k; r0 += kWave) {
    int i = r0 + lane;
    int cnt = (i < k) ? S.rowcnt[i] : 0;
    int incl = wave_incl_scan_i32(cnt) + carry;
    if (i < k) {
      int pos = incl - cnt;
      int base = S.o1[i] * k;
      int w2 = S.roww[i];
      for (int j = 0; j < cnt; ++j) dst[pos + j] = (base + S.o2[j]) | ((j < w2 ? 2 : 1) << 24);
    }
    carry = __shfl(incl, kWave - 1, kWave);
  }
  if (lane == 0) {
    ncell[static_cast<long long>(q) * m + sub] = total;
    retrieved[static_cast<long long>(q) * m + sub] = retr;
  }
}

// ---------------------------------------------------------------------------
// A3/A4: collision counting in LDS.  One block per (id tile, query).
// The tile's uint8 counters are packed four per dword and incremented with
// ds_add_u32 of (w << 8 * (id & 3)); scores never exceed 2M <= 254.
// Work items are (subspace, activated cell) pairs; each contributes the
// slice of the cell's posting list that falls inside the tile (from the
// load-time cell x tile table), flattened over the block by a prefix sum.
//
// pass 0: threshold tau, write the tile's candidates, histogram of scores >= tau
// pass 1: queries flagged for the fallback only: histogram of scores >= 1
// pass 2: queries flagged only: threshold tau_eff, write candidates
// ---------------------------------------------------------------------------
constexpr int kCountThreads = 256;
constexpr int kItems = 1024;

struct CountShared {
  long long start[kItems];
  int pref[kItems + 1];
  unsigned char w[kItems];
  int mbase[129];
  int hist[256];
  int tmp[kCountThreads / kWave + 1];
  int wtot[kCountThreads / kWave + 1];
};

__global__ void __launch_bounds__(kCountThreads) k_count(
    const int32_t *__restrict__ ncell, const int32_t *__restrict__ cells, int m, int ncells,
    const int32_t *__restrict__ offsets, const int32_t *__restrict__ ids, long long n,
    const int32_t *__restrict__ tile_off, int ntiles, int tile_ids, int pass, int tau,
    const int32_t *__restrict__ flag, const int32_t *__restrict__ tau_eff,
    int32_t *__restrict__ seg_ids, uint8_t *__restrict__ seg_score, int32_t *__restrict__ tile_cnt,
    int32_t *__restrict__ hist) {
  extern __shared__ uint32_t cnt[];
  __shared__ CountShared S;
  const int tile = blockIdx.x, q = blockIdx.y, tid = threadIdx.x;
  if (pass != 0 && flag[q] == 0) return;
  const long long t0 = static_cast<long long>(tile) * tile_ids;
  const int tlen = static_cast<int>(min(static_cast<long long>(tile_ids), n - t0));
  const int ndw = (tlen + 3) >> 2;
  const int thr = (pass == 0) ? tau : (pass == 1 ? 1 : tau_eff[q]);
  for (int i = tid; i < ndw; i += kCountThreads) cnt[i] = 0u;
  for (int i = tid; i < 256; i += kCountThreads) S.hist[i] = 0;
  if (tid == 0) {
    S.mbase[0] = 0;
    for (int s = 0; s < m; ++s) S.mbase[s + 1] = S.mbase[s] + ncell[static_cast<long long>(q) * m + s];
  }
  __syncthreads();
  const int total_items = S.mbase[m];
  for (int b0 = 0; b0 < total_items; b0 += kItems) {
    const int nb = min(kItems, total_items - b0);
    for (int it = tid; it < kItems; it += kCountThreads) {
      int len = 0;
      long long start = 0;
      int w = 0;
      if (it < nb) {
        int g = b0 + it;
        int s = upper_bound_minus1(S.mbase, m + 1, g);
        int packed = cells[(static_cast<long long>(q) * m + s) * ncells + (g - S.mbase[s])];
        int cell = packed & 0xFFFFFF;
        w = packed >> 24;
        const int32_t *to = tile_off + (static_cast<long long>(s) * ncells + cell) * (ntiles + 1);
        int a = to[tile];
        len = to[tile + 1] - a;
        start = static_cast<long long>(s) * n + offsets[static_cast<long long>(s) * (ncells + 1) + cell] + a;
      }
      S.pref[it] = len;
      S.start[it] = start;
      S.w[it] = static_cast<unsigned char>(w);
    }
    __syncthreads();
    const int tot = block_exclusive_scan(S.pref, kItems, S.tmp);
    if (tid == 0) S.pref[kItems] = tot;
    __syncthreads();
    for (int p = tid; p < tot; p += kCountThreads) {
      int j = upper_bound_minus1(S.pref, kItems + 1, p);
      int id = ids[S.start[j] + (p - S.pref[j])];
      int loc = id - static_cast<int>(t0);
      if (static_cast<unsigned>(loc) < static_cast<unsigned>(tlen))
        atomicAdd(&cnt[loc >> 2], static_cast<uint32_t>(S.w[j]) << ((loc & 3) * 8));
    }
    __syncthreads();
  }

  // ---- scan: threshold, histogram, ordered compaction -----------------------
  const int lane = lane_id(), wv = wave_id();
  const int nw = kCountThreads / kWave;
  const int per = ((ndw + nw - 1) / nw + kWave - 1) / kWave * kWave;
  const int dw0 = wv * per, dw1 = min(ndw, dw0 + per);
  const unsigned long long below = lanes_below_mask();
  int wcount = 0;
  for (int dw = dw0; dw < dw1; dw += kWave) {
    int i = dw + lane;
    int c = 0;
    if (i < dw1) {
      uint32_t v = cnt[i];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        int sc = (v >> (8 * b)) & 255;
        bool valid = (i * 4 + b) < tlen;
        if (valid && sc >= thr) {
          ++c;
          if (pass != 2 && sc >= 1) atomicAdd(&S.hist[sc], 1);
        }
      }
    }
    wcount += wave_sum_i32(c);
  }
  if (lane == 0) S.wtot[wv] = wcount;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < nw; ++w) { int t = S.wtot[w]; S.wtot[w] = run; run += t; }
    S.wtot[nw] = run;
  }
  __syncthreads();
  if (pass != 1) {
    int32_t *dst = seg_ids + static_cast<long long>(q) * n + t0;
    uint8_t *dsc = seg_score + static_cast<long long>(q) * n + t0;
    int run = S.wtot[wv];
    for (int dw = dw0; dw < dw1; dw += kWave) {
      int i = dw + lane;
      uint32_t v = (i < dw1) ? cnt[i] : 0u;
      int c = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        int sc = (v >> (8 * b)) & 255;
        c += (i < dw1 && (i * 4 + b) < tlen && sc >= thr) ? 1 : 0;
      }
      unsigned long long b0m = __ballot(c & 1), b1m = __ballot(c & 2), b2m = __ballot(c & 4);
      int pre = __popcll(b0m & below) + 2 * __popcll(b1m & below) + 4 * __popcll(b2m & below);
      int wt = __popcll(b0m) + 2 * __popcll(b1m) + 4 * __popcll(b2m);
      int pos = run + pre;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        int sc = (v >> (8 * b)) & 255;
        if (i < dw1 && (i * 4 + b) < tlen && sc >= thr) {
          dst[pos] = static_cast<int32_t>(t0) + i * 4 + b;
          dsc[pos] = static_cast<uint8_t>(sc);
          ++pos;
        }
      }
      run += wt;
    }
    if (tid == 0) tile_cnt[static_cast<long long>(q) * ntiles + tile] = S.wtot[nw];
  }
  if (pass != 2) {
    __syncthreads();
    const int nb = 2 * m + 1;
    for (int s = tid; s < nb; s += kCountThreads)
      if (S.hist[s]) atomicAdd(&hist[static_cast<long long>(q) * nb + s], S.hist[s]);
  }
}

// Per query: |C| at tau; flag the fallback when fewer than k points reach it.
__global__ void k_flag(const int32_t *__restrict__ tile_cnt, int ntiles, int nq, int k, int tau,
                       int32_t *__restrict__ flag, int32_t *__restrict__ tau_eff, int32_t *__restrict__ hist,
                       int nbins) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int tot = 0;
  for (int t = 0; t < ntiles; ++t) tot += tile_cnt[static_cast<long long>(q) * ntiles + t];
  int f = (tot < k && tau > 1) ? 1 : 0;
  flag[q] = f;
  tau_eff[q] = tau;
  if (f)
    for (int s = 0; s < nbins; ++s) hist[static_cast<long long>(q) * nbins + s] = 0;
}

// Flagged queries: tau_eff = largest s <= tau with at least k points scoring
// >= s, else 1; keep the histogram only from tau_eff up.
__global__ void k_tau_eff(const int32_t *__restrict__ flag, int nq, int k, int tau, int nbins,
                          int32_t *__restrict__ hist, int32_t *__restrict__ tau_eff,
                          int32_t *__restrict__ tile_cnt, int ntiles) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq || flag[q] == 0) return;
  int32_t *hq = hist + static_cast<long long>(q) * nbins;
  int ge = 0;
  for (int s = nbins - 1; s > tau; --s) ge += hq[s];
  int se = 1;
  for (int s = tau; s >= 1; --s) {
    ge += hq[s];
    if (ge >= k) { se = s; break; }
  }
  tau_eff[q] = se;
  for (int s = 0; s < se; ++s) hq[s] = 0;
  for (int t = 0; t < ntiles; ++t) tile_cnt[static_cast<long long>(q) * ntiles + t] = 0;
}

// Concatenate the per-tile candidate segments into one ascending list.
__global__ void k_compact(const int32_t *__restrict__ seg_ids, const uint8_t *__restrict__ seg_score,
                          const int32_t *__restrict__ tile_cnt, int ntiles, int tile_ids, long long n,
                          int32_t *__restrict__ cand, uint8_t *__restrict__ score, int32_t *__restrict__ ncand) {
  __shared__ int base[1025];
  const int q = blockIdx.x;
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < ntiles; ++t) { base[t] = run; run += tile_cnt[static_cast<long long>(q) * ntiles + t]; }
    base[ntiles] = run;
    ncand[q] = run;
  }
  __syncthreads();
  const long long qo = static_cast<long long>(q) * n;
  for (int t = 0; t < ntiles; ++t) {
    int c = base[t + 1] - base[t];
    long long src = qo + static_cast<long long>(t) * tile_ids;
    for (int i = threadIdx.x; i < c; i += blockDim.x) {
      cand[qo + base[t] + i] = seg_ids[src + i];
      score[qo + base[t] + i] = seg_score[src + i];
    }
  }
}

// ---------------------------------------------------------------------------
// A5: Hamming order.  One block per query.  The query's sign code is built by
// ballots over q' (bit i%64 of word i/64 = [q'_i > 0]); each candidate's
// distance is popcount(xor) over its code row; candidates (ascending id) are
// placed by a stable counting sort on the distance, giving (hamming, id) order.
// ---------------------------------------------------------------------------
constexpr int kOrderThreads = 256;

__global__ void __launch_bounds__(kOrderThreads) k_hamming_order(
    const float *__restrict__ qrot, int d, const uint64_t *__restrict__ codes, const int32_t *__restrict__ ncand,
    const int32_t *__restrict__ cand, long long n, int32_t *__restrict__ hm_tmp, int32_t *__restrict__ order,
    int32_t *__restrict__ ham_sorted) {
  extern __shared__ int bins[];          // d + 1
  __shared__ uint64_t qc[128];
  __shared__ int chunk[kOrderThreads];
  __shared__ int tmp[kOrderThreads / kWave + 1];
  const int q = blockIdx.x, tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int words = d / 64;
  const int nc = ncand[q];
  const long long qo = static_cast<long long>(q) * n;
  for (int w = wv; w < words; w += kOrderThreads / kWave) {
    unsigned long long b = __ballot(qrot[static_cast<long long>(q) * d + w * 64 + lane] > 0.0f);
    if (lane == 0) qc[w] = b;
  }
  for (int i = tid; i <= d; i += kOrderThreads) bins[i] = 0;
  __syncthreads();
  for (int i = tid; i < nc; i += kOrderThreads) {
    const uint64_t *row = codes + static_cast<long long>(cand[qo + i]) * words;
    int hsum = 0;
    for (int w = 0; w < words; ++w) hsum += __popcll(qc[w] ^ row[w]);
    hm_tmp[qo + i] = hsum;
    atomicAdd(&bins[hsum], 1);
  }
  __syncthreads();
  block_exclusive_scan(bins, d + 1, tmp);
  for (int b0 = 0; b0 < nc; b0 += kOrderThreads) {
    const int i = b0 + tid;
    const int cnt = min(kOrderThreads, nc - b0);
    const int hv = (i < nc) ? hm_tmp[qo + i] : -1;
    chunk[tid] = hv;
    __syncthreads();
    int before = 0, after = 0;
    for (int t = 0; t < cnt; ++t) {
      int u = chunk[t];
      before += (t < tid && u == hv);
      after += (t > tid && u == hv);
    }
    if (i < nc) {
      int pos = bins[hv] + before;
      order[qo + pos] = cand[qo + i];
      ham_sorted[qo + pos] = hv;
    }
    __syncthreads();
    if (i < nc && after == 0) bins[hv] += before + 1;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// A6/A7: re-rank.  One block (4 waves) per query; q' staged in LDS.
//
// First pass per candidate: float32 squared distance, each lane summing D/64
// terms with fmaf, then a 6-level butterfly.  Its distance to the float64 key
// d_canon is at most eps * d_f + abs with eps = (D/64 + 16) 2^-24 (recursive
// summation of non-negative terms: one rounding for the difference, the
// D/64 + 6 additions on any term's path, and the float64 key's own error),
// abs = 4 D 2^-149 for gradual underflow.  Whenever that band could change a
// comparison, d_canon is recomputed exactly as defined.
// ---------------------------------------------------------------------------
constexpr int kRerankThreads = 256;
constexpr int kRerankWaves = kRerankThreads / kWave;
constexpr int kChunk = 256;

struct Band {
  double lo, hi;
};

__device__ __forceinline__ Band band_of(float df, int d) {
  const double eps = (d / 64 + 16) * 5.9604644775390625e-08;  // 2^-24
  const double absb = 4.0 * d * 1.401298464324817e-45;        // 2^-149
  if (!(df <= 3.0e38f)) return Band{0.0, __longlong_as_double(0x7ff0000000000000LL)};
  double v = static_cast<double>(df);
  return Band{v - v * eps - absb, v + v * eps + absb};
}

// float32 distance of one row, whole wave; result in every lane.  Loads are
// issued eight at a time before they are consumed so that several are in
// flight per lane.
__device__ __forceinline__ float row_dist_f32(const float *__restrict__ sq, const float *__restrict__ x, int d) {
  const int lane = lane_id();
  float acc = 0.0f;
  if ((d & 255) == 0) {
    const float4 *xr = reinterpret_cast<const float4 *>(x);
    const float4 *qq = reinterpret_cast<const float4 *>(sq);
    const int nv = d / 4;
    for (int r0 = lane; r0 < nv; r0 += kWave * 8) {
      float4 a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int r = r0 + u * kWave;
        a[u] = (r < nv) ? xr[r] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int r = r0 + u * kWave;
        if (r < nv) {
          float4 b = qq[r];
          float e0 = b.x - a[u].x, e1 = b.y - a[u].y, e2 = b.z - a[u].z, e3 = b.w - a[u].w;
          acc = fmaf(e0, e0, acc);
          acc = fmaf(e1, e1, acc);
          acc = fmaf(e2, e2, acc);
          acc = fmaf(e3, e3, acc);
        }
      }
    }
  } else {
    for (int e0 = lane; e0 < d; e0 += kWave * 8) {
      float a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int e = e0 + u * kWave;
        a[u] = (e < d) ? x[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        int e = e0 + u * kWave;
        if (e < d) {
          float t = sq[e] - a[u];
          acc = fmaf(t, t, acc);
        }
      }
    }
  }
  return wave_sum_f32(acc);
}

// d_canon of one row, whole wave; result in every lane.  Loads are batched
// sixteen at a time; the float64 accumulation order is the definition's.
__device__ __forceinline__ double row_dist_canon(const float *__restrict__ sq, const float *__restrict__ x, int d) {
  const int lane = lane_id();
  const int nr = d / kWave;
  double p = 0.0;
  for (int r0 = 0; r0 < nr; r0 += 16) {
    float xv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) xv[u] = (r0 + u < nr) ? x[(r0 + u) * kWave + lane] : 0.f;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (r0 + u < nr) {
        double t = static_cast<double>(sq[(r0 + u) * kWave + lane]) - static_cast<double>(xv[u]);
        double s2 = t * t;
        p = p + s2;
      }
    }
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    double v = __shfl_down(p, s, kWave);
    if (lane < s) p = p + v;
  }
  return __shfl(p, 0, kWave);
}

__device__ __forceinline__ bool key_less(double da, int ia, double db, int ib) {
  return da < db || (da == db && ia < ib);
}

struct RerankShared {
  float df[kChunk];
  int hist[256];
  int misc[16];
  unsigned int umisc[4];
};

__global__ void __launch_bounds__(kRerankThreads) k_rerank(
    int mode, const float *__restrict__ qrot, int d, const float *__restrict__ base,
    const int32_t *__restrict__ ncand, const int32_t *__restrict__ list, long long n, int k, int patience,
    const int32_t *__restrict__ limits, float *__restrict__ dws, int32_t *__restrict__ sidx,
    double *__restrict__ sd, int64_t *__restrict__ out_ids, float *__restrict__ out_d,
    int32_t *__restrict__ examined, int32_t *__restrict__ last_upd, int32_t *__restrict__ stopped) {
  extern __shared__ __align__(16) unsigned char dyn[];
  float *sq = reinterpret_cast<float *>(dyn);                          // d floats
  double *top_d = reinterpret_cast<double *>(dyn + static_cast<size_t>(d) * 4);   // k doubles
  int *top_i = reinterpret_cast<int *>(dyn + static_cast<size_t>(d) * 4 + static_cast<size_t>(k) * 8);
  __shared__ RerankShared S;
  const int q = blockIdx.x, tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const long long qo = static_cast<long long>(q) * n;
  for (int i = tid; i < d; i += kRerankThreads) sq[i] = qrot[static_cast<long long>(q) * d + i];
  const int nc = ncand[q];
  __syncthreads();
  int64_t *oi = out_ids + static_cast<long long>(q) * k;
  float *od = out_d + static_cast<long long>(q) * k;

  if (mode == 0) {
    // ---- Guaranteed: every candidate --------------------------------------
    for (int i = wv; i < nc; i += kRerankWaves) {
      float df = row_dist_f32(sq, base + static_cast<long long>(list[qo + i]) * d, d);
      if (lane == 0) dws[qo + i] = df;
    }
    __syncthreads();
    // k-th smallest first-pass distance (radix select on the float bits).
    double ucut = __longlong_as_double(0x7ff0000000000000LL);
    if (nc > k) {
      unsigned int prefix = 0u, mask = 0u;
      int kk = k;
      for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += kRerankThreads) S.hist[b] = 0;
        __syncthreads();
        for (int i = tid; i < nc; i += kRerankThreads) {
          unsigned int bits = __float_as_uint(dws[qo + i]);
          if ((bits & mask) == prefix) atomicAdd(&S.hist[(bits >> shift) & 255], 1);
        }
        __syncthreads();
        if (tid == 0) {
          int cum = 0, b = 0;
          for (; b < 256; ++b) {
            if (cum + S.hist[b] >= kk) break;
            cum += S.hist[b];
          }
          S.umisc[0] = prefix | (static_cast<unsigned int>(b) << shift);
          S.misc[0] = kk - cum;
        }
        __syncthreads();
        prefix = S.umisc[0];
        kk = S.misc[0];
        mask |= 255u << shift;
        __syncthreads();
      }
      ucut = band_of(__uint_as_float(prefix), d).hi;
    }
    // Survivors: lower band <= the k-th smallest upper band.
    if (tid == 0) S.misc[1] = 0;
    __syncthreads();
    for (int i = tid; i < nc; i += kRerankThreads) {
      if (band_of(dws[qo + i], d).lo <= ucut) {
        int p = atomicAdd(&S.misc[1], 1);
        sidx[qo + p] = i;
      }
    }
    __syncthreads();
    const int ns = S.misc[1];
    for (int j = wv; j < ns; j += kRerankWaves) {
      int id = list[qo + sidx[qo + j]];
      double dc = row_dist_canon(sq, base + static_cast<long long>(id) * d, d);
      if (lane == 0) sd[qo + j] = dc;
    }
    __syncthreads();
    for (int j = tid; j < ns; j += kRerankThreads) {
      double dj = sd[qo + j];
      int ij = list[qo + sidx[qo + j]];
      int rank = 0;
      for (int t = 0; t < ns; ++t) {
        double dt = sd[qo + t];
        int it = list[qo + sidx[qo + t]];
        rank += key_less(dt, it, dj, ij) ? 1 : 0;
      }
      if (rank < k) { oi[rank] = ij; od[rank] = static_cast<float>(dj); }
    }
    for (int r = ns + tid; r < k; r += kRerankThreads) {
      oi[r] = -1;
      od[r] = __int_as_float(0x7f800000);
    }
    if (tid == 0) {
      examined[q] = nc;
      last_upd[q] = 0;
      stopped[q] = 0;
    }
    return;
  }

  // ---- Optimized: Hamming order with patience ------------------------------
  int lim = nc;
  if (limits != nullptr) {
    int l = limits[q];
    if (l > 0 && l < lim) lim = l;
  }
  if (tid == 0) { S.misc[2] = 0; S.misc[3] = 0; S.misc[4] = 0; S.misc[5] = 0; S.misc[6] = 0; }
  __syncthreads();
  int tn = 0, run = 0, last = 0, stop = 0, pos = 0;
  for (int c0 = 0; c0 < lim; c0 += kChunk) {
    const int cnt = min(kChunk, lim - c0);
    for (int t = wv; t < cnt; t += kRerankWaves) {
      float df = row_dist_f32(sq, base + static_cast<long long>(list[qo + c0 + t]) * d, d);
      if (lane == 0) S.df[t] = df;
    }
    __syncthreads();
    if (wv == 0) {
      tn = S.misc[2]; run = S.misc[3]; last = S.misc[4];
      pos = c0;
      for (int t = 0; t < cnt; ++t) {
        const int id = list[qo + c0 + t];
        const Band bd = band_of(S.df[t], d);
        bool upd;
        bool have = false;
        double dc = 0.0;
        if (tn < k) {
          upd = true;
        } else {
          const double kd = top_d[k - 1];
          const int kid = top_i[k - 1];
          if (bd.hi < kd) upd = true;
          else if (bd.lo > kd) upd = false;
          else {
            dc = row_dist_canon(sq, base + static_cast<long long>(id) * d, d);
            have = true;
            upd = key_less(dc, id, kd, kid);
          }
        }
        pos = c0 + t + 1;
        if (upd) {
          if (!have) dc = row_dist_canon(sq, base + static_cast<long long>(id) * d, d);
          if (lane == 0) {
            int p = (tn < k) ? tn : k - 1;
            while (p > 0 && key_less(dc, id, top_d[p - 1], top_i[p - 1])) {
              top_d[p] = top_d[p - 1];
              top_i[p] = top_i[p - 1];
              --p;
            }
            top_d[p] = dc;
            top_i[p] = id;
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          if (tn < k) ++tn;
          run = 0;
          last = pos;
        } else {
          ++run;
        }
        if (run >= patience) { stop = 1; break; }
      }
      if (lane == 0) {
        S.misc[2] = tn; S.misc[3] = run; S.misc[4] = last; S.misc[5] = stop; S.misc[6] = pos;
      }
    }
    __syncthreads();
    if (S.misc[5]) break;
  }
  __syncthreads();
  tn = S.misc[2];
  for (int r = tid; r < k; r += kRerankThreads) {
    if (r < tn) { oi[r] = top_i[r]; od[r] = static_cast<float>(top_d[r]); }
    else { oi[r] = -1; od[r] = __int_as_float(0x7f800000); }
  }
  if (tid == 0) {
    examined[q] = S.misc[6];
    last_upd[q] = S.misc[4];
    stopped[q] = S.misc[5];
  }
}

// ---------------------------------------------------------------------------
// Load-time: CSR validation and the cell x tile table.
// ---------------------------------------------------------------------------
__global__ void k_validate_csr(const int32_t *__restrict__ offsets, const int32_t *__restrict__ ids, int m,
                               int ncells, long long n, int32_t *__restrict__ err) {
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(m) * ncells) return;
  int sub = static_cast<int>(t / ncells), c = static_cast<int>(t % ncells);
  const int32_t *off = offsets + static_cast<long long>(sub) * (ncells + 1);
  int a = off[c], b = off[c + 1];
  int bad = 0;
  if (c == 0 && a != 0) bad = 1;
  if (c == ncells - 1 && static_cast<long long>(b) != n) bad = 1;
  if (a > b || a < 0 || static_cast<long long>(b) > n) bad = 1;
  if (!bad) {
    const int32_t *row = ids + static_cast<long long>(sub) * n;
    int prev = -1;
    for (int p = a; p < b; ++p) {
      int v = row[p];
      if (v <= prev || static_cast<long long>(v) >= n) { bad = 1; break; }
      prev = v;
    }
  }
  if (bad) atomicOr(err, 1);
}

__global__ void k_tile_offsets(const int32_t *__restrict__ offsets, const int32_t *__restrict__ ids, int m,
                               int ncells, long long n, int ntiles, int tile_ids, int32_t *__restrict__ tile_off) {
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(m) * ncells) return;
  int sub = static_cast<int>(t / ncells), c = static_cast<int>(t % ncells);
  const int32_t *off = offsets + static_cast<long long>(sub) * (ncells + 1);
  const int32_t *row = ids + static_cast<long long>(sub) * n + off[c];
  int len = off[c + 1] - off[c];
  int32_t *dst = tile_off + t * (ntiles + 1);
  for (int tt = 0; tt <= ntiles; ++tt) {
    long long bound = static_cast<long long>(tt) * tile_ids;
    int lo = 0, hi = len;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (row[mid] < bound) lo = mid + 1; else hi = mid;
    }
    dst[tt] = lo;
  }
}

}  // namespace crisp
