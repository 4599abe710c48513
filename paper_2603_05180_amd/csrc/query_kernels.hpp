// Query-path kernels of the CRISP engine (Algorithm 1, Sections 4.3.1-4.3.2).
//
//   k_rotate_rows   (A0) x' = x R, float64 ascending-i accumulation per output
//                   on float64 matrix cores
//   k_select_cells  (A1/A2) Dist_1 / Dist_2 of every half-centroid, then the
//                   Multi-Sequence cell set + rank weights per (query, subspace)
//   k_count         (A3/A4) LDS collision counters per (query, id tile),
//                   threshold, ordered compaction, score histogram
//   k_flag / k_tau_eff / k_compact (A4) fallback rule and candidate lists
//   k_hamming_dist / k_hamming_order (A5) Hamming distances, then the
//                   (distance, id) order placed as far as the walk reads it
//   k_rerank        (A6/A7) exact float64 keys, top-k / patience walk; the
//                   bfloat16 variant first bounds every row from a bfloat16
//                   copy and reads float32 rows only where the bound matters
#pragma once

#include "common.hpp"

namespace crisp {

// ---------------------------------------------------------------------------
// A0: rotation on float64 matrix cores.  v_mfma_f64_16x16x4_f64 adds its four
// products to the accumulator one after another in k order, rounding after
// each addition (checked bit for bit on gfx950), and products of two float32
// values are exact in float64; so chaining the instructions in ascending k
// gives every output exactly the ascending-k float64 sum of its definition.
// Two kernels compute the same values:
//
// k_rotate_rows: 128x128 output tile per 256-thread block, 64x64 per
// wavefront (4x4 tiles of 16x16), two waves per SIMD.  The k dimension goes
// through LDS in 16-deep float32 slabs loaded by global_load_lds_dwordx4
// straight into LDS (no staging registers), double buffered: after the
// barrier each wave reads all of its fragments of the slab into registers,
// then issues the next slab's loads into the other buffer (so no LDS read
// follows a load in flight), then runs its 64 matrix instructions; the loads
// are waited for at the next barrier.  A lane's 16-byte load lands at a fixed
// LDS position (lane x 16 bytes from the instruction's base), so the layout
// is chosen through the source address: the four 16-byte chunks of an A row
// and the 32 of a B row are XOR-swizzled by the row so that the fragment
// reads (16 rows x 4 k, or 4 k x 16 columns) hit 64 different banks.  Needs
// 16-byte aligned rows and enough blocks to fill the chip (the host picks).
//
// k_rotate_rows_small: 128x64 tile per block, 64x32 per wavefront, 8-deep
// slabs staged through registers, four waves per SIMD: twice the blocks of
// the kernel above for small grids (few rows, or D below 1,024).
// ---------------------------------------------------------------------------
constexpr int kRotBM = 128, kRotBN = 128, kRotBK = 16;
constexpr int kRotCpr = kRotBK / 4, kRotRpl = 64 / kRotBK, kRotLoads = kRotBK / 8;  // chunks per A row, A rows per 64 banks, loads per wave per operand
typedef double rot_acc_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;

// live: NULL, or a device count of the rows to produce (rows beyond it are skipped).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_rotate_rows(const float *__restrict__ x, long long rows, int d, const float *__restrict__ r,
              float *__restrict__ out, const int32_t *__restrict__ live) {
  __shared__ __align__(16) float sa[2][kRotBM * kRotBK];
  __shared__ __align__(16) float sb[2][kRotBK * kRotBN];
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int fi = lane & 15, fk = lane >> 4;          // fragment row (column) / k of this lane
  const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64; // the wavefront's 64x64 sub-tile
  const long long row0 = static_cast<long long>(blockIdx.y) * kRotBM;
  const int col0 = blockIdx.x * kRotBN;
  if (live) rows = min(rows, static_cast<long long>(*live));
  if (row0 >= rows) return;
  // Sources of this lane's loads.  A: load g covers rows 16g .. 16g + 15 of
  // the tile, four lanes per row, LDS slot `slot` of row `row` holding k chunk
  // slot ^ swizzle(row).  B: load g covers k rows 2g, 2g + 1, 32 lanes per
  // row, slot holding column chunk slot ^ 4 (k & 3).  Rows past the last are
  // clamped (never stored); columns past D are clamped (never stored).
  const float *ga[kRotLoads], *gb[kRotLoads];
#pragma unroll
  for (int e = 0; e < kRotLoads; ++e) {
    const int g = wv * kRotLoads + e;
    const int row = g * (64 / kRotCpr) + lane / kRotCpr, slot = lane % kRotCpr;
    const int chunk = slot ^ ((row / kRotRpl) % kRotCpr);
    const long long gr = min(row0 + row, rows - 1);
    ga[e] = x + gr * d + chunk * 4;
    const int kr = g * 2 + (lane >> 5), bslot = lane & 31;
    const int bchunk = bslot ^ ((kr & 3) << 2);
    gb[e] = r + static_cast<long long>(kr) * d + min(col0 + bchunk * 4, d - 4);
  }
  auto issue = [&](int buf) {
#pragma unroll
    for (int e = 0; e < kRotLoads; ++e)
      __builtin_amdgcn_global_load_lds(ga[e], (lds_void_t *)&sa[buf][(wv * kRotLoads + e) * 256], 16, 0, 0);
#pragma unroll
    for (int e = 0; e < kRotLoads; ++e)
      __builtin_amdgcn_global_load_lds(gb[e], (lds_void_t *)&sb[buf][(wv * kRotLoads + e) * 256], 16, 0, 0);
#pragma unroll
    for (int e = 0; e < kRotLoads; ++e) {
      ga[e] += kRotBK;
      gb[e] += static_cast<long long>(kRotBK) * d;
    }
  };
  rot_acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = rot_acc_t{0.0, 0.0, 0.0, 0.0};
  const int swa = (fi / kRotRpl) % kRotCpr;          // swizzle of this lane's A rows
  const int abase = (wr + fi) * kRotBK + fk;
  int boff[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) boff[j] = fk * kRotBN + wc + ((j ^ fk) << 4) + fi;
  const int nslab = d / kRotBK;
  issue(0);
  for (int s = 0; s < nslab; ++s) {
    const int cur = s & 1;
    __syncthreads();  // slab s is in LDS (each wave waits for its loads); every wave is done with slab s - 1
    const float *A = sa[cur], *B = sb[cur];
    float fa[kRotBK / 4][4], fb[kRotBK / 4][4];
#pragma unroll
    for (int t = 0; t < kRotBK / 4; ++t) {
      const int ao = abase + ((t ^ swa) << 2);
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[t][i] = A[ao + i * 16 * kRotBK];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[t][j] = B[boff[j] + t * 4 * kRotBN];
    }
    if (s + 1 < nslab) issue(cur ^ 1);
#pragma unroll
    for (int t = 0; t < kRotBK / 4; ++t) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = static_cast<double>(fa[t][i]);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = static_cast<double>(fb[t][j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // Accumulator element v of lane l holds row fk + 4v, column fi of its tile.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long gr = row0 + wr + i * 16 + fk + 4 * v;
        const int gc = col0 + wc + j * 16 + fi;
        if (gr < rows && gc < d) out[gr * d + gc] = static_cast<float>(acc[i][j][v]);
      }
}

constexpr int kRotSmBM = 128, kRotSmBN = 64, kRotSmBK = 8, kRotSmPad = 16;
constexpr int kRotSmEA = kRotSmBM * kRotSmBK / 256, kRotSmEB = kRotSmBK * kRotSmBN / 256;  // staged floats per thread

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_rotate_rows_small(const float *__restrict__ x, long long rows, int d, const float *__restrict__ r,
                    float *__restrict__ out, const int32_t *__restrict__ live) {
  __shared__ __align__(16) float sa[2][kRotSmBK][kRotSmBM + kRotSmPad];
  __shared__ __align__(16) float sb[2][kRotSmBK][kRotSmBN + kRotSmPad];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int fi = lane & 15, fk = lane >> 4;
  const int wr = (wv >> 1) * 64, wc = (wv & 1) * 32;  // the wavefront's 64x32 sub-tile
  const long long row0 = static_cast<long long>(blockIdx.y) * kRotSmBM;
  const int col0 = blockIdx.x * kRotSmBN;
  if (live) rows = min(rows, static_cast<long long>(*live));
  if (row0 >= rows) return;
  rot_acc_t acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = rot_acc_t{0.0, 0.0, 0.0, 0.0};
  float ra[kRotSmEA], rb[kRotSmEB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < kRotSmEA; ++e) {
      const int idx = tid + e * 256;
      const int rr = idx / kRotSmBK, kk = idx % kRotSmBK;
      long long gr = row0 + rr;
      gr = gr < rows ? gr : rows - 1;            // clamped; such rows are never stored
      ra[e] = x[gr * d + k0 + kk];
    }
#pragma unroll
    for (int e = 0; e < kRotSmEB; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx / kRotSmBN, cc = idx % kRotSmBN;
      rb[e] = r[static_cast<long long>(k0 + kk) * d + col0 + cc];
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int e = 0; e < kRotSmEA; ++e) {
      const int idx = tid + e * 256;
      sa[b][idx % kRotSmBK][idx / kRotSmBK] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < kRotSmEB; ++e) {
      const int idx = tid + e * 256;
      sb[b][idx / kRotSmBN][idx % kRotSmBN] = rb[e];
    }
  };
  const int nslab = d / kRotSmBK;
  gload(0);
  store(0);
  __syncthreads();
  for (int s = 0; s < nslab; ++s) {
    const int cur = s & 1;
    if (s + 1 < nslab) gload((s + 1) * kRotSmBK);
#pragma unroll
    for (int kk = 0; kk < kRotSmBK; kk += 4) {
      double a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = static_cast<double>(sa[cur][kk + fk][wr + i * 16 + fi]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = static_cast<double>(sb[cur][kk + fk][wc + j * 16 + fi]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (s + 1 < nslab) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long gr = row0 + wr + i * 16 + fk + 4 * v;
        if (gr < rows) out[gr * d + col0 + wc + j * 16 + fi] = static_cast<float>(acc[i][j][v]);
      }
}

// Plain 16-byte copy: the reference kernel hardware byte counters are
// calibrated against (it reads and writes exactly its size).
__global__ void __launch_bounds__(256) k_copy_probe(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     long long n) {
  const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) dst[i] = src[i];
}

__global__ void k_copy_f32(const float *__restrict__ src, float *__restrict__ dst, long long n,
                           const int32_t *__restrict__ live, long long row_len) {
  if (live) n = min(n, static_cast<long long>(*live) * row_len);
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
// A1 + A2: half distances and cell selection.  One wavefront per
// (query, subspace).
//
// Dist_1 / Dist_2 are computed from the rotated sub-vector (staged in LDS)
// and a load-time transposed copy of the half-codebooks ([M][2][h][K], so the
// lanes of a wave read consecutive centroids), accumulated over the h
// coordinates in ascending order exactly as defined.
//
// The heap of Algorithm 1 pops cells in ascending key (cost, i, j) with
// cost = d1s[i] + d2s[j].  For K <= 64 the pops are replayed directly (one
// lane per sorted row, a wavefront argmin per pop) while they number at most
// kPopCap.  Otherwise: since cost is monotone in i and in j the popped
// prefix is exactly {cells with key <= key of the cutoff cell}.  The cutoff
// is the smallest key whose prefix holds >= budget ids.  It is found by
// bisection over the bit patterns of the float64 cost (monotone for
// non-negative values): for a threshold theta each row i of the sorted grid
// contributes the prefix j < n_i(theta) (binary search, cost monotone in j)
// whose size is read from a per-row prefix-size table.  Equal costs are then
// ordered by (i, j).  The k_size-th key (rank weights) is found the same way
// counting cells instead of ids.
// ---------------------------------------------------------------------------
constexpr int kPopCap = 256;  // cells the direct enumeration may pop before bisection takes over

struct SelectLds {
  double *d1s, *d2s, *hd;
  int *o1, *o2, *rowcnt, *roww, *pops;
  double *qs;  // the subspace's 2h coordinates of q', widened once
};

__host__ __device__ inline size_t select_lds_bytes(int k, int h) {
  size_t b = 0;
  b += 8 * static_cast<size_t>(k) * 4;                      // d1s, d2s, hd (2k)
  b += 4 * static_cast<size_t>(k) * 4;                      // o1, o2, rowcnt, roww
  b += (k <= 64) ? 4 * static_cast<size_t>(kPopCap) : 0;      // pops
  b += 8 * 2 * static_cast<size_t>(h);                      // qs
  return (b + 15) / 16 * 16;
}

__device__ __forceinline__ int row_count_le(const double *d1s, const double *d2s, int k, int i, double th) {
  const double a = d1s[i];
  int lo = 0, hi = k;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a + d2s[mid] <= th) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Certified pre-scoring of the half-codebook distances on bfloat16 matrix
// cores (precision 2, K <= 64).  Each coordinate is split into two bfloat16
// terms, x = x_hi + x_lo + r_x (x_hi = bf16(x), x_lo = bf16(x - x_hi)), and
// q.c is approximated by q_hi.c_hi + q_lo.c_hi + q_hi.c_lo with three
// v_mfma_f32_16x16x16_bf16 per 16-coordinate step (products of bfloat16 are
// exact in float32).  With d~ = |q|^2 + |c|^2 - 2 q.c~ the distance
// |q - c|^2 differs from d~ by at most
//   2 (|q_lo||c_lo| + |q_hi + q_lo||r_c| + |r_q||c|)      omitted terms
//   + 2 (3h + 16) 2^-22 |q~||c~|                             float32 sums
//   + (4 nks + 4) 2^-23 (|q|^2 + |c|^2) + 2^-21 (|q|^2 + |c|^2 + 2|q.c~|)
// (norms and the final expression in float32), and the canonical float64
// half distance differs from |q - c|^2 by far less than 2^-40 of the same
// scale.  The bound used is twice that sum plus that last term, and the
// interval [d~ - E, d~ + E] is stored in float rounded outward.
// One wavefront per (16 queries, subspace); lane l holds query row l & 15 of
// the A operand and centroid column l & 15 of the B operand.
// ---------------------------------------------------------------------------
typedef short score_s4 __attribute__((ext_vector_type(4)));
typedef float score_f4 __attribute__((ext_vector_type(4)));
constexpr int kScoreRanks = 4;  // ranks per half certified before the exact pass

__device__ __forceinline__ void split_bf16(float x, short &hi, short &lo, float &hf, float &lf) {
  const uint16_t h = bf16_bits(x);
  hf = __uint_as_float(static_cast<uint32_t>(h) << 16);
  const uint16_t l = bf16_bits(x - hf);
  lf = __uint_as_float(static_cast<uint32_t>(l) << 16);
  hi = static_cast<short>(h);
  lo = static_cast<short>(l);
}

__global__ void __launch_bounds__(64) k_score_bf16x3(const float *__restrict__ qrot, int d,
                                                     const float *__restrict__ cent_t, int m, int k, int h, int cq,
                                                     float *__restrict__ out_lb, float *__restrict__ out_ub,
                                                     const int32_t *__restrict__ live) {
  const int lane = threadIdx.x, r = lane & 15, kq = lane >> 4;
  const int q0 = blockIdx.x * 16, sub = blockIdx.y;
  const int nl = live ? min(cq, *live) : cq;
  if (q0 >= nl) return;
  const int nks = (h + 15) / 16;
  const int qa = q0 + r;                        // this lane's query row of the A operand
  const float *qrow = qrot + static_cast<long long>(min(qa, nl - 1)) * d + sub * 2 * h;
  const float sacc = 3.f * static_cast<float>(3 * 16 * nks + 16) * 0x1p-22f;
  const float snorm = static_cast<float>(4 * nks + 4) * 0x1p-23f;
  for (int s = 0; s < 2; ++s) {
    const float *ct = cent_t + static_cast<long long>(sub * 2 + s) * h * k;
    for (int c0 = 0; c0 < k; c0 += 16) {
      const int c = c0 + r;                     // this lane's centroid column of the B operand
      score_f4 acc = score_f4{0.f, 0.f, 0.f, 0.f};
      // partial norms over this lane's coordinates: |x|^2, |x_lo|^2, |r_x|^2, |x_hi + x_lo|^2
      float nq = 0.f, nqlo = 0.f, nqr = 0.f, nqt = 0.f;
      float nc = 0.f, nclo = 0.f, ncr = 0.f, nct = 0.f;
      for (int ks = 0; ks < nks; ++ks) {
        score_s4 qh, ql, ch, cl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int dd = ks * 16 + 4 * kq + e;
          const float xq = (dd < h && qa < nl) ? qrow[s * h + dd] : 0.f;
          const float xc = (dd < h && c < k) ? ct[static_cast<long long>(dd) * k + c] : 0.f;
          short hi, lo;
          float hf, lf;
          split_bf16(xq, hi, lo, hf, lf);
          qh[e] = hi;
          ql[e] = lo;
          float rr = (xq - hf) - lf;
          nq = fmaf(xq, xq, nq);
          nqlo = fmaf(lf, lf, nqlo);
          nqr = fmaf(rr, rr, nqr);
          nqt = fmaf(hf + lf, hf + lf, nqt);
          split_bf16(xc, hi, lo, hf, lf);
          ch[e] = hi;
          cl[e] = lo;
          rr = (xc - hf) - lf;
          nc = fmaf(xc, xc, nc);
          nclo = fmaf(lf, lf, nclo);
          ncr = fmaf(rr, rr, ncr);
          nct = fmaf(hf + lf, hf + lf, nct);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qh, ch, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ql, ch, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(qh, cl, acc, 0, 0, 0);
      }
      // the four lanes of a row / column (kq = 0..3) hold its four partial sums
#pragma unroll
      for (int sh = 16; sh <= 32; sh <<= 1) {
        nq += __shfl_xor(nq, sh, kWave);
        nqlo += __shfl_xor(nqlo, sh, kWave);
        nqr += __shfl_xor(nqr, sh, kWave);
        nqt += __shfl_xor(nqt, sh, kWave);
        nc += __shfl_xor(nc, sh, kWave);
        nclo += __shfl_xor(nclo, sh, kWave);
        ncr += __shfl_xor(ncr, sh, kWave);
        nct += __shfl_xor(nct, sh, kWave);
      }
      // acc[i]: query q0 + 4 kq + i, centroid c
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 4 * kq + i;
        const float vq = __shfl(nq, row, kWave), vqlo = __shfl(nqlo, row, kWave);
        const float vqr = __shfl(nqr, row, kWave), vqt = __shfl(nqt, row, kWave);
        const int qq = q0 + row;
        if (qq < nl && c < k) {
          const float dot = acc[i];
          const float dt = vq + nc - 2.f * dot;
          const float omit = sqrtf(vqlo * nclo) + sqrtf(vqt * ncr) + sqrtf(vqr * nc);
          const float sums = sacc * (sqrtf(vqt) + sqrtf(vqlo)) * (sqrtf(nct) + sqrtf(nclo));
          const float scale = vq + nc + 2.f * fabsf(dot);
          const double e = 2.0 * (2.0 * (static_cast<double>(omit) + sums) + static_cast<double>(snorm) * (vq + nc) +
                                  0x1p-21 * scale) +
                           0x1p-40 * scale + 1e-300;
          const double lo = fmax(0.0, static_cast<double>(dt) - e);
          const double hi = static_cast<double>(dt) + e;
          float lf = static_cast<float>(lo), hf = static_cast<float>(hi);
          if (static_cast<double>(lf) > lo) lf = nextafterf(lf, 0.f);
          if (static_cast<double>(hf) < hi) hf = nextafterf(hf, __int_as_float(0x7f800000));
          const long long o = (static_cast<long long>(qq) * m + sub) * 2 * k + s * k + c;
          out_lb[o] = lf;
          out_ub[o] = hf;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same certified pre-scoring on FP8 (OCP e4m3) matrix cores (precision 3,
// K <= 64).  Per (query, half) and per half-codebook a power-of-two scale
// maps the largest magnitude to [128, 256) (exact), each scaled coordinate is
// split into two e4m3 terms, x = x_hi + x_lo + r_x (x_hi = e4m3(x), x_lo =
// e4m3(x - x_hi), both round to nearest even; r_x exact in float32), and q.c
// is approximated by q_hi.c_hi + q_lo.c_hi + q_hi.c_lo with three
// v_mfma_f32_16x16x32_fp8_fp8 per 32-coordinate step (products of two e4m3
// values are exact in float32).  The bound has the form of the bfloat16
// kernel's: the omitted terms |q_lo.c_lo| + |(q_hi + q_lo).r_c| + |r_q.c| by
// Cauchy-Schwarz from the exact residual norms, the float32 sum errors of
// the three products ((3 * 32 nks + 32) 2^-22 per unit of the products'
// absolute sum, nks = 32-coordinate steps), the float32 norms and the final
// expression; doubled, plus 2^-40 of the scale for the canonical float64
// half distance.  One wavefront per (16 queries, subspace); lane l holds
// query row l & 15 (A) and centroid column l & 15 (B), coordinates
// 8 (l >> 4) .. + 7 of each 32-coordinate step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float pow2_scale_for(float amax) {
  // 2^e with amax * 2^e in [128, 256); 1 when amax is 0 or not finite
  if (!(amax > 0.f) || !(amax < 3.0e38f)) return 1.f;
  const int e = 7 - ilogbf(amax);
  return ldexpf(1.f, max(-60, min(60, e)));  // two scales multiply without overflow
}

// Two e4m3 terms of one float (already scaled): bytes hi, lo; their float
// values hf, lf (exact).
__device__ __forceinline__ void split_fp8(float x, int &hb, int &lb, float &hf, float &lf) {
  const int ph = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false);
  hf = __builtin_amdgcn_cvt_f32_fp8(ph, 0);
  const int pl = __builtin_amdgcn_cvt_pk_fp8_f32(x - hf, 0.f, 0, false);
  lf = __builtin_amdgcn_cvt_f32_fp8(pl, 0);
  hb = ph & 0xff;
  lb = pl & 0xff;
}

__global__ void __launch_bounds__(64) k_score_fp8(const float *__restrict__ qrot, int d,
                                                  const float *__restrict__ cent_t, int m, int k, int h, int cq,
                                                  float *__restrict__ out_lb, float *__restrict__ out_ub,
                                                  const int32_t *__restrict__ live) {
  const int lane = threadIdx.x, r = lane & 15, kq = lane >> 4;
  const int q0 = blockIdx.x * 16, sub = blockIdx.y;
  const int nl = live ? min(cq, *live) : cq;
  if (q0 >= nl) return;
  const int nks = (h + 31) / 32;
  const int qa = q0 + r;
  const float *qrow = qrot + static_cast<long long>(min(qa, nl - 1)) * d + sub * 2 * h;
  // Sum error of the FP8 matrix-core products: the 32-product dot of one
  // instruction is not exact in float32 on gfx950 (measured up to 4.1e-4,
  // 2^-11.2, of the products' absolute sum over 131,072 tiles of random
  // codes and of two-term splits); 2^-8 of it per instruction, plus the
  // float32 accumulation over the 3 nks instructions.
  const float sacc = 0x1p-8f + static_cast<float>(3 * nks + 4) * 0x1p-22f;
  const float snorm = static_cast<float>(4 * nks + 4) * 0x1p-23f;
  for (int s = 0; s < 2; ++s) {
    const float *ct = cent_t + static_cast<long long>(sub * 2 + s) * h * k;
    // scales: this lane's query row (its four lanes share the row), the codebook
    float aq = 0.f;
    for (int t = kq; t < h; t += 4) aq = fmaxf(aq, fabsf(qa < nl ? qrow[s * h + t] : 0.f));
    aq = fmaxf(aq, __shfl_xor(aq, 16, kWave));
    aq = fmaxf(aq, __shfl_xor(aq, 32, kWave));
    float ac = 0.f;
    for (int t = lane; t < h * k; t += kWave) ac = fmaxf(ac, fabsf(ct[t]));
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) ac = fmaxf(ac, __shfl_xor(ac, sh, kWave));
    const float sq = pow2_scale_for(aq), sc = pow2_scale_for(ac);
    for (int c0 = 0; c0 < k; c0 += 16) {
      const int c = c0 + r;
      score_f4 acc = score_f4{0.f, 0.f, 0.f, 0.f};
      float nq = 0.f, nqlo = 0.f, nqr = 0.f, nqt = 0.f;
      float nc = 0.f, nclo = 0.f, ncr = 0.f, nct = 0.f;
      for (int ks = 0; ks < nks; ++ks) {
        long qh = 0, ql = 0, ch = 0, cl = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int dd = ks * 32 + 8 * kq + e;
          const float xq = (dd < h && qa < nl) ? qrow[s * h + dd] : 0.f;
          const float xc = (dd < h && c < k) ? ct[static_cast<long long>(dd) * k + c] : 0.f;
          int hb, lb;
          float hf, lf;
          split_fp8(xq * sq, hb, lb, hf, lf);
          qh |= static_cast<long>(hb) << (8 * e);
          ql |= static_cast<long>(lb) << (8 * e);
          // unscaled terms (power-of-two scale: exact)
          float uh = hf / sq, ul = lf / sq;
          float rr = (xq - uh) - ul;
          nq = fmaf(xq, xq, nq);
          nqlo = fmaf(ul, ul, nqlo);
          nqr = fmaf(rr, rr, nqr);
          nqt = fmaf(uh + ul, uh + ul, nqt);
          split_fp8(xc * sc, hb, lb, hf, lf);
          ch |= static_cast<long>(hb) << (8 * e);
          cl |= static_cast<long>(lb) << (8 * e);
          uh = hf / sc;
          ul = lf / sc;
          rr = (xc - uh) - ul;
          nc = fmaf(xc, xc, nc);
          nclo = fmaf(ul, ul, nclo);
          ncr = fmaf(rr, rr, ncr);
          nct = fmaf(uh + ul, uh + ul, nct);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(qh, ch, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ql, ch, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(qh, cl, acc, 0, 0, 0);
      }
#pragma unroll
      for (int sh = 16; sh <= 32; sh <<= 1) {
        nq += __shfl_xor(nq, sh, kWave);
        nqlo += __shfl_xor(nqlo, sh, kWave);
        nqr += __shfl_xor(nqr, sh, kWave);
        nqt += __shfl_xor(nqt, sh, kWave);
        nc += __shfl_xor(nc, sh, kWave);
        nclo += __shfl_xor(nclo, sh, kWave);
        ncr += __shfl_xor(ncr, sh, kWave);
        nct += __shfl_xor(nct, sh, kWave);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 4 * kq + i;
        const float vq = __shfl(nq, row, kWave), vqlo = __shfl(nqlo, row, kWave);
        const float vqr = __shfl(nqr, row, kWave), vqt = __shfl(nqt, row, kWave);
        const float vs = __shfl(sq, row, kWave);
        const int qq = q0 + row;
        if (qq < nl && c < k) {
          const float dot = acc[i] / (vs * sc);   // power-of-two unscaling: exact
          const float dt = vq + nc - 2.f * dot;
          const float omit = sqrtf(vqlo * nclo) + sqrtf(vqt * ncr) + sqrtf(vqr * nc);
          const float sums = sacc * (sqrtf(vqt) + sqrtf(vqlo)) * (sqrtf(nct) + sqrtf(nclo));
          const float scale = vq + nc + 2.f * fabsf(dot);
          const double e = 2.0 * (2.0 * (static_cast<double>(omit) + sums) + static_cast<double>(snorm) * (vq + nc) +
                                  0x1p-21 * scale) +
                           0x1p-40 * scale + 1e-300;
          const double lo = fmax(0.0, static_cast<double>(dt) - e);
          const double hi = static_cast<double>(dt) + e;
          float lf = static_cast<float>(lo), hf = static_cast<float>(hi);
          if (static_cast<double>(lf) > lo) lf = nextafterf(lf, 0.f);
          if (static_cast<double>(hf) < hi) hf = nextafterf(hf, __int_as_float(0x7f800000));
          const long long o = (static_cast<long long>(qq) * m + sub) * 2 * k + s * k + c;
          out_lb[o] = lf;
          out_ub[o] = hf;
        }
      }
    }
  }
}

__global__ void __launch_bounds__(64) k_select_cells(const float *__restrict__ qrot, int d,
                                                     const float *__restrict__ cent_t, int m, int k, int h,
                                                     const int32_t *__restrict__ offsets, int budget, int ksize,
                                                     int phi, double *__restrict__ hdist_out,
                                                     int32_t *__restrict__ ptab_g, int32_t *__restrict__ ncell,
                                                     int32_t *__restrict__ cells_out,
                                                     int32_t *__restrict__ retrieved,
                                                     double *__restrict__ sstat, const int32_t *__restrict__ live,
                                                     const float *__restrict__ sc_lb,
                                                     const float *__restrict__ sc_ub,
                                                     int32_t *__restrict__ sfall) {
  extern __shared__ __align__(16) unsigned char dyn[];
  SelectLds S;
  {
    unsigned char *p = dyn;
    S.d1s = reinterpret_cast<double *>(p); p += 8 * k;
    S.d2s = reinterpret_cast<double *>(p); p += 8 * k;
    S.hd = reinterpret_cast<double *>(p); p += 16 * k;
    S.o1 = reinterpret_cast<int *>(p); p += 4 * k;
    S.o2 = reinterpret_cast<int *>(p); p += 4 * k;
    S.rowcnt = reinterpret_cast<int *>(p); p += 4 * k;
    S.roww = reinterpret_cast<int *>(p); p += 4 * k;
    S.pops = reinterpret_cast<int *>(p); p += (k <= 64) ? 4 * kPopCap : 0;
    S.qs = reinterpret_cast<double *>(p);
  }
  const int sub = blockIdx.x, q = blockIdx.y, lane = threadIdx.x;
  if (live && q >= *live) return;
  const int ncells = k * k;
  const float *qa = qrot + static_cast<long long>(q) * d + sub * 2 * h;
  for (int t = lane; t < 2 * h; t += kWave) S.qs[t] = static_cast<double>(qa[t]);
  __syncthreads();
  // ---- certified pre-scoring (precision 2, K <= 64) ------------------------
  // From the bounds of k_score_bf16x3: T_s >= the R-th smallest upper bound of
  // half s; every centroid whose lower bound is <= T_s gets its exact float64
  // distance (X_s, all of X_0 and X_1 in one pass when they fit a wavefront).
  // The R nearest of each half lie in X_s (the R smallest upper bounds
  // belong to centroids whose distances are <= T_s, and every centroid
  // outside X_s is farther), so ranks 0..R-1 are exact, and lb_s = min(exact
  // values of X_s at ranks >= R, lower bounds outside X_s) bounds rank R from
  // below.  The pops then run on the known ranks; whenever a cell with an
  // unknown rank (row R, or column R of a started row) could come next, or
  // the pops run out, the exact path below redoes the subspace.
  if (sc_lb != nullptr && k <= kWave) {
    const long long so = (static_cast<long long>(q) * m + sub) * 2 * k;
    const bool inb = lane < k;
    const float finf = __int_as_float(0x7f800000);
    const double dinf = __longlong_as_double(0x7ff0000000000000ll);
    const float lb0 = inb ? sc_lb[so + lane] : finf, ub0 = inb ? sc_ub[so + lane] : finf;
    const float lb1 = inb ? sc_lb[so + k + lane] : finf, ub1 = inb ? sc_ub[so + k + lane] : finf;
    const int R = min(k, kScoreRanks);
    // T_s >= the R-th smallest upper bound: bisection over the top 12 bits
    // of the (non-negative) float patterns, T_s = the top of the first
    // bucket by which R upper bounds have appeared (at most 1/8 above it).
    auto kth_ub = [&](float ub) -> float {
      uint32_t lo = 0u, hi = 0x7f800000u >> 20;
      const uint32_t bucket = __float_as_uint(ub) >> 20;
      while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (__popcll(__ballot(inb && bucket <= mid)) >= R) hi = mid; else lo = mid + 1;
      }
      return lo >= (0x7f800000u >> 20) ? __int_as_float(0x7f800000) : __uint_as_float(((lo + 1u) << 20) - 1u);
    };
    const float t0 = kth_ub(ub0), t1 = kth_ub(ub1);
    const unsigned long long x0 = __ballot(inb && lb0 <= t0), x1 = __ballot(inb && lb1 <= t1);
    const int n0 = __popcll(x0), n1 = __popcll(x1), nx = n0 + n1;
    if (nx <= kWave) {
      int *xl = S.rowcnt;  // 2K ints: entry t = half << 6 | centroid, half 0 first
      const unsigned long long below = lanes_below_mask();
      if ((x0 >> lane) & 1ull) xl[__popcll(x0 & below)] = lane;
      if ((x1 >> lane) & 1ull) xl[n0 + __popcll(x1 & below)] = 64 | lane;
      __syncthreads();
      int es = 0, ec = 0;
      double ex = dinf;
      if (lane < nx) {
        const int e = xl[lane];
        es = e >> 6;
        ec = e & 63;
        const float *ctp = cent_t + static_cast<long long>(sub * 2 + es) * h * k + ec;
        double acc = 0.0;
        for (int t = 0; t < h; ++t) {
          double delta = S.qs[es * h + t] - static_cast<double>(ctp[t * k]);
          double sq = delta * delta;
          acc = acc + sq;
        }
        ex = acc;
        S.hd[lane] = acc;
      }
      __syncthreads();
      int rank = 0;
      if (lane < nx) {
        const int b0 = es ? n0 : 0, b1 = es ? nx : n0;
        for (int t = b0; t < b1; ++t) {
          const double v = S.hd[t];
          const int c2 = xl[t] & 63;
          rank += (v < ex) || (v == ex && c2 < ec);
        }
        if (rank < R) {
          if (es == 0) { S.d1s[rank] = ex; S.o1[rank] = ec; }
          else { S.d2s[rank] = ex; S.o2[rank] = ec; }
        }
      }
      double l0 = (lane < nx && es == 0 && rank >= R) ? ex : dinf;
      double l1 = (lane < nx && es == 1 && rank >= R) ? ex : dinf;
      if (inb && !((x0 >> lane) & 1ull)) l0 = fmin(l0, static_cast<double>(lb0));
      if (inb && !((x1 >> lane) & 1ull)) l1 = fmin(l1, static_cast<double>(lb1));
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) {
        l0 = fmin(l0, __shfl_xor(l0, sh, kWave));
        l1 = fmin(l1, __shfl_xor(l1, sh, kWave));
      }
      __syncthreads();
      const int32_t *off = offsets + static_cast<long long>(sub) * (ncells + 1);
      const bool more = R < k;                          // ranks R.. exist and are not known exactly
      const bool rowl = lane < R;
      const double a = rowl ? S.d1s[lane] : 0.0;
      const int cbase = rowl ? S.o1[lane] * k : 0;
      int j = 0;
      int cell = rowl ? cbase + S.o2[0] : 0;
      int size = rowl ? off[cell + 1] - off[cell] : 0;
      double cost = rowl ? a + S.d2s[0] : dinf;
      double pend = dinf;                               // lower bound of the next cell once column R is reached
      const double urow = more ? l0 + S.d2s[0] : dinf;  // lower bound of row R's first cell
      int npop = 0, retr = 0, started = 0;
      double ccut = 0.0;
      bool met = false;
      while (npop < kPopCap) {
        double bc = dinf, bu = (started >= R) ? urow : dinf;
        int bi = -1;
        const int last = min(started, R - 1);
        for (int i = 0; i <= last; ++i) {
          const double ci = readlane_f64(cost, i);
          if (ci < bc) { bc = ci; bi = i; }
          bu = fmin(bu, readlane_f64(pend, i));
        }
        if (bi < 0 || bu <= bc) break;                 // an unknown rank could come next
        if (bi == started) ++started;
        const int psz = __builtin_amdgcn_readlane(size, bi);
        const int pcell = __builtin_amdgcn_readlane(cell, bi);
        if (lane == 0) S.pops[npop] = pcell | ((phi == 1 && npop < ksize ? 2 : 1) << 24);
        ++npop;
        retr += psz;
        ccut = bc;
        if (lane == bi) {
          ++j;
          if (j < R) {
            cell = cbase + S.o2[j];
            size = off[cell + 1] - off[cell];
            cost = a + S.d2s[j];
          } else {
            cost = dinf;
            if (more) pend = a + l1;
          }
        }
        if (retr >= budget) { met = true; break; }
      }
      if (met) {
        __syncthreads();
        int32_t *dst = cells_out + (static_cast<long long>(q) * m + sub) * ncells;
        double *st = sstat + (static_cast<long long>(q) * m + sub) * 4;
        for (int t = lane; t < npop; t += kWave) dst[t] = S.pops[t];
        if (lane == 0) {
          const double c1 = S.d1s[0] + S.d2s[0];
          double c2 = c1;
          if (k > 1) {
            const double u = S.d1s[0] + S.d2s[1], v = S.d1s[1] + S.d2s[0];
            c2 = u < v ? u : v;
          }
          ncell[static_cast<long long>(q) * m + sub] = npop;
          retrieved[static_cast<long long>(q) * m + sub] = retr;
          st[0] = c1;
          st[1] = c2;
          st[2] = ccut;
          const int cc = S.o1[0] * k + S.o2[0];
          st[3] = static_cast<double>(off[cc + 1] - off[cc]);
        }
        return;
      }
      __syncthreads();
    }
  }

  // the certified path did not decide this subspace: count it
  if (sc_lb != nullptr && sfall != nullptr && lane == 0) atomicAdd(&sfall[q], 1);
  // ---- Dist_1 / Dist_2 -----------------------------------------------------
  double *hout = hdist_out + (static_cast<long long>(q) * m + sub) * 2 * k;
  for (int s = 0; s < 2; ++s) {
    const float *ct = cent_t + static_cast<long long>(sub * 2 + s) * h * k;
    for (int c = lane; c < k; c += kWave) {
      double acc = 0.0;
      for (int t = 0; t < h; ++t) {
        double delta = S.qs[s * h + t] - static_cast<double>(ct[t * k + c]);
        double sq = delta * delta;
        acc = acc + sq;
      }
      S.hd[s * k + c] = acc;
      hout[s * k + c] = acc;
    }
  }
  __syncthreads();
  // ---- sort both halves by (distance, index) via ranks -----------------------
  for (int c = lane; c < k; c += kWave) {
    double v1 = S.hd[c], v2 = S.hd[k + c];
    int r1 = 0, r2 = 0;
    for (int c2 = 0; c2 < k; ++c2) {
      double u1 = S.hd[c2], u2 = S.hd[k + c2];
      r1 += (u1 < v1) || (u1 == v1 && c2 < c);
      r2 += (u2 < v2) || (u2 == v2 && c2 < c);
    }
    S.d1s[r1] = v1; S.o1[r1] = c;
    S.d2s[r2] = v2; S.o2[r2] = c;
  }
  __syncthreads();
  const int32_t *off = offsets + static_cast<long long>(sub) * (ncells + 1);
  int32_t *dst = cells_out + (static_cast<long long>(q) * m + sub) * ncells;
  double *st = sstat + (static_cast<long long>(q) * m + sub) * 4;
  const double c1 = S.d1s[0] + S.d2s[0];
  double c2 = c1;
  if (k > 1) {
    const double a = S.d1s[0] + S.d2s[1], b = S.d1s[1] + S.d2s[0];
    c2 = a < b ? a : b;
  }

  // ---- direct enumeration (K <= 64: lane i owns sorted row i) ---------------
  // Each step pops the smallest (cost, i) over the rows' next cells (within
  // a row cost and j ascend together), i.e. exactly the heap's order, until
  // the budget is met; typical budgets need a handful of cells.  If kPopCap
  // cells do not meet it, the bisection below decides instead.
  if (k <= kWave) {
    const bool row = lane < k;
    const double a = row ? S.d1s[lane] : 0.0;
    const int cbase = row ? S.o1[lane] * k : 0;
    int j = 0;
    int cell = row ? cbase + S.o2[0] : 0;
    int size = row ? off[cell + 1] - off[cell] : 0;
    double cost = row ? a + S.d2s[0] : __longlong_as_double(0x7ff0000000000000ll);
    int npop = 0, retr = 0;
    double ccut = 0.0;
    bool met = false;
    // Rows start in order (an unstarted row's cost d1s[i] + d2s[0] is
    // nondecreasing in i, so of the unstarted rows only the first can hold
    // the smallest (cost, row)); each pop therefore takes the smallest
    // (cost, row) over the started rows and the first unstarted one, read
    // from their lanes in ascending row order (strict < keeps the lower row
    // on equal costs).
    int started = 0;
    while (npop < kPopCap) {
      double bc = __longlong_as_double(0x7ff0000000000000ll);
      int bi = -1;
      const int last = min(started, k - 1);
      for (int i = 0; i <= last; ++i) {
        const double ci = readlane_f64(cost, i);
        if (ci < bc) { bc = ci; bi = i; }
      }
      if (bi < 0) break;                    // every cell popped: cannot happen before the budget is met
      if (bi == started) ++started;
      const int psz = __builtin_amdgcn_readlane(size, bi);
      const int pcell = __builtin_amdgcn_readlane(cell, bi);
      if (lane == 0) S.pops[npop] = pcell | ((phi == 1 && npop < ksize ? 2 : 1) << 24);
      ++npop;
      retr += psz;
      ccut = bc;
      if (lane == bi) {
        ++j;
        if (j < k) {
          cell = cbase + S.o2[j];
          size = off[cell + 1] - off[cell];
          cost = a + S.d2s[j];
        } else {
          cost = __longlong_as_double(0x7ff0000000000000ll);
        }
      }
      if (retr >= budget) { met = true; break; }
    }
    if (met) {
      __syncthreads();
      for (int t = lane; t < npop; t += kWave) dst[t] = S.pops[t];
      if (lane == 0) {
        ncell[static_cast<long long>(q) * m + sub] = npop;
        retrieved[static_cast<long long>(q) * m + sub] = retr;
        st[0] = c1;
        st[1] = c2;
        st[2] = ccut;
        const int c0 = S.o1[0] * k + S.o2[0];
        st[3] = static_cast<double>(off[c0 + 1] - off[c0]);
      }
      return;
    }
  }

  // Prefix sums of the cell sizes along each sorted row: a table in global
  // memory for K > 64; for K <= 64 (where this bisection runs only when the
  // direct enumeration ran out of pops) summed from the offsets on demand,
  // which keeps the kernel's LDS small for the common path.
  int *P = (k <= 64) ? nullptr : (ptab_g + (static_cast<long long>(q) * m + sub) * k * (k + 1));
  if (P) {
    for (int i = lane; i < k; i += kWave) {
      int base = S.o1[i] * k, acc = 0;
      P[i * (k + 1)] = 0;
      for (int j = 0; j < k; ++j) {
        int c = base + S.o2[j];
        acc += off[c + 1] - off[c];
        P[i * (k + 1) + j + 1] = acc;
      }
    }
  }
  __syncthreads();
  auto psum = [&](int i, int j) -> int {   // sizes of the first j cells of sorted row i
    if (P) return P[i * (k + 1) + j];
    const int base = S.o1[i] * k;
    int acc = 0;
    for (int jj = 0; jj < j; ++jj) {
      const int c = base + S.o2[jj];
      acc += off[c + 1] - off[c];
    }
    return acc;
  };

  auto size_le = [&](unsigned long long bits) -> int {
    double th = from_dbits(bits);
    int tot = 0;
    for (int i = lane; i < k; i += kWave) tot += psum(i, row_count_le(S.d1s, S.d2s, k, i, th));
    return wave_sum_i32(tot);
  };
  auto count_le = [&](unsigned long long bits) -> int {
    double th = from_dbits(bits);
    int tot = 0;
    for (int i = lane; i < k; i += kWave) tot += row_count_le(S.d1s, S.d2s, k, i, th);
    return wave_sum_i32(tot);
  };

  // ---- budget cutoff -------------------------------------------------------
  const unsigned long long top_bits = dbits(S.d1s[k - 1] + S.d2s[k - 1]);
  unsigned long long lo = dbits(S.d1s[0] + S.d2s[0]), hi = top_bits;
  if (lo > 0) --lo;  // the smallest key itself may be the cutoff
  while (lo < hi) {
    unsigned long long mid = lo + ((hi - lo) >> 1);
    if (size_le(mid) >= budget) hi = mid; else lo = mid + 1;
  }
  const unsigned long long cstar = hi;
  const int s_lt = (cstar > 0) ? size_le(cstar - 1) : 0;
  int istar = -1, jstar = -1;
  {
    int carry = 0;
    for (int r0 = 0; r0 < k && istar < 0; r0 += kWave) {
      int i = r0 + lane;
      int tlo = 0, thi = 0, tsz = 0;
      if (i < k) {
        thi = row_count_le(S.d1s, S.d2s, k, i, from_dbits(cstar));
        tlo = (cstar > 0) ? row_count_le(S.d1s, S.d2s, k, i, from_dbits(cstar - 1)) : 0;
        tsz = psum(i, thi) - psum(i, tlo);
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
          acc += psum(row, j + 1) - psum(row, j);
          if (acc >= budget) break;
        }
        istar = row;
        jstar = j;
      }
      carry = __shfl(incl, kWave - 1, kWave);
    }
  }
  for (int i = lane; i < k; i += kWave) {
    int n;
    if (i < istar) n = row_count_le(S.d1s, S.d2s, k, i, from_dbits(cstar));
    else if (i == istar) n = jstar + 1;
    else n = (cstar > 0) ? row_count_le(S.d1s, S.d2s, k, i, from_dbits(cstar - 1)) : 0;
    S.rowcnt[i] = n;
  }
  __syncthreads();
  int total = 0, retr = 0;
  for (int i = lane; i < k; i += kWave) {
    total += S.rowcnt[i];
    retr += psum(i, S.rowcnt[i]);
  }
  total = wave_sum_i32(total);
  retr = wave_sum_i32(retr);

  // ---- rank weights (Optimized Mode) ----------------------------------------
  if (phi == 1 && ksize >= total) {
    for (int i = lane; i < k; i += kWave) S.roww[i] = S.rowcnt[i];
  } else if (phi == 1) {
    unsigned long long lo2 = dbits(S.d1s[0] + S.d2s[0]), hi2 = top_bits;
    if (lo2 > 0) --lo2;
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
        thi = row_count_le(S.d1s, S.d2s, k, i, from_dbits(ck));
        tlo = (ck > 0) ? row_count_le(S.d1s, S.d2s, k, i, from_dbits(ck - 1)) : 0;
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
      if (i < ik) n = row_count_le(S.d1s, S.d2s, k, i, from_dbits(ck));
      else if (i == ik) n = jk + 1;
      else n = (ck > 0) ? row_count_le(S.d1s, S.d2s, k, i, from_dbits(ck - 1)) : 0;
      S.roww[i] = n;
    }
  } else {
    for (int i = lane; i < k; i += kWave) S.roww[i] = 0;
  }
  __syncthreads();

  // ---- emit (cell | weight << 24), rows in order ----------------------------
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
    // statistics for the learned budget: two smallest cell costs, the
    // cutoff cost, and the size of the cheapest cell
    st[0] = c1;
    st[1] = c2;
    st[2] = from_dbits(cstar);
    st[3] = static_cast<double>(psum(0, 1));
  }
}

// ---------------------------------------------------------------------------
// A3/A4: collision counting in LDS.  One 1024-thread block per (id tile,
// query).  The tile's uint8 counters are packed four per dword and
// incremented with ds_add_u32 of w shifted to the id's byte; scores never
// exceed 2M <= 254.  Within each group of 32 ids, id 8j + i (j < 4, i < 8)
// is byte j of the group's dword i, so that the threshold test of a dword
// lands, with one shift, on the bits that keep a lane's 64 counters in id
// order.  The posting lists are read in a load-time form: per entry, the
// uint16 byte position of its id's counter inside a 65,536-id tile (the
// layout above, which permutes only within groups of 32, so the position in
// a tile of 2^t <= 65,536 ids is the low t bits); a counter update is then an
// AND, two shifts and the atomic.  Work items are (subspace, activated cell)
// pairs; each contributes the slice of the cell's posting list inside the
// tile (from the load-time cell x tile table).  The block cuts the slices
// into sub-slices of at most 64 entries and lists them in LDS; waves take
// eight consecutive sub-slices at a time, round robin, with each record in
// scalar registers, and issue the eight 64-lane loads before the first
// counter update, so that a wave waits for memory once per eight
// sub-slices.  The block's setup costs two dependent round trips to memory
// when every subspace activates at most 1024 / M cells (counts and cells
// loaded together, then the table), three otherwise.
// Each of the 16 waves then scans its sixteenth of the counters (64 per lane
// per step, four bytes of a dword tested by one 32-bit add when 2M < 128,
// else in two 16-bit fields) and writes the ids reaching the threshold, in
// ascending order, to its own segment; segment counts go to
// seg_cnt[q][tile][wave].
//
// pass 0: threshold tau, write candidates, histogram of scores >= max(tau, 1)
// pass 1: queries flagged for the fallback only: histogram of scores >= 1
// pass 2: queries flagged only: threshold tau_eff, write candidates
// ---------------------------------------------------------------------------
constexpr int kCountThreads = 1024;
constexpr int kCountWaves = kCountThreads / kWave;
constexpr int kSub = 1280;    // sub-slices (<= 64 entries) per batch
constexpr int kG = 8;         // sub-slices per wave per round (loads in flight)
static_assert(kG > 0 && kG <= kWave && (kG & (kG - 1)) == 0, "a wave's lanes u < kG read its kG records");

// LDS byte offset of the counter of tile-local id loc (the layout above).
__device__ __forceinline__ int cnt_dword_bytes(int loc) { return (loc & ~31) | ((loc << 2) & 31); }
__device__ __forceinline__ int cnt_byte(int loc) { return cnt_dword_bytes(loc) | ((loc >> 3) & 3); }

// A posting-list entry in global memory (a pointer formed from values read
// back from LDS would otherwise be treated as generic and loaded with flat
// instructions).
typedef const uint16_t __attribute__((address_space(1))) *global_u16_ptr;
typedef uint32_t __attribute__((address_space(3))) *lds_u32_ptr;

// Adds v to the LDS dword at byte address addr.
__device__ __forceinline__ void lds_add(uint32_t addr, uint32_t v) {
  __hip_atomic_fetch_add(reinterpret_cast<lds_u32_ptr>(static_cast<uintptr_t>(addr)), v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct CountShared {
  // per sub-slice: element offset of its first entry in the position array;
  // length << 8 | rank weight.  kG empty entries follow the last one.
  uint32_t soff[kSub + kG], slw[kSub + kG];
  int mbase[129];
  int hist[256];
  int tmp[kCountWaves + 1];
  int wide[kCountWaves];
  int misc;
};

#define CRISP_COUNT_PARAMS                                                                                      \
  const int32_t *__restrict__ ncell, const int32_t *__restrict__ cells, int m, int ncells,                      \
      const uint16_t *__restrict__ pos, long long n, const int32_t *__restrict__ tile_off, int ntiles,         \
      int tile_ids, int tau, const int32_t *__restrict__ flag, const int32_t *__restrict__ tau_eff,            \
      int32_t *__restrict__ seg_ids, uint8_t *__restrict__ seg_score, int32_t *__restrict__ seg_cnt,           \
      int32_t *__restrict__ hist, const int32_t *__restrict__ live
#define CRISP_COUNT_ARGS                                                                                 \
  ncell, cells, m, ncells, pos, n, tile_off, ntiles, tile_ids, tau, flag, tau_eff, seg_ids, seg_score, seg_cnt, \
      hist, live

// The block's counting rounds over the sub-slice list (total_sub records in
// S.soff / S.slw, followed by kG empty ones).  Waves take kG consecutive
// sub-slices at a time, round robin; lane u < kG reads record c0 + u, which
// then goes to scalar registers.  All kG loads are issued before the first
// counter update; they are unconditional (a lane past the end of its
// sub-slice reads the entries that follow, which exist: the position array
// ends with 64 spare entries; an empty record reads the first 64), so that
// no value register carries over between rounds and the loads overlap.
template <typename Shared>
__device__ __forceinline__ void count_rounds(const Shared &S, int total_sub, const uint16_t *__restrict__ pos,
                                             uint32_t amask) {
  const int lane = lane_id();
  const int wave0 = __builtin_amdgcn_readfirstlane(wave_id());
  for (int c0 = wave0 * kG; c0 < total_sub; c0 += kG * kCountWaves) {
    const int mi = c0 + (lane & (kG - 1));
    const int moff = static_cast<int>(S.soff[mi]), mlw = static_cast<int>(S.slw[mi]);
    uint32_t pv[kG];
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const uint32_t o = static_cast<uint32_t>(__builtin_amdgcn_readlane(moff, u));
      pv[u] = *(global_u16_ptr)(reinterpret_cast<const char *>(pos) + 2u * (o + static_cast<uint32_t>(lane)));
    }
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const uint32_t l = static_cast<uint32_t>(__builtin_amdgcn_readlane(mlw, u));
      if (lane < static_cast<int>(l >> 8)) lds_add(pv[u] & amask, (l & 255u) << ((pv[u] << 3) & 31));
    }
  }
}

// Sum of v[0 .. 15] (the block's per-wave values) and of v[0 .. w - 1], w
// uniform over the wave: lane j < 16 reads v[j], then a wave scan.
__device__ __forceinline__ int2 waves_total_and_before(const int *v, int w) {
  const int lane = lane_id();
  const int sc = wave_incl_scan_i32(lane < kCountWaves ? v[lane] : 0);
  const int total = __builtin_amdgcn_readlane(sc, kCountWaves - 1);
  const int before = w > 0 ? __builtin_amdgcn_readlane(sc, w - 1) : 0;
  return make_int2(total, before);
}

// Writes the sub-slices of one activated cell's slice (element offset off,
// length len, rank weight w) from record index at.
template <typename Shared>
__device__ __forceinline__ void put_subslices(Shared &S, int at, uint32_t off, int len, uint32_t w) {
  for (int k = 0; k * kWave < len; ++k) {
    S.soff[at + k] = off + static_cast<uint32_t>(k * kWave);
    S.slw[at + k] = (static_cast<uint32_t>(min(kWave, len - k * kWave)) << 8) | w;
  }
}

// Threshold scan of one tile's counters: each of the 16 waves scans its
// sixteenth (64 counters per lane per step, four bytes of a dword tested by
// one 32-bit add when 2M < 128, else in two 16-bit fields), counts the scores
// >= 1 reached into the block's histogram (passes 0 and 1) and writes the ids
// reaching the threshold, in ascending order, to its own segment (passes 0
// and 2); returns the wave's candidate count.
template <int kPass, typename Shared>
__device__ __forceinline__ int scan_tile(Shared &S, const uint32_t *cnt, int q, long long t0, int tlen, int ndw,
                                         int m, int thr, long long n, int32_t *__restrict__ seg_ids,
                                         uint8_t *__restrict__ seg_score) {
  constexpr int pass = kPass;
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(wave_id());
  const int per_wave = ndw / kCountWaves;            // dwords per wave (tiles of 2^12..2^16 ids: a multiple of 256)
  const int dw0 = wv * per_wave;
  // The wave's segment; candidates are stored at 32-bit offsets from it.
  char *dst = reinterpret_cast<char *>(seg_ids + static_cast<long long>(q) * n + t0 + static_cast<long long>(dw0) * 4);
  char *dsc = reinterpret_cast<char *>(seg_score + static_cast<long long>(q) * n + t0 + static_cast<long long>(dw0) * 4);
  int run = 0;
  // Bytes >= thr, four at a time.  When 2M < 128 adding 128 - thr to every
  // byte of a dword sets each byte's bit 7 exactly when the byte is >= thr
  // (no carry leaves a byte).  Otherwise the even and odd bytes sit in
  // 16-bit fields, and adding 256 - thr to a field sets its bit 8 exactly
  // when the byte is >= thr.
  const bool narrow = 2 * m < 128;
  const uint32_t add4 = static_cast<uint32_t>(0x80 - thr) * 0x01010101u;
  const uint32_t add = static_cast<uint32_t>(0x100 - thr) * 0x00010001u;
  const uint8_t *cnt8 = reinterpret_cast<const uint8_t *>(cnt);
  const uint4 *cnt4 = reinterpret_cast<const uint4 *>(cnt);
  constexpr int kScanDw = 8;                         // dwords (32 counters, one group of 32 ids) per lane per step
  for (int v0 = 0; v0 < per_wave; v0 += kScanDw * kWave) {
    const int dwl = v0 + kScanDw * lane;             // this lane's first dword within the wave range
    uint32_t words[kScanDw];
#pragma unroll
    for (int u = 0; u < kScanDw / 4; ++u) {
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (dwl < per_wave) v = cnt4[((dw0 + dwl) >> 2) + u];
      words[4 * u] = v.x; words[4 * u + 1] = v.y; words[4 * u + 2] = v.z; words[4 * u + 3] = v.w;
    }
    const int idbase = (dw0 + dwl) * 4;              // tile-local id of the first counter (a multiple of 32)
    // Bit 8j + i of sel (dword i, byte j) is the counter of id idbase + 8j + i.
    uint32_t sel = 0u;
    if (narrow) {
#pragma unroll
      for (int j = 0; j < kScanDw; ++j) sel |= ((words[j] + add4) >> (7 - j)) & (0x01010101u << j);
    } else {
#pragma unroll
      for (int j = 0; j < kScanDw; ++j) {
        const uint32_t ge = (words[j] & 0x00FF00FFu) + add;           // bytes 0, 2 -> bits 8, 24
        const uint32_t go = ((words[j] >> 8) & 0x00FF00FFu) + add;    // bytes 1, 3 -> bits 8, 24
        sel |= ((ge >> (8 - j)) & (0x00010001u << j)) | ((go << j) & (0x01000100u << j));
      }
    }
    const int nvalid = (dwl < per_wave) ? min(max(tlen - idbase, 0), 4 * kScanDw) : 0;
    sel &= (nvalid >= 32) ? ~0u : ((1u << nvalid) - 1u);
    const int c = __popc(sel);
    int pos = run;
    if (pass != 1) {
      // exclusive prefix of c over the lanes, and the step's total
      const int incl = wave_incl_scan_dpp(c);
      pos += incl - c;
      run += __builtin_amdgcn_readlane(incl, kWave - 1);
    }
    while (sel) {
      const int e = __builtin_ctz(sel);               // id idbase + e: dword e & 7, byte e >> 3 of the group
      sel &= sel - 1u;
      const int sc = cnt8[idbase + ((e & 7) << 2) + (e >> 3)];
      if (pass != 2 && sc >= 1) atomicAdd(&S.hist[sc], 1);
      if (pass != 1) {
        *reinterpret_cast<int32_t *>(dst + 4u * static_cast<uint32_t>(pos)) = static_cast<int32_t>(t0) + idbase + e;
        *reinterpret_cast<uint8_t *>(dsc + static_cast<uint32_t>(pos)) = static_cast<uint8_t>(sc);
        ++pos;
      }
    }
  }
  return run;
}

// One block's work: tiles tile_lo .. tile_hi - 1 of query q, in turn; every
// early return is uniform over the block.
template <int kPass>
__device__ __forceinline__ void count_block(const int tile_lo, const int tile_hi, const int q, CRISP_COUNT_PARAMS) {
  constexpr int pass = kPass;
  // dynamic LDS: the tile's counters first, then the block's shared records.
  // The kernel has no static LDS (checked on the host at index load), so the
  // counters start at LDS address 0 and a counter's byte position within the
  // tile is its LDS address.
  extern __shared__ __align__(16) uint32_t cnt[];
  CountShared &S = *reinterpret_cast<CountShared *>(reinterpret_cast<char *>(cnt) + tile_ids);
  const int tid = threadIdx.x;
  if (live && q >= *live) return;
  if (pass != 0 && flag[q] == 0) return;
  const int ndw = tile_ids >> 2;  // counters allocated for a full tile
  const int thr = (pass == 0) ? tau : (pass == 1 ? 1 : tau_eff[q]);
  const int lane = lane_id();
  const int wv0 = wave_id();
  const long long qm = static_cast<long long>(q) * m;
  // Counter dword of a position: its low t bits with the byte bits cleared;
  // the byte's shift (8 x its low two bits) is what a 32-bit shift keeps of
  // the position times 8.
  const uint32_t amask = static_cast<uint32_t>(tile_ids - 1) & ~3u;
  // Direct slots: thread t stands for cell t % J of subspace t / J, with J =
  // 1024 / m rounded down to a power of two.  Its subspace's count and the
  // cell are loaded together (the cell speculatively: in bounds, used only
  // when t % J is below the count), then the cell's row of the cell x tile
  // table, whose entry for the next tile is always loaded one tile ahead.
  const int jl = 31 - __builtin_clz(static_cast<unsigned>(kCountThreads / m));   // log2 J
  const int fs = tid >> jl, fj = tid & ((1 << jl) - 1);
  int nco = 0, fpk = 0;
  if (fs < m) {
    nco = ncell[qm + fs];
    if (fj < ncells) fpk = cells[(qm + fs) * ncells + fj];
  }
  const bool valid = fs < m && fj < nco;
  // the slot's row of the cell x tile table (an element index)
  const uint32_t row = valid ? static_cast<uint32_t>((fs * ncells + (fpk & 0xFFFFFF)) * (ntiles + 1)) : 0u;
  int ta = 0, tb = 0;                                      // the slot's slice of the current tile
  if (valid) {
    ta = tile_off[row + tile_lo];
    tb = tile_off[row + tile_lo + 1];
  }
  for (int i = tid; i < 256; i += kCountThreads) S.hist[i] = 0;
  bool general = false, have_mbase = false;
  for (int tile = tile_lo; tile < tile_hi; ++tile) {
    const long long t0 = static_cast<long long>(tile) * tile_ids;
    const int tlen = static_cast<int>(min(static_cast<long long>(tile_ids), n - t0));
    const int tn = (valid && tile + 2 <= ntiles) ? tile_off[row + tile + 2] : 0;   // next tile's end, loaded ahead
    uint4 *cnt4 = reinterpret_cast<uint4 *>(cnt);
    for (int i = tid; i < (ndw >> 2); i += kCountThreads) cnt4[i] = make_uint4(0u, 0u, 0u, 0u);
    const int len = tb - ta;
    const int nsub = valid ? (len + kWave - 1) / kWave : 0;
    const int incl = wave_incl_scan_i32(nsub);
    if (tile == tile_lo) {
      const bool wide = __builtin_amdgcn_ballot_w64(fs < m && fj == 0 && nco > (1 << jl)) != 0;
      if (lane == 0) S.wide[wv0] = wide;
    }
    if (lane == kWave - 1) S.tmp[wv0] = incl;
    __syncthreads();
    const int2 tb2 = waves_total_and_before(S.tmp, wv0);
    const int total = tb2.x, excl = incl - nsub + tb2.y;
    if (tile == tile_lo) general = __builtin_amdgcn_ballot_w64(lane < kCountWaves && S.wide[lane] != 0) != 0;
    // Common case: every activated cell has a direct slot and all the
    // tile's sub-slices fit in the list (one round of the loop below).
    // Otherwise the activated cells are taken in subspace order (item g lies
    // in subspace s with mbase[s] <= g < mbase[s + 1]), in batches whose
    // sub-slices fit in the list.
    const bool batched = general || total > kSub;
    int total_items = 0;
    if (batched) {
      __syncthreads();                                     // every wave has read S.tmp
      if (!have_mbase) {
        // Per-subspace counts -> prefix mbase[0..m] (m <= 127: waves 0 and
        // 1 load and scan them in parallel).
        const int v = (tid < m) ? ncell[qm + tid] : 0;
        const int inc = wave_incl_scan_i32(v);
        if (tid == kWave - 1) S.tmp[0] = inc;
        __syncthreads();
        if (tid < 2 * kWave) S.mbase[tid + 1] = inc + (tid >= kWave ? S.tmp[0] : 0);
        if (tid == 0) S.mbase[0] = 0;
        __syncthreads();
        have_mbase = true;
      }
      total_items = S.mbase[m];
    }
    for (int b0 = 0;;) {
      int total_sub = total, taken = 0;
      if (!batched) {
        if (nsub > 0)
          put_subslices(S, excl, static_cast<uint32_t>(static_cast<long long>(fs) * n + ta), len,
                        static_cast<uint32_t>(fpk) >> 24);
        if (tid < kG) {
          S.soff[total + tid] = 0;
          S.slw[total + tid] = 0;
        }
        __syncthreads();
      } else {
        if (b0 >= total_items) break;
        // Items b0 .. b0 + nb - 1, one per thread; the items whose
        // sub-slices fit in the list are taken (at least the first: a slice
        // has at most 65,536 / 64 = 1,024 <= kSub of them).
        const int nb = min(kCountThreads, total_items - b0);
        uint32_t goff = 0, glw = 0;
        int gsub = 0;
        if (tid < nb) {
          const int g = b0 + tid;
          const int s = upper_bound_minus1(S.mbase, m + 1, g);
          const int packed = cells[(qm + s) * ncells + (g - S.mbase[s])];
          const int32_t *gto = tile_off + (static_cast<long long>(s) * ncells + (packed & 0xFFFFFF)) * (ntiles + 1);
          const int a = gto[tile];
          const int gl = gto[tile + 1] - a;
          goff = static_cast<uint32_t>(static_cast<long long>(s) * n + a);   // M x N < 2^31
          glw = (static_cast<uint32_t>(gl) << 8) | (static_cast<uint32_t>(packed) >> 24);
          gsub = (gl + kWave - 1) / kWave;
        }
        const int inc = wave_incl_scan_i32(gsub);
        if (lane == kWave - 1) S.tmp[wv0] = inc;
        __syncthreads();
        const int gex = inc - gsub + waves_total_and_before(S.tmp, wv0).y;
        const bool fits = tid < nb && gex + gsub <= kSub;
        const unsigned long long fb = __builtin_amdgcn_ballot_w64(fits);
        __syncthreads();                                   // every wave has read S.tmp
        if (lane == 0) S.tmp[wv0] = __popcll(fb);
        __syncthreads();
        taken = waves_total_and_before(S.tmp, 0).x;
        if (fits) {
          if (gsub > 0) put_subslices(S, gex, goff, static_cast<int>(glw >> 8), glw & 255u);
          if (tid == taken - 1) {                          // the last item taken closes the list
            S.misc = gex + gsub;
            for (int k = 0; k < kG; ++k) {
              S.soff[gex + gsub + k] = 0;
              S.slw[gex + gsub + k] = 0;
            }
          }
        }
        __syncthreads();
        total_sub = S.misc;
      }
      count_rounds(S, total_sub, pos, amask);
      __syncthreads();
      if (!batched) break;
      b0 += taken;
    }
    const int run = scan_tile<kPass>(S, cnt, q, t0, tlen, ndw, m, thr, n, seg_ids, seg_score);
    if (pass != 1 && lane == 0) seg_cnt[(static_cast<long long>(q) * ntiles + tile) * kCountWaves + wv0] = run;
    __syncthreads();                                       // the counters are read before the next tile clears them
    ta = tb;
    tb = tn;
  }
  if (pass != 2) {
    const int nb = 2 * m + 1;
    for (int s = tid; s < nb; s += kCountThreads)
      if (S.hist[s]) atomicAdd(&hist[static_cast<long long>(q) * nb + s], S.hist[s]);
  }
}

// pass 0: grid (tile groups, queries), each block counting tiles_per_block
// consecutive tiles of its query.  Passes 1 and 2 concern the queries k_flag
// listed (flist[0 .. *nflag)), usually none: a grid of (tile groups, a few
// hundred) blocks walks the list instead of launching a block for every
// query.
// At most 80 scalar registers: with more, two 16-wave blocks do not fit on a
// compute unit together (measured: 96 registers left one resident block per
// unit and took 1.5x as long; the few values over the budget go to lanes of
// a vector register).
template <int kPass>
__global__ void __launch_bounds__(kCountThreads) __attribute__((amdgpu_num_sgpr(80)))
k_count(CRISP_COUNT_PARAMS, const int32_t *__restrict__ flist, const int32_t *__restrict__ nflag,
        int tiles_per_block) {
  const int tile_lo = blockIdx.x * tiles_per_block;
  const int tile_hi = min(tile_lo + tiles_per_block, ntiles);
  if constexpr (kPass == 0) {
    count_block<0>(tile_lo, tile_hi, blockIdx.y, CRISP_COUNT_ARGS);
  } else {
    const int nf = *nflag;
    for (int i = blockIdx.y; i < nf; i += gridDim.y) {
      count_block<kPass>(tile_lo, tile_hi, flist[i], CRISP_COUNT_ARGS);
      __syncthreads();
    }
  }
}

// Per query (one wavefront): |C| at tau; flag the fallback when fewer than k
// points reach it, and list the flagged queries.
__global__ void k_flag(const int32_t *__restrict__ seg_cnt, int nseg, int nq, int k, int tau,
                       int32_t *__restrict__ flag, int32_t *__restrict__ tau_eff, int32_t *__restrict__ hist,
                       int nbins, const int32_t *__restrict__ live, int32_t *__restrict__ flist,
                       int32_t *__restrict__ nflag) {
  const int q = blockIdx.x * (blockDim.x / kWave) + wave_id();
  if (q >= nq || (live && q >= *live)) return;
  const int lane = lane_id();
  int tot = 0;
  for (int t = lane; t < nseg; t += kWave) tot += seg_cnt[static_cast<long long>(q) * nseg + t];
  tot = wave_sum_i32(tot);
  const int f = (tot < k && tau > 1) ? 1 : 0;
  if (lane == 0) {
    flag[q] = f;
    tau_eff[q] = tau;
    if (f) flist[atomicAdd(nflag, 1)] = q;   // nflag is zero at launch
  }
  if (f)
    for (int s = lane; s < nbins; s += kWave) hist[static_cast<long long>(q) * nbins + s] = 0;
}

// Flagged queries: tau_eff = largest s <= tau with at least k points scoring
// >= s, else 1; keep the histogram only from tau_eff up.
__global__ void k_tau_eff(const int32_t *__restrict__ flag, int nq, int k, int tau, int nbins,
                          int32_t *__restrict__ hist, int32_t *__restrict__ tau_eff,
                          int32_t *__restrict__ seg_cnt, int nseg, const int32_t *__restrict__ live) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq || (live && q >= *live) || flag[q] == 0) return;
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
  for (int t = 0; t < nseg; ++t) seg_cnt[static_cast<long long>(q) * nseg + t] = 0;
}

// Concatenate the per-(tile, wave) candidate segments into one ascending list.
constexpr int kCompactThreads = 256;

// cap: capacity of a query's candidate list (its stride in cand / score);
// a query with more candidates keeps the first cap, and its index in the
// batch (q_base + q) is appended to ovf_list (count in *ovf_count, which the
// caller clears) to be searched again with lists of n entries.
__global__ void __launch_bounds__(kCompactThreads) k_compact(
    const int32_t *__restrict__ seg_ids, const uint8_t *__restrict__ seg_score, const int32_t *__restrict__ seg_cnt,
    int nseg, int seg_len, long long n, long long cap, int32_t *__restrict__ cand, uint8_t *__restrict__ score,
    int32_t *__restrict__ ncand, const int32_t *__restrict__ live, int32_t *__restrict__ ovf_count,
    int32_t *__restrict__ ovf_list, long long q_base) {
  __shared__ int base[kCompactThreads + 1];
  __shared__ int tmp[kCompactThreads / kWave + 1];
  __shared__ int carry;
  const int q = blockIdx.x, tid = threadIdx.x;
  if (live && q >= *live) return;
  const long long qs = static_cast<long long>(q) * n;     // the query's segments
  const long long qo = static_cast<long long>(q) * cap;   // its candidate list
  const int32_t *sc = seg_cnt + static_cast<long long>(q) * nseg;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int s0 = 0; s0 < nseg; s0 += kCompactThreads) {
    const int ns = min(kCompactThreads, nseg - s0);
    base[tid] = (tid < ns) ? sc[s0 + tid] : 0;
    __syncthreads();
    const int tot = block_exclusive_scan(base, kCompactThreads, tmp);
    // copy the ns segments: thread t writes list positions carry + j for
    // j = t, t + 256, ... (segment of j by binary search over the prefix),
    // kU positions in flight per thread
    const int lim = static_cast<int>(max(0ll, min(static_cast<long long>(tot), cap - carry)));
    constexpr int kU = 8;
    for (int j0 = 0; j0 < lim; j0 += kCompactThreads * kU) {
      int32_t iv[kU];
      uint8_t sv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = min(j0 + u * kCompactThreads + tid, lim - 1);   // clamped: every load is issued
        const int sg = upper_bound_minus1(base, ns, j);                // base[sg] <= j < base[sg + 1]
        const long long src = qs + static_cast<long long>(s0 + sg) * seg_len + (j - base[sg]);
        iv[u] = seg_ids[src];
        sv[u] = seg_score[src];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * kCompactThreads + tid;
        if (j < lim) {
          cand[qo + carry + j] = iv[u];
          score[qo + carry + j] = sv[u];
        }
      }
    }
    __syncthreads();
    if (tid == 0) carry += tot;
    __syncthreads();
  }
  if (tid == 0) {
    ncand[q] = static_cast<int32_t>(min(static_cast<long long>(carry), cap));
    if (carry > cap) ovf_list[atomicAdd(ovf_count, 1)] = static_cast<int32_t>(q_base + q);
  }
}

// Run order of a chunk's queries for the stages that read candidate rows
// (Hamming distances, re-rank): ascending smallest candidate id, ties by query
// index, queries past the live count and queries with no candidates last, so
// live queries fill the first live-count positions.  Queries whose candidate
// sets overlap then run side by side and find the shared code and base rows
// in L2 / the last-level cache instead of HBM.  It only decides which query
// a block takes: every per-query result is the same in any order.  One
// block, bitonic sort of (key << 12 | q) in LDS.
constexpr int kQueryOrderMax = 4096;
constexpr int kQueryOrderThreads = 1024;
constexpr int kQueryOrderBits = 12;
static_assert(kQueryOrderMax <= (1 << kQueryOrderBits), "query index must fit its field");

// cap: the stride of a query's candidate list; n: a key above every id.
// Bitonic network over kQueryOrderMax keys (padded with the largest key),
// thread t holding keys 4t .. 4t + 3 in registers: exchanges at distance 1
// and 2 stay in the thread, distances 4 .. 128 are lane shuffles within the
// wavefront, and only the ten stages at distance >= 256 go through LDS.
__global__ void __launch_bounds__(kQueryOrderThreads) k_query_order(int cq, const int32_t *__restrict__ ncand,
                                                                    const int32_t *__restrict__ cand, long long n,
                                                                    long long cap, int32_t *__restrict__ order,
                                                                    const int32_t *__restrict__ live) {
  static_assert(kQueryOrderMax == 4 * kQueryOrderThreads, "four keys per thread");
  __shared__ long long key[kQueryOrderMax];
  const int nl = live ? min(cq, *live) : cq;
  const int tid = threadIdx.x;
  long long v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * tid + e;
    long long x = 0x7fffffffffffffffll;
    if (i < cq) {
      const long long first = (i < nl && ncand[i] > 0) ? cand[static_cast<long long>(i) * cap] : n;
      x = (first << kQueryOrderBits) | i;
    }
    v[e] = x;
  }
  // key i takes the smaller of (i, i ^ j) when i is the lower index of the
  // pair in an ascending run (i & len == 0), or the higher one in a
  // descending run; the larger otherwise
  for (int len = 2; len <= kQueryOrderMax; len <<= 1) {
    for (int j = len >> 1; j > 0; j >>= 1) {
      long long w[4];
      if (j >= 256) {
#pragma unroll
        for (int e = 0; e < 4; ++e) key[4 * tid + e] = v[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = key[(4 * tid + e) ^ j];
        __syncthreads();
      } else if (j >= 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = __shfl_xor(v[e], j >> 2, kWave);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = v[e ^ j];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 4 * tid + e;
        const bool lower = (i & j) == 0, up = (i & len) == 0;
        const bool take_min = lower == up;
        v[e] = take_min ? min(v[e], w[e]) : max(v[e], w[e]);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * tid + e;
    if (i < cq) order[i] = static_cast<int32_t>(v[e] & ((1ll << kQueryOrderBits) - 1));
  }
}

// ---------------------------------------------------------------------------
// A5: Hamming order, in two kernels.
//
// k_hamming_dist: gx blocks per query (gx chosen from the batch size so that a
// small batch still spreads over the chip), in run order, dealt to the XCDs
// in contiguous ranges.  Each wavefront takes 64
// consecutive candidates at a time (one coalesced id load, ids passed
// between lanes by shuffles), striding over the query's list with the
// other gx * 4 - 1 wavefronts of its query.  The query's sign code is built
// by ballots over q' (bit i%64 of word i/64 = [q'_i > 0]).  A code row is
// read by L lanes (L = the largest power of two with kVec * L <= min(16,
// words)), each reading kVec consecutive 64-bit words per load (kVec = 2,
// 16-byte loads, when rows have an even number of words); four rows times
// up to four loads per lane are in flight per batch, and the partial
// popcounts are reduced over the row's L lanes.
//
// k_hamming_order (below) places the candidates in (distance, id) order.
// ---------------------------------------------------------------------------
constexpr int kOrderThreads = 256;
constexpr int kOrderSpan = 1024;  // distance bins placed by all four waves (per-wave counts)
constexpr int kOrderWaves = kOrderThreads / kWave;

template <int kVec>
struct CodeVec;
template <>
struct CodeVec<1> {
  using T = unsigned long long;
  static __device__ __forceinline__ int pop(const uint64_t *qc, int w, T v) { return __popcll(qc[w] ^ v); }
};
template <>
struct CodeVec<2> {
  using T = ulonglong2;
  static __device__ __forceinline__ int pop(const uint64_t *qc, int w, T v) {
    return __popcll(qc[w] ^ v.x) + __popcll(qc[w + 1] ^ v.y);
  }
};

__host__ __device__ inline int hamming_vec(int words) { return (words % 2 == 0) ? 2 : 1; }

constexpr int kHamRows = 4, kHamLoads = 4;  // code rows per lane step, loads per row in flight

// Lanes per code row and loads per row per lane for rows of `words` 64-bit
// words read kVec at a time.
__host__ __device__ inline int hamming_lanes(int words, int vec) {
  const int span = words / vec;
  return span >= 8 ? 8 : span >= 4 ? 4 : span >= 2 ? 2 : 1;
}
__host__ __device__ inline int hamming_loads(int words, int vec) {
  const int span = words / vec, L = hamming_lanes(words, vec);
  return (span + L - 1) / L;
}

// kJ > 0: every lane makes exactly kJ (at most kHamLoads) loads per row
// (D <= 4096), so the lane's query words stay in registers and each row's
// loads are issued unconditionally (a row past the list is read as a clamped
// one and not stored; a load past the row's end is read clamped and not
// counted).  kJ = 0: any row length.
template <int kVec, int kJ>
__global__ void __launch_bounds__(kOrderThreads) k_hamming_dist(
    const float *__restrict__ qrot, int d, const uint64_t *__restrict__ codes, const int32_t *__restrict__ ncand,
    const int32_t *__restrict__ cand, long long cap, int32_t *__restrict__ hm_tmp, const int32_t *__restrict__ live,
    const int32_t *__restrict__ order, int gx, int cq) {
  using V = typename CodeVec<kVec>::T;
  __shared__ __align__(16) uint64_t qc[128];
  const int lb = xcd_major(blockIdx.x, gridDim.x);
  if (lb >= gx * cq) return;
  const int bx = lb % gx, pos = lb / gx;
  const int q = order ? order[pos] : pos, lane = lane_id(), wv = wave_id();
  if (live && q >= *live) return;
  const int words = d / 64;
  const int nc = ncand[q];
  const long long qo = static_cast<long long>(q) * cap;
  for (int w = wv; w < words; w += kOrderWaves) {
    unsigned long long b = __ballot(qrot[static_cast<long long>(q) * d + w * 64 + lane] > 0.0f);
    if (lane == 0) qc[w] = b;
  }
  __syncthreads();
  const int span = words / kVec;                      // loads that cover a row
  const int L = hamming_lanes(words, kVec);
  const int rows_per = kWave / L;
  const int sub = lane % L, rsel = lane / L;
  const int J = (span + L - 1) / L;                   // loads per row per lane
  const int stride = gx * kOrderWaves * kWave;
  if constexpr (kJ > 0) {
    V qv[kJ];
    bool ve[kJ];
    int vo[kJ];
#pragma unroll
    for (int e = 0; e < kJ; ++e) {
      const int v = sub + e * L;
      ve[e] = v < span;
      vo[e] = min(v, span - 1);
      qv[e] = reinterpret_cast<const V *>(qc)[vo[e]];
    }
    for (int base = (bx * kOrderWaves + wv) * kWave; base < nc; base += stride) {
      const int my_id = cand[qo + min(base + lane, nc - 1)];
      for (int s0 = 0; s0 < L; s0 += kHamRows) {
        V cw[kHamRows][kJ];
#pragma unroll
        for (int u = 0; u < kHamRows; ++u) {
          const int r = min(s0 + u, L - 1) * rows_per + rsel;
          const V *row = reinterpret_cast<const V *>(codes + static_cast<long long>(__shfl(my_id, r, kWave)) * words);
#pragma unroll
          for (int e = 0; e < kJ; ++e) cw[u][e] = row[vo[e]];
        }
#pragma unroll
        for (int u = 0; u < kHamRows; ++u) {
          int h = 0;
#pragma unroll
          for (int e = 0; e < kJ; ++e) {
            int c;
            if constexpr (kVec == 2) c = __popcll(qv[e].x ^ cw[u][e].x) + __popcll(qv[e].y ^ cw[u][e].y);
            else c = __popcll(qv[e] ^ cw[u][e]);
            h += ve[e] ? c : 0;
          }
          for (int s2 = L >> 1; s2 >= 1; s2 >>= 1) h += __shfl_xor(h, s2, kWave);
          const int row_at = base + (s0 + u) * rows_per + rsel;
          if (sub == 0 && s0 + u < L && row_at < nc) hm_tmp[qo + row_at] = h;
        }
      }
    }
    return;
  }
  for (int base = (bx * kOrderWaves + wv) * kWave; base < nc; base += stride) {
    const int my_id = cand[qo + min(base + lane, nc - 1)];
    for (int s0 = 0; s0 < L; s0 += kHamRows) {
      int hs[kHamRows], idr[kHamRows];
      bool rok[kHamRows];
#pragma unroll
      for (int u = 0; u < kHamRows; ++u) {
        const int st = s0 + u;
        const int r = st * rows_per + rsel;
        rok[u] = st < L && base + r < nc;
        idr[u] = __shfl(my_id, rok[u] ? r : 0, kWave);
        hs[u] = 0;
      }
      for (int j0 = 0; j0 < J; j0 += kHamLoads) {
        V cw[kHamRows][kHamLoads];
#pragma unroll
        for (int u = 0; u < kHamRows; ++u) {
          const V *row = reinterpret_cast<const V *>(codes + static_cast<long long>(idr[u]) * words);
#pragma unroll
          for (int e = 0; e < kHamLoads; ++e) {
            const int v = sub + (j0 + e) * L;
            cw[u][e] = row[(rok[u] && v < span) ? v : 0];   // clamped: every load is issued
          }
        }
#pragma unroll
        for (int u = 0; u < kHamRows; ++u)
#pragma unroll
          for (int e = 0; e < kHamLoads; ++e) {
            const int v = sub + (j0 + e) * L;
            if (rok[u] && v < span) hs[u] += CodeVec<kVec>::pop(qc, v * kVec, cw[u][e]);
          }
      }
#pragma unroll
      for (int u = 0; u < kHamRows; ++u) {
        int h = hs[u];
        for (int s2 = L >> 1; s2 >= 1; s2 >>= 1) h += __shfl_xor(h, s2, kWave);
        if (sub == 0 && rok[u]) hm_tmp[qo + base + (s0 + u) * rows_per + rsel] = h;
      }
    }
  }
}

// Candidates in ascending (Hamming distance, id) order, placed only as far
// as the walk is expected to read.  One block per query (or per entry of a
// query list): a histogram of the distances over all candidates (LDS, D + 1
// bins) and its exclusive scan give every bin's first position; the order
// statistics the learned budget uses are read from it (the distance at
// positions 1, 2, 4, ..., 2048 and at the median); then the candidates of
// the bins that cover the first `plen` positions (whole bins) are placed
// stably, in id order within a bin: a lane's rank among the lanes with the
// same distance comes from ballots over the distance's bits, each bin's
// cursor is in LDS (the four waves take four contiguous id ranges when the
// placed bins span at most kOrderSpan distances, else one wave places all).
// avail[q] = positions placed.
constexpr int kHamStats = 13;  // positions 1, 2, 4, ..., 2048, then the median

__global__ void __launch_bounds__(kOrderThreads) k_hamming_order(
    int d, const int32_t *__restrict__ ncand, const int32_t *__restrict__ cand, long long cap,
    const int32_t *__restrict__ hm_tmp, int plen, int32_t *__restrict__ order, int32_t *__restrict__ ham_sorted,
    int32_t *__restrict__ avail, int32_t *__restrict__ hstat, const int32_t *__restrict__ live,
    const int32_t *__restrict__ qlist, const int32_t *__restrict__ qcount) {
  // d + 1 bins (or, while placing, the per-wave counts and starts of the
  // placed bins and the waves' staging lists), then the scan's scratch
  extern __shared__ __align__(16) int hist[];
  int *tmp = hist + max(d + 1, (kOrderWaves + 2) * kOrderSpan);
  const int nl = live ? *live : 0x7fffffff;
  const int nitems = qcount ? *qcount : static_cast<int>(gridDim.x);
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int q = qlist ? qlist[item] : item;
    if (q >= nl) return;                  // uniform over the block
    const int nc = ncand[q];
    const long long qo = static_cast<long long>(q) * cap;
    const int32_t *hq = hm_tmp + qo;
    for (int h = tid; h <= d; h += kOrderThreads) hist[h] = 0;
    __syncthreads();
    // histogram: one LDS atomic per candidate (a crowded bin serializes its
    // lanes, at most 64 per instruction)
    {
      constexpr int U = 8;  // steps per batch; the next batch is loaded while this one is counted
      int hv[U], hn[U];
      const int first = wv * kWave * U;
#pragma unroll
      for (int u = 0; u < U; ++u) hv[u] = nc > 0 ? hq[min(first + u * kWave + lane, nc - 1)] : 0;  // clamped
      for (int i0 = first; i0 < nc; i0 += kOrderThreads * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) hn[u] = hq[min(i0 + kOrderThreads * U + u * kWave + lane, nc - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (i0 + u * kWave + lane < nc) atomicAdd(&hist[hv[u]], 1);
#pragma unroll
        for (int u = 0; u < U; ++u) hv[u] = hn[u];
      }
    }
    __syncthreads();
    block_exclusive_scan(hist, d + 1, tmp);  // hist[h] = first position of bin h
    // order statistics: the bin holding position p - 1 (largest h with start <= p - 1)
    if (tid < kHamStats) {
      int v = 0;
      if (nc > 0) {
        const int p = tid < kHamStats - 1 ? min(1 << tid, nc) : (nc + 1) / 2;
        v = upper_bound_minus1(hist, d + 1, p - 1);
      }
      hstat[static_cast<long long>(q) * kHamStats + tid] = v;
    }
    const int want = min(nc, plen);
    const int hcut = want > 0 ? upper_bound_minus1(hist, d + 1, want - 1) : -1;
    const int placed = hcut < 0 ? 0 : (hcut < d ? hist[hcut + 1] : nc);
    if (tid == 0) avail[q] = placed;
    __syncthreads();
    // Placement of bins hmin .. hcut in (h, id) order.  When they span at
    // most kOrderSpan distances the four waves place four contiguous ranges
    // of the candidates (in id order) at once: each counts its range per
    // bin, a prefix over the waves gives each wave its first position in
    // every bin, then each places its range in order.  Otherwise wave 0
    // places all of them.
    const int hmin = hcut >= 0 ? upper_bound_minus1(hist, d + 1, 0) : 0;   // the first non-empty bin
    const int span = hcut - hmin + 1;
    if (hcut >= 0 && span <= kOrderSpan) {
      int *wcnt = hist;                        // [kOrderWaves][kOrderSpan]: counts, then first positions
      int *bst = hist + kOrderWaves * kOrderSpan;   // [kOrderSpan]: first position of each bin
      int sv[kOrderSpan / kOrderThreads];
#pragma unroll
      for (int u = 0; u < kOrderSpan / kOrderThreads; ++u) {
        const int j = tid + u * kOrderThreads;
        sv[u] = j < span ? hist[hmin + j] : 0;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kOrderSpan / kOrderThreads; ++u) bst[tid + u * kOrderThreads] = sv[u];
      const int per = (nc + kOrderWaves * kWave - 1) / (kOrderWaves * kWave) * kWave;
      const int r0 = wv * per, r1 = min(nc, r0 + per);
      int *mine = wcnt + wv * kOrderSpan;
      for (int j = lane; j < span; j += kWave) mine[j] = 0;   // the wave's own counters
      __builtin_amdgcn_wave_barrier();
      if (r0 < r1) {
        constexpr int U = 8;  // steps per batch; the next batch is loaded while this one is counted
        int hv[U], hn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) hv[u] = hq[min(r0 + u * kWave + lane, r1 - 1)];  // clamped: every load is issued
        for (int i0 = r0; i0 < r1; i0 += kWave * U) {
#pragma unroll
          for (int u = 0; u < U; ++u) hn[u] = hq[min(i0 + kWave * U + u * kWave + lane, r1 - 1)];
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (i0 + u * kWave + lane < r1 && hv[u] <= hcut) atomicAdd(&mine[hv[u] - hmin], 1);
#pragma unroll
          for (int u = 0; u < U; ++u) hv[u] = hn[u];
        }
      }
      __syncthreads();
      for (int j = tid; j < span; j += kOrderThreads) {
        int run = bst[j];
#pragma unroll
        for (int w = 0; w < kOrderWaves; ++w) {
          const int c = wcnt[w * kOrderSpan + j];
          wcnt[w * kOrderSpan + j] = run;
          run += c;
        }
      }
      __syncthreads();
      // Each wave walks its range 256 candidates at a time: the placed ones
      // (h <= hcut) are packed, in id order, into the wave's staging lists
      // (bin offset and id, in the space the bin starts used), then ranked 64
      // at a time among equal bins by ballots over the bin offset's bits.
      int nbits = 0;
      while ((1 << nbits) < span) ++nbits;
      const unsigned long long below = lanes_below_mask();
      int *sbin = bst + wv * (kOrderSpan / kOrderWaves), *sid = bst + kOrderSpan + wv * (kOrderSpan / kOrderWaves);
      constexpr int U = kOrderSpan / kOrderWaves / kWave;  // steps per batch (256 candidates)
      int hv[U], iv[U], hn[U], in_[U];
      if (r0 < r1) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = min(r0 + u * kWave + lane, r1 - 1);  // clamped: every load is issued
          hv[u] = hq[i];
          iv[u] = cand[qo + i];
        }
      }
      for (int i0 = r0; i0 < r1; i0 += kWave * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {  // the next batch, loaded while this one is placed
          const int i = min(i0 + kWave * U + u * kWave + lane, r1 - 1);
          hn[u] = hq[i];
          in_[u] = cand[qo + i];
        }
        int nin = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool in = i0 + u * kWave + lane < r1 && hv[u] <= hcut;
          const unsigned long long m = __ballot(in);
          if (in) {
            const int at = nin + __popcll(m & below);
            sbin[at] = hv[u] - hmin;
            sid[at] = iv[u];
          }
          nin += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
        for (int j0 = 0; j0 < nin; j0 += kWave) {
          const bool ok = j0 + lane < nin;
          const int bb = ok ? sbin[j0 + lane] : 0, id = ok ? sid[j0 + lane] : 0;
          unsigned long long same = __ballot(ok);
          for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (bb >> bit) & 1;
            const unsigned long long bm = __ballot(on);
            same &= on ? bm : ~bm;
          }
          if (ok) {
            const int pos = mine[bb] + __popcll(same & below);
            order[qo + pos] = id;
            ham_sorted[qo + pos] = bb + hmin;
          }
          __builtin_amdgcn_wave_barrier();
          if (ok && (same & below) == 0) mine[bb] += __popcll(same);
          __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          hv[u] = hn[u];
          iv[u] = in_[u];
        }
      }
    } else if (wv == 0 && hcut >= 0) {
      int nbits = 0;
      while ((1 << nbits) <= hcut) ++nbits;
      const unsigned long long below = lanes_below_mask();
      constexpr int U = 8;  // steps whose distances and ids are loaded together
      for (int i0 = 0; i0 < nc; i0 += kWave * U) {
        int hv[U], iv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = min(i0 + u * kWave + lane, nc - 1);  // clamped: every load is issued
          hv[u] = hq[i];
          iv[u] = cand[qo + i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int h = hv[u];
          const bool in = i0 + u * kWave + lane < nc && h <= hcut;
          unsigned long long same = __ballot(in);
          if (same == 0ull) continue;  // wave-uniform
          for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (h >> bit) & 1;
            const unsigned long long bb = __ballot(on);
            same &= on ? bb : ~bb;
          }
          if (in) {
            const int pos = hist[h] + __popcll(same & below);
            order[qo + pos] = iv[u];
            ham_sorted[qo + pos] = h;
          }
          __builtin_amdgcn_wave_barrier();
          if (in && (same & below) == 0) hist[h] += __popcll(same);
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
    __syncthreads();
  }
}

__host__ __device__ inline size_t hamming_order_lds(int d) {
  const size_t bins = static_cast<size_t>(d) + 1, part = static_cast<size_t>(kOrderWaves + 2) * kOrderSpan;
  return ((bins > part ? bins : part) + kOrderWaves + 1) * sizeof(int);
}

// ---------------------------------------------------------------------------
// A6/A7: re-rank.  One block (4 waves) per query; q' staged in LDS.
//
// The distance key of a row is the squared L2 distance summed in float64
// over the dimensions in ascending order, one rounding per operation
// (Section 4.3.2, Stage 3: exact L2).  A wavefront computes the same D terms
// t_i = (q'_i - x_i)^2 but adds them lane-parallel (lane l sums the 4-element
// groups l, l + 64, ... in order, then a halving tree), with up to 16
// sixteen-byte loads in flight per lane.  Every t_i >= 0, so any summation
// tree of depth h <= D is within gamma_D = D u / (1 - D u) (u = 2^-53) of the
// exact sum T of the terms (the standard bound for recursive and pairwise
// summation of non-negative terms), both the wave's value p and the defined
// key s lie within gamma_D T of T, and |p - s| <= 2 gamma_D T / (1 - gamma_D)
// p.  The key is therefore known to lie in the interval [p (1 - c), p (1 + c)]
// with c = (2D + 16) u (which also covers the rounding of the two products).
// Decisions are taken on the intervals: a comparison whose intervals overlap,
// or a returned float32 value that the interval does not fix (f32 of its two
// ends differ), is decided on s itself, computed by the definition
// (row_dist_seq, one thread, ascending i).  Guaranteed Mode selects the
// top-k of all candidate keys (radix select on the key bits, the band around
// the k-th key made exact when it is ambiguous, ties by id); Optimized Mode
// walks the Hamming order chunk by chunk, computing a chunk's keys in
// parallel and applying the patience rule to them in order.
// ---------------------------------------------------------------------------
constexpr int kRerankThreads = 256;
constexpr int kRerankWaves = kRerankThreads / kWave;
constexpr int kChunk = 256;
constexpr int kWalkGrain = 16;  // walk chunks are whole multiples of this many rows

template <int B>
__device__ __forceinline__ double canon_partial(const float4 *__restrict__ qq, const float4 *__restrict__ xr, int nv,
                                                int lane) {
  double p = 0.0;
  for (int r0 = 0; r0 * kWave < nv; r0 += B) {
    float4 xv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int g = (r0 + u) * kWave + lane;
      xv[u] = xr[g < nv ? g : 0];              // clamped: every load is issued
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int g = (r0 + u) * kWave + lane;
      const bool ok = g < nv;
      const float4 qv = qq[ok ? g : 0];
      const double t0 = ok ? static_cast<double>(qv.x) - static_cast<double>(xv[u].x) : 0.0;
      const double t1 = ok ? static_cast<double>(qv.y) - static_cast<double>(xv[u].y) : 0.0;
      const double t2 = ok ? static_cast<double>(qv.z) - static_cast<double>(xv[u].z) : 0.0;
      const double t3 = ok ? static_cast<double>(qv.w) - static_cast<double>(xv[u].w) : 0.0;
      double s0 = t0 * t0; p = p + s0;
      double s1 = t1 * t1; p = p + s1;
      double s2 = t2 * t2; p = p + s2;
      double s3 = t3 * t3; p = p + s3;
    }
  }
  return p;
}

// Wave key p of one row (the key's terms added lane-parallel), whole wave;
// result in every lane.  Lane l owns the 4-element groups g = l, l + 64, ... (one 16-byte load each, all of a batch
// issued before use); groups past the end contribute exact zeros.
// kWide = false keeps at most 4 loads in flight per lane (fewer registers,
// for kernels that read few rows this way).
template <bool kWide = true>
__device__ __forceinline__ double row_dist_canon(const float *__restrict__ sq, const float *__restrict__ x, int d) {
  const int lane = lane_id();
  const int nv = d >> 2;
  const float4 *qq = reinterpret_cast<const float4 *>(sq);
  const float4 *xr = reinterpret_cast<const float4 *>(x);
  double p = (!kWide || nv <= 4 * kWave) ? canon_partial<4>(qq, xr, nv, lane) : canon_partial<16>(qq, xr, nv, lane);
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

// Relative half-width c of the interval around a wave key (see above).
__host__ __device__ inline double key_band(int d) { return (2.0 * d + 16.0) * 0x1p-53; }
__device__ __forceinline__ double key_lo(double p, double c) { return p * (1.0 - c); }
__device__ __forceinline__ double key_hi(double p, double c) { return p * (1.0 + c); }

// The defined key of one row: ascending i, acc = acc + (q'_i - x_i)^2 in
// float64, one thread.  Used only where a wave key's interval cannot decide.
__device__ inline double row_dist_seq(const float *__restrict__ sq, const float *__restrict__ x, int d) {
  const float4 *qq = reinterpret_cast<const float4 *>(sq);
  const float4 *xr = reinterpret_cast<const float4 *>(x);
  double acc = 0.0;
  for (int g = 0; g < (d >> 2); ++g) {
    const float4 xv = xr[g];
    const float4 qv = qq[g];
    const double t0 = static_cast<double>(qv.x) - static_cast<double>(xv.x);
    const double s0 = t0 * t0;
    acc = acc + s0;
    const double t1 = static_cast<double>(qv.y) - static_cast<double>(xv.y);
    const double s1 = t1 * t1;
    acc = acc + s1;
    const double t2 = static_cast<double>(qv.z) - static_cast<double>(xv.z);
    const double s2 = t2 * t2;
    acc = acc + s2;
    const double t3 = static_cast<double>(qv.w) - static_cast<double>(xv.w);
    const double s3 = t3 * t3;
    acc = acc + s3;
  }
  return acc;
}

// True when the float32 rounding of every value in the key's interval is
// the same (then it is f32 of the defined key).
__device__ __forceinline__ bool f32_fixed(double p, double c) {
  return static_cast<float>(key_lo(p, c)) == static_cast<float>(key_hi(p, c));
}

// ---------------------------------------------------------------------------
// ADSampling (Eq. (2)): a walked candidate is pruned at the first t = 32, 64,
// ... below D with d_t^2 > r_k^2 * factor_t, where d_t^2 is the distance
// key's running sum after t dimensions, r_k^2 the k-th key of the top-k when
// the candidate is walked and factor_t = (t/D)(1 + eps_0/sqrt(t))^2 (table
// from the host, eps_0 = 2.1).  fl(r * factor_t) is monotone in r, so a row
// pruned against a larger r is pruned against every smaller one.
// ---------------------------------------------------------------------------
constexpr int kAdsStep = 32;
constexpr double kAdsMargin = 0x1p-50;  // covers the roundings of L / factor and r * factor

// Inclusive prefix sum of a double across the 64 lanes.
__device__ __forceinline__ double wave_incl_scan_f64(double v) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    const double u = __shfl_up(v, s, kWave);
    if (lane >= s) v = v + u;
  }
  return v;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = fmax(v, __shfl_xor(v, s, kWave));
  return v;
}

struct AdsRow {
  double key, mlo, mhi;
  int dims;
  bool pruned;
};

// One row, whole wave, read in 256-dimension blocks two at a time (lane l
// holds dimensions 256b + 4l .. + 3 of block b).  After each block the lanes'
// partial sums are scanned: lane 8j + 7 then holds the wave value p_t of
// d_t^2 at t = 256b + 32(j + 1), whose defined value lies in [p_t(1 - c_t),
// p_t(1 + c_t)], c_t = (2t + 16) u (the same argument as the key's, t
// terms).  The row is pruned for certain when some t has p_t(1 - c_t) >
// fl(rhi * factor_t) (rhi an upper end of r_k^2); otherwise it is read to the
// end and gets its wave key and the bounds mlo <= max_t d_t^2 / factor_t <=
// mhi (widened by kAdsMargin).  dims = dimensions loaded.
__device__ inline AdsRow ads_row(const float *__restrict__ sq, const float *__restrict__ x, int d, double rhi,
                                 const double *__restrict__ fac) {
  const int lane = lane_id();
  const int nv = d >> 2;
  const int nblk = (d + 255) >> 8;
  const float4 *qq = reinterpret_cast<const float4 *>(sq);
  const float4 *xr = reinterpret_cast<const float4 *>(x);
  double carry = 0.0, mlo = 0.0, mhi = 0.0;
  AdsRow r{0.0, 0.0, 0.0, d, false};
  for (int b0 = 0; b0 < nblk; b0 += 2) {
    float4 xv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int g = (b0 + u) * kWave + lane;
      xv[u] = xr[g < nv ? g : 0];  // clamped: every load is issued
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int b = b0 + u;
      if (b >= nblk) break;
      const int g = b * kWave + lane;
      const bool ok = g < nv;
      const float4 qv = qq[ok ? g : 0];
      double v = 0.0;
      if (ok) {
        const double t0 = static_cast<double>(qv.x) - static_cast<double>(xv[u].x);
        const double t1 = static_cast<double>(qv.y) - static_cast<double>(xv[u].y);
        const double t2 = static_cast<double>(qv.z) - static_cast<double>(xv[u].z);
        const double t3 = static_cast<double>(qv.w) - static_cast<double>(xv[u].w);
        const double s0 = t0 * t0, s1 = t1 * t1, s2 = t2 * t2, s3 = t3 * t3;
        v = s0;
        v = v + s1;
        v = v + s2;
        v = v + s3;
      }
      const double p = carry + wave_incl_scan_f64(v);
      const int t = (g + 1) * 4;  // dimensions summed through this lane's group
      bool cut = false;
      if ((lane & 7) == 7 && t < d) {
        const double ct = (2.0 * t + 16.0) * 0x1p-53;
        const double f = fac[t / kAdsStep - 1];
        const double lo = p * (1.0 - ct), hi = p * (1.0 + ct);
        cut = lo > rhi * f;
        mlo = fmax(mlo, lo / f);
        mhi = fmax(mhi, hi / f);
      }
      if (__ballot(cut)) {
        r.pruned = true;
        r.dims = min(d, (b0 + 2) * 256);
        return r;
      }
      carry = readlane_f64(p, kWave - 1);
    }
  }
  r.key = carry;
  r.mlo = wave_max_f64(mlo) * (1.0 - kAdsMargin);
  r.mhi = wave_max_f64(mhi) * (1.0 + kAdsMargin);
  return r;
}

// The ADSampling decision by the definition: the running float64 sum in
// ascending dimension order against fl(r * factor_t) at every test point.
__device__ inline bool ads_pruned_seq(const float *__restrict__ sq, const float *__restrict__ x, int d, double r,
                                      const double *__restrict__ fac) {
  double acc = 0.0;
  for (int i = 0; i < d; ++i) {
    const double t = static_cast<double>(sq[i]) - static_cast<double>(x[i]);
    const double s = t * t;
    acc = acc + s;
    if ((i + 1) % kAdsStep == 0 && i + 1 < d && acc > r * fac[(i + 1) / kAdsStep - 1]) return true;
  }
  return false;
}

struct RerankShared {
  double dk[kChunk];
  int dx[kChunk];  // dk[t] is the defined key (1) or a wave key (0)
  double amlo[kChunk], amhi[kChunk];  // ADSampling: bounds of max_t d_t^2 / factor_t of a surviving row
  unsigned long long rbytes;          // bytes of stored rows read for this query
  int sid[kChunk];
  float serr[kChunk];
  int plist[kChunk];
  int hist[256];
  int misc[16];
  unsigned long long umisc[2];
  double bd;
};

// ---------------------------------------------------------------------------
// Mixed precision: a bfloat16 first pass whose every decision is certified.
//
// Row x has a bfloat16 copy x~ (round to nearest even) and a stored
// e_x >= ||x - x~||.  The float32 value t of ||q' - x~||^2 (each lane sums
// L <= ceil(D/512) * 8 fused squares in order, then a 6-level tree; every
// term is >= 0) satisfies |t - ||q' - x~||^2| <= g ||q' - x~||^2 with
// g = gamma_{L+10} = (L+10)u / (1 - (L+10)u), u = 2^-24.  The triangle
// inequality then gives
//     (sqrt(t (1 - g)) - e_x)_+^2  <=  ||q' - x||^2  <=  (sqrt(t (1 + 2g)) + e_x)^2.
// The defined key and the wave key are both within a relative (D + 4) 2^-53
// (< 2^-39.9 for D <= 8192) of ||q' - x||^2; both bounds are widened by a
// relative 2^-36 (that, plus the float64 rounding of the bound) and an
// absolute 2^-100 (float32 subnormals flushed to zero), so lb <= key <= ub
// holds for every row.  A row is read in float32 only if its lower bound
// does not exclude it; every comparison that decides a result is taken on
// the float32 row's key, so the results equal the float32-only path bit for
// bit.
// ---------------------------------------------------------------------------
constexpr double kBoundRel = 1.0 / 68719476736.0;          // 2^-36
constexpr double kBoundAbs = 7.888609052210118e-31;         // 2^-100

// ||q' - x~||^2 in float32 for two bfloat16 rows at once (2 x 8 sixteen-byte
// loads in flight per lane: one row alone leaves the wave latency-bound);
// whole wave, results in every lane (an xor butterfly adds the same pair in
// both lanes).
__device__ __forceinline__ float2 row_dist_bf16_x2(const float *__restrict__ sq, const uint16_t *__restrict__ xa16,
                                                   const uint16_t *__restrict__ xb16, int d) {
  const int lane = lane_id();
  const int nv = d >> 3;  // 16-byte groups of eight bfloat16
  const uint4 *xa = reinterpret_cast<const uint4 *>(xa16);
  const uint4 *xb = reinterpret_cast<const uint4 *>(xb16);
  const float4 *qq = reinterpret_cast<const float4 *>(sq);
  constexpr int B = 8;
  float pa = 0.f, pb = 0.f;
  for (int r0 = 0; r0 * kWave < nv; r0 += B) {
    uint4 va[B], vb[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int g = (r0 + u) * kWave + lane;
      const int gg = g < nv ? g : 0;  // clamped: every load is issued
      va[u] = xa[gg];
      vb[u] = xb[gg];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int g = (r0 + u) * kWave + lane;
      const bool ok = g < nv;
      const int gg = ok ? g : 0;
      const float4 q0 = qq[2 * gg], q1 = qq[2 * gg + 1];
      const float qs[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
      const uint32_t wa[4] = {va[u].x, va[u].y, va[u].z, va[u].w};
      const uint32_t wb[4] = {vb[u].x, vb[u].y, vb[u].z, vb[u].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float a0 = ok ? qs[2 * e] - __uint_as_float(wa[e] << 16) : 0.f;
        const float a1 = ok ? qs[2 * e + 1] - __uint_as_float(wa[e] & 0xFFFF0000u) : 0.f;
        const float b0 = ok ? qs[2 * e] - __uint_as_float(wb[e] << 16) : 0.f;
        const float b1 = ok ? qs[2 * e + 1] - __uint_as_float(wb[e] & 0xFFFF0000u) : 0.f;
        pa = fmaf(a0, a0, pa);
        pa = fmaf(a1, a1, pa);
        pb = fmaf(b0, b0, pb);
        pb = fmaf(b1, b1, pb);
      }
    }
  }
  return make_float2(wave_sum_f32(pa), wave_sum_f32(pb));
}

__device__ __forceinline__ void bf16_bounds(float t32, float ex, double g, double &lb, double &ub) {
  const double t = static_cast<double>(t32);
  const double e = static_cast<double>(ex);
  const double slo = sqrt(fmax(0.0, t * (1.0 - g))) - e;
  lb = (slo > 0.0 ? slo * slo : 0.0) * (1.0 - kBoundRel) - kBoundAbs;
  const double shi = sqrt(t * (1.0 + 2.0 * g)) + e;
  ub = shi * shi * (1.0 + kBoundRel) + kBoundAbs;
}

__device__ __forceinline__ void base_bf16_row(const float *__restrict__ base, long long row, int d,
                                              uint16_t *__restrict__ b16, float *__restrict__ err) {
  const int lane = lane_id();
  const float *x = base + row * d;
  uint16_t *y = b16 + row * d;
  double s = 0.0;
  for (int i = lane; i < d; i += kWave) {
    const float v = x[i];
    const uint16_t b = bf16_bits(v);
    y[i] = b;
    const double diff = static_cast<double>(v) - static_cast<double>(__uint_as_float(static_cast<uint32_t>(b) << 16));
    s = s + diff * diff;
  }
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) s = s + __shfl_xor(s, sh, kWave);
  if (lane == 0) {
    const double e = sqrt(s) * (1.0 + kBoundRel);
    float f = static_cast<float>(e);
    if (static_cast<double>(f) < e) f = nextafterf(f, __int_as_float(0x7f800000));
    err[row] = f;
  }
}

// One wavefront per row, striding over the rows (capped grid): bfloat16
// copy and an upper bound of ||x - x~|| (float64 sum of exact squared
// differences, widened, rounded up to float).
__global__ void __launch_bounds__(256) k_base_bf16(const float *__restrict__ base, long long n, int d,
                                                    uint16_t *__restrict__ b16, float *__restrict__ err) {
  const long long step = static_cast<long long>(gridDim.x) * (256 / kWave);
  for (long long row = static_cast<long long>(blockIdx.x) * (256 / kWave) + wave_id(); row < n; row += step)
    base_bf16_row(base, row, d, b16, err);
}

// Dynamic LDS of k_rerank: q' (D floats) | top-k keys (k doubles) | top-k ids
// (k ints) | top-k exactness flags (k ints) | [bfloat16 pass] lower / upper
// bounds and certification flags of a chunk.
struct RerankLds {
  size_t top_d, top_i, top_x, lb, ub, pc, total;
};
__host__ __device__ inline RerankLds rerank_lds(int d, int k, bool bf16) {
  RerankLds L{};
  size_t o = static_cast<size_t>(d) * 4;
  L.top_d = o; o += static_cast<size_t>(k) * 8;
  L.top_i = o; o += static_cast<size_t>(k) * 4;
  L.top_x = o; o += static_cast<size_t>(k) * 4;
  o = (o + 15) & ~static_cast<size_t>(15);
  if (bf16) {
    L.lb = o; o += kChunk * 8;
    L.ub = o; o += kChunk * 8;
    L.pc = o; o += kChunk * 4;
  }
  L.total = o;
  return L;
}

// kk-th smallest (1-based, kk <= n) by bit pattern of the n doubles whose
// bits under `mask0` equal `prefix0` (all of them when both are 0; the
// candidates must be non-negative, or all carry the sign bit, which then
// orders them by magnitude): radix select, 8 bits per round.  Whole block.
// Returns the value and, in *need_eq, how many entries equal to it are among
// the kk smallest.
__device__ inline double radix_kth(const double *__restrict__ keys, int n, int kk, RerankShared &S, int *need_eq,
                                   unsigned long long prefix0 = 0ull, unsigned long long mask0 = 0ull) {
  const int tid = threadIdx.x;
  unsigned long long prefix = prefix0, mask = mask0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = tid; b < 256; b += kRerankThreads) S.hist[b] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kRerankThreads) {
      const unsigned long long bits = dbits(keys[i]);
      if ((bits & mask) == prefix) atomicAdd(&S.hist[(bits >> shift) & 255], 1);
    }
    __syncthreads();
    if (tid == 0) {
      int cum = 0, b = 0;
      for (; b < 255; ++b) {
        if (cum + S.hist[b] >= kk) break;
        cum += S.hist[b];
      }
      S.umisc[0] = (prefix & ~(255ull << shift)) | (static_cast<unsigned long long>(b) << shift);
      S.misc[0] = kk - cum;
    }
    __syncthreads();
    prefix = S.umisc[0];
    kk = S.misc[0];
    mask |= 255ull << shift;
    __syncthreads();
  }
  *need_eq = kk;
  return from_dbits(prefix);
}

// Block-wide sum of one int per thread (every thread gets the total).
__device__ inline int block_sum_i32(int v, RerankShared &S) {
  v = wave_sum_i32(v);
  __syncthreads();
  if (lane_id() == 0) S.hist[wave_id()] = v;
  __syncthreads();
  int t = 0;
  for (int w = 0; w < kRerankWaves; ++w) t += S.hist[w];
  __syncthreads();
  return t;
}

constexpr unsigned long long kSignBit = 0x8000000000000000ull;

// Sorts the ns (<= k) rows held in top_d / top_i / top_x by (key, id) and
// writes them (padded with id -1 / +inf to k).  A wave key (top_x = 0) is
// made exact when its interval overlaps another row's or does not fix its
// float32 value; one round suffices, since making a key exact only shrinks
// its interval.  Whole block.
__device__ inline void write_topk(int ns, int k, double c, const float *sq, const float *__restrict__ base, int d,
                                  double *top_d, int *top_i, int *top_x, int64_t *__restrict__ oi,
                                  float *__restrict__ od) {
  const int tid = threadIdx.x;
  bool amb[(1024 + kRerankThreads - 1) / kRerankThreads];
#pragma unroll
  for (int u = 0; u < (1024 + kRerankThreads - 1) / kRerankThreads; ++u) {
    const int j = tid + u * kRerankThreads;
    amb[u] = false;
    if (j < ns && !top_x[j]) {
      const double p = top_d[j], lo = key_lo(p, c), hi = key_hi(p, c);
      bool a = !f32_fixed(p, c);
      for (int t = 0; t < ns && !a; ++t) {
        if (t == j) continue;
        const double pt = top_d[t];
        const double lt = top_x[t] ? pt : key_lo(pt, c), ht = top_x[t] ? pt : key_hi(pt, c);
        a = lt <= hi && lo <= ht;
      }
      amb[u] = a;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < (1024 + kRerankThreads - 1) / kRerankThreads; ++u) {
    const int j = tid + u * kRerankThreads;
    if (amb[u]) {
      top_d[j] = row_dist_seq(sq, base + static_cast<long long>(top_i[j]) * d, d);
      top_x[j] = 1;
    }
  }
  __syncthreads();
  for (int j = tid; j < ns; j += kRerankThreads) {
    const double dj = top_d[j];
    const int ij = top_i[j];
    int rank = 0;
    for (int t = 0; t < ns; ++t) rank += key_less(top_d[t], top_i[t], dj, ij) ? 1 : 0;
    oi[rank] = ij;
    od[rank] = static_cast<float>(dj);
  }
  for (int r = ns + tid; r < k; r += kRerankThreads) {
    oi[r] = -1;
    od[r] = __int_as_float(0x7f800000);
  }
}

// Top-k by (key, id) of n rows with wave keys, whose ids are ascending in
// list order; writes the k results (padded with id -1 / +inf).  Whole block.
// With v the k-th smallest wave key, a row whose interval lies wholly below
// v's interval is below the k-th defined key (set A, all taken), a row whose
// interval lies wholly above it is not in the top-k, and the band between
// holds every other row of the top-k.  When the band holds exactly the
// k - |A| rows still needed, all of them are taken; otherwise the band's
// keys are made exact (stored negated in `keys`, so the sign marks the band:
// a band key is 0 only when no row is in A) and its k - |A| smallest by
// (key, id) are taken.
__device__ inline void select_topk(double *__restrict__ keys, const int32_t *__restrict__ kid, int n, int k,
                                   double c, const float *sq, const float *__restrict__ base, int d,
                                   RerankShared &S, double *top_d, int *top_i, int *top_x,
                                   int64_t *__restrict__ oi, float *__restrict__ od) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  double vlo = 0.0, vhi = 0.0;
  bool exact_band = false;
  int need = 0, need_eq = 0;
  unsigned long long vb = 0ull;
  if (n > k) {
    int unused;
    const double vk = radix_kth(keys, n, k, S, &unused);
    vlo = key_lo(vk, c);
    vhi = key_hi(vk, c);
    int na = 0, nb = 0;
    for (int i = tid; i < n; i += kRerankThreads) {
      const double p = keys[i];
      if (key_hi(p, c) < vlo) ++na;
      else if (key_lo(p, c) <= vhi) ++nb;
    }
    na = block_sum_i32(na, S);
    nb = block_sum_i32(nb, S);
    if (na + nb > k) {
      exact_band = true;
      need = k - na;
      for (int i = tid; i < n; i += kRerankThreads) {
        const double p = keys[i];
        if (!(key_hi(p, c) < vlo) && key_lo(p, c) <= vhi)
          keys[i] = -row_dist_seq(sq, base + static_cast<long long>(kid[i]) * d, d);
      }
      __syncthreads();
      vb = dbits(radix_kth(keys, n, need, S, &need_eq, kSignBit, kSignBit));
    }
  }
  // Rows taken: all (n <= k); A and the band; or A, band keys below vb and
  // the first need_eq band keys equal to it in list order.
  if (tid == 0) { S.misc[1] = 0; S.misc[2] = 0; }
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += kRerankThreads) {
    const int i = i0 + tid;
    const double di = (i < n) ? keys[i] : 0.0;
    const unsigned long long bi = dbits(di);
    const bool band_x = exact_band && (bi & kSignBit) != 0;
    bool take = false, eq = false;
    if (i < n) {
      if (n <= k) take = true;
      else if (!band_x) take = key_hi(di, c) < vlo || (!exact_band && key_lo(di, c) <= vhi);
      else if (bi < vb) take = true;
      else eq = bi == vb;
    }
    const unsigned long long bm = __ballot(eq);
    const int eq_before = __popcll(bm & lanes_below_mask());
    if (lane == kWave - 1) S.hist[wv] = __popcll(bm);
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wv; ++w) wbase += S.hist[w];
    int eq_total_block = 0;
    for (int w = 0; w < kRerankWaves; ++w) eq_total_block += S.hist[w];
    const int eq_seen = S.misc[2];
    __syncthreads();
    if (take || (eq && eq_seen + wbase + eq_before < need_eq)) {
      const int p = atomicAdd(&S.misc[1], 1);
      top_d[p] = band_x ? -di : di;
      top_i[p] = kid[i];
      top_x[p] = band_x ? 1 : 0;
    }
    __syncthreads();
    if (tid == 0) S.misc[2] = eq_seen + eq_total_block;
    __syncthreads();
  }
  write_topk(S.misc[1], k, c, sq, base, d, top_d, top_i, top_x, oi, od);
}

// kMode: 0 Guaranteed, 1 Optimized.  kBf16 = false: every verified row read
// in float32.  kBf16 = true: every row first in bfloat16; float32 only where
// the bounds cannot exclude it.
#define CRISP_RERANK_PARAMS                                                                              \
  const float *__restrict__ qrot, int d, const float *__restrict__ base, const uint16_t *__restrict__ base16, \
      const float *__restrict__ rerr, double gam, const int32_t *__restrict__ ncand,                          \
      const int32_t *__restrict__ list, long long cap, int k, int patience, const int32_t *__restrict__ limits,\
      double *__restrict__ dkey, float *__restrict__ lbuf, int32_t *__restrict__ rbuf,                        \
      int64_t *__restrict__ out_ids, float *__restrict__ out_d, int32_t *__restrict__ examined,              \
      int32_t *__restrict__ last_upd, int32_t *__restrict__ stopped, int32_t *__restrict__ refined,           \
      const double *__restrict__ ads_fac, long long *__restrict__ row_bytes, const int32_t *__restrict__ avail, \
      int32_t *__restrict__ redo, int32_t *__restrict__ nredo
#define CRISP_RERANK_ARGS                                                                                 \
  qrot, d, base, base16, rerr, gam, ncand, list, cap, k, patience, limits, dkey, lbuf, rbuf, out_ids, out_d, \
      examined, last_upd, stopped, refined, ads_fac, row_bytes, avail, redo, nredo

// One query, whole block.  kAds (Optimized Mode, float32 rows): walked
// candidates are verified with ADSampling.
template <int kMode, bool kBf16, bool kAds>
__device__ __forceinline__ void rerank_query(const int q, CRISP_RERANK_PARAMS) {
  extern __shared__ __align__(16) unsigned char dyn[];
  const RerankLds LL = rerank_lds(d, k, kBf16);
  float *sq = reinterpret_cast<float *>(dyn);
  double *top_d = reinterpret_cast<double *>(dyn + LL.top_d);
  int *top_i = reinterpret_cast<int *>(dyn + LL.top_i);
  int *top_x = reinterpret_cast<int *>(dyn + LL.top_x);
  double *xlb = reinterpret_cast<double *>(dyn + LL.lb);
  double *xub = reinterpret_cast<double *>(dyn + LL.ub);
  int *xpc = reinterpret_cast<int *>(dyn + LL.pc);
  __shared__ RerankShared S;
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const long long qo = static_cast<long long>(q) * cap;
  const double cb = key_band(d);
  for (int i = tid; i < d; i += kRerankThreads) sq[i] = qrot[static_cast<long long>(q) * d + i];
  const int nc = ncand[q];
  __syncthreads();
  int64_t *oi = out_ids + static_cast<long long>(q) * k;
  float *od = out_d + static_cast<long long>(q) * k;

  if constexpr (kMode == 0) {
    // ---- Guaranteed: every candidate --------------------------------------
    const int32_t *kid = list + qo;
    int nk = nc;
    if constexpr (kBf16) {
      // Bounds of every candidate; the k-th smallest upper bound T caps the
      // k-th key, so only rows with lower bound <= T can be in the top-k.
      for (int i = 2 * wv; i < nc; i += 2 * kRerankWaves) {
        const int ida = list[qo + i];
        const int idb = list[qo + min(i + 1, nc - 1)];
        const float2 t = row_dist_bf16_x2(sq, base16 + static_cast<long long>(ida) * d,
                                          base16 + static_cast<long long>(idb) * d, d);
        if (lane < 2 && i + lane < nc) {
          const int id = lane ? idb : ida;
          double lb, ub;
          bf16_bounds(lane ? t.y : t.x, rerr[id], gam, lb, ub);
          dkey[qo + i + lane] = ub;
          float lf = static_cast<float>(lb);
          if (static_cast<double>(lf) > lb) lf = nextafterf(lf, -__int_as_float(0x7f800000));
          lbuf[qo + i + lane] = lf;
        }
      }
      __syncthreads();
      double thr = __longlong_as_double(0x7ff0000000000000ll);
      if (nc > k) {
        int unused;
        thr = radix_kth(dkey + qo, nc, k, S, &unused);
      }
      // Refinement set, in list order (ascending id).
      if (tid == 0) S.misc[3] = 0;
      __syncthreads();
      for (int i0 = 0; i0 < nc; i0 += kRerankThreads) {
        const int i = i0 + tid;
        const bool keep = i < nc && static_cast<double>(lbuf[qo + i]) <= thr;
        const unsigned long long bm = __ballot(keep);
        if (lane == 0) S.hist[wv] = __popcll(bm);
        __syncthreads();
        int before = S.misc[3];
        for (int w = 0; w < wv; ++w) before += S.hist[w];
        if (keep) rbuf[qo + before + __popcll(bm & lanes_below_mask())] = list[qo + i];
        __syncthreads();
        if (tid == 0) {
          int tot = 0;
          for (int w = 0; w < kRerankWaves; ++w) tot += S.hist[w];
          S.misc[3] += tot;
        }
        __syncthreads();
      }
      nk = S.misc[3];
      kid = rbuf + qo;
      for (int j = wv; j < nk; j += kRerankWaves) {
        const double dc = row_dist_canon<false>(sq, base + static_cast<long long>(kid[j]) * d, d);
        if (lane == 0) dkey[qo + j] = dc;
      }
    } else {
      for (int i = wv; i < nc; i += kRerankWaves) {
        const double dc = row_dist_canon(sq, base + static_cast<long long>(list[qo + i]) * d, d);
        if (lane == 0) dkey[qo + i] = dc;
      }
    }
    __syncthreads();
    select_topk(dkey + qo, kid, nk, k, cb, sq, base, d, S, top_d, top_i, top_x, oi, od);
    if (tid == 0) {
      examined[q] = nc;
      last_upd[q] = 0;
      stopped[q] = 0;
      if (refined) refined[q] = nk;
      if (row_bytes) row_bytes[q] = static_cast<long long>(d) * (kBf16 ? 2ll * nc + 4ll * nk : 4ll * nc);
    }
    return;
  }

  if constexpr (kMode == 1) {
    // ---- Optimized: Hamming order with patience ------------------------------
    int lim0 = nc;
    if (limits != nullptr) {
      const int l = limits[q];
      if (l > 0 && l < lim0) lim0 = l;
    }
    // only the first avail[q] positions of the order are placed; a walk that
    // reaches them without stopping is redone on the full order
    const int lim = avail != nullptr ? min(lim0, avail[q]) : lim0;
    if (tid == 0) {
      S.misc[2] = 0; S.misc[3] = 0; S.misc[4] = 0; S.misc[5] = 0; S.misc[6] = 0; S.misc[8] = 0;
      S.rbytes = 0;
    }
    __syncthreads();
    for (int c0 = 0, cnt = 0; c0 < lim; c0 += cnt) {
      // The walk cannot stop within the next patience - run candidates, so a
      // chunk of that many (rounded up to kWalkGrain rows, at most kChunk) is
      // always walked in full; fewer rows are read past the stopping point.
      const int need = max(patience - S.misc[3], 1);
      cnt = min(min(kChunk, (need + kWalkGrain - 1) / kWalkGrain * kWalkGrain), lim - c0);
      const int tn0 = S.misc[2];
      const int free_slots = max(0, k - tn0);
      // (a0) the chunk's ids (and row error bounds) staged in LDS by one
      // coalesced load, so that no row load waits on an id load
      if (tid < cnt) {
        const int id = list[qo + c0 + tid];
        S.sid[tid] = id;
        if constexpr (kBf16) S.serr[tid] = rerr[id];
      }
      __syncthreads();
      if constexpr (kBf16) {
        // (a) bounds of the chunk from the bfloat16 rows
        for (int t = 2 * wv; t < cnt; t += 2 * kRerankWaves) {
          const int ida = S.sid[t];
          const int idb = S.sid[min(t + 1, cnt - 1)];
          const float2 tt = row_dist_bf16_x2(sq, base16 + static_cast<long long>(ida) * d,
                                             base16 + static_cast<long long>(idb) * d, d);
          if (lane < 2 && t + lane < cnt) {
            double lb, ub;
            bf16_bounds(lane ? tt.y : tt.x, S.serr[t + lane], gam, lb, ub);
            xlb[t + lane] = lb;
            xub[t + lane] = ub;
          }
        }
        __syncthreads();
        // When candidate t is walked, the k-th key is at most the k-th smallest
        // of (the top-k keys at the chunk start, upper bounds of the chunk
        // before t); a row whose lower bound exceeds that cannot update.  The
        // lower bound is at most that k-th smallest exactly when fewer than k
        // of those values lie below it: each thread counts them for its own
        // row, and the certified rows are then listed in order.
        {
          static_assert(kChunk <= kRerankThreads, "one row per thread");
          const int t = tid;
          bool cert = false;
          if (t < cnt) {
            const double lb = xlb[t];
            int c = 0;
            for (int e = 0; e < tn0 && c < k; ++e) c += key_hi(top_d[e], cb) < lb ? 1 : 0;
            for (int j = 0; j < t && c < k; ++j) c += xub[j] < lb ? 1 : 0;
            cert = c < k;
            xpc[t] = cert ? 1 : 0;
          }
          const unsigned long long bm = __ballot(cert);
          if (lane == 0) S.hist[wv] = __popcll(bm);
          __syncthreads();
          int before = 0;
          for (int w = 0; w < wv; ++w) before += S.hist[w];
          if (cert) S.plist[before + __popcll(bm & lanes_below_mask())] = t;
          if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < kRerankWaves; ++w) tot += S.hist[w];
            S.misc[7] = tot;
          }
        }
        __syncthreads();
        const int np = S.misc[7];
        if (tid == 0) S.rbytes += static_cast<unsigned long long>(d) * (2ull * cnt + 4ull * np);
        for (int e = wv; e < np; e += kRerankWaves) {
          const int t = S.plist[e];
          const double dc = row_dist_canon<false>(sq, base + static_cast<long long>(S.sid[t]) * d, d);
          if (lane == 0) { S.dk[t] = dc; S.dx[t] = 0; }
        }
      } else if constexpr (kAds) {
        // (a) ADSampling against the k-th key at the chunk start: the walk's
        // k-th key is never larger, so a row pruned here is pruned in the
        // walk; the others are read in full and decided again in (c)
        const double rhi = tn0 >= k ? key_hi(top_d[k - 1], cb) : __longlong_as_double(0x7ff0000000000000ll);
        for (int t = wv; t < cnt; t += kRerankWaves) {
          const AdsRow r = ads_row(sq, base + static_cast<long long>(S.sid[t]) * d, d, rhi, ads_fac);
          if (lane == 0) {
            S.dk[t] = r.pruned ? __longlong_as_double(0x7ff0000000000000ll) : r.key;
            S.dx[t] = 0;
            S.amlo[t] = r.mlo;
            S.amhi[t] = r.mhi;
            atomicAdd(&S.rbytes, static_cast<unsigned long long>(r.dims) * 4ull);
            if (!r.pruned) atomicAdd(&S.misc[8], 1);
          }
        }
      } else {
        if (tid == 0) S.rbytes += static_cast<unsigned long long>(d) * 4ull * cnt;
        // (a) exact keys of the chunk, in parallel
        for (int t = wv; t < cnt; t += kRerankWaves) {
          const double dc = row_dist_canon(sq, base + static_cast<long long>(S.sid[t]) * d, d);
          if (lane == 0) { S.dk[t] = dc; S.dx[t] = 0; }
        }
      }
      __syncthreads();
      // (b) candidates that can update the top-k.  With a full top-k, only keys
      // below its k-th key at the chunk start; while it fills, the first `free`
      // candidates always update and later ones only below the k-th key of
      // (top-k so far + those `free`), which bounds the k-th key from then on.
      // Taken on the intervals: a row whose lower end exceeds the upper end of
      // that bound cannot update; the rest are decided in (c).
      if (tid == 0) {
        if (tn0 >= k) {
          S.bd = key_hi(top_d[k - 1], cb);
        } else if (cnt > free_slots) {
          double bd = 0.0;
          for (int e = 0; e < tn0; ++e) bd = fmax(bd, key_hi(top_d[e], cb));
          for (int e = 0; e < free_slots; ++e) bd = fmax(bd, key_hi(S.dk[e], cb));
          S.bd = bd;
        }
      }
      __syncthreads();
      {
        const int t = tid;
        bool pot = t < cnt;
        if constexpr (kBf16) pot = pot && xpc[t] != 0;
        pot = pot && (t < free_slots || key_lo(S.dk[t], cb) <= S.bd);
        const unsigned long long bm = __ballot(pot);
        if (lane == 0) S.hist[wv] = __popcll(bm);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wv; ++w) before += S.hist[w];
        if (pot) S.plist[before + __popcll(bm & lanes_below_mask())] = t;
        if (tid == 0) {
          int tot = 0;
          for (int w = 0; w < kRerankWaves; ++w) tot += S.hist[w];
          S.misc[7] = tot;
        }
      }
      __syncthreads();
      // (c) the patience rule in order over those candidates; every candidate
      // between two of them is a non-update and only advances the run.  A
      // comparison whose intervals overlap is taken on the defined keys.
      if (tid == 0) {
        // (key, id) of chunk row t before top-k entry e
        auto before_top = [&](int t, int e) -> bool {
          if (!(S.dx[t] && top_x[e])) {
            const double a = S.dk[t], b = top_d[e];
            const double alo = S.dx[t] ? a : key_lo(a, cb), ahi = S.dx[t] ? a : key_hi(a, cb);
            const double blo = top_x[e] ? b : key_lo(b, cb), bhi = top_x[e] ? b : key_hi(b, cb);
            if (ahi < blo) return true;
            if (bhi < alo) return false;
            if (!S.dx[t]) {
              S.dk[t] = row_dist_seq(sq, base + static_cast<long long>(S.sid[t]) * d, d);
              S.dx[t] = 1;
            }
            if (!top_x[e]) {
              top_d[e] = row_dist_seq(sq, base + static_cast<long long>(top_i[e]) * d, d);
              top_x[e] = 1;
            }
          }
          return key_less(S.dk[t], S.sid[t], top_d[e], top_i[e]);
        };
        // ADSampling of chunk row t against the current k-th key (top-k full)
        auto ads_cut = [&](int t) -> bool {
          const double r = top_d[k - 1];
          const double rl = top_x[k - 1] ? r : key_lo(r, cb), rh = top_x[k - 1] ? r : key_hi(r, cb);
          if (S.amlo[t] > rh * (1.0 + kAdsMargin)) return true;
          if (S.amhi[t] < rl * (1.0 - kAdsMargin)) return false;
          if (!top_x[k - 1]) {
            top_d[k - 1] = row_dist_seq(sq, base + static_cast<long long>(top_i[k - 1]) * d, d);
            top_x[k - 1] = 1;
          }
          return ads_pruned_seq(sq, base + static_cast<long long>(S.sid[t]) * d, d, top_d[k - 1], ads_fac);
        };
        int tn = S.misc[2], run = S.misc[3], last = S.misc[4], stop = 0, pos = c0 + cnt, prev = -1;
        const int np = S.misc[7];
        for (int e = 0; e <= np; ++e) {
          const int t = (e < np) ? S.plist[e] : cnt;
          const int gap = t - prev - 1;
          if (gap > 0 && run + gap >= patience) {
            pos = c0 + prev + 1 + (patience - run);
            stop = 1;
            break;
          }
          run += gap;
          if (e == np) break;
          bool cut = false;
          if constexpr (kAds) cut = tn >= k && ads_cut(t);
          if (!cut && (tn < k || before_top(t, k - 1))) {
            int p = (tn < k) ? tn : k - 1;
            while (p > 0 && before_top(t, p - 1)) {
              top_d[p] = top_d[p - 1];
              top_i[p] = top_i[p - 1];
              top_x[p] = top_x[p - 1];
              --p;
            }
            top_d[p] = S.dk[t];
            top_i[p] = S.sid[t];
            top_x[p] = S.dx[t];
            if (tn < k) ++tn;
            run = 0;
            last = c0 + t + 1;
          } else if (++run >= patience) {
            pos = c0 + t + 1;
            stop = 1;
            break;
          }
          prev = t;
        }
        S.misc[2] = tn; S.misc[3] = run; S.misc[4] = last; S.misc[5] = stop; S.misc[6] = pos;
      }
      __syncthreads();
      if constexpr (kBf16) {
        // float32 rows inside the verified prefix
        const bool f = tid < cnt && c0 + tid < S.misc[6] && xpc[tid] != 0;
        const unsigned long long bm = __ballot(f);
        if (lane == 0 && bm) atomicAdd(&S.misc[8], __popcll(bm));
        __syncthreads();
      }
      if (S.misc[5]) break;
    }
    __syncthreads();
    // The top-k is in (key, id) order; write_topk fixes the float32 values.
    write_topk(S.misc[2], k, cb, sq, base, d, top_d, top_i, top_x, oi, od);
    if (tid == 0 && redo != nullptr && lim < lim0 && !S.misc[5]) redo[atomicAdd(nredo, 1)] = q;
    if (tid == 0) {
      examined[q] = S.misc[6];
      last_upd[q] = S.misc[4];
      stopped[q] = S.misc[5];
      if (refined) refined[q] = (kBf16 || kAds) ? S.misc[8] : S.misc[6];
      if (row_bytes) row_bytes[q] = static_cast<long long>(S.rbytes);
    }
  }
}

// Positions: queue == NULL, the grid is padded to a multiple of 8 and each
// XCD takes a contiguous range of positions; otherwise the grid is
// persistent (about as many blocks as fit on the chip at once) and every
// block pulls the next position from the device counter *queue (zero at
// launch) until the live positions are exhausted; every block then exits.
// Position i re-ranks query order[i] (order from k_query_order, which keeps
// live queries first), or query i when order is NULL.
template <int kMode, bool kBf16, bool kAds = false>
__global__ void __launch_bounds__(kRerankThreads) __attribute__((amdgpu_waves_per_eu((kBf16 || kAds) ? 4 : 1)))
k_rerank(CRISP_RERANK_PARAMS, const int32_t *__restrict__ live, int nq,
                                                           int32_t *__restrict__ queue, const int32_t *__restrict__ order) {
  // One call site, so the per-query code is inlined once.
  const int nl = live ? min(nq, *live) : nq;
  __shared__ int next;
  int q = queue ? 0 : xcd_major(blockIdx.x, gridDim.x);
  if (queue != nullptr) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1);
    __syncthreads();
    q = next;
    __syncthreads();
  }
  while (q < nl) {
    rerank_query<kMode, kBf16, kAds>(order ? order[q] : q, CRISP_RERANK_ARGS);
    if (queue == nullptr) break;
    __syncthreads();
    if (threadIdx.x == 0) next = atomicAdd(queue, 1);
    __syncthreads();
    q = next;
    __syncthreads();
  }
}

// Transposed half-codebooks for the scoring wavefronts: [M][2][K][h] -> [M][2][h][K].
__global__ void k_transpose_centroids(const float *__restrict__ cent, int m, int k, int h, float *__restrict__ cent_t) {
  long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  long long total = static_cast<long long>(m) * 2 * k * h;
  if (t >= total) return;
  int i = static_cast<int>(t % h);
  long long r = t / h;
  int c = static_cast<int>(r % k);
  long long ms = r / k;
  cent_t[(ms * h + i) * k + c] = cent[t];
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
    dst[tt] = off[c] + lo;  // position in the subspace's id array
  }
}

// Per posting-list entry: the uint16 byte position of its id's collision
// counter inside a 65,536-id tile (the counting kernel's layout).
__global__ void k_count_positions(const int32_t *__restrict__ ids, long long total, uint16_t *__restrict__ pos) {
  for (long long j = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; j < total;
       j += static_cast<long long>(gridDim.x) * blockDim.x)
    pos[j] = static_cast<uint16_t>(cnt_byte(ids[j] & 0xFFFF));
}

}  // namespace crisp
