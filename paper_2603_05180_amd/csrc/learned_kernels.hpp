// Learned verification budget for Optimized Mode (an addition on top of the
// paper's patience rule, Section 4.3.2 Stage 3): per-query features from the
// search's own intermediates, a 2-layer MLP (64 hidden units) trained in
// float32 by the kernels below, and bfloat16 MFMA inference that turns the
// predicted log prefix length into a per-query verification limit.
//
// Parameter layout (float32, flat): w1 [F][64] | b1 [64] | w2 [64] | b2 [1].
#pragma once

#include "common.hpp"

namespace crisp {

constexpr int kHidden = 64;

__host__ __device__ inline int mlp_param_count(int f) { return f * kHidden + 2 * kHidden + 1; }
constexpr int kHamPos = 12;  // Hamming distances at positions 1, 2, 4, ..., 2048, then the median
__host__ __device__ inline int n_features(int m) { return 1 + 16 + 3 * m + kHamPos + 1; }

// One thread per query.  sstat [q][m][4] = (c1, c2, c_cut, size of the
// cheapest cell); hist [q][2M+1]; hstat [q][kHamPos + 1] = the Hamming
// distances at positions 1, 2, 4, ..., 2048 (clipped to |C|) and at the
// median of the Hamming order.
__global__ void k_features(int nq, int m, int d, int k, int have_ham, const int32_t *__restrict__ ncand,
                           const int32_t *__restrict__ hist, const int32_t *__restrict__ tau_eff,
                           const double *__restrict__ sstat, const int32_t *__restrict__ hstat,
                           float *__restrict__ feat, const int32_t *__restrict__ live) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq || (live && q >= *live)) return;
  const int nf = n_features(m);
  float *f = feat + static_cast<long long>(q) * nf;
  const int nc = ncand[q];
  f[0] = static_cast<float>(log1p(static_cast<double>(nc)));
  const int floor_s = max(tau_eff[q], 1);
  const int nb = 2 * m + 1;
  for (int j = 0; j < 16; ++j) {
    const int s = 2 * m - j;
    f[1 + j] = (s >= floor_s) ? static_cast<float>(log1p(static_cast<double>(hist[static_cast<long long>(q) * nb + s])))
                              : 0.0f;
  }
  for (int sub = 0; sub < m; ++sub) {
    const double *st = sstat + (static_cast<long long>(q) * m + sub) * 4;
    const double den = st[0] > 1e-30 ? st[0] : 1e-30;
    f[17 + 3 * sub] = static_cast<float>((st[1] - st[0]) / den);
    f[18 + 3 * sub] = static_cast<float>((st[2] - st[0]) / den);
    f[19 + 3 * sub] = static_cast<float>(log1p(st[3]));
  }
  const int base = 17 + 3 * m;
  if (have_ham && nc > 0) {
    const int32_t *hs = hstat + static_cast<long long>(q) * (kHamPos + 1);
    for (int j = 0; j <= kHamPos; ++j) f[base + j] = static_cast<float>(static_cast<double>(hs[j]) / d);
  } else {
    for (int j = 0; j <= kHamPos; ++j) f[base + j] = 0.0f;
  }
}

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x) { return static_cast<short>(bf16_bits(x)); }

// Inference: one wavefront per 16 queries.  x_norm = (f - mean) / std in
// float32, rounded to bfloat16 with W1; h = relu(x W1 + b1) on
// v_mfma_f32_16x16x16_bf16 (float32 accumulation); y = h . w2 + b2;
// limit = clamp(ceil(exp(y + delta)), k, |C|) (|C| = 0 -> 0).
__global__ void __launch_bounds__(64) k_mlp_limits(int nq, int nf, const float *__restrict__ feat,
                                                   const float *__restrict__ mean, const float *__restrict__ sdev,
                                                   const float *__restrict__ params, double delta, int k,
                                                   const int32_t *__restrict__ ncand, int32_t *__restrict__ limits,
                                                   float *__restrict__ yout, const int32_t *__restrict__ live) {
  const int lane = threadIdx.x;
  const int q0 = blockIdx.x * 16;
  const int row = lane & 15, kq = lane >> 4;          // A: row of the tile, k quad
  const float *w1 = params;
  const float *b1 = params + nf * kHidden;
  const float *w2 = b1 + kHidden;
  const float b2 = w2[kHidden];
  float4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int qa = q0 + row;
  for (int kb = 0; kb < nf; kb += 16) {
    short4_t a;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int fi = kb + 4 * kq + e;
      float v = 0.f;
      if (fi < nf && qa < nq) v = (feat[static_cast<long long>(qa) * nf + fi] - mean[fi]) / sdev[fi];
      a[e] = bf16_rne(v);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      short4_t b;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int fi = kb + 4 * kq + e;
        b[e] = bf16_rne(fi < nf ? w1[fi * kHidden + t * 16 + row] : 0.f);
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  // acc[t][i] = pre-activation of query q0 + 4*kq + i, hidden unit t*16 + row.
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int u = t * 16 + row;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float h = fmaxf(acc[t][i] + b1[u], 0.f);
      part[i] += h * w2[u];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) part[i] += __shfl_xor(part[i], s, kWave);
  if (row == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + 4 * kq + i;
      if (q < nq && (!live || q < *live)) {
        const float y = part[i] + b2;
        if (yout) yout[q] = y;
        const int nc = ncand[q];
        double lim = ceil(exp(static_cast<double>(y) + delta));
        lim = lim < k ? k : lim;
        lim = lim > nc ? nc : lim;
        limits[q] = static_cast<int32_t>(lim);
      }
    }
  }
}

// ---- training (float32) ------------------------------------------------------
// Forward: one block of 64 threads per sample; thread j = hidden unit.
__global__ void __launch_bounds__(64) k_mlp_fwd(int b, int nf, const float *__restrict__ x,
                                                const float *__restrict__ params, float *__restrict__ pre,
                                                float *__restrict__ y) {
  const int s = blockIdx.x, j = threadIdx.x;
  if (s >= b) return;
  const float *w1 = params;
  const float *b1 = params + nf * kHidden;
  const float *w2 = b1 + kHidden;
  const float *xs = x + static_cast<long long>(s) * nf;
  float acc = b1[j];
  for (int f = 0; f < nf; ++f) acc = fmaf(xs[f], w1[f * kHidden + j], acc);
  pre[static_cast<long long>(s) * kHidden + j] = acc;
  float c = fmaxf(acc, 0.f) * w2[j];
  c = wave_sum_f32(c);
  if (j == 0) y[s] = c + w2[kHidden];
}

// Gradients of the mean squared error; every sum over the batch runs in
// ascending sample order (one thread per output).
__global__ void k_mlp_bwd(int b, int nf, const float *__restrict__ x, const float *__restrict__ t,
                          const float *__restrict__ params, const float *__restrict__ pre,
                          const float *__restrict__ y, float *__restrict__ grad) {
  const int np = mlp_param_count(nf);
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= np) return;
  const float *w2 = params + nf * kHidden + kHidden;
  const float inv = 2.0f / static_cast<float>(b);
  float acc = 0.f;
  if (o < nf * kHidden) {                    // dW1[f][j]
    const int f = o / kHidden, j = o % kHidden;
    for (int s = 0; s < b; ++s) {
      const float p = pre[static_cast<long long>(s) * kHidden + j];
      if (p > 0.f) acc = fmaf(x[static_cast<long long>(s) * nf + f], (y[s] - t[s]) * inv * w2[j], acc);
    }
  } else if (o < nf * kHidden + kHidden) {   // db1[j]
    const int j = o - nf * kHidden;
    for (int s = 0; s < b; ++s)
      if (pre[static_cast<long long>(s) * kHidden + j] > 0.f) acc += (y[s] - t[s]) * inv * w2[j];
  } else if (o < nf * kHidden + 2 * kHidden) {  // dw2[j]
    const int j = o - nf * kHidden - kHidden;
    for (int s = 0; s < b; ++s)
      acc = fmaf(fmaxf(pre[static_cast<long long>(s) * kHidden + j], 0.f), (y[s] - t[s]) * inv, acc);
  } else {                                   // db2
    for (int s = 0; s < b; ++s) acc += (y[s] - t[s]) * inv;
  }
  grad[o] = acc;
}

__global__ void k_mlp_adam(int np, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                           float *__restrict__ m2, float lr, float beta1, float beta2, float eps, float c1, float c2) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= np) return;
  const float gg = g[o];
  const float a = beta1 * m1[o] + (1.f - beta1) * gg;
  const float v = beta2 * m2[o] + (1.f - beta2) * gg * gg;
  m1[o] = a;
  m2[o] = v;
  w[o] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace crisp
