// GPU twin of the synthetic-input generator in synth/__init__.py.
//
// Philox4x32-10 (Salmon et al., SC'11) keyed by the seed, counter
// (j_lo, j_hi, tag, block); Irwin-Hall(12) normals; mixture rows assembled
// with float64 sequential accumulation of exact float32 x float32 products,
// rounded once to float32.  Bit-identical to the numpy twin.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

struct U4 {
  uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ double normal_at(uint64_t seed, uint32_t tag, uint64_t j) {
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const uint32_t lo = static_cast<uint32_t>(j), hi = static_cast<uint32_t>(j >> 32);
  uint64_t s = 0;
#pragma unroll
  for (uint32_t b = 0; b < 3; ++b) {
    U4 o = philox(lo, hi, tag, b, k0, k1);
    s += static_cast<uint64_t>(o.a) + o.b + o.c + o.d;
  }
  return static_cast<double>(s) * 2.3283064365386963e-10 - 6.0;  // 2^-32
}

__device__ __forceinline__ uint32_t u32_at(uint64_t seed, uint32_t tag, uint64_t j) {
  return philox(static_cast<uint32_t>(j), static_cast<uint32_t>(j >> 32), tag, 0u, static_cast<uint32_t>(seed),
                static_cast<uint32_t>(seed >> 32)).a;
}

__global__ void k_normals_f64(uint64_t seed, uint32_t tag, uint64_t start, long long count, double *out) {
  long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = normal_at(seed, tag, start + static_cast<uint64_t>(i));
}

__global__ void k_normals_f32(uint64_t seed, uint32_t tag, uint64_t start, long long count, double scale, float *out) {
  long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = static_cast<float>(normal_at(seed, tag, start + static_cast<uint64_t>(i)) * scale);
}

// One block per row.  kind 0: local factors (mu [C][D], fac [C][D][R]);
// kind 1: global low rank (fac = B [D][R], nu [C][R]).
__global__ void __launch_bounds__(256) k_rows(int kind, uint64_t seed, int ncomp, int rank, int d, float sigma,
                                              uint64_t row0, const float *__restrict__ mu,
                                              const float *__restrict__ fac, const float *__restrict__ nu,
                                              float *__restrict__ out) {
  __shared__ float z[256];
  __shared__ int lab_s;
  const uint64_t row = row0 + blockIdx.x;
  if (threadIdx.x == 0) {
    uint64_t u = u32_at(seed, 3u, row);
    lab_s = static_cast<int>((u * static_cast<uint64_t>(ncomp)) >> 32);
  }
  __syncthreads();
  const int lab = lab_s;
  for (int r = threadIdx.x; r < rank; r += blockDim.x) {
    float zr = static_cast<float>(normal_at(seed, 2u, row * rank + r));
    if (kind == 1) zr = static_cast<float>(static_cast<double>(nu[lab * rank + r]) + static_cast<double>(zr));
    z[r] = zr;
  }
  __syncthreads();
  float *dst = out + static_cast<long long>(blockIdx.x) * d;
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double acc;
    const float *f;
    if (kind == 0) {
      acc = static_cast<double>(mu[static_cast<long long>(lab) * d + j]);
      f = fac + (static_cast<long long>(lab) * d + j) * rank;
    } else {
      acc = 0.0;
      f = fac + static_cast<long long>(j) * rank;
    }
    for (int r = 0; r < rank; ++r) {
      double p = static_cast<double>(f[r]) * static_cast<double>(z[r]);
      acc = acc + p;
    }
    float eps = static_cast<float>(normal_at(seed, 1u, row * static_cast<uint64_t>(d) + j));
    double e = static_cast<double>(sigma) * static_cast<double>(eps);
    acc = acc + e;
    dst[j] = static_cast<float>(acc);
  }
}

}  // namespace

extern "C" {

int synth_normals_f64(uint64_t seed, uint32_t tag, uint64_t start, long long count, double *out, void *stream) {
  if (!out || count < 0) return -1;
  if (count == 0) return 0;
  k_normals_f64<<<static_cast<unsigned>((count + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
      seed, tag, start, count, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int synth_normals_f32(uint64_t seed, uint32_t tag, uint64_t start, long long count, double scale, float *out,
                      void *stream) {
  if (!out || count < 0) return -1;
  if (count == 0) return 0;
  k_normals_f32<<<static_cast<unsigned>((count + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
      seed, tag, start, count, scale, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int synth_rows(int kind, uint64_t seed, int ncomp, int rank, int d, float sigma, uint64_t row0, long long nrows,
               const float *mu, const float *fac, const float *nu, float *out, void *stream) {
  if (!out || !fac || nrows < 0 || rank < 1 || rank > 256 || ncomp < 1 || d < 1) return -1;
  if (kind == 0 && !mu) return -1;
  if (kind == 1 && !nu) return -1;
  if (kind != 0 && kind != 1) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long step = 1ll << 30;
  for (long long r0 = 0; r0 < nrows; r0 += step) {
    long long nr = nrows - r0 < step ? nrows - r0 : step;
    k_rows<<<static_cast<unsigned>(nr), 256, 0, st>>>(kind, seed, ncomp, rank, d, sigma, row0 + r0, mu, fac, nu,
                                                      out + r0 * d);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  return 0;
}

}  // extern "C"
