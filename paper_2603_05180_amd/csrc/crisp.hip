// C ABI of the CRISP engine: validation, workspace layout and launch order.
// Every entry point is declared and documented in include/crisp.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "build_kernels.hpp"
#include "common.hpp"
#include "learned_kernels.hpp"
#include "query_kernels.hpp"

using namespace crisp;

namespace {

thread_local std::string g_err;

crisp_status fail(crisp_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
crisp_status fail(crisp_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(CRISP_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

#define LAUNCH_TRY(name)                                                                     \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess) return fail(CRISP_E_HIP, "launch %s: %s", name, hipGetErrorString(e_)); \
  } while (0)

constexpr int kDefaultTile = 65536;
constexpr int kDefaultChunk = 2048;

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

inline unsigned grid1(long long n, int block) {
  long long g = (n + block - 1) / block;
  return static_cast<unsigned>(std::max<long long>(1, std::min<long long>(g, 0x7fffffffll)));
}

// Blocks for a grid-stride kernel of 256-thread blocks: a dispatch must hold
// fewer than 2^32 threads, and 65536 blocks keep every CU busy.
inline unsigned grid_stride(long long n, int per_block) {
  return static_cast<unsigned>(std::max<long long>(1, std::min<long long>((n + per_block - 1) / per_block, 65536)));
}

crisp_status check_shape(int64_t n, int32_t d, int32_t m, int32_t k) {
  if (n < 1 || d < 1 || m < 1 || k < 1) return fail(CRISP_E_INVALID, "n, d, m, k must be positive");
  if (n >= (int64_t(1) << 31)) return fail(CRISP_E_UNSUPPORTED, "N must be < 2^31");
  if (d % 64 != 0) return fail(CRISP_E_UNSUPPORTED, "D must be a multiple of 64");
  if (d > 8192) return fail(CRISP_E_UNSUPPORTED, "D must be <= 8192");
  if (m > 127) return fail(CRISP_E_UNSUPPORTED, "M must be <= 127");
  if (static_cast<int64_t>(m) * n >= (int64_t(1) << 31)) return fail(CRISP_E_UNSUPPORTED, "M x N must be < 2^31");
  if (d % (2 * m) != 0) return fail(CRISP_E_UNSUPPORTED, "D must be a multiple of 2M");
  if (k > 256) return fail(CRISP_E_UNSUPPORTED, "K must be <= 256");
  // The selection's path for K > 64 (prefix-size tables in device memory)
  // faulted the GPU in a search at N = 1M, D = 960, K = 256; the cause is
  // not found yet, so that path is switched off.
  if (k > 64) return fail(CRISP_E_UNSUPPORTED, "K > 64 is switched off (an unexplained GPU fault at K = 256)");
  return CRISP_OK;
}

int resolve_tile(int32_t tile_ids) { return tile_ids > 0 ? tile_ids : kDefaultTile; }

// ADSampling (Eq. (2)): eps_0 = 2.1, a test every 32 dimensions below D.
// factor_t = (t / D) * (b * b) with b = 1 + eps_0 / sqrt(t), float64.
constexpr double kAdsEps0 = 2.1;
std::vector<double> ads_factors(int d) {
  std::vector<double> f;
  for (int t = kAdsStep; t < d; t += kAdsStep) {
    const double b = 1.0 + kAdsEps0 / std::sqrt(static_cast<double>(t));
    f.push_back((static_cast<double>(t) / static_cast<double>(d)) * (b * b));
  }
  return f;
}
size_t ads_table_bytes(int d) { return align_up(static_cast<size_t>(d / kAdsStep + 1) * sizeof(double)); }

}  // namespace

// Scratch of crisp_search_static: one copy per GPU, held until the process
// ends.  Host code never takes its name as an address; each device's
// address comes from hipGetSymbolAddress (static_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[CRISP_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per
// device.
crisp_status static_scratch_ptr(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CRISP_E_UNSUPPORTED, "device ordinal %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CRISP_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CRISP_OK;
}
}  // namespace

struct crisp_index {
  int64_t n;
  int d, m, k, h, ncells, tile, ntiles;
  const float *rot, *cent, *base;
  const int32_t *off, *ids;
  const uint64_t *codes;
  const uint16_t *base16 = nullptr;  // bfloat16 copy of the rows (crisp_index_enable_bf16)
  const float *rerr = nullptr;       // per-row bound of the bfloat16 rounding error
  int32_t *tile_off;
  uint16_t *pos16;  // counter byte position of every posting-list entry (load-time form)
  float *cent_t;  // [M][2][h][K]
  double *ads_fac;  // ADSampling factors (t/D)(1 + eps_0/sqrt(t))^2, t = 32, 64, ... < D
  int ncu = 256;  // compute units of the device the index was loaded on
  void *scratch = nullptr;  // that device's static scratch (crisp_search_static)
  // Bumped whenever state a captured plan bakes in changes (budget model,
  // bfloat16 copy); plans re-capture buckets captured under an older value.
  uint64_t gen = 0;
  std::string scratch_err;  // why it is unavailable
  hipStream_t aux = nullptr;  // second chunk pipeline (overlap = 1)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // learned budget model (borrowed device pointers; null when unset)
  const float *mlp_params = nullptr, *mlp_mean = nullptr, *mlp_std = nullptr;
  int mlp_nf = 0;
  double mlp_delta = 0.0;
  // stage timing (crisp_profile_begin / crisp_profile_end)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_stage;
  size_t prof_used = 0;
  int64_t prof_dropped = 0;
};

namespace {
// Records a start event on construction and a stop event on stop() when the
// index is being profiled and the pool has room.
struct StageTimer {
  crisp_index *ix;
  hipStream_t st;
  long slot = -1;
  StageTimer(crisp_index *ix_, int stage, hipStream_t st_) : ix(ix_), st(st_) {
    if (!ix->prof_on) return;
    if (ix->prof_used + 2 > ix->prof_ev.size()) { ++ix->prof_dropped; return; }
    slot = static_cast<long>(ix->prof_used);
    ix->prof_used += 2;
    ix->prof_stage[slot / 2] = stage;
    (void)hipEventRecord(ix->prof_ev[slot], st);
  }
  void stop() {
    if (slot >= 0) (void)hipEventRecord(ix->prof_ev[slot + 1], st);
    slot = -1;
  }
};
}  // namespace

// Workspace layout for one chunk of qc queries.
struct Layout {
  size_t qrot, hdist, ptab, ncell, cells, retr, tilecnt, hist, flag, taueff, ncand, segids, segscore, cand,
      score, regA, regB, regC, examined, lastupd, stopped, refined, sstat, feat, lim, queue, order, sclb, scub,
      flist, nflag, rbytes, sfall, avail, hstat, redo, nredo, total;
};

// cap: capacity of each query's candidate list (entries of cand, score,
// the Hamming distances and order, the float64 keys); n when uncapped.
static Layout make_layout(const crisp_index *ix, long long qc, long long cap) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  const long long n = ix->n;
  L.qrot = take(qc * ix->d * 4);
  L.hdist = take(qc * ix->m * 2 * ix->k * 8);
  L.ptab = take(ix->k > 64 ? qc * ix->m * ix->k * (ix->k + 1) * 4 : 0);
  L.ncell = take(qc * ix->m * 4);
  L.cells = take(qc * ix->m * ix->ncells * 4);
  L.retr = take(qc * ix->m * 4);
  L.tilecnt = take(qc * ix->ntiles * kCountWaves * 4);
  L.hist = take(qc * (2 * ix->m + 1) * 4);
  L.flag = take(qc * 4);
  L.taueff = take(qc * 4);
  L.ncand = take(qc * 4);
  L.segids = take(qc * n * 4);     // per-tile segments; later the Hamming order (stride cap)
  L.segscore = take(qc * n);
  L.cand = take(qc * cap * 4);
  L.score = take(qc * cap);
  L.regA = take(qc * cap * 4);     // mode 1: Hamming distance per candidate
  L.regB = take(qc * cap * 4);     // mode 1: Hamming distances in order
  L.regC = take(qc * cap * 8);     // mode 0: float64 keys of the candidates
  L.examined = take(qc * 4);
  L.lastupd = take(qc * 4);
  L.stopped = take(qc * 4);
  L.refined = take(qc * 4);
  L.sstat = take(qc * ix->m * 4 * 8);
  L.feat = take(qc * n_features(ix->m) * 4);
  L.lim = take(qc * 4);
  L.queue = take(4);
  L.order = take(qc * 4);
  L.sclb = take(ix->k <= kWave ? qc * ix->m * 2 * ix->k * 4 : 0);
  L.scub = take(ix->k <= kWave ? qc * ix->m * 2 * ix->k * 4 : 0);
  L.flist = take(qc * 4);
  L.nflag = take(4);
  L.rbytes = take(qc * 8);
  L.sfall = take(qc * 4);
  L.avail = take(qc * 4);
  L.hstat = take(qc * kHamStats * 4);
  L.redo = take(qc * 4);
  L.nredo = take(4);
  L.total = o;
  return L;
}

static long long chunk_of(const crisp_search_params *p, long long nq) {
  long long c = (p && p->max_chunk > 0) ? p->max_chunk : kDefaultChunk;
  return std::max<long long>(1, std::min<long long>(c, std::max<long long>(nq, 1)));
}

static long long cap_of(const crisp_index *ix, const crisp_search_params *p) {
  return (p && p->max_candidates > 0 && p->max_candidates < ix->n) ? p->max_candidates : ix->n;
}

// Workspace of one search of nq queries: the chunk pipelines (two with
// overlap), the list of queries whose candidates overflowed the cap (a count,
// then their indexes), and, with a cap, one uncapped query's workspace in
// which those queries are searched again.
struct SearchWs {
  Layout L;
  size_t ovf, retry, retry_bytes, total;
};
static size_t retry_bytes_of(const crisp_index *ix) { return make_layout(ix, 1, ix->n).total + align_up(8); }
static SearchWs search_ws(const crisp_index *ix, long long nq, const crisp_search_params *p) {
  SearchWs W{};
  const long long cap = cap_of(ix, p);
  W.L = make_layout(ix, chunk_of(p, nq), cap);
  W.ovf = W.L.total * (p->overlap == 1 ? 2 : 1);
  W.retry = W.ovf + align_up(4 + 4 * static_cast<size_t>(std::max<long long>(nq, 1)));
  W.retry_bytes = cap < ix->n ? retry_bytes_of(ix) : 0;
  W.total = W.retry + W.retry_bytes;
  return W;
}

extern "C" {

const char *crisp_last_error(void) { return g_err.c_str(); }
const char *crisp_version(void) { return "crisp-gfx950 0.1"; }

crisp_status crisp_index_derived_bytes(const crisp_index_desc *desc, int32_t tile_ids, size_t *bytes) {
  if (!desc || !bytes) return fail(CRISP_E_INVALID, "null argument");
  crisp_status s = check_shape(desc->n, desc->d, desc->m, desc->k_half);
  if (s != CRISP_OK) return s;
  int tile = resolve_tile(tile_ids);
  if (tile < 4096 || tile > 65536 || (tile & (tile - 1)))
    return fail(CRISP_E_INVALID, "tile_ids must be a power of two in [4096, 65536]");
  long long ntiles = (desc->n + tile - 1) / tile;
  if (ntiles > 1024) return fail(CRISP_E_UNSUPPORTED, "N / tile_ids must be <= 1024");
  long long ncells = static_cast<long long>(desc->k_half) * desc->k_half;
  const size_t h = static_cast<size_t>(desc->d) / (2 * desc->m);
  *bytes = align_up(static_cast<size_t>(desc->m) * ncells * (ntiles + 1) * 4) +
           align_up(static_cast<size_t>(desc->m) * 2 * desc->k_half * h * 4) + ads_table_bytes(desc->d) +
           align_up(static_cast<size_t>(desc->m) * desc->n * 2 + 128) + 256;
  return CRISP_OK;
}

crisp_status crisp_index_load(const crisp_index_desc *desc, int32_t tile_ids, void *derived, size_t derived_bytes,
                              void *hip_stream, crisp_index **out) {
  if (!desc || !out || !derived) return fail(CRISP_E_INVALID, "null argument");
  size_t need = 0;
  crisp_status s = crisp_index_derived_bytes(desc, tile_ids, &need);
  if (s != CRISP_OK) return s;
  if (derived_bytes < need) return fail(CRISP_E_WORKSPACE, "derived buffer %zu < %zu bytes", derived_bytes, need);
  if (!desc->centroids || !desc->offsets || !desc->ids || !desc->base)
    return fail(CRISP_E_INVALID, "centroids, offsets, ids and base are required");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int tile = resolve_tile(tile_ids);
  const int ncells = desc->k_half * desc->k_half;
  const int ntiles = static_cast<int>((desc->n + tile - 1) / tile);
  int32_t *tile_off = static_cast<int32_t *>(derived);
  int32_t *err = reinterpret_cast<int32_t *>(static_cast<char *>(derived) + need - 256);
  const long long cellsm = static_cast<long long>(desc->m) * ncells;
  k_fill<int32_t><<<1, 64, 0, st>>>(err, 1, 0);
  LAUNCH_TRY("k_fill");
  k_validate_csr<<<grid1(cellsm, 256), 256, 0, st>>>(desc->offsets, desc->ids, desc->m, ncells, desc->n, err);
  LAUNCH_TRY("k_validate_csr");
  int32_t herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (herr) return fail(CRISP_E_FORMAT, "CSR arrays inconsistent (offsets/ids)");
  // Only validated offsets are used to address the id arrays.
  k_tile_offsets<<<grid1(cellsm, 256), 256, 0, st>>>(desc->offsets, desc->ids, desc->m, ncells, desc->n, ntiles,
                                                      tile, tile_off);
  LAUNCH_TRY("k_tile_offsets");
  const int hh = desc->d / (2 * desc->m);
  float *cent_t = reinterpret_cast<float *>(static_cast<char *>(derived) +
                                            align_up(static_cast<size_t>(desc->m) * ncells * (ntiles + 1) * 4));
  const long long ncent = static_cast<long long>(desc->m) * 2 * desc->k_half * hh;
  k_transpose_centroids<<<grid1(ncent, 256), 256, 0, st>>>(desc->centroids, desc->m, desc->k_half, hh, cent_t);
  LAUNCH_TRY("k_transpose_centroids");
  // ADSampling factors of Eq. (2), formed on the host in IEEE float64 (one
  // correctly rounded square root each); the copy completes before returning.
  double *ads_fac = reinterpret_cast<double *>(reinterpret_cast<char *>(cent_t) +
                                               align_up(static_cast<size_t>(desc->m) * 2 * desc->k_half * hh * 4));
  // Counter positions of the posting-list entries (uint16 each).
  uint16_t *pos16 = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(ads_fac) + ads_table_bytes(desc->d));
  const long long npos = static_cast<long long>(desc->m) * desc->n;
  k_count_positions<<<grid_stride(npos, 256), 256, 0, st>>>(desc->ids, npos, pos16);
  LAUNCH_TRY("k_count_positions");
  k_fill<uint16_t><<<1, 64, 0, st>>>(pos16 + npos, 64, 0);   // spare entries read past the last sub-slice
  LAUNCH_TRY("k_fill");
  std::vector<double> fac = ads_factors(desc->d);
  if (!fac.empty()) {
    HIP_TRY(hipMemcpyAsync(ads_fac, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  {
    // the counting kernels address their counters from LDS address 0
    const void *kc[3] = {reinterpret_cast<const void *>(&k_count<0>), reinterpret_cast<const void *>(&k_count<1>),
                         reinterpret_cast<const void *>(&k_count<2>)};
    for (int i = 0; i < 3; ++i) {
      hipFuncAttributes fa{};
      HIP_TRY(hipFuncGetAttributes(&fa, kc[i]));
      if (fa.sharedSizeBytes != 0) return fail(CRISP_E_HIP, "k_count<%d> has %zu bytes of static LDS", i, fa.sharedSizeBytes);
    }
  }
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_count<0>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              tile + static_cast<int>(sizeof(CountShared))));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_count<1>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              tile + static_cast<int>(sizeof(CountShared))));
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_count<2>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              tile + static_cast<int>(sizeof(CountShared))));
  {
    const void *rr[5] = {reinterpret_cast<const void *>(&k_rerank<0, false>),
                         reinterpret_cast<const void *>(&k_rerank<0, true>),
                         reinterpret_cast<const void *>(&k_rerank<1, false>),
                         reinterpret_cast<const void *>(&k_rerank<1, true>),
                         reinterpret_cast<const void *>(&k_rerank<1, false, true>)};
    for (int i = 0; i < 5; ++i)
      HIP_TRY(hipFuncSetAttribute(rr[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(rerank_lds(desc->d, 1024, i < 4 && (i & 1) != 0).total)));
  }
  crisp_index *ix = new (std::nothrow) crisp_index{};
  if (!ix) return fail(CRISP_E_INVALID, "out of host memory");
  ix->n = desc->n; ix->d = desc->d; ix->m = desc->m; ix->k = desc->k_half;
  ix->h = desc->d / (2 * desc->m); ix->ncells = ncells; ix->tile = tile; ix->ntiles = ntiles;
  ix->rot = desc->rotation; ix->cent = desc->centroids; ix->base = desc->base;
  ix->off = desc->offsets; ix->ids = desc->ids; ix->codes = desc->codes; ix->tile_off = tile_off;
  ix->pos16 = pos16;
  ix->cent_t = cent_t;
  ix->ads_fac = ads_fac;
  {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      ix->ncu = cu;
  }
  if (static_scratch_ptr(&ix->scratch) != CRISP_OK) {
    ix->scratch = nullptr;
    ix->scratch_err = g_err;
  }
  if (hipStreamCreateWithFlags(&ix->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ix->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ix->ev_join, hipEventDisableTiming) != hipSuccess) {
    crisp_index_free(ix);
    return fail(CRISP_E_HIP, "stream or event creation failed");
  }
  *out = ix;
  return CRISP_OK;
}

crisp_status crisp_index_bf16_bytes(const crisp_index *ix, size_t *bytes) {
  if (!ix || !bytes) return fail(CRISP_E_INVALID, "null argument");
  *bytes = align_up(static_cast<size_t>(ix->n) * ix->d * 2) + align_up(static_cast<size_t>(ix->n) * 4);
  return CRISP_OK;
}

crisp_status crisp_index_enable_bf16(crisp_index *ix, void *buffer, size_t bytes, void *hip_stream) {
  if (!ix) return fail(CRISP_E_INVALID, "null index");
  if (!buffer) {
    ix->base16 = nullptr;
    ix->rerr = nullptr;
    ++ix->gen;
    return CRISP_OK;
  }
  size_t need = 0;
  crisp_status s = crisp_index_bf16_bytes(ix, &need);
  if (s != CRISP_OK) return s;
  if (bytes < need) return fail(CRISP_E_WORKSPACE, "bfloat16 buffer %zu < %zu bytes", bytes, need);
  if (reinterpret_cast<uintptr_t>(buffer) % 16 != 0) return fail(CRISP_E_INVALID, "buffer must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  uint16_t *b16 = static_cast<uint16_t *>(buffer);
  float *err = reinterpret_cast<float *>(static_cast<char *>(buffer) +
                                         align_up(static_cast<size_t>(ix->n) * ix->d * 2));
  k_base_bf16<<<grid_stride(ix->n, 256 / kWave), 256, 0, st>>>(ix->base, ix->n, ix->d, b16, err);
  LAUNCH_TRY("k_base_bf16");
  ix->base16 = b16;
  ix->rerr = err;
  ++ix->gen;
  return CRISP_OK;
}

crisp_status crisp_index_free(crisp_index *index) {
  if (index) {
    for (auto &e : index->prof_ev) (void)hipEventDestroy(e);
    if (index->ev_fork) (void)hipEventDestroy(index->ev_fork);
    if (index->ev_join) (void)hipEventDestroy(index->ev_join);
    if (index->aux) (void)hipStreamDestroy(index->aux);
  }
  delete index;
  return CRISP_OK;
}

static crisp_status check_params(const crisp_index *ix, int64_t nq, int32_t k, const crisp_search_params *p) {
  if (!ix || !p) return fail(CRISP_E_INVALID, "null argument");
  if (nq < 0) return fail(CRISP_E_INVALID, "nq must be >= 0");
  if (k < 1 || k > 1024 || k > ix->n) return fail(CRISP_E_INVALID, "k must be in [1, min(N, 1024)]");
  if (p->mode != 0 && p->mode != 1) return fail(CRISP_E_INVALID, "mode must be 0 or 1");
  if (!(p->alpha > 0.0) || p->alpha > 1.0) return fail(CRISP_E_INVALID, "alpha must be in (0, 1]");
  if (p->tau < 0 || p->tau > 2 * ix->m) return fail(CRISP_E_INVALID, "tau must be in [0, 2M]");
  if (p->mode == 1 && p->patience_factor < 1) return fail(CRISP_E_INVALID, "patience_factor must be >= 1");
  if (p->mode == 1 && !ix->codes) return fail(CRISP_E_UNSUPPORTED, "Optimized Mode needs sign codes");
  if (p->max_chunk < 0) return fail(CRISP_E_INVALID, "max_chunk must be >= 0");
  if (p->budget_source != 0 && p->budget_source != 1) return fail(CRISP_E_INVALID, "budget_source must be 0 or 1");
  if (p->budget_source == 1 && p->mode != 1) return fail(CRISP_E_INVALID, "the learned budget applies to Optimized Mode");
  if (p->budget_source == 1 && !ix->mlp_params) return fail(CRISP_E_INVALID, "no budget model set");
  if (p->precision < 0 || p->precision > 3) return fail(CRISP_E_INVALID, "precision must be 0, 1, 2 or 3");
  if (p->precision >= 1 && !ix->base16)
    return fail(CRISP_E_INVALID, "precision 1, 2 and 3 need crisp_index_enable_bf16");
  if (p->persistent != 0 && p->persistent != 1) return fail(CRISP_E_INVALID, "persistent must be 0 or 1");
  if (p->overlap != 0 && p->overlap != 1) return fail(CRISP_E_INVALID, "overlap must be 0 or 1");
  if (p->walk_order != 0 && p->walk_order != 1) return fail(CRISP_E_INVALID, "walk_order must be 0 or 1");
  if (p->walk_order == 1 && p->budget_source == 1)
    return fail(CRISP_E_INVALID, "the learned budget's features need the Hamming order (walk_order 0)");
  if (p->verify != 0 && p->verify != 1) return fail(CRISP_E_INVALID, "verify must be 0 or 1");
  if (p->order_prefix < 0) return fail(CRISP_E_INVALID, "order_prefix must be >= 0");
  if (p->count_tiles < 0) return fail(CRISP_E_INVALID, "count_tiles must be >= 0");
  if (p->max_candidates < 0) return fail(CRISP_E_INVALID, "max_candidates must be >= 0");
  if (p->verify == 1 && p->mode != 1) return fail(CRISP_E_INVALID, "ADSampling (verify 1) is for Optimized Mode");
  if (p->verify == 1 && p->precision != 0) return fail(CRISP_E_INVALID, "ADSampling (verify 1) needs precision 0");
  return CRISP_OK;
}

crisp_status crisp_search_workspace_bytes(const crisp_index *index, int64_t nq, int32_t k,
                                          const crisp_search_params *params, size_t *bytes) {
  if (!bytes) return fail(CRISP_E_INVALID, "null argument");
  crisp_status s = check_params(index, nq, k, params);
  if (s != CRISP_OK) return s;
  *bytes = search_ws(index, nq, params).total;
  return CRISP_OK;
}

// A0 launch.  The direct-to-LDS kernel needs 16-byte aligned rows and pays
// off once its 128x128 tiles give every compute unit a block; smaller grids
// (few rows, small D) run the small-tile kernel, which has twice the blocks.
static void launch_rotate(const float *x, long long rows, int d, const float *r, float *out, const int32_t *live,
                          int ncu, hipStream_t st) {
  const long long tiles = static_cast<long long>((d + kRotBN - 1) / kRotBN) * ((rows + kRotBM - 1) / kRotBM);
  const bool aligned = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(r)) & 15u) == 0;
  if (aligned && tiles >= ncu) {
    dim3 g((d + kRotBN - 1) / kRotBN, static_cast<unsigned>((rows + kRotBM - 1) / kRotBM));
    k_rotate_rows<<<g, 256, 0, st>>>(x, rows, d, r, out, live);
  } else {
    dim3 g(d / kRotSmBN, static_cast<unsigned>((rows + kRotSmBM - 1) / kRotSmBM));
    k_rotate_rows_small<<<g, 256, 0, st>>>(x, rows, d, r, out, live);
  }
}

static crisp_status tap_copy(void *dst, const void *src, size_t bytes, hipStream_t st) {
  if (!dst || bytes == 0) return CRISP_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
  return CRISP_OK;
}

// rows of `width` bytes from a pitch of spitch to one of dpitch
static crisp_status tap_copy_rows(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                                  size_t rows, hipStream_t st) {
  if (!dst || width == 0 || rows == 0) return CRISP_OK;
  HIP_TRY(hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, hipMemcpyDeviceToDevice, st));
  return CRISP_OK;
}

// The taps of query qi of a batch (each array advanced by qi rows).
static const crisp_taps *taps_at(crisp_taps *t, const crisp_taps *src, const crisp_index *ix, long long qi) {
  *t = *src;
  const long long n = ix->n, hk = 2LL * ix->m * ix->k;
  auto adv = [qi](auto *&ptr, long long row) {
    if (ptr) ptr += qi * row;
  };
  adv(t->q_rot, ix->d); adv(t->half_dist, hk); adv(t->n_cells, ix->m);
  adv(t->cells, static_cast<long long>(ix->m) * ix->ncells); adv(t->retrieved, ix->m); adv(t->hist, 2LL * ix->m + 1);
  adv(t->tau_eff, 1); adv(t->n_cand, 1); adv(t->cand, n); adv(t->cand_score, n); adv(t->order, n);
  adv(t->hamming, n); adv(t->examined, 1); adv(t->last_update, 1); adv(t->stopped, 1);
  adv(t->features, n_features(ix->m)); adv(t->limits, 1); adv(t->refined, 1); adv(t->score_lb, hk);
  adv(t->score_ub, hk); adv(t->row_bytes, 1); adv(t->score_fallback, 1);
  return t;
}

}  // extern "C"

// The search pipeline.  live: NULL, or a device array with one count per
// chunk of qc queries; kernels then skip the queries of chunk c at or beyond
// live[c] (a captured graph sized for a batch-size bucket runs any smaller
// batch this way).
// redo: search the queries whose candidates overflowed max_candidates again
// (host-synchronous); a graph capture passes false and its caller redoes
// them after the replay (plan_redo).
static crisp_status search_impl(crisp_index *ix, const float *queries, int64_t nq, int32_t k,
                                const crisp_search_params *p, int64_t *ids, float *dists, void *workspace,
                                size_t ws_bytes, const crisp_taps *taps, hipStream_t st0, const int32_t *live_base,
                                bool redo_overflow);
static crisp_status redo_overflow(crisp_index *ix, const float *queries, int64_t nq, int32_t k,
                                  const crisp_search_params *p, int64_t *ids, float *dists, void *workspace,
                                  const crisp_taps *taps, hipStream_t st) {
  const SearchWs W = search_ws(ix, nq, p);
  if (W.retry_bytes == 0) return CRISP_OK;
  const int32_t *count = reinterpret_cast<const int32_t *>(static_cast<char *>(workspace) + W.ovf);
  int32_t h = 0;
  HIP_TRY(hipMemcpyAsync(&h, count, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h <= 0) return CRISP_OK;
  std::vector<int32_t> list(static_cast<size_t>(h));
  HIP_TRY(hipMemcpyAsync(list.data(), count + 1, 4 * static_cast<size_t>(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  crisp_search_params p1 = *p;
  p1.max_chunk = 1;
  p1.overlap = 0;
  p1.max_candidates = 0;
  for (const int32_t qi : list) {
    p1.limits = p->limits ? p->limits + qi : nullptr;
    crisp_taps t1{};
    const crisp_taps *tp = taps ? taps_at(&t1, taps, ix, qi) : nullptr;
    crisp_status s = search_impl(ix, queries + static_cast<long long>(qi) * ix->d, 1, k, &p1,
                                 ids + static_cast<long long>(qi) * k, dists + static_cast<long long>(qi) * k,
                                 static_cast<char *>(workspace) + W.retry, W.retry_bytes, tp, st, nullptr, false);
    if (s != CRISP_OK) return s;
  }
  return CRISP_OK;
}

static crisp_status search_impl(crisp_index *ix, const float *queries, int64_t nq, int32_t k,
                                const crisp_search_params *p, int64_t *ids, float *dists, void *workspace,
                                size_t ws_bytes, const crisp_taps *taps, hipStream_t st0, const int32_t *live_base,
                                bool redo_overflow_now) {
  crisp_status s = CRISP_OK;
  const long long qc = chunk_of(p, nq);
  const SearchWs W = search_ws(ix, nq, p);
  const Layout &L = W.L;
  const long long cap = cap_of(ix, p);
  // Two chunk pipelines (this stream and the index's second stream, each
  // with its own workspace) when the batch has more than one chunk.
  const bool two = p->overlap == 1 && nq > qc;
  if (ws_bytes < W.total) return fail(CRISP_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, W.total);
  int32_t *ovf_count = reinterpret_cast<int32_t *>(static_cast<char *>(workspace) + W.ovf);
  k_fill<int32_t><<<1, 64, 0, st0>>>(ovf_count, 1, 0);
  LAUNCH_TRY("k_fill");
  if (two) {
    HIP_TRY(hipEventRecord(ix->ev_fork, st0));
    HIP_TRY(hipStreamWaitEvent(ix->aux, ix->ev_fork, 0));
  }
  const int nf = n_features(ix->m);
  const int d = ix->d, m = ix->m, kh = ix->k, nb = 2 * m + 1;
  const long long n = ix->n;
  const int budget = static_cast<int>(std::max<double>(1.0, std::ceil(p->alpha * static_cast<double>(n))));
  const int patience =
      p->mode == 1 ? static_cast<int>(std::min<long long>(static_cast<long long>(p->patience_factor) * k, INT32_MAX)) : 0;
  const size_t count_lds = static_cast<size_t>(ix->tile) + sizeof(CountShared);
  const int nseg = ix->ntiles * kCountWaves;
  const bool bf16 = p->precision >= 1;
  // precision 2: certified bfloat16 matrix-core pre-scoring of the half
  // distances (K <= 64); the selection ignores it while the exact half
  // distances are tapped
  const bool score = p->precision >= 2 && ix->k <= kWave;
  const bool score_used = score && !(taps && taps->half_dist);
  const size_t rr_lds = rerank_lds(d, k, bf16).total;
  // Hamming order: positions placed before the walk (whole distance bins
  // covering them); all of them when the order or its distances are tapped
  const bool full_order = taps && (taps->order || taps->hamming);
  const long long plen_auto = 2ll * patience + 1024;
  const int plen = full_order ? INT32_MAX
                              : static_cast<int>(std::min<long long>(p->order_prefix > 0 ? p->order_prefix : plen_auto,
                                                                     INT32_MAX));
  // float32 error factor of the bfloat16 row distance: gamma_{L+10}, L = terms per lane
  const double lterms = static_cast<double>((d / 8 + kWave - 1) / kWave * 8 + 10) * 5.9604644775390625e-08;
  const double gam = lterms / (1.0 - lterms);
  auto rerank0 = bf16 ? k_rerank<0, true> : k_rerank<0, false>;
  auto rerank1 = bf16 ? k_rerank<1, true> : (p->verify == 1 ? k_rerank<1, false, true> : k_rerank<1, false>);
  // Persistent re-rank: as many blocks as fit on the chip at once.
  int rr_resident = 0;
  if (p->persistent) {
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(p->mode == 0 ? rerank0 : rerank1), kRerankThreads, rr_lds));
    rr_resident = std::max(1, per_cu) * ix->ncu;
  }

  for (long long q0 = 0; q0 < nq; q0 += qc) {
    const bool odd = two && ((q0 / qc) & 1);
    hipStream_t st = odd ? ix->aux : st0;
    char *ws = static_cast<char *>(workspace) + (odd ? L.total : 0);
    float *qrot = reinterpret_cast<float *>(ws + L.qrot);
    double *hdist = reinterpret_cast<double *>(ws + L.hdist);
    int32_t *ptab = reinterpret_cast<int32_t *>(ws + L.ptab);
    int32_t *ncell = reinterpret_cast<int32_t *>(ws + L.ncell);
    int32_t *cells = reinterpret_cast<int32_t *>(ws + L.cells);
    int32_t *retr = reinterpret_cast<int32_t *>(ws + L.retr);
    int32_t *tilecnt = reinterpret_cast<int32_t *>(ws + L.tilecnt);
    int32_t *hist = reinterpret_cast<int32_t *>(ws + L.hist);
    int32_t *flag = reinterpret_cast<int32_t *>(ws + L.flag);
    int32_t *taueff = reinterpret_cast<int32_t *>(ws + L.taueff);
    int32_t *ncand = reinterpret_cast<int32_t *>(ws + L.ncand);
    int32_t *segids = reinterpret_cast<int32_t *>(ws + L.segids);
    uint8_t *segscore = reinterpret_cast<uint8_t *>(ws + L.segscore);
    int32_t *cand = reinterpret_cast<int32_t *>(ws + L.cand);
    uint8_t *score = reinterpret_cast<uint8_t *>(ws + L.score);
    int32_t *regA = reinterpret_cast<int32_t *>(ws + L.regA);
    int32_t *regB = reinterpret_cast<int32_t *>(ws + L.regB);
    double *regC = reinterpret_cast<double *>(ws + L.regC);
    int32_t *exam = reinterpret_cast<int32_t *>(ws + L.examined);
    int32_t *lastu = reinterpret_cast<int32_t *>(ws + L.lastupd);
    int32_t *stopd = reinterpret_cast<int32_t *>(ws + L.stopped);
    int32_t *refd = reinterpret_cast<int32_t *>(ws + L.refined);
    int32_t *queue = reinterpret_cast<int32_t *>(ws + L.queue);
    int32_t *qord = reinterpret_cast<int32_t *>(ws + L.order);
    float *sclb = reinterpret_cast<float *>(ws + L.sclb);
    float *scub = reinterpret_cast<float *>(ws + L.scub);
    int32_t *flist = reinterpret_cast<int32_t *>(ws + L.flist);
    int32_t *nflag = reinterpret_cast<int32_t *>(ws + L.nflag);
    double *sstat = reinterpret_cast<double *>(ws + L.sstat);
    float *feat = reinterpret_cast<float *>(ws + L.feat);
    int32_t *llim = reinterpret_cast<int32_t *>(ws + L.lim);
    long long *rbytes = reinterpret_cast<long long *>(ws + L.rbytes);
    int32_t *sfall = reinterpret_cast<int32_t *>(ws + L.sfall);
    int32_t *avail = reinterpret_cast<int32_t *>(ws + L.avail);
    int32_t *hstat = reinterpret_cast<int32_t *>(ws + L.hstat);
    int32_t *redo = reinterpret_cast<int32_t *>(ws + L.redo);
    int32_t *nredo = reinterpret_cast<int32_t *>(ws + L.nredo);
    const int cq = static_cast<int>(std::min<long long>(qc, nq - q0));
    const float *qin = queries + q0 * d;
    const int32_t *lv = live_base ? live_base + q0 / qc : nullptr;
    // A0
    StageTimer t0(ix, 0, st);
    if (ix->rot) {
      launch_rotate(qin, cq, d, ix->rot, qrot, lv, ix->ncu, st);
      LAUNCH_TRY("k_rotate_rows");
    } else {
      k_copy_f32<<<grid1(static_cast<long long>(cq) * d, 256), 256, 0, st>>>(qin, qrot, static_cast<long long>(cq) * d,
                                                                             lv, d);
      LAUNCH_TRY("k_copy_f32");
    }
    t0.stop();
    // A1 + A2
    {
      StageTimer t2(ix, 2, st);
      if (score) {
        k_fill<int32_t><<<grid1(cq, 256), 256, 0, st>>>(sfall, cq, 0);
        LAUNCH_TRY("k_fill");
        if (p->precision == 3) {
          k_score_fp8<<<dim3((cq + 15) / 16, m), 64, 0, st>>>(qrot, d, ix->cent_t, m, kh, ix->h, cq, sclb, scub, lv);
          LAUNCH_TRY("k_score_fp8");
        } else {
          k_score_bf16x3<<<dim3((cq + 15) / 16, m), 64, 0, st>>>(qrot, d, ix->cent_t, m, kh, ix->h, cq, sclb, scub, lv);
          LAUNCH_TRY("k_score_bf16x3");
        }
      }
      dim3 g(m, cq);
      k_select_cells<<<g, 64, select_lds_bytes(kh, ix->h), st>>>(qrot, d, ix->cent_t, m, kh, ix->h, ix->off,
                                                                  budget, k, p->mode, hdist, ptab, ncell, cells,
                                                                  retr, sstat, lv, score_used ? sclb : nullptr,
                                                                  score_used ? scub : nullptr, sfall);
      LAUNCH_TRY("k_select_cells");
      t2.stop();
    }
    // A3 / A4: the first counting pass is stage 3; clearing, the fallback
    // passes, compaction and the run order are stage 7
    {
      StageTimer t7(ix, 7, st);
      k_fill<int32_t><<<grid1(static_cast<long long>(cq) * nb, 256), 256, 0, st>>>(hist, static_cast<long long>(cq) * nb, 0);
      LAUNCH_TRY("k_fill");
      k_fill<int32_t><<<1, 64, 0, st>>>(nflag, 1, 0);
      LAUNCH_TRY("k_fill");
      t7.stop();
    }
    {
      // Tiles per counting block: given, or up to 4 (a power of two) while
      // at least 16 blocks per compute unit remain (measured on N = 1M,
      // D = 4096: 1, 4, 8, 16 tiles -> 3.46, 3.15, 3.20, 3.18 ms per 10k
      // queries).
      int tpb = 1;
      if (p->count_tiles > 0) {
        tpb = std::min(p->count_tiles, ix->ntiles);
      } else {
        while (tpb * 2 <= std::min(ix->ntiles, 4) &&
               static_cast<long long>(cq) * ((ix->ntiles + 2 * tpb - 1) / (2 * tpb)) >= 16LL * ix->ncu)
          tpb *= 2;
      }
      dim3 g((ix->ntiles + tpb - 1) / tpb, cq);
      StageTimer t3(ix, 3, st);
      k_count<0><<<g, kCountThreads, count_lds, st>>>(ncell, cells, m, ix->ncells, ix->pos16, n, ix->tile_off,
                                                      ix->ntiles, ix->tile, p->tau, flag, taueff, segids, segscore,
                                                      tilecnt, hist, lv, flist, nflag, tpb);
      LAUNCH_TRY("k_count pass 0");
      t3.stop();
      StageTimer t7(ix, 7, st);
      k_flag<<<grid1(cq, 4), 256, 0, st>>>(tilecnt, nseg, cq, k, p->tau, flag, taueff, hist, nb, lv, flist, nflag);
      LAUNCH_TRY("k_flag");
      // the fallback passes walk the flagged queries' list
      const dim3 gf(ix->ntiles, std::min(cq, 256));
      k_count<1><<<gf, kCountThreads, count_lds, st>>>(ncell, cells, m, ix->ncells, ix->pos16, n, ix->tile_off,
                                                      ix->ntiles, ix->tile, p->tau, flag, taueff, segids, segscore,
                                                      tilecnt, hist, lv, flist, nflag, 1);
      LAUNCH_TRY("k_count pass 1");
      k_tau_eff<<<grid1(cq, 256), 256, 0, st>>>(flag, cq, k, p->tau, nb, hist, taueff, tilecnt, nseg, lv);
      LAUNCH_TRY("k_tau_eff");
      k_count<2><<<gf, kCountThreads, count_lds, st>>>(ncell, cells, m, ix->ncells, ix->pos16, n, ix->tile_off,
                                                      ix->ntiles, ix->tile, p->tau, flag, taueff, segids, segscore,
                                                      tilecnt, hist, lv, flist, nflag, 1);
      LAUNCH_TRY("k_count pass 2");
      k_compact<<<cq, kCompactThreads, 0, st>>>(segids, segscore, tilecnt, nseg, ix->tile / kCountWaves, n, cap,
                                                 cand, score, ncand, lv, ovf_count, ovf_count + 1, q0);
      LAUNCH_TRY("k_compact");
      if (cq <= kQueryOrderMax) {
        k_query_order<<<1, kQueryOrderThreads, 0, st>>>(cq, ncand, cand, n, cap, qord, lv);
        LAUNCH_TRY("k_query_order");
      } else {
        qord = nullptr;
      }
      t7.stop();
    }
    const int32_t *lim = p->limits ? p->limits + q0 : nullptr;
    // walk_order 1 (ablation): the walk takes the candidates in id order
    const bool ham = p->walk_order == 0;
    if (p->mode == 1 && ham) {
      // A5
      StageTimer t4(ix, 4, st);  // distances
      {
        const int gx = static_cast<int>(std::max(1, std::min(64, (4096 + cq - 1) / cq)));
        const int g = xcd_pad(gx * cq);
        const int vec = hamming_vec(d / 64), jl = hamming_loads(d / 64, vec);
#define CRISP_HAM_ARGS qrot, d, ix->codes, ncand, cand, cap, regA, lv, qord, gx, cq
        if (vec == 2) {
          if (jl == 4) k_hamming_dist<2, 4><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else if (jl == 3) k_hamming_dist<2, 3><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else if (jl == 2) k_hamming_dist<2, 2><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else if (jl == 1) k_hamming_dist<2, 1><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else k_hamming_dist<2, 0><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
        } else {
          if (jl == 4) k_hamming_dist<1, 4><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else if (jl == 3) k_hamming_dist<1, 3><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else if (jl == 2) k_hamming_dist<1, 2><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else if (jl == 1) k_hamming_dist<1, 1><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
          else k_hamming_dist<1, 0><<<g, kOrderThreads, 0, st>>>(CRISP_HAM_ARGS);
        }
#undef CRISP_HAM_ARGS
        LAUNCH_TRY("k_hamming_dist");
      }
      t4.stop();
      StageTimer t1(ix, 1, st);  // order
      k_fill<int32_t><<<1, 64, 0, st>>>(nredo, 1, 0);
      LAUNCH_TRY("k_fill");
      k_hamming_order<<<cq, kOrderThreads, hamming_order_lds(d), st>>>(d, ncand, cand, cap, regA, plen, segids, regB,
                                                                       avail, hstat, lv, nullptr, nullptr);
      LAUNCH_TRY("k_hamming_order");
      t1.stop();
    }
    if (p->mode == 1) {
      // learned budget: features, then bfloat16 MFMA inference -> limits
      if (ham && (p->budget_source == 1 || (taps && taps->features))) {
        StageTimer t6(ix, 6, st);
        k_features<<<grid1(cq, 256), 256, 0, st>>>(cq, m, d, k, 1, ncand, hist, taueff, sstat, hstat, feat, lv);
        LAUNCH_TRY("k_features");
        if (p->budget_source == 1) {
          k_mlp_limits<<<(cq + 15) / 16, 64, 0, st>>>(cq, nf, feat, ix->mlp_mean, ix->mlp_std, ix->mlp_params,
                                                      ix->mlp_delta, k, ncand, llim, nullptr, lv);
          LAUNCH_TRY("k_mlp_limits");
          if (!lim) lim = llim;
        }
        t6.stop();
      }
      // A6 / A7
      StageTimer t5(ix, 5, st);
      if (p->persistent) {
        k_fill<int32_t><<<1, 64, 0, st>>>(queue, 1, 0);
        LAUNCH_TRY("k_fill");
      }
      rerank1<<<p->persistent ? std::min(cq, rr_resident) : xcd_pad(cq), kRerankThreads, rr_lds, st>>>(qrot, d, ix->base, ix->base16, ix->rerr, gam, ncand,
                                                        ham ? segids : cand, cap, k, patience, lim, regC, nullptr, nullptr,
                                                        ids + q0 * k,
                                                        dists + q0 * k, exam, lastu, stopd, refd, ix->ads_fac,
                                                        rbytes, ham ? avail : nullptr, ham ? redo : nullptr, nredo,
                                                        lv, cq, p->persistent ? queue : nullptr, qord);
      LAUNCH_TRY("k_rerank");
      if (ham && plen < cap) {
        // walks that reached the end of the placed prefix: full order, walk again
        k_hamming_order<<<std::min(cq, 256), kOrderThreads, hamming_order_lds(d), st>>>(
            d, ncand, cand, cap, regA, INT32_MAX, segids, regB, avail, hstat, lv, redo, nredo);
        LAUNCH_TRY("k_hamming_order (redo)");
        rerank1<<<xcd_pad(cq), kRerankThreads, rr_lds, st>>>(qrot, d, ix->base, ix->base16, ix->rerr, gam, ncand,
                                                             segids, cap, k, patience, lim, regC, nullptr, nullptr,
                                                             ids + q0 * k, dists + q0 * k, exam, lastu, stopd, refd,
                                                             ix->ads_fac, rbytes, nullptr, nullptr, nullptr, nredo,
                                                             cq, nullptr, redo);
        LAUNCH_TRY("k_rerank (redo)");
      }
      t5.stop();
    } else {
      StageTimer t5(ix, 5, st);
      if (p->persistent) {
        k_fill<int32_t><<<1, 64, 0, st>>>(queue, 1, 0);
        LAUNCH_TRY("k_fill");
      }
      rerank0<<<p->persistent ? std::min(cq, rr_resident) : xcd_pad(cq), kRerankThreads, rr_lds, st>>>(qrot, d, ix->base, ix->base16, ix->rerr, gam, ncand,
                                                        cand, cap, k, patience, lim, regC,
                                                        reinterpret_cast<float *>(regA), regB, ids + q0 * k,
                                                        dists + q0 * k, exam, lastu, stopd, refd, ix->ads_fac,
                                                        rbytes, nullptr, nullptr, nullptr, lv, cq,
                                                        p->persistent ? queue : nullptr, qord);
      LAUNCH_TRY("k_rerank");
      t5.stop();
    }
    if (taps) {
      const size_t un = static_cast<size_t>(n), uc = static_cast<size_t>(cap);
      if ((s = tap_copy(taps->q_rot ? taps->q_rot + q0 * d : nullptr, qrot, size_t(cq) * d * 4, st))) return s;
      if ((s = tap_copy(taps->half_dist ? taps->half_dist + q0 * m * 2 * kh : nullptr, hdist, size_t(cq) * m * 2 * kh * 8, st))) return s;
      if ((s = tap_copy(taps->n_cells ? taps->n_cells + q0 * m : nullptr, ncell, size_t(cq) * m * 4, st))) return s;
      if ((s = tap_copy(taps->cells ? taps->cells + q0 * m * ix->ncells : nullptr, cells, size_t(cq) * m * ix->ncells * 4, st))) return s;
      if ((s = tap_copy(taps->retrieved ? taps->retrieved + q0 * m : nullptr, retr, size_t(cq) * m * 4, st))) return s;
      if ((s = tap_copy(taps->hist ? taps->hist + q0 * nb : nullptr, hist, size_t(cq) * nb * 4, st))) return s;
      if ((s = tap_copy(taps->tau_eff ? taps->tau_eff + q0 : nullptr, taueff, size_t(cq) * 4, st))) return s;
      if ((s = tap_copy(taps->n_cand ? taps->n_cand + q0 : nullptr, ncand, size_t(cq) * 4, st))) return s;
      // candidate-indexed taps: rows of n entries, filled up to the cap
      if ((s = tap_copy_rows(taps->cand ? taps->cand + q0 * n : nullptr, un * 4, cand, uc * 4, uc * 4, cq, st))) return s;
      if ((s = tap_copy_rows(taps->cand_score ? taps->cand_score + q0 * n : nullptr, un, score, uc, uc, cq, st)))
        return s;
      if (p->mode == 1 && ham) {
        if ((s = tap_copy_rows(taps->order ? taps->order + q0 * n : nullptr, un * 4, segids, uc * 4, uc * 4, cq, st)))
          return s;
        if ((s = tap_copy_rows(taps->hamming ? taps->hamming + q0 * n : nullptr, un * 4, regB, uc * 4, uc * 4, cq, st)))
          return s;
      }
      if ((s = tap_copy(taps->examined ? taps->examined + q0 : nullptr, exam, size_t(cq) * 4, st))) return s;
      if ((s = tap_copy(taps->last_update ? taps->last_update + q0 : nullptr, lastu, size_t(cq) * 4, st))) return s;
      if ((s = tap_copy(taps->stopped ? taps->stopped + q0 : nullptr, stopd, size_t(cq) * 4, st))) return s;
      if ((s = tap_copy(taps->refined ? taps->refined + q0 : nullptr, refd, size_t(cq) * 4, st))) return s;
      if ((s = tap_copy(taps->row_bytes ? taps->row_bytes + q0 : nullptr, rbytes, size_t(cq) * 8, st))) return s;
      if (score_used && (s = tap_copy(taps->score_fallback ? taps->score_fallback + q0 : nullptr, sfall,
                                      size_t(cq) * 4, st))) return s;
      if (score) {
        const size_t sb = size_t(cq) * m * 2 * kh * 4;
        if ((s = tap_copy(taps->score_lb ? taps->score_lb + q0 * m * 2 * kh : nullptr, sclb, sb, st))) return s;
        if ((s = tap_copy(taps->score_ub ? taps->score_ub + q0 * m * 2 * kh : nullptr, scub, sb, st))) return s;
      }
      if (p->mode == 1 && ham && (s = tap_copy(taps->features ? taps->features + q0 * nf : nullptr, feat,
                                        size_t(cq) * nf * 4, st))) return s;
      if (p->budget_source == 1 && (s = tap_copy(taps->limits ? taps->limits + q0 : nullptr, llim,
                                                 size_t(cq) * 4, st))) return s;
    }
  }
  if (two) {
    HIP_TRY(hipEventRecord(ix->ev_join, ix->aux));
    HIP_TRY(hipStreamWaitEvent(st0, ix->ev_join, 0));
  }
  if (redo_overflow_now) return redo_overflow(ix, queries, nq, k, p, ids, dists, workspace, taps, st0);
  return CRISP_OK;
}

__global__ void k_set_live(int32_t *__restrict__ live, int nq, int qc, int nch) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nch) live[c] = max(0, min(qc, nq - c * qc));
}

// A batch executor: one captured graph per batch-size bucket.
struct crisp_plan {
  crisp_index *ix = nullptr;
  int max_batch = 0, k = 0, nbuckets = 0;
  crisp_search_params p{};
  char *ws = nullptr;
  size_t ws_bytes = 0;
  float *q_stage = nullptr;
  int64_t *id_stage = nullptr;
  float *d_stage = nullptr;
  int32_t *live = nullptr;
  hipStream_t cap = nullptr;  // private stream the graphs are captured on
  std::vector<hipGraphExec_t> exec;
  std::vector<uint64_t> exec_gen;  // index generation each bucket was captured under
};

namespace {
struct PlanLayout {
  size_t ws, q, ids, dists, live, total;
};
PlanLayout plan_layout(const crisp_index *ix, int max_batch, int k, const crisp_search_params *p) {
  PlanLayout L{};
  const long long qc = chunk_of(p, max_batch);
  const long long nch = (max_batch + qc - 1) / qc;
  L.ws = 0;
  L.q = align_up(search_ws(ix, max_batch, p).total);
  L.ids = L.q + align_up(static_cast<size_t>(max_batch) * ix->d * 4);
  L.dists = L.ids + align_up(static_cast<size_t>(max_batch) * k * 8);
  L.live = L.dists + align_up(static_cast<size_t>(max_batch) * k * 4);
  L.total = L.live + align_up(static_cast<size_t>(nch) * 4);
  return L;
}
int bucket_of(const crisp_plan *pl, int64_t nq) {
  int b = 0;
  while ((1ll << b) < nq) ++b;
  return std::min(b, pl->nbuckets - 1);
}
long long bucket_size(const crisp_plan *pl, int b) { return std::min<long long>(1ll << b, pl->max_batch); }
}  // namespace

extern "C" {

crisp_status crisp_search(crisp_index *ix, const float *queries, int64_t nq, int32_t k,
                          const crisp_search_params *p, int64_t *ids, float *dists, void *workspace,
                          size_t ws_bytes, const crisp_taps *taps, void *hip_stream) {
  crisp_status s = check_params(ix, nq, k, p);
  if (s != CRISP_OK) return s;
  if (nq == 0) return CRISP_OK;
  if (!queries || !ids || !dists || !workspace) return fail(CRISP_E_INVALID, "null argument");
  return search_impl(ix, queries, nq, k, p, ids, dists, workspace, ws_bytes, taps,
                     static_cast<hipStream_t>(hip_stream), nullptr, true);
}

crisp_status crisp_search_static(crisp_index *ix, const float *queries, int64_t nq, int32_t k,
                                 const crisp_search_params *p, int64_t *ids, float *dists, void *hip_stream) {
  crisp_status s = check_params(ix, nq, k, p);
  if (s != CRISP_OK) return s;
  if (!ix->scratch) return fail(CRISP_E_HIP, "static scratch unavailable: %s", ix->scratch_err.c_str());
  const size_t room = CRISP_STATIC_SCRATCH_BYTES;
  crisp_search_params q = *p;
  q.overlap = 0;
  q.max_chunk = 1;
  const size_t one = search_ws(ix, nq, &q).total;
  if (one > room)
    return fail(CRISP_E_WORKSPACE, "one query needs %zu bytes of workspace; the static scratch holds %zu", one, room);
  if (nq == 0) return CRISP_OK;
  if (!queries || !ids || !dists) return fail(CRISP_E_INVALID, "null argument");
  // Largest chunk (up to the requested one) whose workspace fits.
  long long lo = 1, hi = chunk_of(p, nq);
  while (lo < hi) {
    const long long mid = (lo + hi + 1) / 2;
    q.max_chunk = static_cast<int32_t>(mid);
    if (search_ws(ix, nq, &q).total <= room) lo = mid; else hi = mid - 1;
  }
  q.max_chunk = static_cast<int32_t>(lo);
  return search_impl(ix, queries, nq, k, &q, ids, dists, ix->scratch, room, nullptr,
                     static_cast<hipStream_t>(hip_stream), nullptr, true);
}

crisp_status crisp_plan_bytes(const crisp_index *ix, int32_t max_batch, int32_t k, const crisp_search_params *p,
                              size_t *bytes) {
  if (!bytes) return fail(CRISP_E_INVALID, "null argument");
  if (max_batch < 1) return fail(CRISP_E_INVALID, "max_batch must be >= 1");
  crisp_status s = check_params(ix, max_batch, k, p);
  if (s != CRISP_OK) return s;
  if (p->limits) return fail(CRISP_E_INVALID, "plans take no per-query limits (use budget_source 1)");
  *bytes = plan_layout(ix, max_batch, k, p).total;
  return CRISP_OK;
}

crisp_status crisp_plan_create(crisp_index *ix, int32_t max_batch, int32_t k, const crisp_search_params *p,
                               void *buffer, size_t bytes, crisp_plan **out) {
  if (!out || !buffer) return fail(CRISP_E_INVALID, "null argument");
  size_t need = 0;
  crisp_status s = crisp_plan_bytes(ix, max_batch, k, p, &need);
  if (s != CRISP_OK) return s;
  if (bytes < need) return fail(CRISP_E_WORKSPACE, "plan buffer %zu < %zu bytes", bytes, need);
  const PlanLayout L = plan_layout(ix, max_batch, k, p);
  crisp_plan *pl = new (std::nothrow) crisp_plan{};
  if (!pl) return fail(CRISP_E_INVALID, "out of host memory");
  char *b = static_cast<char *>(buffer);
  pl->ix = ix; pl->max_batch = max_batch; pl->k = k; pl->p = *p;
  pl->ws = b + L.ws; pl->ws_bytes = L.q - L.ws;
  pl->q_stage = reinterpret_cast<float *>(b + L.q);
  pl->id_stage = reinterpret_cast<int64_t *>(b + L.ids);
  pl->d_stage = reinterpret_cast<float *>(b + L.dists);
  pl->live = reinterpret_cast<int32_t *>(b + L.live);
  while ((1ll << pl->nbuckets) < max_batch) ++pl->nbuckets;
  ++pl->nbuckets;
  pl->exec.assign(pl->nbuckets, nullptr);
  pl->exec_gen.assign(pl->nbuckets, 0);
  hipError_t e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete pl;
    return fail(CRISP_E_HIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
  }
  *out = pl;
  return CRISP_OK;
}

static crisp_status plan_capture(crisp_plan *pl, int b) {
  const long long nb = bucket_size(pl, b);
  crisp_index *ix = pl->ix;
  const bool prof = ix->prof_on;
  ix->prof_on = false;
  HIP_TRY(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
  crisp_status s = search_impl(ix, pl->q_stage, nb, pl->k, &pl->p, pl->id_stage, pl->d_stage, pl->ws, pl->ws_bytes,
                               nullptr, pl->cap, pl->live, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(pl->cap, &g);
  ix->prof_on = prof;
  if (s != CRISP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(CRISP_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(CRISP_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  pl->exec[b] = x;
  pl->exec_gen[b] = ix->gen;
  return CRISP_OK;
}

crisp_status crisp_plan_search(crisp_plan *pl, const float *queries, int64_t nq, int64_t *ids, float *dists,
                               void *hip_stream) {
  if (!pl) return fail(CRISP_E_INVALID, "null plan");
  if (nq < 0 || nq > pl->max_batch) return fail(CRISP_E_INVALID, "nq must be in [0, max_batch]");
  if (nq == 0) return CRISP_OK;
  if (!queries || !ids || !dists) return fail(CRISP_E_INVALID, "null argument");
  // The index's state may have changed since the plan was made (a budget
  // model cleared, the bfloat16 copy dropped): validate again.
  crisp_status sv = check_params(pl->ix, nq, pl->k, &pl->p);
  if (sv != CRISP_OK) return sv;
  const int b = bucket_of(pl, nq);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (pl->exec[b] && pl->exec_gen[b] != pl->ix->gen) {
    // Captured before the budget model or bfloat16 copy changed: earlier
    // replays are ordered on this stream, so wait for them and capture anew.
    HIP_TRY(hipStreamSynchronize(st));
    (void)hipGraphExecDestroy(pl->exec[b]);
    pl->exec[b] = nullptr;
  }
  if (!pl->exec[b]) {
    crisp_status s = plan_capture(pl, b);
    if (s != CRISP_OK) return s;
  }
  const long long qc = chunk_of(&pl->p, bucket_size(pl, b));
  const int nch = static_cast<int>((bucket_size(pl, b) + qc - 1) / qc);
  const int d = pl->ix->d, k = pl->k;
  HIP_TRY(hipMemcpyAsync(pl->q_stage, queries, static_cast<size_t>(nq) * d * 4, hipMemcpyDeviceToDevice, st));
  k_set_live<<<grid1(nch, 64), 64, 0, st>>>(pl->live, static_cast<int>(nq), static_cast<int>(qc), nch);
  LAUNCH_TRY("k_set_live");
  HIP_TRY(hipGraphLaunch(pl->exec[b], st));
  HIP_TRY(hipMemcpyAsync(ids, pl->id_stage, static_cast<size_t>(nq) * k * 8, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(dists, pl->d_stage, static_cast<size_t>(nq) * k * 4, hipMemcpyDeviceToDevice, st));
  // queries whose candidates overflowed max_candidates: searched again,
  // uncapped, into the caller's outputs (the replay's overflow list is in
  // the workspace laid out for the bucket)
  return redo_overflow(pl->ix, queries, bucket_size(pl, b), k, &pl->p, ids, dists, pl->ws, nullptr, st);
}

crisp_status crisp_plan_free(crisp_plan *pl) {
  if (!pl) return CRISP_OK;
  for (auto &x : pl->exec)
    if (x) (void)hipGraphExecDestroy(x);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  delete pl;
  return CRISP_OK;
}

crisp_status crisp_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (!dst || !src) return fail(CRISP_E_INVALID, "null argument");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
    return fail(CRISP_E_INVALID, "bytes and both pointers must be multiples of 16");
  const long long n = static_cast<long long>(bytes / 16);
  if (n == 0) return CRISP_OK;
  k_copy_probe<<<grid_stride(n, 256), 256, 0, static_cast<hipStream_t>(hip_stream)>>>(
      static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
  LAUNCH_TRY("k_copy_probe");
  return CRISP_OK;
}

int32_t crisp_mlp_param_count(int32_t f) { return f > 0 ? mlp_param_count(f) : -1; }

int32_t crisp_feature_count(int32_t m) { return m > 0 ? n_features(m) : -1; }

crisp_status crisp_set_budget_model(crisp_index *ix, const float *params, int32_t f, const float *feat_mean,
                                    const float *feat_std, double delta) {
  if (!ix) return fail(CRISP_E_INVALID, "null index");
  if (!params) {
    ix->mlp_params = ix->mlp_mean = ix->mlp_std = nullptr;
    ix->mlp_nf = 0;
    ++ix->gen;
    return CRISP_OK;
  }
  if (f != n_features(ix->m)) return fail(CRISP_E_INVALID, "model has %d features, the index needs %d", f,
                                          n_features(ix->m));
  if (!feat_mean || !feat_std) return fail(CRISP_E_INVALID, "feature mean and std are required");
  if (!std::isfinite(delta)) return fail(CRISP_E_INVALID, "delta must be finite");
  ix->mlp_params = params; ix->mlp_mean = feat_mean; ix->mlp_std = feat_std; ix->mlp_nf = f; ix->mlp_delta = delta;
  ++ix->gen;
  return CRISP_OK;
}

crisp_status crisp_mlp_forward(const float *x, int64_t b, int32_t f, const float *params, float *pre, float *y,
                               void *hip_stream) {
  if (!x || !params || !pre || !y) return fail(CRISP_E_INVALID, "null argument");
  if (b < 1 || f < 1) return fail(CRISP_E_INVALID, "b and f must be positive");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  k_mlp_fwd<<<static_cast<unsigned>(b), kHidden, 0, st>>>(static_cast<int>(b), f, x, params, pre, y);
  LAUNCH_TRY("k_mlp_fwd");
  return CRISP_OK;
}

crisp_status crisp_mlp_backward(const float *x, const float *t, int64_t b, int32_t f, const float *params,
                                const float *pre, const float *y, float *grad, void *hip_stream) {
  if (!x || !t || !params || !pre || !y || !grad) return fail(CRISP_E_INVALID, "null argument");
  if (b < 1 || f < 1) return fail(CRISP_E_INVALID, "b and f must be positive");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int np = mlp_param_count(f);
  k_mlp_bwd<<<grid1(np, 128), 128, 0, st>>>(static_cast<int>(b), f, x, t, params, pre, y, grad);
  LAUNCH_TRY("k_mlp_bwd");
  return CRISP_OK;
}

crisp_status crisp_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t f, int32_t step,
                            float lr, void *hip_stream) {
  if (!params || !grad || !m1 || !m2) return fail(CRISP_E_INVALID, "null argument");
  if (f < 1 || step < 1 || !(lr > 0.f)) return fail(CRISP_E_INVALID, "f >= 1, step >= 1, lr > 0");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int np = mlp_param_count(f);
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = static_cast<float>(1.0 - std::pow(0.9, step));
  const float c2 = static_cast<float>(1.0 - std::pow(0.999, step));
  k_mlp_adam<<<grid1(np, 256), 256, 0, st>>>(np, params, grad, m1, m2, lr, b1, b2, 1e-8f, c1, c2);
  LAUNCH_TRY("k_mlp_adam");
  return CRISP_OK;
}

crisp_status crisp_profile_begin(crisp_index *ix, int32_t max_intervals) {
  if (!ix || max_intervals < 1) return fail(CRISP_E_INVALID, "bad argument");
  if (ix->prof_on) return fail(CRISP_E_INVALID, "profiling already active");
  ix->prof_ev.assign(static_cast<size_t>(max_intervals) * 2, nullptr);
  ix->prof_stage.assign(static_cast<size_t>(max_intervals), 0);
  for (auto &e : ix->prof_ev) HIP_TRY(hipEventCreate(&e));
  ix->prof_used = 0;
  ix->prof_dropped = 0;
  ix->prof_on = true;
  return CRISP_OK;
}

crisp_status crisp_profile_end(crisp_index *ix, crisp_profile *out) {
  if (!ix || !out) return fail(CRISP_E_INVALID, "null argument");
  if (!ix->prof_on) return fail(CRISP_E_INVALID, "profiling not active");
  std::memset(out, 0, sizeof *out);
  crisp_status rc = CRISP_OK;
  for (size_t i = 0; i + 1 < ix->prof_used; i += 2) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(ix->prof_ev[i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ix->prof_ev[i], ix->prof_ev[i + 1]);
    if (e != hipSuccess) { rc = fail(CRISP_E_HIP, "event timing: %s", hipGetErrorString(e)); break; }
    int stg = ix->prof_stage[i / 2];
    out->ms[stg] += ms;
    out->intervals[stg] += 1;
  }
  out->dropped = ix->prof_dropped;
  for (auto &e : ix->prof_ev) (void)hipEventDestroy(e);
  ix->prof_ev.clear();
  ix->prof_stage.clear();
  ix->prof_used = 0;
  ix->prof_on = false;
  return rc;
}

crisp_status crisp_rotate_rows(const float *x, int64_t rows, int32_t d, const float *r, float *out, void *hip_stream) {
  if (!x || !r || !out) return fail(CRISP_E_INVALID, "null argument");
  if (rows < 0 || d < 64 || d % 64 != 0) return fail(CRISP_E_UNSUPPORTED, "rows >= 0, D a positive multiple of 64");
  if (rows == 0) return CRISP_OK;
  if ((rows + kRotBM - 1) / kRotBM > 65535) return fail(CRISP_E_UNSUPPORTED, "too many rows for one call");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 256;
  launch_rotate(x, rows, d, r, out, nullptr, ncu, st);
  LAUNCH_TRY("k_rotate_rows");
  return CRISP_OK;
}

crisp_status crisp_build_covariance(const float *x, int64_t n, int32_t d, const int64_t *rows, int64_t s, double *cov,
                                    void *hip_stream) {
  if (!x || !rows || !cov) return fail(CRISP_E_INVALID, "null argument");
  if (n < 1 || s < 2 || d < 64 || d % 64 != 0) return fail(CRISP_E_INVALID, "need s >= 2 and D a multiple of 64");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double *mean = cov + static_cast<long long>(d) * d;  // caller provides d*d + d doubles
  k_sample_mean<<<grid1(d, 256), 256, 0, st>>>(x, d, rows, s, mean);
  LAUNCH_TRY("k_sample_mean");
  dim3 g(d / 64, d / 64);
  k_covariance<<<g, 256, 0, st>>>(x, d, rows, s, mean, cov);
  LAUNCH_TRY("k_covariance");
  return CRISP_OK;
}

crisp_status crisp_build_assign(const float *x, int64_t n, int32_t d, int32_t col0, int32_t h, const int64_t *rows,
                                int64_t s, const float *cent, int32_t k, int32_t *label, void *hip_stream) {
  if (!x || !cent || !label) return fail(CRISP_E_INVALID, "null argument");
  if (k < 1 || h < 1 || col0 < 0 || col0 + h > d || s < 0) return fail(CRISP_E_INVALID, "bad half or sizes");
  if (static_cast<size_t>(k) * h * 4 > 64 * 1024) return fail(CRISP_E_UNSUPPORTED, "K * h too large");
  if (s == 0) return CRISP_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  k_assign<<<grid1(s, 256), 256, static_cast<size_t>(k) * h * 4, st>>>(x, d, col0, h, rows, s, cent, k, label);
  LAUNCH_TRY("k_assign");
  return CRISP_OK;
}

crisp_status crisp_build_update(const float *x, int64_t n, int32_t d, int32_t col0, int32_t h, const int64_t *rows,
                                const int32_t *member_off, const int32_t *members, int32_t k, float *cent,
                                void *hip_stream) {
  if (!x || !member_off || !members || !cent) return fail(CRISP_E_INVALID, "null argument");
  if (k < 1 || h < 1 || col0 < 0 || col0 + h > d) return fail(CRISP_E_INVALID, "bad half or sizes");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  k_update<<<grid1(static_cast<long long>(k) * h, 256), 256, 0, st>>>(x, d, col0, h, rows, member_off, members, k, cent);
  LAUNCH_TRY("k_update");
  return CRISP_OK;
}

static long long csr_block(int64_t n, int32_t cells) {
  long long blk = 256;
  while ((n + blk - 1) / blk * static_cast<long long>(cells) > (16ll << 20)) blk *= 2;
  return blk;
}

int64_t crisp_build_csr_scratch(int64_t n, int32_t cells) {
  long long blk = csr_block(n, cells);
  return (n + blk - 1) / blk * static_cast<long long>(cells) + cells;
}

crisp_status crisp_build_csr(const int32_t *cell_of, int64_t n, int32_t cells, int32_t *offsets, int32_t *ids,
                             int32_t *scratch, void *hip_stream) {
  if (!cell_of || !offsets || !ids || !scratch) return fail(CRISP_E_INVALID, "null argument");
  if (n < 1 || cells < 1) return fail(CRISP_E_INVALID, "n and cells must be positive");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const long long blk = csr_block(n, cells);
  const long long nblk = (n + blk - 1) / blk;
  int32_t *table = scratch;
  int32_t *totals = scratch + nblk * cells;
  k_fill<int32_t><<<grid1(nblk * cells, 256), 256, 0, st>>>(table, nblk * cells, 0);
  LAUNCH_TRY("k_fill");
  k_csr_count<<<grid1(n, 256), 256, 0, st>>>(cell_of, n, cells, static_cast<int>(blk), table);
  LAUNCH_TRY("k_csr_count");
  k_csr_scan_blocks<<<grid1(cells, 256), 256, 0, st>>>(table, static_cast<int>(nblk), cells, totals);
  LAUNCH_TRY("k_csr_scan_blocks");
  k_csr_offsets<<<1, 1024, 0, st>>>(totals, cells, offsets);
  LAUNCH_TRY("k_csr_offsets");
  k_csr_place<<<grid1(nblk, 64), 64, 0, st>>>(cell_of, n, cells, static_cast<int>(blk), offsets, table, ids);
  LAUNCH_TRY("k_csr_place");
  return CRISP_OK;
}

crisp_status crisp_build_combine(const int32_t *left, const int32_t *right, int64_t n, int32_t k, int32_t *cell_of,
                                 void *hip_stream) {
  if (!left || !right || !cell_of) return fail(CRISP_E_INVALID, "null argument");
  if (n < 0 || k < 1) return fail(CRISP_E_INVALID, "bad sizes");
  if (n == 0) return CRISP_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  k_combine<<<grid1(n, 256), 256, 0, st>>>(left, right, n, k, cell_of);
  LAUNCH_TRY("k_combine");
  return CRISP_OK;
}

crisp_status crisp_build_codes(const float *x, int64_t n, int32_t d, uint64_t *codes, void *hip_stream) {
  if (!x || !codes) return fail(CRISP_E_INVALID, "null argument");
  if (n < 0 || d < 64 || d % 64 != 0) return fail(CRISP_E_UNSUPPORTED, "D must be a positive multiple of 64");
  if (n == 0) return CRISP_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  long long waves = n * (d / 64);
  k_codes<<<grid_stride(waves, 4), 256, 0, st>>>(x, n, d, codes);
  LAUNCH_TRY("k_codes");
  return CRISP_OK;
}

}  // extern "C"
