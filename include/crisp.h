/*
 * crisp.h -- C ABI of the MI355X (gfx950) CRISP query engine.
 *
 * CRISP ("Correlation-Resilient Indexing via Subspace Partitioning",
 * Dimitropoulos, Michalopoulos, Tsitsigkos, Mamoulis) answers approximate
 * k-nearest-neighbour queries under squared Euclidean distance with a
 * subspace-collision index: M subspaces, each split into two halves with a
 * K-centroid codebook per half; a point's cell in a subspace is the pair of
 * its nearest half-centroids; per subspace a CSR inverted index lists the ids
 * of every cell (Section 4.2).  A query (Algorithm 1, Section 4.3) rotates
 * itself when the index was built with a rotation (Section 4.1), scores its
 * sub-vectors against the half-codebooks, walks the cells of each subspace in
 * ascending cost until a per-subspace id budget is met, counts per-point
 * collisions (Eq. 1; rank-weighted in Optimized Mode), keeps points reaching
 * a threshold tau, and re-ranks them by exact L2 -- all of them (Guaranteed
 * Mode) or in Hamming order with patience termination (Optimized Mode).
 *
 * Conventions for every entry point
 * ---------------------------------
 * * Every call returns crisp_status; CRISP_OK (0) on success.  Nothing throws
 *   across the ABI.  crisp_last_error() returns a thread-local message for
 *   the last non-OK status of the calling thread.
 * * Pointers named "device" are HIP device pointers.  The caller owns every
 *   input, output and workspace buffer; the library owns only the opaque
 *   crisp_index host structure.  The library never allocates device memory.
 * * hip_stream is a hipStream_t (NULL = the default stream).  Work is enqueued
 *   asynchronously on it; results are valid after the stream is synchronised.
 *   Launch failures are reported as CRISP_E_HIP; faults inside kernels surface
 *   at the caller's next synchronisation.
 * * Arguments are validated before anything is enqueued; on any error no
 *   output is written.
 * * Limits: D % 64 == 0, D % (2M) == 0, 1 <= M <= 127 (scores fit in 8 bits),
 *   1 <= K <= 64, 1 <= N < 2^31, D <= 8192.  Violations return
 *   CRISP_E_UNSUPPORTED.  (The selection also has a path for 64 < K <= 256,
 *   switched off: a search with it faulted the GPU at N = 1M, K = 256 and
 *   the cause is not found yet.)
 *
 * Floating-point definitions shared with the CPU reference
 * --------------------------------------------------------
 * * Rotation (Section 3 "Randomized Orthogonal Rotation", Section 4.1):
 *   x'_j = f32( sum_i x_i R_ij ), float64 accumulation in ascending i.  Both
 *   factors are float32, so every product is exact in float64.
 * * Half distance (Algorithm 1, Dist_1 / Dist_2): float64, for t ascending
 *   acc = acc + (f64(a_t) - f64(c_t))^2, unfused.
 * * Cell order inside a subspace (Section 4.3.1, Multi-Sequence traversal):
 *   ascending (d1s[i] + d2s[j], i, j) with i, j the ranks of the left / right
 *   centroids in their half's (distance, index) order; cell id = iL * K + iR.
 * * Distance key (Section 4.3.2, Stage 3, exact L2): the squared L2
 *   distance summed in float64 over the dimensions in ascending order,
 *   acc = acc + (f64(q'_i) - f64(x_i))^2, unfused.  Results are ordered by
 *   (key, id); returned distances are f32(key).  The kernels add the same
 *   terms lane-parallel and use that value only where its rounding
 *   interval decides a comparison or the float32 result; elsewhere they
 *   compute the key by the definition.
 */
#ifndef CRISP_H_
#define CRISP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CRISP_OK = 0,
  CRISP_E_INVALID = -1,     /* bad argument (null pointer, out-of-range value) */
  CRISP_E_WORKSPACE = -2,   /* workspace smaller than the size query returned */
  CRISP_E_HIP = -3,         /* a HIP runtime call failed */
  CRISP_E_FORMAT = -4,      /* index arrays inconsistent (CSR check failed) */
  CRISP_E_UNSUPPORTED = -5  /* shape outside the documented limits */
} crisp_status;

typedef struct crisp_index crisp_index;   /* opaque; freed by crisp_index_free */

/*
 * Index arrays (Section 4.2).  All pointers are device pointers BORROWED for
 * the lifetime of the index; the caller keeps them alive and unchanged.
 *   rotation  -- float32 [D][D] row-major, x' = x R; NULL when the correlation
 *                check did not fire (Section 4.1).
 *   centroids -- float32 [M][2][K][h], h = D / (2M); half 0 covers the first h
 *                dimensions of subspace m (dims m*2h .. m*2h+h-1).
 *   offsets   -- int32 [M][K*K + 1]; offsets[m][0] = 0, non-decreasing,
 *                offsets[m][K*K] = N ("Offsets", size K^2 + 1).
 *   ids       -- int32 [M][N]; cell-major, ascending inside a cell ("Vector IDs").
 *   base      -- float32 [N][D] row-major, in rotated space when rotated.
 *   codes     -- uint64 [N][D/64], bit (i % 64) of word (i / 64) = [base_i > 0]
 *                (Section 3, Binary Quantization).  Required for Optimized Mode.
 */
typedef struct {
  int64_t n;
  int32_t d, m, k_half;
  const float *rotation;
  const float *centroids;
  const int32_t *offsets;
  const int32_t *ids;
  const float *base;
  const uint64_t *codes;
} crisp_index_desc;

/*
 * Bytes of the device buffer crisp_index_load needs for derived per-index
 * tables: per cell and id tile, where each posting list crosses tile
 * boundaries; and the posting lists in the counting kernel's form, 2 bytes
 * per entry (M x N entries).  tile_ids: ids per collision-counting tile (a
 * power of two in [4096, 65536]; 0 = library default).
 */
crisp_status crisp_index_derived_bytes(const crisp_index_desc *desc, int32_t tile_ids,
                                       size_t *bytes);

/*
 * Validates the CSR arrays on the device (offsets monotone with the documented
 * end points; every id in range and ascending inside its cell) and builds the
 * derived tables into `derived` (device, caller-owned, at least the bytes
 * returned above, kept alive until crisp_index_free).  Synchronises
 * hip_stream once to read the validation result.  Returns CRISP_E_FORMAT if
 * the arrays are inconsistent.
 */
crisp_status crisp_index_load(const crisp_index_desc *desc, int32_t tile_ids, void *derived,
                              size_t derived_bytes, void *hip_stream, crisp_index **out);

crisp_status crisp_index_free(crisp_index *index);

/*
 * Mixed-precision verification (Section 4.3.2, Stage 3 reads rows at full
 * width; this halves the bytes of rows that cannot enter the result).
 * crisp_index_bf16_bytes: bytes of the buffer crisp_index_enable_bf16 needs
 * (2 N D for a bfloat16 copy of the rows, round to nearest even, then 4 N for
 * a per-row float32 upper bound of ||x - bf16(x)||).
 * crisp_index_enable_bf16: fills `buffer` (device, caller-owned, 16-byte
 * aligned, kept alive while searches use precision 1) from the index rows on
 * hip_stream and lets searches use precision = 1.  buffer == NULL disables it.
 * The rows must be finite.
 */
crisp_status crisp_index_bf16_bytes(const crisp_index *index, size_t *bytes);
crisp_status crisp_index_enable_bf16(crisp_index *index, void *buffer, size_t bytes, void *hip_stream);

/*
 * Search parameters (Table 1; Section 4.3.2; Section 6 parameter ranges).
 *   mode            -- 0 Guaranteed (phi = 0), 1 Optimized (phi = 1).
 *   alpha           -- retrieval fraction per subspace, 0 < alpha <= 1:
 *                      budget = max(1, ceil(alpha * N)) ids per subspace.
 *   tau             -- integer collision threshold, 0 <= tau <= 2M.
 *   patience_factor -- Optimized Mode stops after patience_factor * k
 *                      consecutive non-updating verifications (paper: 40).
 *   limits          -- optional device int32 [nq]: per-query cap on the number
 *                      of candidates verified in Optimized Mode (the learned
 *                      budget); values < 1 mean "no cap".  NULL = none.
 *   max_chunk       -- queries processed per internal chunk (0 = default);
 *                      the workspace scales with it.
 *   budget_source   -- 0: patience rule only; 1: Optimized Mode also stops
 *                      at the prefix predicted by the model set with
 *                      crisp_set_budget_model (explicit `limits` take
 *                      precedence).
 *   precision       -- 0: every verified row is read in float32.  1: every
 *                      verified row is first read from the bfloat16 copy
 *                      (crisp_index_enable_bf16) to bound its distance, and
 *                      in float32 only where the bound cannot exclude it
 *                      from the result.  Both give identical ids and
 *                      distances (every deciding comparison uses the exact
 *                      float64 key); 1 reads fewer bytes.  2: as 1, and
 *                      for K <= 64 the half-codebook distances (Algorithm 1,
 *                      Dist_1 / Dist_2) are first scored on bfloat16 matrix
 *                      cores (three-term split, float32 accumulation) with a
 *                      certified error bound; the exact float64 distance is
 *                      then computed only for centroids whose bound lets
 *                      them be among the 4 nearest of their half, and the
 *                      cell walk falls back to all exact distances whenever
 *                      it needs a rank the bounds leave open.  Same ids,
 *                      distances and stage outputs; half_dist is only filled
 *                      for every centroid when that tap is requested (which
 *                      then takes the exact path).  3: as 2 with the
 *                      pre-scoring on FP8 (OCP e4m3) matrix cores: per
 *                      (query, half) and per half-codebook power-of-two
 *                      scales, each coordinate split into two e4m3 terms,
 *                      three v_mfma_f32_16x16x32_fp8_fp8 per 32 coordinates,
 *                      float32 accumulation, the same kind of certified
 *                      bound; wider bounds, so more subspaces take the exact
 *                      path (the score_fallback tap counts them).
 *   persistent      -- 0: the re-rank launches one block per query.  1: it
 *                      launches about as many blocks as fit on the chip,
 *                      each pulling queries from a device-side counter (same
 *                      results; the batch executor's tuner picks per bucket).
 *   overlap         -- 0: query chunks run one after another on hip_stream.
 *                      1: odd chunks run on a second stream owned by the
 *                      index, with their own half of a doubled workspace, so
 *                      the kernels of two chunks overlap (same results).  The
 *                      second stream joins hip_stream before the call's work
 *                      completes; calls with overlap on one index must be
 *                      ordered on one stream.
 *   walk_order      -- Optimized Mode only.  0: candidates are verified in
 *                      ascending (Hamming distance, id) order (Section
 *                      4.3.2, Stage 2).  1: in ascending id order, the
 *                      Hamming stage skipped (the ablation of Section 6.4
 *                      without Hamming re-ranking); not with budget_source 1,
 *                      whose features are Hamming distances.
 *   verify          -- Optimized Mode only.  0: every walked candidate is
 *                      verified by its exact L2 distance key.  1: ADSampling
 *                      (Section 3, Eq. (2); Section 4.3.2, Stage 3): once the
 *                      top-k holds k items, a walked candidate is pruned at
 *                      the first t = 32, 64, ... below D where the key's
 *                      running sum over its first t dimensions exceeds
 *                      r_k^2 (t/D)(1 + eps_0/sqrt(t))^2, eps_0 = 2.1, r_k^2
 *                      the k-th key at that moment (the product in float64);
 *                      a pruned candidate counts as a non-update, the others
 *                      are verified exactly.  Needs precision 0.
 *   order_prefix    -- Optimized Mode: positions of the Hamming order placed
 *                      before the walk (whole distance bins covering them;
 *                      0 = 2 P + 1024, P the patience).  A walk that reaches
 *                      their end without stopping is walked again on the
 *                      full order, so results never depend on it.
 *   count_tiles     -- id tiles that one block of the collision-counting
 *                      stage counts in turn (the activated cells are read
 *                      once for them; 0 = chosen from the chunk size and the
 *                      number of compute units).  Results do not depend on
 *                      it.
 *   max_candidates  -- capacity of a query's candidate list in the workspace
 *                      (0, or N or more: N, uncapped).  The candidate-indexed
 *                      buffers (candidates, their scores, Hamming distances
 *                      and order, float64 keys: 21 bytes per entry) shrink
 *                      from N to this many entries per query; the per-tile
 *                      counting segments stay N (5 bytes per id).  A query
 *                      with more candidates is searched again, alone, with
 *                      N-entry lists in a reserved part of the workspace,
 *                      after the batch (crisp_search waits for the batch to
 *                      find them: one host synchronisation per call, and
 *                      one per crisp_plan_search).  Results and taps do not
 *                      depend on it.
 */
typedef struct {
  int32_t mode;
  double alpha;
  int32_t tau;
  int32_t patience_factor;
  const int32_t *limits;
  int32_t max_chunk;
  int32_t budget_source;
  int32_t precision;
  int32_t persistent;
  int32_t overlap;
  int32_t walk_order;
  int32_t verify;
  int32_t order_prefix;
  int32_t count_tiles;
  int32_t max_candidates;
} crisp_search_params;

/*
 * Optional stage outputs for verification (device pointers, each may be NULL).
 * Sizes are per query; rows are laid out query-major for all nq queries.
 *   q_rot       float32 [nq][D]        rotated query (A0)
 *   half_dist   float64 [nq][M][2][K]  Dist_1 / Dist_2 (A1)
 *   n_cells     int32  [nq][M]         activated cells per subspace (A2)
 *   cells       int32  [nq][M][K*K]    activated cell | weight << 24, any order
 *   retrieved   int32  [nq][M]         ids in the activated cells of subspace m
 *   hist        int32  [nq][2M+1]      number of points with each score
 *   tau_eff     int32  [nq]            threshold after the fallback rule
 *   n_cand      int32  [nq]            |C|
 *   cand        int32  [nq][N]         candidates, ascending id (first n_cand)
 *   cand_score  uint8  [nq][N]         their scores
 *   order       int32  [nq][N]         candidates in (Hamming, id) order (mode 1)
 *   hamming     int32  [nq][N]         their Hamming distances (mode 1)
 *   examined    int32  [nq]            candidates verified
 *   last_update int32  [nq]            1-based position of the last top-k update
 *   stopped     int32  [nq]            1 if the patience rule ended the walk
 *   features    float32 [nq][F]        learned-budget features (mode 1), F = 17 + 3M + 13
 *   limits      int32  [nq]            predicted verification limits (budget_source 1)
 *   refined     int32  [nq]            verified rows read in float32 (precision 0:
 *                                      every one; 1: those the bfloat16 bound kept;
 *                                      verify 1: those ADSampling did not prune)
 *   row_bytes   int64  [nq]            bytes of stored rows the verification read
 *                                      (rows of a walk chunk past the stop included)
 *   score_fallback int32 [nq]          precision 2 and 3: subspaces whose cell
 *                                      selection the certified bounds did not
 *                                      decide (computed on the exact path)
 *   score_lb    float32 [nq][M][2][K]  precision 2, K <= 64: certified lower and
 *   score_ub    float32 [nq][M][2][K]  upper bounds of Dist_1 / Dist_2 from the
 *                                      bfloat16 matrix-core scoring
 */
typedef struct {
  float *q_rot;
  double *half_dist;
  int32_t *n_cells;
  int32_t *cells;
  int32_t *retrieved;
  int32_t *hist;
  int32_t *tau_eff;
  int32_t *n_cand;
  int32_t *cand;
  uint8_t *cand_score;
  int32_t *order;
  int32_t *hamming;
  int32_t *examined;
  int32_t *last_update;
  int32_t *stopped;
  float *features;
  int32_t *limits;
  int32_t *refined;
  float *score_lb;
  float *score_ub;
  int64_t *row_bytes;
  int32_t *score_fallback;
} crisp_taps;

/* Bytes of workspace crisp_search needs for this index, batch and parameters. */
crisp_status crisp_search_workspace_bytes(const crisp_index *index, int64_t nq, int32_t k,
                                          const crisp_search_params *params, size_t *bytes);

/*
 * Algorithm 1 for a batch of queries.
 *   queries -- device float32 [nq][D] (original, unrotated space)
 *   ids     -- device int64 [nq][k], ascending (key, id); -1 padding
 *   dists   -- device float32 [nq][k], f32(key) squared L2; +inf padding
 *   workspace -- device, >= crisp_search_workspace_bytes(...)
 *   taps    -- NULL, or stage outputs to fill (see crisp_taps)
 * Padding occurs only when fewer than k points collide at all.
 * 1 <= k <= min(N, 1024); nq >= 0 (nq == 0 is a no-op).
 */
crisp_status crisp_search(crisp_index *index, const float *queries, int64_t nq, int32_t k,
                          const crisp_search_params *params, int64_t *ids, float *dists,
                          void *workspace, size_t ws_bytes, const crisp_taps *taps,
                          void *hip_stream);

/*
 * crisp_search without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP stream capture, tight serving
 * loops, hosts that forbid allocation).  The pipeline's scratch is a static
 * device array of CRISP_STATIC_SCRATCH_BYTES per GPU, which every GPU the
 * library is loaded on holds until the process ends; its address is taken
 * once per device when an index is loaded there.  Arguments as for
 * crisp_search (device pointers, caller-owned); params->overlap is ignored
 * (one pipeline) and there are no taps.  Queries run in chunks of at most
 * params->max_chunk (0 = the default), fewer when a chunk's workspace would
 * not fit the array; CRISP_E_WORKSPACE when even one query's workspace does
 * not fit (it grows with N: crisp_search_workspace_bytes(index, 1, ...)).
 * Results equal crisp_search's bit for bit.  Calls on one GPU share the
 * array: calls that overlap in time on that GPU (other streams, other
 * threads, other indexes) race and must be serialised by the caller.  Never
 * calls hipMalloc or hipFree.
 */
#define CRISP_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
crisp_status crisp_search_static(crisp_index *index, const float *queries, int64_t nq, int32_t k,
                                 const crisp_search_params *params, int64_t *ids, float *dists,
                                 void *hip_stream);

/*
 * Batch executor for uneven batch sizes (serving; each query still runs
 * Algorithm 1 exactly as crisp_search does, with identical results).
 * A plan serves batches of 1..max_batch queries with fixed k and parameters
 * (params->limits must be NULL; the learned budget uses budget_source 1).
 * Batch sizes are grouped in power-of-two buckets; the first batch of a
 * bucket captures the whole search pipeline for the bucket's largest size
 * into a HIP graph (on a private stream), and every later batch of that
 * bucket replays it: the queries are copied into the plan's staging buffer,
 * a device-side count of live queries makes the kernels skip the padding,
 * and the results are copied out.
 *   crisp_plan_bytes  -- device bytes the plan's buffer needs (workspace for
 *                        max_batch queries, staging for queries and results).
 *   crisp_plan_create -- `buffer` (device, caller-owned, kept alive until
 *                        crisp_plan_free) is carved into those parts.  The
 *                        index must outlive the plan.
 *   crisp_plan_search -- enqueues one batch on hip_stream (device pointers:
 *                        queries nq*D float32, ids nq*k int64, dists nq*k
 *                        float32); 0 <= nq <= max_batch.  Batches of one
 *                        plan must be stream-ordered: they share the staging
 *                        buffers.  Capturing a new bucket synchronises the
 *                        private stream only.  The parameters are checked
 *                        against the index again on every call (a budget
 *                        model cleared since, a bfloat16 copy dropped:
 *                        CRISP_E_INVALID).  A bucket captured before the
 *                        index's budget model or bfloat16 copy last changed
 *                        (crisp_set_budget_model, crisp_index_enable_bf16) is
 *                        captured anew: that call first synchronises
 *                        hip_stream, where the earlier batches ran.
 *   crisp_plan_free   -- releases the graphs and the private stream.
 */
typedef struct crisp_plan crisp_plan;
crisp_status crisp_plan_bytes(const crisp_index *index, int32_t max_batch, int32_t k,
                              const crisp_search_params *params, size_t *bytes);
crisp_status crisp_plan_create(crisp_index *index, int32_t max_batch, int32_t k,
                               const crisp_search_params *params, void *buffer, size_t bytes,
                               crisp_plan **out);
crisp_status crisp_plan_search(crisp_plan *plan, const float *queries, int64_t nq, int64_t *ids,
                               float *dists, void *hip_stream);
crisp_status crisp_plan_free(crisp_plan *plan);

/*
 * Row rotation x' = x R with the float64 ascending-order definition above
 * (Section 3; used for queries, and for the data set when building).
 *   x -- device float32 [rows][d]; r -- device float32 [d][d]; out -- device
 *   float32 [rows][d] (must not alias x).  Any 4-byte alignment is accepted;
 *   x and r 16-byte aligned with at least one 128 x 128 output tile per
 *   compute unit take the faster kernel (same results).
 * Errors: CRISP_E_INVALID for a null pointer; CRISP_E_UNSUPPORTED when d is
 * not a positive multiple of 64 or rows exceed 128 x 65,535 in one call.
 */
crisp_status crisp_rotate_rows(const float *x, int64_t rows, int32_t d, const float *r,
                               float *out, void *hip_stream);

/* ---- Index build on the GPU (Sections 3, 4.1, 4.2) ---------------------- */

/*
 * Centred sample covariance (Section 4.1): cov_ij = sum_s (x_si - mu_i)
 * (x_sj - mu_j) / (S - 1) over the sampled rows, accumulated in float64.
 *   x -- device float32 [n][d]; rows -- device int64 [s] sampled row indices;
 *   cov -- device float64 [d*d + d]: the [d][d] covariance followed by the d
 *   column means.  s >= 2.
 */
crisp_status crisp_build_covariance(const float *x, int64_t n, int32_t d, const int64_t *rows,
                                    int64_t s, double *cov, void *hip_stream);

/*
 * One Lloyd assignment on sampled rows of one half (k-means, Section 3):
 * label[i] = argmin_c halfdist(x[rows[i]][col0 .. col0+h), cent[c]) with the
 * lowest index on ties.
 *   x -- device float32 [n][d]; rows -- device int64 [s] (NULL: rows 0..s-1);
 *   cent -- device float32 [k][h]; label -- device int32 [s].
 */
crisp_status crisp_build_assign(const float *x, int64_t n, int32_t d, int32_t col0, int32_t h,
                                const int64_t *rows, int64_t s, const float *cent, int32_t k,
                                int32_t *label, void *hip_stream);

/*
 * Lloyd update: cent[c] = f32( (float64 sum of the member rows in the order
 * listed) / count ) for every non-empty cluster; empty clusters keep their
 * centroid.  member_off -- device int32 [k + 1], members -- device int32
 * sample positions grouped by cluster (ascending inside a cluster, as
 * crisp_build_csr produces from the labels); row = rows[member] (rows NULL:
 * row = member).
 */
crisp_status crisp_build_update(const float *x, int64_t n, int32_t d, int32_t col0, int32_t h,
                                const int64_t *rows, const int32_t *member_off,
                                const int32_t *members, int32_t k, float *cent, void *hip_stream);

/*
 * Stable counting sort of cell labels into CSR (Section 4.2): offsets int32
 * [cells + 1], ids int32 [n] (cell-major, ascending ids inside a cell).
 * cell_of -- device int32 [n] in [0, cells); scratch -- device int32 of at
 * least crisp_build_csr_scratch(n, cells) ints.
 */
int64_t crisp_build_csr_scratch(int64_t n, int32_t cells);
crisp_status crisp_build_csr(const int32_t *cell_of, int64_t n, int32_t cells, int32_t *offsets,
                             int32_t *ids, int32_t *scratch, void *hip_stream);

/* cell_of[i] = left[i] * k + right[i] (Combine). */
crisp_status crisp_build_combine(const int32_t *left, const int32_t *right, int64_t n, int32_t k,
                                 int32_t *cell_of, void *hip_stream);

/* Sign codes (Section 3): codes uint64 [n][d/64] from x float32 [n][d]. */
crisp_status crisp_build_codes(const float *x, int64_t n, int32_t d, uint64_t *codes,
                               void *hip_stream);

/* ---- Learned verification budget (Optimized Mode) ----------------------- */

/*
 * An addition on top of the patience rule of Section 4.3.2 (Stage 3): a
 * 2-layer MLP (64 hidden units, ReLU) predicts y = log(L*), L* being the
 * 1-based position of the last top-k update of the plain walk, from F =
 * 17 + 3M + 13 per-query features (log1p |C|; log1p of the counts at the 16
 * highest score levels; per subspace (c2-c1)/c1, (c_cut-c1)/c1 and log1p of
 * the cheapest cell's size; Hamming distances at positions 1, 2, 4, ...,
 * 2048 (clamped to |C|) and at the median position, over D).  The walk stops at min(patience stop, clamp(ceil(exp(y + delta)),
 * k, |C|)).  Inference rounds the standardised features and W1 to bfloat16
 * and runs on MFMA with float32 accumulation.
 *
 * Parameters: one float32 array of crisp_mlp_param_count(F) values laid out
 * w1 [F][64] | b1 [64] | w2 [64] | b2 [1].
 */
int32_t crisp_feature_count(int32_t m);
int32_t crisp_mlp_param_count(int32_t f);

/*
 * Uses `params`, `feat_mean`, `feat_std` (device float32, borrowed until
 * replaced or cleared) for searches with budget_source = 1; features are
 * standardised as (f - mean) / std.  params == NULL clears the model.
 */
crisp_status crisp_set_budget_model(crisp_index *index, const float *params, int32_t f, const float *feat_mean,
                                    const float *feat_std, double delta);

/*
 * Training kernels (float32, device pointers).  x [b][f] standardised
 * features, t [b] targets; pre [b][64] pre-activations and y [b] outputs of
 * the forward pass; grad has the parameter layout (mean squared error,
 * sums over the batch in sample order); Adam with beta1 0.9, beta2 0.999,
 * eps 1e-8, step >= 1, moments m1, m2 zero-initialised by the caller.
 */
crisp_status crisp_mlp_forward(const float *x, int64_t b, int32_t f, const float *params, float *pre, float *y,
                               void *hip_stream);
crisp_status crisp_mlp_backward(const float *x, const float *t, int64_t b, int32_t f, const float *params,
                                const float *pre, const float *y, float *grad, void *hip_stream);
crisp_status crisp_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t f, int32_t step,
                            float lr, void *hip_stream);

/* ---- Measurement --------------------------------------------------------- */

/*
 * Plain device-to-device copy of `bytes` (a multiple of 16; both pointers
 * 16-byte aligned; the ranges must not overlap) by the kernel k_copy_probe,
 * which reads and writes exactly `bytes`.  Hardware byte counters
 * (FETCH_SIZE, WRITE_SIZE) read for it give the factor that turns the
 * counters read for another kernel in the same run into bytes.
 */
crisp_status crisp_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream);

/* ---- Stage timing ------------------------------------------------------ */

/*
 * GPU time per query stage, measured with HIP events recorded on the search
 * stream around each stage's launches.  Stages: 0 rotation, 1 Hamming
 * order placement, 2 half distances + cell selection, 3 collision counting
 * (the first counting pass alone), 4 Hamming distances, 5 re-rank (exact
 * keys, top-k or patience walk), 6 learned-budget features and inference,
 * 7 candidate lists (score histogram clear, fallback flag, the two fallback
 * counting passes, effective threshold, compaction, query run order).
 */
typedef struct {
  double ms[8];
  int64_t intervals[8];
  int64_t dropped;       /* intervals not timed because the event pool was full */
} crisp_profile;

/*
 * Starts timing the index's subsequent crisp_search calls: creates a pool of
 * 2 * max_intervals HIP events (host-side driver objects; no device memory).
 * Calls that overlap on several streams are timed per stream interval.
 */
crisp_status crisp_profile_begin(crisp_index *index, int32_t max_intervals);

/* Waits for the recorded events, writes the sums to *out, releases the pool. */
crisp_status crisp_profile_end(crisp_index *index, crisp_profile *out);

/* Thread-local message for the last non-OK status. */
const char *crisp_last_error(void);

/* Library version string. */
const char *crisp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CRISP_H_ */
