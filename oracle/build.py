"""Oracle index build (test infrastructure only).

Follows the paper's three build steps:

* Section 4.1 (Correlation-Aware Preprocessing): covariance of a random sample
  of min(0.1 N, 1e5) rows, eigen-decomposition, cumulative explained variance
  (CEV) of the top floor(0.2 D) eigenvalues; if CEV exceeds tau_CEV = 0.85 the
  data are rotated by the Q factor of a Gaussian matrix (Section 3,
  Randomized Orthogonal Rotation) and the rotation is kept with the index.
* Section 3 (Subspace Collision Framework) and Section 4.2: M equal
  contiguous subspaces, each split in two halves with a K-centroid k-means
  codebook per half; a point's cell in subspace m is the pair of its nearest
  half-centroids, combined as i_L * K + i_R.
* Section 4.2 (Cache-Coherent CSR Indexing): per subspace, (cell, id) pairs
  sorted by cell, ids ascending inside a cell; Offsets of size K^2 + 1 and a
  Vector-IDs array of size N.
* Section 3 (Binary Quantization): sign bits b_i(x) = [x_i > 0] of the stored
  (rotated) vector, packed 64 per word, dimension i in word i // 64, bit i % 64.

Floating-point conventions (readings where the paper is silent):

* Rotation of a row (data or query): x'_j = f32( sum_i x_i R_ij ) with the sum
  accumulated in float64 in ascending i.  x_i and R_ij are float32, so every
  product is exact in float64 and fused/unfused evaluation agree.
* Half-distance (used for k-means assignment here and for query scoring):
  acc = 0; for t ascending: delta = f64(a_t) - f64(c_t); acc = acc + delta*delta
  (float64, no fused multiply-add).
* k-means: Lloyd iterations on the sampled rows; assignment to the lowest
  centroid index on ties; each centroid update is the float64 sum of its
  members in ascending sample order divided by the member count, rounded to
  float32; an empty cluster keeps its previous centroid.
"""
from __future__ import annotations

import numpy as np

TAU_CEV = 0.85          # Section 4.1
KMEANS_ITERS = 25       # the paper gives no iteration count (reading)
CEV_SAMPLE_CAP = 100_000
KMEANS_SAMPLE_CAP = 100_000


def cev_sample_size(n: int) -> int:
    """min(0.1 N, 1e5) rows, at least 2 (Section 4.1)."""
    return int(max(2, min(n // 10, CEV_SAMPLE_CAP)))


def cumulative_explained_variance(sample: np.ndarray) -> float:
    """CEV = sum of the top floor(0.2 D) eigenvalues / sum of all (Section 4.1).

    ``sample`` is the (S, D) sampled rows; the covariance is centred and
    normalised by S - 1.
    """
    s = np.asarray(sample, dtype=np.float64)
    d = s.shape[1]
    centred = s - s.mean(axis=0, keepdims=True)
    cov = centred.T @ centred / (s.shape[0] - 1)
    lam = np.linalg.eigvalsh(cov)[::-1]
    top = int(np.floor(0.2 * d))
    return float(lam[:top].sum() / lam.sum())


def needs_rotation(cev: float) -> bool:
    """Rotate iff the CEV exceeds tau_CEV (strictly greater, Section 4.1)."""
    return cev > TAU_CEV


def rotation_from_gaussian(g: np.ndarray) -> np.ndarray:
    """R <- Q where G = Q R' (Section 3); stored as float32."""
    q, _ = np.linalg.qr(np.asarray(g, dtype=np.float64))
    return q.astype(np.float32)


def rotate_rows(x: np.ndarray, r: np.ndarray) -> np.ndarray:
    """x' = x R per row, float64 accumulation in ascending i, rounded to f32."""
    x64 = np.asarray(x, dtype=np.float32).astype(np.float64)
    r64 = np.asarray(r, dtype=np.float32).astype(np.float64)
    acc = np.zeros((x64.shape[0], r64.shape[1]), dtype=np.float64)
    for i in range(r64.shape[0]):
        acc = acc + x64[:, i:i + 1] * r64[i:i + 1, :]
    return acc.astype(np.float32)


def half_distances(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Squared distances of rows a (n, h) to centroids c (K, h), float64.

    Sequential over the h coordinates, unfused (see the module docstring).
    """
    a64 = np.asarray(a, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(c, dtype=np.float32).astype(np.float64)
    acc = np.zeros((a64.shape[0], c64.shape[0]), dtype=np.float64)
    for t in range(a64.shape[1]):
        delta = a64[:, t:t + 1] - c64[None, :, t]
        sq = delta * delta
        acc = acc + sq
    return acc


def nearest_centroid(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Index of the nearest centroid, lowest index on ties."""
    return np.argmin(half_distances(a, c), axis=1).astype(np.int64)


def kmeans(a: np.ndarray, init_rows: np.ndarray, iters: int = KMEANS_ITERS) -> np.ndarray:
    """Lloyd's k-means on rows ``a`` (S, h) starting from a[init_rows]; f32 centroids."""
    a32 = np.asarray(a, dtype=np.float32)
    cent = a32[np.asarray(init_rows)].copy()
    k = cent.shape[0]
    for _ in range(iters):
        lab = nearest_centroid(a32, cent)
        sums = np.zeros((k, a32.shape[1]), dtype=np.float64)
        np.add.at(sums, lab, a32.astype(np.float64))   # in ascending sample order
        cnt = np.bincount(lab, minlength=k)
        upd = cnt > 0
        cent[upd] = (sums[upd] / cnt[upd, None]).astype(np.float32)
    return cent


def build_csr(cells: np.ndarray, n_cells: int):
    """Offsets (n_cells + 1) and ids (N): cell-major, ascending ids in a cell."""
    cells = np.asarray(cells, dtype=np.int64)
    ids = np.argsort(cells, kind="stable").astype(np.int32)
    counts = np.bincount(cells, minlength=n_cells)
    offsets = np.zeros(n_cells + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return offsets.astype(np.int32), ids


def sign_codes(x: np.ndarray) -> np.ndarray:
    """b_i = [x_i > 0], dimension i -> word i // 64, bit i % 64 (uint64)."""
    bits = (np.asarray(x) > 0).astype(np.uint8)
    n, d = bits.shape
    assert d % 64 == 0
    packed = np.packbits(bits, axis=1, bitorder="little")      # (n, d/8) bytes
    return np.ascontiguousarray(packed).view("<u8").reshape(n, d // 64).astype(np.uint64)


def build_index(x: np.ndarray, m: int, k_half: int, *, g: np.ndarray | None,
                cev_rows: np.ndarray, km_rows: np.ndarray, km_init: np.ndarray,
                force_rotation: bool | None = None, iters: int = KMEANS_ITERS) -> dict:
    """Build a CRISP index.

    x        -- (N, D) float32 data
    g        -- (D, D) Gaussian matrix for the rotation (or a callable returning
                it), required only if the rotation fires
    cev_rows -- sampled row indices for the correlation check
    km_rows  -- sampled row indices for k-means training
    km_init  -- K positions into km_rows used as initial centroids
    force_rotation -- None: decide by CEV; True/False: override (tests)
    """
    x = np.asarray(x, dtype=np.float32)
    n, d = x.shape
    assert d % (2 * m) == 0 and d % 64 == 0
    h = d // (2 * m)
    cev = cumulative_explained_variance(x[cev_rows])
    rotate = needs_rotation(cev) if force_rotation is None else bool(force_rotation)
    rot = None
    if rotate:
        rot = rotation_from_gaussian(g() if callable(g) else g)
        x = rotate_rows(x, rot)
    cent = np.zeros((m, 2, k_half, h), dtype=np.float32)
    assign = np.zeros((m, n), dtype=np.int32)
    offsets = np.zeros((m, k_half * k_half + 1), dtype=np.int32)
    ids = np.zeros((m, n), dtype=np.int32)
    for sub in range(m):
        halves = []
        for s in range(2):
            lo = sub * 2 * h + s * h
            part = x[:, lo:lo + h]
            c = kmeans(part[km_rows], km_init, iters)
            cent[sub, s] = c
            halves.append(nearest_centroid(part, c))
        cell = halves[0] * k_half + halves[1]
        assign[sub] = cell
        offsets[sub], ids[sub] = build_csr(cell, k_half * k_half)
    return {
        "n": n, "d": d, "m": m, "k_half": k_half, "cev": cev,
        "rotation": rot, "centroids": cent, "offsets": offsets, "ids": ids,
        "base": x, "codes": sign_codes(x), "assign": assign,
    }


def build_index_for(w, x: np.ndarray, **kw) -> dict:
    """Build with the workload's own seeded random draws (see ``synth``)."""
    import synth
    n = x.shape[0]
    cev_rows = synth.sample_indices(w.seed_index, synth.TAG["cev_sample"], n, cev_sample_size(n))
    km_rows = synth.sample_indices(w.seed_index, synth.TAG["kmeans_sample"], n, min(n, KMEANS_SAMPLE_CAP))
    km_init = synth.permutation_prefix(w.seed_index, synth.TAG["kmeans_init"], np.arange(km_rows.size), w.k_half)
    g = kw.pop("g", None)
    if g is None:
        def g():
            return synth.gaussian_matrix(w.seed_index, w.d)
    return build_index(x, w.m, w.k_half, g=g, cev_rows=cev_rows, km_rows=km_rows,
                       km_init=km_init, **kw)
