"""Seeded synthetic workloads: the inputs shared by the oracle and the GPU engine.

This module holds no arithmetic of the CRISP method.  It only draws random
numbers and assembles synthetic correlated Gaussian-mixture data sets, query
sets and the random draws the index build consumes (the Gaussian matrix G
whose QR factor becomes the rotation, and sample / initialisation indices).

Generator
---------
Every random number comes from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), a counter-based
generator: output = Philox(counter, key), so any element of any array can be
produced independently and in any order.  The numpy implementation here and
the HIP implementation in ``synth/csrc/synth_gpu.hip`` follow the published
definition and agree bit for bit (tested against the paper's known-answer
vectors and against each other).

* key     = (seed & 0xffffffff, seed >> 32)
* counter = (j & 0xffffffff, j >> 32, tag, block) for element j of a stream
  identified by ``tag``.

A standard normal variate is approximated by the Irwin-Hall sum of twelve
uniforms minus six: three Philox blocks give twelve 32-bit words u_0..u_11 and
z = (sum u_i) * 2^-32 - 6, which is exact in float64 (mean 0, variance 1,
support [-6, 6]).  Using only exact integer arithmetic keeps the CPU and GPU
twins identical without relying on transcendental functions.

Mixtures
--------
All component parameters are float32.  A row is assembled in float64 by
sequential accumulation (every product is float32 x float32, hence exact in
float64, so fused and unfused evaluation agree) and rounded once to float32:

* local factors (``kind == "local"``):
    x_d = mu[c,d] + sum_r A[c,d,r] * z_r + sigma * eps_d
* global low rank (``kind == "global"``):
    y_r = f32(nu[c,r] + eta_r),  x_d = sum_r B[d,r] * y_r + sigma * eps_d

with c the row's component label, z/eta/eps standard normals rounded to
float32, mu = 2 N(0, I) (so means ~ N(0, 4I)), A ~ N(0, 1) unscaled,
B = N(0, 1) / 8 (1/sqrt(64)), nu = s N(0, I) with s the workload's
``center_scale`` (2 unless stated; a power of two keeps the float32 draw
exact on both generators).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "philox4x32", "uniform_u32", "normals", "Workload", "WORKLOADS",
    "mixture_params", "rows", "TAG",
]

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Stream tags (third counter word).
TAG = {
    "noise": 1, "latent": 2, "label": 3, "mean": 4, "factor": 5, "center": 6,
    "rotation": 7, "cev_sample": 8, "kmeans_sample": 9, "kmeans_init": 10,
    "mlp_init": 11, "mlp_shuffle": 12, "batch": 13, "batch_k": 14,
}


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on arrays of counters; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = np.uint64(k0)
    k1 = np.uint64(k1)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        n0 = (p1 >> _S32) ^ c1 ^ k0
        n2 = (p0 >> _S32) ^ c3 ^ k1
        c0, c1, c2, c3 = n0, p1 & _MASK, n2, p0 & _MASK
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform_u32(seed: int, tag: int, idx) -> np.ndarray:
    """One 32-bit word per element index (block 0, word 0)."""
    idx = np.asarray(idx, dtype=np.uint64)
    k0, k1 = _key(seed)
    lo = idx & _MASK
    hi = idx >> _S32
    out = philox4x32(lo, hi, np.full_like(idx, tag), np.zeros_like(idx), k0, k1)
    return out[0]


def normals(seed: int, tag: int, idx) -> np.ndarray:
    """Irwin-Hall(12) approximate standard normals, exact float64 values."""
    idx = np.asarray(idx, dtype=np.uint64)
    k0, k1 = _key(seed)
    lo = idx & _MASK
    hi = idx >> _S32
    t = np.full_like(idx, tag)
    s = np.zeros(idx.shape, dtype=np.uint64)
    for b in range(3):
        words = philox4x32(lo, hi, t, np.full_like(idx, b), k0, k1)
        for w in words:
            s += w.astype(np.uint64)
    return s.astype(np.float64) * (2.0 ** -32) - 6.0


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic data set + query set + index parameters."""
    name: str
    n: int                 # data set cardinality N
    d: int                 # dimensionality D
    n_comp: int            # mixture components
    rank: int              # factor rank (local) or global latent rank
    noise_var: float       # isotropic noise variance
    kind: str              # "local" | "global"
    seed_data: int
    seed_query: int
    seed_index: int
    m: int                 # subspaces M
    k_half: int            # centroids per half-codebook K
    n_query: int
    k: int                 # neighbours per query
    center_scale: float = 2.0  # global kind: component centres nu = center_scale * N(0, I)

    @property
    def sigma32(self) -> np.float32:
        return np.float32(math.sqrt(self.noise_var))

    def scaled(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    # Plain Guaranteed Mode, CPU-fast size (local rank-8 factors, 20 comps).
    "d128": Workload("d128", 10_000, 128, 20, 8, 0.1, "local",
                     1001, 2001, 4001, 8, 8, 100, 10),
    # Plain engine at scale (local rank-32 factors, 100 comps), D=960.
    "d960": Workload("d960", 1_000_000, 960, 100, 32, 0.1, "local",
                     1002, 2002, 4002, 16, 16, 10_000, 10),
    # The same data with K = 256 centroids per half (65,536 cells per subspace).
    "d960k256": Workload("d960k256", 1_000_000, 960, 100, 32, 0.1, "local",
                         1002, 2002, 4002, 16, 256, 10_000, 10),
    # Strongly correlated global rank-64 data, D=4096: the rotation fires.
    "d4096": Workload("d4096", 1_000_000, 4096, 100, 64, 0.05, "global",
                     1003, 2003, 4003, 32, 50, 10_000, 10),
    # Uneven batching workload, D=3072.
    "d3072": Workload("d3072", 2_000_000, 3072, 200, 64, 0.05, "global",
                     1005, 2005, 4005, 32, 50, 50_000, 10),
    # Overlapping components (centres at scale 0.5 against unit spread in the
    # 64-dim latent space), D=1024: the candidate set depends on alpha and tau.
    "d1024mix": Workload("d1024mix", 1_000_000, 1024, 100, 64, 0.05, "global",
                         1006, 2006, 4006, 16, 50, 10_000, 10, center_scale=0.5),
}


def mixture_params(w: Workload) -> dict:
    """float32 component parameters drawn from the data seed."""
    s = w.seed_data
    if w.kind == "local":
        mu = (2.0 * normals(s, TAG["mean"], np.arange(w.n_comp * w.d))).astype(np.float32)
        a = normals(s, TAG["factor"], np.arange(w.n_comp * w.d * w.rank)).astype(np.float32)
        return {"mu": mu.reshape(w.n_comp, w.d), "a": a.reshape(w.n_comp, w.d, w.rank)}
    if w.kind == "global":
        b = (normals(s, TAG["factor"], np.arange(w.d * w.rank)) / 8.0).astype(np.float32)
        nu = (w.center_scale * normals(s, TAG["center"], np.arange(w.n_comp * w.rank))).astype(np.float32)
        return {"b": b.reshape(w.d, w.rank), "nu": nu.reshape(w.n_comp, w.rank)}
    raise ValueError(w.kind)


def rows(w: Workload, seed: int, start: int, stop: int, params: dict | None = None) -> np.ndarray:
    """Rows [start, stop) of the mixture sample drawn with ``seed`` (float32)."""
    if params is None:
        params = mixture_params(w)
    n_idx = np.arange(start, stop, dtype=np.uint64)
    nr = stop - start
    r = w.rank
    lab = (uniform_u32(seed, TAG["label"], n_idx).astype(np.uint64) * np.uint64(w.n_comp)) >> _S32
    lab = lab.astype(np.int64)
    lat_idx = (n_idx[:, None] * np.uint64(r) + np.arange(r, dtype=np.uint64)[None, :])
    z = normals(seed, TAG["latent"], lat_idx).astype(np.float32)          # (nr, r)
    if w.kind == "global":
        z = (params["nu"][lab].astype(np.float64) + z.astype(np.float64)).astype(np.float32)
    eps_idx = n_idx[:, None] * np.uint64(w.d) + np.arange(w.d, dtype=np.uint64)[None, :]
    eps = normals(seed, TAG["noise"], eps_idx).astype(np.float32)         # (nr, d)
    if w.kind == "local":
        acc = params["mu"][lab].astype(np.float64)                       # (nr, d)
        fac = params["a"][lab]                                           # (nr, d, r)
        for t in range(r):
            acc = acc + fac[:, :, t].astype(np.float64) * z[:, t:t + 1].astype(np.float64)
    else:
        acc = np.zeros((nr, w.d), dtype=np.float64)
        b = params["b"].astype(np.float64)
        for t in range(r):
            acc = acc + b[None, :, t] * z[:, t:t + 1].astype(np.float64)
    acc = acc + np.float64(w.sigma32) * eps.astype(np.float64)
    return acc.astype(np.float32)


def gaussian_matrix(seed: int, d: int) -> np.ndarray:
    """The D x D matrix G ~ N(0, 1) whose QR factor is the random rotation."""
    return normals(seed, TAG["rotation"], np.arange(d * d, dtype=np.uint64)).reshape(d, d)


def sample_indices(seed: int, tag: int, n: int, s: int) -> np.ndarray:
    """``s`` distinct row indices of [0, n), ascending, drawn without replacement.

    Rows are ranked by the key (u32 draw, row index), which is unique, and the
    ``s`` smallest are kept.
    """
    if s >= n:
        return np.arange(n, dtype=np.int64)
    u = uniform_u32(seed, tag, np.arange(n, dtype=np.uint64)).astype(np.uint64)
    key = (u << _S32) | np.arange(n, dtype=np.uint64)
    pick = np.argpartition(key, s - 1)[:s]
    return np.sort(pick).astype(np.int64)


def permutation_prefix(seed: int, tag: int, pool: np.ndarray, s: int) -> np.ndarray:
    """The first ``s`` items of a random order of ``pool`` (distinct items)."""
    pool = np.asarray(pool, dtype=np.int64)
    u = uniform_u32(seed, tag, np.arange(pool.size, dtype=np.uint64)).astype(np.uint64)
    key = (u << _S32) | np.arange(pool.size, dtype=np.uint64)
    order = np.argsort(key, kind="stable")
    return pool[order[:s]]


def batch_ks(seed: int, count: int, choices=(1, 10, 100)) -> list[int]:
    """k of each batch, uniform over ``choices`` (uneven-batching workload)."""
    u = uniform_u32(seed, TAG["batch_k"], np.arange(count, dtype=np.uint64))
    return [int(choices[int(v) % len(choices)]) for v in u]


def batch_sizes(seed: int, total: int, max_batch: int = 4096) -> list[int]:
    """Log-uniform batch sizes in [1, max_batch] summing to ``total``.

    b = floor(exp(u * ln(max_batch + 1))) with u uniform in [0, 1); the last
    batch is truncated.  Used for the uneven-batching workload.
    """
    out, t, i = [], 0, 0
    lim = math.log(max_batch + 1)
    while t < total:
        u = float(uniform_u32(seed, TAG["batch"], np.array([i], dtype=np.uint64))[0]) * 2.0 ** -32
        b = max(1, min(max_batch, int(math.floor(math.exp(u * lim)))))
        b = min(b, total - t)
        out.append(b)
        t += b
        i += 1
    return out
