"""Exact k-nearest-neighbour ground truth (test infrastructure only).

The problem statement of Section 3 (Exact and Approximate Similarity Search):
NN(q) = argmin_x dist(q, x) under Euclidean distance, extended to the k
nearest.  Distances here are plain float64 sums ``((q - x)**2).sum()``
(numpy's own summation order), independent of the engine's canonical key, and
ties are broken by ascending id.
"""
from __future__ import annotations

import numpy as np


def knn(base: np.ndarray, queries: np.ndarray, k: int, chunk: int = 4096):
    """Exact kNN by brute force; returns (ids (Q, k) int64, sq. dists (Q, k) f64)."""
    base64 = np.asarray(base, dtype=np.float64)
    qs = np.asarray(queries, dtype=np.float64).reshape(-1, base64.shape[1])
    ids = np.zeros((qs.shape[0], k), dtype=np.int64)
    dd = np.zeros((qs.shape[0], k), dtype=np.float64)
    for qi in range(qs.shape[0]):
        best_d = np.empty(0)
        best_i = np.empty(0, dtype=np.int64)
        for s in range(0, base64.shape[0], chunk):
            diff = base64[s:s + chunk] - qs[qi][None, :]
            d = (diff * diff).sum(axis=1)
            cat_d = np.concatenate([best_d, d])
            cat_i = np.concatenate([best_i, np.arange(s, s + d.size)])
            o = np.lexsort((cat_i, cat_d))[:k]
            best_d, best_i = cat_d[o], cat_i[o]
        ids[qi, :best_i.size] = best_i
        dd[qi, :best_d.size] = best_d
    return ids, dd


def recall_at_k(found: np.ndarray, truth: np.ndarray) -> float:
    """Mean fraction of the true k neighbours present in the returned k."""
    k = truth.shape[1]
    hits = 0
    for f, t in zip(found, truth):
        hits += len(set(int(a) for a in f if a >= 0) & set(int(b) for b in t))
    return hits / float(truth.shape[0] * k)
