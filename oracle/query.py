"""Oracle query engine (test infrastructure only).

Executes CRISP's dual-mode query (Algorithm 1; Sections 4.3.1-4.3.2) one query
at a time, in the paper's order and notation:

  1. q' = q R when the index holds a rotation (Section 4.1: the rotation is
     kept in the index metadata so queries are mapped into the same space).
  2. For every subspace m: split q'^(m) into its left / right halves, compute
     Dist_1 and Dist_2 against the two half-codebooks, and take the cells the
     Multi-Sequence traversal activates: in ascending cost until the ids
     gathered reach the per-subspace budget, each cell one rank, weight 2 when
     the mode flag phi = 1 and rank <= k_size (else 1); add the weight to the
     score of every id in the cell's CSR posting list.
  3. Candidates C = {x : V[x] >= tau}, with the robustness fallback that keeps
     |C| >= k (Section 4.3.2, Stage 1).
  4. phi = 1: order C by Hamming distance of sign codes (Stage 2).
  5. Verify: phi = 0 computes the exact L2 distance of every candidate;
     phi = 1 walks the Hamming order and stops after P = patience_factor * k
     consecutive candidates that leave the top-k unchanged (Stage 3), each
     candidate verified by exact L2 (the paper's "Hamming re-ranking with
     exact L2" variant, Section 6.4) or, with ads=True, by ADSampling
     (Eq. (2): prune once a partial distance exceeds the scaled k-th key).
  6. Return the top-k.

Readings where the paper is silent (each is also listed in the design notes):

* Budget: budget = max(1, ceil(alpha * N)) ids per subspace; whole cells are
  added, so the last cell may overshoot it; empty cells still consume a rank.
* Order of cells: ascending (cost, i, j) where i, j are ranks in the sorted
  half-distance lists, each sorted by (distance, centroid index).
* tau is one integer threshold for both modes.
* Fallback: if fewer than k points reach tau, use the largest s <= tau with at
  least k points scoring >= s; if even s = 1 has fewer than k, C = {V >= 1}
  and the output is padded with id -1 / distance +inf.
* Distance key: the squared L2 distance summed in float64 over the dimensions
  in ascending order (``canonical_sqdist``); the result order is ascending
  (key, id).  Returned distances are f32(key).
* Patience: a candidate "updates" the top-k iff the top-k holds fewer than k
  items or its key is below the current k-th key; the counter of consecutive
  non-updates resets on an update and the walk stops when it reaches P.
* Learned budget: the walk additionally stops after ``limit`` candidates.
* ADSampling: the test of Eq. (2) runs every 32 dimensions below D with
  eps_0 = 2.1; r_k^2 is the k-th key of the top-k at the moment the
  candidate is verified (none while the top-k holds fewer than k items, so
  nothing is pruned then); d_t^2 is the key's own float64 running sum after
  t dimensions, the threshold r_k^2 * (t/D)(1 + eps_0/sqrt(t))^2 a float64
  product with the factor formed as in ``ads_factors``.  A pruned candidate
  counts as a non-update; one that passes every test is verified exactly.
"""
from __future__ import annotations

import math

import numpy as np

from .build import half_distances, rotate_rows

def budget_for(alpha: float, n: int) -> int:
    """Per-subspace retrieval budget: max(1, ceil(alpha * N)), in float64."""
    return max(1, int(math.ceil(float(alpha) * float(n))))


def rotate_query(index: dict, q: np.ndarray) -> np.ndarray:
    """q' = q R if the index has a rotation, else q (float32)."""
    q = np.asarray(q, dtype=np.float32).reshape(-1, index["d"])
    if index["rotation"] is None:
        return q.copy()
    return rotate_rows(q, index["rotation"])


def subspace_half_distances(index: dict, qp: np.ndarray) -> np.ndarray:
    """Dist_1 / Dist_2 of one rotated query for every subspace: (M, 2, K) f64."""
    m, kh = index["m"], index["k_half"]
    h = index["d"] // (2 * m)
    out = np.zeros((m, 2, kh), dtype=np.float64)
    for sub in range(m):
        for s in range(2):
            lo = sub * 2 * h + s * h
            out[sub, s] = half_distances(qp[None, lo:lo + h], index["centroids"][sub, s])[0]
    return out


def multi_sequence(d1: np.ndarray, d2: np.ndarray, sizes: np.ndarray, budget: int,
                   k_size: int, phi: int):
    """Activated cells of one subspace and their weights (Section 4.3.1).

    d1, d2 -- half distances (K,) of the left / right half
    sizes  -- (K*K,) posting-list length of cell i_L * K + i_R
    Returns a list of (cell, weight) in visit order.

    The Multi-Sequence traversal visits the cells of the K x K grid in
    ascending cost d1s[i] + d2s[j] (i, j = ranks in each half's list sorted by
    (distance, centroid index)); ties are taken in (i, j) order.  It stops
    after the first cell at which the ids gathered reach the budget, so the
    activated set is the shortest prefix of that order whose posting sizes
    sum to at least the budget (empty cells still take a rank).  Written out
    here as that definition: every cell's cost, one sort, one prefix.  A
    cell's weight is 2 when phi = 1 and its 1-based rank is at most k_size,
    else 1.
    """
    kh = d1.shape[0]
    o1 = np.argsort(d1, kind="stable")        # ascending (distance, index)
    o2 = np.argsort(d2, kind="stable")
    cost = np.add.outer(d1[o1], d2[o2])       # cost[i, j] = d1s[i] + d2s[j]
    ii, jj = np.meshgrid(np.arange(kh), np.arange(kh), indexing="ij")
    visit = np.lexsort((jj.ravel(), ii.ravel(), cost.ravel()))
    cell = (o1[ii.ravel()[visit]] * kh + o2[jj.ravel()[visit]]).astype(np.int64)
    gathered = np.cumsum(np.asarray(sizes, dtype=np.int64)[cell])
    reached = np.flatnonzero(gathered >= budget)
    n_act = int(reached[0]) + 1 if reached.size else cell.size
    rank = np.arange(1, n_act + 1)
    weight = np.where((phi == 1) & (rank <= k_size), 2, 1)
    return [(int(c), int(w)) for c, w in zip(cell[:n_act], weight)]


def collision_scores(index: dict, activated: list) -> np.ndarray:
    """V[x] += w for every id of every activated cell (Eq. 1 / Algorithm 1)."""
    v = np.zeros(index["n"], dtype=np.int64)
    for sub, cells in enumerate(activated):
        off = index["offsets"][sub]
        ids = index["ids"][sub]
        for cell, w in cells:
            v[ids[off[cell]:off[cell + 1]]] += w
    return v


def select_candidates(v: np.ndarray, tau: int, k: int):
    """Threshold + fallback; returns (ascending candidate ids, effective tau)."""
    def count_ge(s):
        return int(np.count_nonzero(v >= s))
    s_eff = tau
    if count_ge(tau) < k:
        s_eff = 1
        for s in range(min(tau, int(v.max(initial=0))), 0, -1):
            if count_ge(s) >= k:
                s_eff = s
                break
    return np.flatnonzero(v >= s_eff).astype(np.int64), s_eff


def hamming(codes_q: np.ndarray, codes_x: np.ndarray) -> np.ndarray:
    """Popcount of XOR of packed sign codes."""
    x = np.bitwise_xor(codes_x, codes_q[None, :])
    return np.unpackbits(x.view(np.uint8), axis=1).sum(axis=1).astype(np.int64)


def hamming_order(index: dict, qp: np.ndarray, cand: np.ndarray):
    """Candidates sorted by (Hamming distance, id) (Section 4.3.2, Stage 2)."""
    from .build import sign_codes
    cq = sign_codes(qp[None, :])[0]
    hd = hamming(cq, index["codes"][cand])
    order = np.lexsort((cand, hd))
    return cand[order], hd[order]


def canonical_sqdist(qp: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Distance key of each row: the squared L2 distance summed in float64
    over the dimensions in ascending order (Section 4.3.2, Stage 3, exact L2).

        acc = 0;  for i = 0 .. D-1:  delta = f64(q'_i) - f64(x_i);  acc = acc + delta * delta

    one rounding per operation, no fused multiply-add.  Results are ordered
    by (key, id) and returned as f32(key).
    """
    q64 = np.asarray(qp, dtype=np.float32).astype(np.float64)
    x64 = np.asarray(rows, dtype=np.float32).astype(np.float64).reshape(-1, q64.shape[0])
    acc = np.zeros(x64.shape[0], dtype=np.float64)
    for i in range(q64.shape[0]):
        delta = q64[i] - x64[:, i]
        sq = delta * delta
        acc = acc + sq
    return acc


# ADSampling (Section 3, Eq. (2); Section 4.3.2, Stage 3): the test runs every
# ADS_STEP dimensions with the safety margin eps_0 = ADS_EPS0 (both the paper's
# settings).
ADS_EPS0 = 2.1
ADS_STEP = 32


def ads_factors(d: int) -> np.ndarray:
    """(t / D) (1 + eps_0 / sqrt(t))^2 of Eq. (2) for t = 32, 64, ... below D,
    in float64: b = 1 + eps_0 / sqrt(t), factor = (t / D) * (b * b)."""
    t = np.arange(ADS_STEP, d, ADS_STEP, dtype=np.float64)
    b = 1.0 + ADS_EPS0 / np.sqrt(t)
    return (t / float(d)) * (b * b)


def sqdist_with_prefixes(qp: np.ndarray, rows: np.ndarray):
    """The distance key of each row (as canonical_sqdist) together with the
    running sum after every ADS_STEP dimensions below D: prefixes[:, j] is
    the partial distance d_t^2 of Eq. (2) at t = ADS_STEP (j + 1), the same
    float64 accumulation stopped early."""
    q64 = np.asarray(qp, dtype=np.float32).astype(np.float64)
    d = q64.shape[0]
    x64 = np.asarray(rows, dtype=np.float32).astype(np.float64).reshape(-1, d)
    acc = np.zeros(x64.shape[0], dtype=np.float64)
    pre = np.zeros((x64.shape[0], max(0, (d - 1) // ADS_STEP)), dtype=np.float64)
    for i in range(d):
        delta = q64[i] - x64[:, i]
        sq = delta * delta
        acc = acc + sq
        if (i + 1) % ADS_STEP == 0 and i + 1 < d:
            pre[:, (i + 1) // ADS_STEP - 1] = acc
    return acc, pre


def ads_walk(ids: np.ndarray, keys: np.ndarray, prefixes: np.ndarray, factors: np.ndarray, k: int,
             patience: int, limit: int | None = None):
    """Optimized Mode verification with ADSampling and patience.

    Candidates are verified in order.  Once the top-k holds k items, with
    r_k^2 its current k-th key, a candidate is pruned at the first t with
    d_t^2 > r_k^2 * factor_t (Eq. (2); the product rounded in float64): it is
    not verified further and counts as a non-update.  A candidate that
    passes every test is verified exactly and updates the top-k iff the
    top-k holds fewer than k items or its (key, id) is below the k-th.  The
    walk stops after `patience` consecutive non-updates.

    Returns (top-k list of (key, id), examined prefix, last update L*, stop
    position or None, candidates pruned, dimensions read).
    """
    top = []
    run = 0
    last_update = 0
    stop = None
    pruned = 0
    dims = 0
    d_full = (prefixes.shape[1] + 1) * ADS_STEP if prefixes.ndim == 2 else 0
    n = ids.size if limit is None else min(ids.size, int(limit))
    pos = 0
    for pos in range(1, n + 1):
        key = (float(keys[pos - 1]), int(ids[pos - 1]))
        cut = None
        if len(top) == k:
            over = np.flatnonzero(prefixes[pos - 1] > top[-1][0] * factors)
            if over.size:
                cut = int(over[0])
        if cut is not None:
            pruned += 1
            dims += (cut + 1) * ADS_STEP
            run += 1
        else:
            dims += d_full
            if len(top) < k or key < top[-1]:
                top.append(key)
                top.sort()
                del top[k:]
                run = 0
                last_update = pos
            else:
                run += 1
        if run >= patience:
            stop = pos
            break
    return top, pos, last_update, stop, pruned, dims


def topk_by_key(ids: np.ndarray, dist: np.ndarray, k: int):
    """Top-k by ascending (key, id), padded with (-1, +inf)."""
    order = np.lexsort((ids, dist))[:k]
    out_i = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, np.inf, dtype=np.float32)
    out_i[:order.size] = ids[order]
    out_d[:order.size] = dist[order].astype(np.float32)
    return out_i, out_d


def patience_walk(ids: np.ndarray, dist: np.ndarray, k: int, patience: int,
                  limit: int | None = None):
    """Sequential verification with patience termination.

    Returns (examined prefix length, position of the last update L*, stop
    position L_stop if the patience rule fired else None).
    """
    top = []                      # sorted list of (d, id), at most k entries
    run = 0
    last_update = 0
    stop = None
    n = ids.size if limit is None else min(ids.size, int(limit))
    pos = 0
    for pos in range(1, n + 1):
        key = (float(dist[pos - 1]), int(ids[pos - 1]))
        if len(top) < k or key < top[-1]:
            top.append(key)
            top.sort()
            del top[k:]
            run = 0
            last_update = pos
        else:
            run += 1
        if run >= patience:
            stop = pos
            break
    return pos, last_update, stop


def search_one(index: dict, q: np.ndarray, k: int, *, mode: int, alpha: float,
               tau: int, patience_factor: int = 40, limit: int | None = None,
               trace: bool = False, hamming: bool = True, ads: bool = False):
    """One query through Algorithm 1.  Returns (ids[k], dists[k], trace).

    hamming=False is the ablation of Section 6.4 without Hamming re-ranking:
    Optimized Mode verifies the candidates in the order C is produced in,
    ascending id (the paper does not name the order; ids are the natural one).
    ads=True verifies with ADSampling (Optimized Mode; Algorithm 1's Verify
    with phi = 1) instead of exact L2 on every walked candidate.
    """
    n, m = index["n"], index["m"]
    budget = budget_for(alpha, n)
    qp = rotate_query(index, q)[0]
    hd = subspace_half_distances(index, qp)
    activated = []
    for sub in range(m):
        sizes = np.diff(index["offsets"][sub].astype(np.int64))
        activated.append(multi_sequence(hd[sub, 0], hd[sub, 1], sizes, budget, k, mode))
    v = collision_scores(index, activated)
    cand, tau_eff = select_candidates(v, tau, k)
    tr = {"q_rot": qp, "half_dist": hd, "activated": activated, "scores": v,
          "candidates": cand, "tau_eff": tau_eff}
    if mode == 0:
        dist = canonical_sqdist(qp, index["base"][cand])
        out_i, out_d = topk_by_key(cand, dist, k)
        tr.update(order=cand, examined=cand.size)
    else:
        if hamming:
            order, hdist = hamming_order(index, qp, cand)
        else:
            order, hdist = cand, None
        if ads:
            dist_all, pre = sqdist_with_prefixes(qp, index["base"][order])
            top, examined, last_upd, stop, pruned, dims = ads_walk(
                order, dist_all, pre, ads_factors(qp.shape[0]), k, patience_factor * k, limit)
            out_i = np.full(k, -1, dtype=np.int64)
            out_d = np.full(k, np.inf, dtype=np.float32)
            for j, (dk, ik) in enumerate(top):
                out_i[j], out_d[j] = ik, np.float32(dk)
            tr.update(ads_pruned=pruned, ads_dims=dims)
        else:
            dist_all = canonical_sqdist(qp, index["base"][order])
            examined, last_upd, stop = patience_walk(order, dist_all, k, patience_factor * k, limit)
            out_i, out_d = topk_by_key(order[:examined], dist_all[:examined], k)
        tr.update(order=order, hamming=hdist, examined=examined, last_update=last_upd,
                  stop=stop, dist_order=dist_all)
    return out_i, out_d, (tr if trace else None)


def search(index: dict, queries: np.ndarray, k: int, *, mode: int, alpha: float, tau: int,
           patience_factor: int = 40, limits=None, trace: bool = False, hamming: bool = True,
           ads: bool = False):
    """All queries; returns ids (Q, k) int64, dists (Q, k) f32 and traces."""
    queries = np.asarray(queries, dtype=np.float32).reshape(-1, index["d"])
    nq = queries.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    dists = np.full((nq, k), np.inf, dtype=np.float32)
    traces = []
    for qi in range(nq):
        # a per-query limit below 1 means "no limit" (the engine's convention)
        lim = None
        if limits is not None and int(limits[qi]) >= 1:
            lim = int(limits[qi])
        i, d, tr = search_one(index, queries[qi], k, mode=mode, alpha=alpha, tau=tau,
                              patience_factor=patience_factor, limit=lim, trace=trace, hamming=hamming,
                              ads=ads and mode == 1)
        ids[qi], dists[qi] = i, d
        traces.append(tr)
    return ids, dists, traces
