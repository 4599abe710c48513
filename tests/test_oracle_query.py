"""Pins of the oracle query engine against the paper, special cases and brute force (CPU)."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import brute, build, query

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _traversal_with_priority_queue(d1, d2, sizes, budget, k_size, phi):
    """Algorithm 1's own traversal, restated independently of the oracle: a
    priority queue keyed (cost, i, j) seeded with the corner cell; popping
    (i, j) pushes its right neighbour (i, j + 1) and, from column 0, the next
    row's first cell (i + 1, 0); every pop is one rank; stop once the ids
    gathered reach the budget."""
    import heapq
    kh = d1.size
    o1, o2 = np.argsort(d1, kind="stable"), np.argsort(d2, kind="stable")
    d1s, d2s = d1[o1], d2[o2]
    heap = [(d1s[0] + d2s[0], 0, 0)]
    out, total, rank = [], 0, 0
    while total < budget and heap:
        _, i, j = heapq.heappop(heap)
        rank += 1
        cell = int(o1[i]) * kh + int(o2[j])
        out.append((cell, 2 if (phi == 1 and rank <= k_size) else 1))
        total += int(sizes[cell])
        if j + 1 < kh:
            heapq.heappush(heap, (d1s[i] + d2s[j + 1], i, j + 1))
        if j == 0 and i + 1 < kh:
            heapq.heappush(heap, (d1s[i + 1] + d2s[0], i + 1, 0))
    return out


@pytest.mark.parametrize("seed", range(12))
def test_multi_sequence_equals_priority_queue_traversal(seed):
    rng = np.random.default_rng(seed)
    kh = int(rng.integers(1, 9))
    d1 = np.round(rng.random(kh) * 4, 1)      # coarse values -> ties
    d2 = np.round(rng.random(kh) * 4, 1)
    sizes = rng.integers(0, 5, kh * kh)
    if sizes.sum() == 0:
        sizes[0] = 1
    budget = int(rng.integers(1, sizes.sum() + 1))
    k_size = int(rng.integers(1, 6))
    for phi in (0, 1):
        got = query.multi_sequence(d1, d2, sizes, budget, k_size, phi)
        assert got == _traversal_with_priority_queue(d1, d2, sizes, budget, k_size, phi)


def test_multi_sequence_budget_and_empty_cells():
    """Whole cells are added and the walk stops after the cell that reaches the
    budget; empty cells still take a rank (and so a weight-2 slot)."""
    d1 = np.array([0.0, 1.0])
    d2 = np.array([0.0, 10.0])
    sizes = np.array([0, 0, 3, 5])            # cells (0,0), (0,1), (1,0), (1,1)
    # order: (0,0) cost 0 [empty], (1,0) cost 1 [3 ids], (0,1) cost 10 [empty], (1,1) 11 [5]
    assert query.multi_sequence(d1, d2, sizes, 1, 1, 1) == [(0, 2), (2, 1)]
    assert query.multi_sequence(d1, d2, sizes, 3, 2, 1) == [(0, 2), (2, 2)]
    assert query.multi_sequence(d1, d2, sizes, 4, 9, 0) == [(0, 1), (2, 1), (1, 1), (3, 1)]


def test_figure3_structure():
    with open(os.path.join(GOLD, "fig3_grid.json")) as f:
        fx = json.load(f)
    kh = fx["k_half"]
    d = np.array(fx["half_distances"], dtype=np.float64)
    sizes = np.ones(kh * kh, dtype=np.int64)
    got = query.multi_sequence(d, d, sizes, fx["activated_ranks"], fx["k_size"], 1)
    assert len(got) == 13
    assert [w for _, w in got] == [2] * 6 + [1] * 7
    cells = [(c // kh, c % kh) for c, _ in got]
    assert set(cells[:6]) == {(i, j) for i in range(kh) for j in range(kh) if i + j <= 2}
    assert set(cells) == {(i, j) for i in range(kh) for j in range(kh) if i + j <= 3} | {(0, 4), (1, 3), (2, 2)}
    guaranteed = query.multi_sequence(d, d, sizes, 13, 6, 0)
    assert [w for _, w in guaranteed] == [1] * 13


def _tiny_index(seed=0, n=600, d=64, m=4, kh=4, rotate=None):
    w = synth.WORKLOADS["d128"].scaled(n=n, d=d, m=m, k_half=kh, seed_data=100 + seed)
    x = synth.rows(w, w.seed_data, 0, n)
    idx = build.build_index_for(w, x, force_rotation=rotate)
    qs = synth.rows(w, 900 + seed, 0, 12)
    return idx, qs, x


def test_collision_scores_equal_direct_counting():
    idx, qs, _ = _tiny_index(1)
    for qi in range(4):
        for mode in (0, 1):
            _, _, tr = query.search_one(idx, qs[qi], 5, mode=mode, alpha=0.1, tau=2, trace=True)
            direct = np.zeros(idx["n"], dtype=np.int64)
            for sub, cells in enumerate(tr["activated"]):
                wmap = dict(cells)
                for x in range(idx["n"]):
                    direct[x] += wmap.get(int(idx["assign"][sub, x]), 0)
            assert np.array_equal(direct, tr["scores"])


def test_threshold_and_fallback():
    v = np.array([0, 1, 1, 2, 3, 0, 2])
    c, s = query.select_candidates(v, 3, 1)
    assert c.tolist() == [4] and s == 3
    c, s = query.select_candidates(v, 3, 3)
    assert c.tolist() == [3, 4, 6] and s == 2
    c, s = query.select_candidates(v, 3, 6)
    assert c.tolist() == [1, 2, 3, 4, 6] and s == 1
    c, s = query.select_candidates(v, 0, 7)
    assert c.tolist() == list(range(7)) and s == 0
    c, s = query.select_candidates(np.zeros(5, dtype=np.int64), 2, 3)
    assert c.size == 0


def test_hamming_against_sign_comparison():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((30, 128)).astype(np.float32)
    q = rng.standard_normal(128).astype(np.float32)
    codes = build.sign_codes(x)
    got = query.hamming(build.sign_codes(q[None])[0], codes)
    ref = ((x > 0) != (q[None] > 0)).sum(axis=1)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("d", [64, 192, 512])
def test_canonical_sqdist_exact_bound(d):
    """The distance key is within the float64 bound of a D-term sum of
    rounded squares (each term rounded once, then at most D - 1 additions)
    of the exact rational squared distance."""
    rng = np.random.default_rng(10 + d)
    q = rng.standard_normal(d).astype(np.float32)
    x = rng.standard_normal((5, d)).astype(np.float32)
    got = query.canonical_sqdist(q, x)
    for i in range(5):
        ex = sum((Fraction(float(q[t])) - Fraction(float(x[i, t]))) ** 2 for t in range(d))
        assert abs(Fraction(got[i]) - ex) <= Fraction(d + 1) * Fraction(2.0 ** -53) * ex
    assert np.allclose(got, ((q[None].astype(np.float64) - x) ** 2).sum(1), rtol=1e-14)


@pytest.mark.parametrize("d", [8, 512, 4096])
def test_canonical_sqdist_sums_in_ascending_dimension_order(d):
    """The key is a left-to-right float64 sum over dimensions 0 .. D-1.  One
    squared term of 1 and D - 1 terms of 2^-54 (a quarter of the unit in the
    last place of 1): added after the 1 each small term rounds away, so the
    key is exactly 1; added before it they sum exactly to (D-1) 2^-54, and the
    final addition rounds 1 + (D-1) 2^-54 to the nearest double.  Any other
    order (pairwise, reversed, lane-strided) gives another value."""
    q = np.zeros(d, dtype=np.float32)
    tiny = np.float32(2.0 ** -27)               # tiny^2 = 2^-54 exactly
    big_first = np.full(d, tiny, dtype=np.float32)
    big_first[0] = 1.0
    big_last = np.full(d, tiny, dtype=np.float32)
    big_last[-1] = 1.0
    got = query.canonical_sqdist(q, np.stack([big_first, big_last]))
    assert got[0] == 1.0
    exact_last = Fraction(1) + Fraction(d - 1, 2 ** 54)
    ulp = Fraction(1, 2 ** 52)
    nearest = round(exact_last / ulp) * ulp    # Python rounds halves to even
    assert Fraction(got[1]) == nearest
    assert got[1] != 1.0


def test_hamming_order_breaks_ties_by_id():
    """Stage 2 orders by Hamming distance; equal distances keep ascending id."""
    d = 64
    codes = np.zeros((10, 1), dtype=np.uint64)
    pops = {1: 1, 2: 1, 5: 2, 7: 0, 9: 2}       # id -> bits set (query code is 0)
    for i, c in pops.items():
        codes[i, 0] = np.uint64((1 << c) - 1)
    idx = {"codes": codes, "d": d}
    qp = -np.ones(d, dtype=np.float32)          # every sign bit 0
    order, hd = query.hamming_order(idx, qp, np.array([1, 2, 5, 7, 9]))
    assert order.tolist() == [7, 1, 2, 5, 9]
    assert hd.tolist() == [0, 1, 1, 2, 2]


def test_query_equal_to_a_point_ranks_its_own_cell_first():
    """A query equal to a stored point is nearest to that point's own
    half-centroids (the build assigns with the same half distances and the
    same lowest-index tie rule), so in every subspace the point's cell is the
    first one the traversal activates: this pins the split of q' into
    subspaces and halves against the build's."""
    idx, _, x = _tiny_index(6, rotate=False)
    for p in (0, 17, 311, idx["n"] - 1):
        _, _, tr = query.search_one(idx, x[p], 5, mode=1, alpha=0.02, tau=1, trace=True)
        for sub in range(idx["m"]):
            assert tr["activated"][sub][0][0] == int(idx["assign"][sub, p])
    ridx, _, _ = _tiny_index(7, rotate=True)
    for p in (3, 200):
        hd = query.subspace_half_distances(ridx, ridx["base"][p])
        kh = ridx["k_half"]
        for sub in range(ridx["m"]):
            cell = int(np.argmin(hd[sub, 0])) * kh + int(np.argmin(hd[sub, 1]))
            assert cell == int(ridx["assign"][sub, p])


def test_guaranteed_alpha_one_is_exact_knn():
    """alpha = 1 activates every cell, so V == M everywhere and C = all points:
    Guaranteed Mode must return the exact k nearest neighbours."""
    idx, qs, x = _tiny_index(2)
    gt_i, gt_d = brute.knn(idx["base"], qs, 7)
    ids, dists, tr = query.search(idx, qs, 7, mode=0, alpha=1.0, tau=idx["m"], trace=True)
    assert all(np.all(t["scores"] == idx["m"]) for t in tr)
    assert np.array_equal(ids, gt_i)
    assert np.allclose(dists, gt_d, rtol=1e-6)


def test_guaranteed_alpha_one_rotated_is_exact_knn():
    idx, qs, x = _tiny_index(3, rotate=True)
    assert idx["rotation"] is not None
    qrot = build.rotate_rows(qs, idx["rotation"])
    gt_i, _ = brute.knn(idx["base"], qrot, 5)
    ids, _, _ = query.search(idx, qs, 5, mode=0, alpha=1.0, tau=1)
    assert np.array_equal(ids, gt_i)


def test_optimized_without_patience_is_topk_of_candidates():
    idx, qs, _ = _tiny_index(4)
    for qi in range(6):
        ids, _, tr = query.search_one(idx, qs[qi], 5, mode=1, alpha=0.08, tau=3,
                                      patience_factor=10 ** 9, trace=True)
        cand = tr["candidates"]
        d = ((idx["base"][cand].astype(np.float64) - tr["q_rot"][None]) ** 2).sum(1)
        ref = cand[np.lexsort((cand, d))[:5]]
        assert ids[:ref.size].tolist() == ref.tolist()


def _patience_reference(keys, k, p):
    """Independent statement of the patience rule: candidate t updates iff
    t < k or its key is below the k-th smallest key among the first t."""
    upd = []
    for t in range(len(keys)):
        if t < k:
            upd.append(True)
        else:
            kth = sorted(keys[:t])[k - 1]
            upd.append(keys[t] < kth)
    run = 0
    for t, u in enumerate(upd):
        run = 0 if u else run + 1
        if run >= p:
            return t + 1, max([i + 1 for i in range(t + 1) if upd[i]], default=0)
    return None, max([i + 1 for i, u in enumerate(upd) if u], default=0)


@pytest.mark.parametrize("seed", range(8))
def test_patience_walk_against_reference(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 120))
    dist = np.round(rng.random(n) * 50)          # ties on distance
    ids = rng.permutation(1000)[:n]
    k = int(rng.integers(1, 6))
    p = int(rng.integers(1, 30))
    keys = list(zip(dist.tolist(), ids.tolist()))
    stop_ref, last_ref = _patience_reference(keys, k, p)
    examined, last, stop = query.patience_walk(ids, dist, k, p)
    assert stop == stop_ref
    assert examined == (stop_ref if stop_ref is not None else n)
    assert last == last_ref or stop_ref is None


def test_learned_limit_truncates_walk():
    idx, qs, _ = _tiny_index(5)
    full_i, _, tr = query.search_one(idx, qs[0], 5, mode=1, alpha=0.1, tau=2, trace=True)
    lim = max(5, tr["last_update"])
    lim_i, _, tr2 = query.search_one(idx, qs[0], 5, mode=1, alpha=0.1, tau=2, limit=lim, trace=True)
    assert tr2["examined"] == min(lim, tr["examined"])
    assert np.array_equal(full_i, lim_i)       # the prefix up to L* reproduces the result


def test_cev_sample_size():
    """Section 4.1 samples 10% of the rows, at most 100,000 (at least two,
    so that a covariance exists)."""
    assert build.cev_sample_size(15) == 2
    assert build.cev_sample_size(1_000) == 100
    assert build.cev_sample_size(999_999) == 99_999
    assert build.cev_sample_size(1_000_000) == 100_000
    assert build.cev_sample_size(2_000_000) == 100_000


def test_budget_rounding():
    assert query.budget_for(0.01, 1000) == 10
    assert query.budget_for(0.0101, 1000) == 11
    assert query.budget_for(1e-9, 1000) == 1
    assert query.budget_for(1.0, 77) == 77


def test_key_on_rows_where_order_matters():
    """Closed forms of the defined key on rows built so that summation order
    changes the result (1 absorbs 2^-54; 1 + 2^-24 is a float32 midpoint)."""
    from parity_util import key_stress_rows
    rows = key_stress_rows(128)
    got = query.canonical_sqdist(np.zeros(128, dtype=np.float32), np.stack([rows["A"], rows["B"], rows["C"]]))
    assert got[0] == 1.0
    assert got[1] == 1.0 + 2.0 ** -52
    assert got[2] == 1.0 + 2.0 ** -24
    assert np.float32(got[2]) == np.float32(1.0)
    # The same terms added pairwise (any order that first combines the small
    # terms) give different values: the rows do separate the orders.
    terms = np.stack([rows["A"], rows["C"]]).astype(np.float64) ** 2
    pair = terms.copy()
    while pair.shape[1] > 1:
        pair = pair[:, 0::2] + pair[:, 1::2]
    assert pair[0, 0] > got[1] > got[0]
    assert np.float32(pair[1, 0]) != np.float32(got[2])


def test_walk_without_hamming_order_is_the_id_order_walk():
    """The Section 6.4 ablation without Hamming re-ranking walks C in ascending
    id order: its trace equals the patience walk over C as produced."""
    import synth
    from oracle import build as obuild
    w = synth.WORKLOADS["d128"].scaled(n=1500, n_query=3)
    p = synth.mixture_params(w)
    x = synth.rows(w, w.seed_data, 0, w.n, p)
    q = synth.rows(w, w.seed_query, 0, w.n_query, p)
    idx = obuild.build_index_for(w, x)
    _, _, tr = query.search(idx, q, 5, mode=1, alpha=0.05, tau=3, patience_factor=2, trace=True, hamming=False)
    for t in tr:
        assert np.array_equal(t["order"], t["candidates"])
        assert np.all(np.diff(t["order"]) > 0)
        d = query.canonical_sqdist(t["q_rot"], idx["base"][t["candidates"]])
        assert query.patience_walk(t["candidates"], d, 5, 10)[0] == t["examined"]


# ---------------------------------------------------------------------------
# ADSampling (Eq. (2), Section 4.3.2 Stage 3)
# ---------------------------------------------------------------------------
def test_ads_factors_match_eq2_in_high_precision():
    """(t/D)(1 + eps0/sqrt(t))^2 against 50-digit decimal arithmetic on the
    same float64 eps0: within a relative 8 u (u = 2^-53; five roundings and
    a square root, each at most u/2, the square doubling b's error)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    for d in (64, 128, 960, 4096):
        f = query.ads_factors(d)
        assert f.size == (d - 1) // 32
        for j, v in enumerate(f):
            t = 32 * (j + 1)
            exact = (Decimal(t) / Decimal(d)) * (1 + Decimal(query.ADS_EPS0) / Decimal(t).sqrt()) ** 2
            assert abs(Decimal(float(v)) - exact) <= exact * Decimal(8) * Decimal(2.0 ** -53)
        # the margin shrinks with t: (1 + eps0/sqrt(t))^2 decreases towards 1
        ratio = f * d / np.arange(32, d, 32)
        assert np.all(np.diff(ratio) < 0) and np.all(ratio > 1)


def test_prefixes_are_the_key_of_the_leading_dimensions():
    """d_t^2 is the key's own running sum: the key of the first t dimensions."""
    rng = np.random.default_rng(3)
    q = rng.standard_normal(160).astype(np.float32)
    x = rng.standard_normal((7, 160)).astype(np.float32)
    key, pre = query.sqdist_with_prefixes(q, x)
    assert np.array_equal(key, query.canonical_sqdist(q, x))
    assert pre.shape == (7, 4)
    for j in range(4):
        t = 32 * (j + 1)
        assert np.array_equal(pre[:, j], query.canonical_sqdist(q[:t], x[:, :t]))


def test_ads_walk_without_pruning_is_the_exact_walk():
    rng = np.random.default_rng(5)
    n, d, k = 300, 96, 5
    ids = rng.permutation(10_000)[:n]
    keys = rng.random(n) * 100
    pre = rng.random((n, 2)) * 100
    for patience in (3, 20, 10_000):
        top, ex, last, stop, pruned, dims = query.ads_walk(ids, keys, pre, np.full(2, np.inf), k, patience)
        assert (ex, last, stop) == query.patience_walk(ids, keys, k, patience)
        oi, od = query.topk_by_key(ids[:ex], keys[:ex], k)
        assert [i for _, i in top] == list(oi) and pruned == 0 and dims == ex * d


def test_ads_walk_prunes_by_eq2_on_constructed_rows():
    """D = 64, k = 1, one test at t = 32 with factor (32/64)(1 + 2.1/sqrt 32)^2
    ~ 0.94: after a first row at key 64 (r_k^2 = 64, threshold ~ 60.1), a row
    with d_32^2 = 128 is pruned at t = 32, a row with d_32^2 = 8 and key 296
    is verified and rejected, a row at key 51.84 updates."""
    d = 64
    q = np.zeros(d, dtype=np.float32)
    rows = np.zeros((4, d), dtype=np.float32)
    rows[0] = 1.0
    rows[1, :32] = 2.0
    rows[2, :32] = 0.5
    rows[2, 32:] = 3.0
    rows[3] = 0.9
    key, pre = query.sqdist_with_prefixes(q, rows)
    f = query.ads_factors(d)
    assert f.size == 1 and 60.0 < 64 * f[0] < 60.2
    ids = np.array([10, 11, 12, 13])
    top, ex, last, stop, pruned, dims = query.ads_walk(ids, key, pre, f, 1, 100)
    assert pruned == 1 and dims == 64 + 32 + 64 + 64
    assert ex == 4 and last == 4 and stop is None
    assert top == [(float(key[3]), 13)]
    # the same rows with the top-k not yet full: nothing is pruned
    top, ex, last, stop, pruned, dims = query.ads_walk(ids, key, pre, f, 2, 100)
    assert pruned == 0


def test_ads_pruning_is_monotone_in_the_kth_key():
    """A candidate pruned under r_k^2 is pruned under any smaller r_k^2."""
    rng = np.random.default_rng(8)
    f = query.ads_factors(4096)
    for _ in range(200):
        p = np.cumsum(rng.random(f.size) * 3)
        r = rng.random() * p[-1]
        if np.any(p > r * f):
            assert np.any(p > (r * rng.random()) * f)


def test_ads_keeps_nearly_all_exact_results_on_rotated_data():
    """The statistical guarantee of ADSampling after a random rotation: the
    walk with Eq. (2) returns almost the same top-k as the exact walk."""
    import synth
    from oracle import build as obuild
    w = synth.WORKLOADS["d128"].scaled(n=3000, n_query=20)
    p = synth.mixture_params(w)
    x = synth.rows(w, w.seed_data, 0, w.n, p)
    q = synth.rows(w, w.seed_query, 0, w.n_query, p)
    idx = obuild.build_index_for(w, x, force_rotation=True)
    kw = dict(mode=1, alpha=0.05, tau=3, patience_factor=40)
    ei, _, _ = query.search(idx, q, 10, **kw)
    ai, _, tr = query.search(idx, q, 10, ads=True, trace=True, **kw)
    same = np.mean([len(set(a) & set(e)) / 10.0 for a, e in zip(ai, ei)])
    assert same >= 0.97
    assert sum(t["ads_pruned"] for t in tr) > 0
    read = sum(t["ads_dims"] for t in tr) / float(sum(t["examined"] for t in tr) * w.d)
    assert read < 0.9
