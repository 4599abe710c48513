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


def _first_cells_by_full_sort(d1, d2, sizes, budget, k_size, phi):
    """Brute force: sort all K^2 cells by (cost, i, j) and take the shortest
    prefix whose total size reaches the budget."""
    kh = d1.size
    o1, o2 = np.argsort(d1, kind="stable"), np.argsort(d2, kind="stable")
    cells = sorted(((d1[o1[i]] + d2[o2[j]], i, j) for i in range(kh) for j in range(kh)))
    out, total = [], 0
    for rank, (_, i, j) in enumerate(cells, start=1):
        cell = int(o1[i]) * kh + int(o2[j])
        out.append((cell, 2 if (phi == 1 and rank <= k_size) else 1))
        total += int(sizes[cell])
        if total >= budget:
            break
    return out


@pytest.mark.parametrize("seed", range(12))
def test_multi_sequence_equals_full_sort(seed):
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
        assert got == _first_cells_by_full_sort(d1, d2, sizes, budget, k_size, phi)


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
    """The distance key is within the float64 summation bound of the exact
    rational value (lane sums of at most 4 ceil(d/256) terms + a 6-level tree)."""
    rng = np.random.default_rng(10 + d)
    q = rng.standard_normal(d).astype(np.float32)
    x = rng.standard_normal((5, d)).astype(np.float32)
    got = query.canonical_sqdist(q, x)
    depth = 4 * ((d + 255) // 256) + 6 + 2
    for i in range(5):
        ex = sum((Fraction(float(q[t])) - Fraction(float(x[i, t]))) ** 2 for t in range(d))
        assert abs(Fraction(got[i]) - ex) <= Fraction(depth) * Fraction(2.0 ** -53) * ex
    assert np.allclose(got, ((q[None].astype(np.float64) - x) ** 2).sum(1), rtol=1e-14)


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


def test_budget_rounding():
    assert query.budget_for(0.01, 1000) == 10
    assert query.budget_for(0.0101, 1000) == 11
    assert query.budget_for(1e-9, 1000) == 1
    assert query.budget_for(1.0, 77) == 77
