"""Theorem 1 (Section 5) pins: the Hoeffding bound against the exact binomial
tail, and an empirical check over rebuilt randomly rotated indexes (CPU)."""
import math

import numpy as np
import pytest

import synth
from oracle import brute, build, query, theory


def test_bound_below_exact_binomial_tail():
    for m in (4, 8, 16, 32, 64):
        for p in np.linspace(0.02, 0.98, 25):
            for tau in range(0, m + 1):
                lb = theory.recall_lower_bound(m, float(p), tau)
                ex = theory.binomial_tail_ge(m, float(p), tau)
                assert lb <= ex + 1e-12
                if m * p <= tau:
                    assert lb == 0.0


def test_bound_closed_form_values():
    assert theory.recall_lower_bound(32, 0.5, 8) == pytest.approx(1 - math.exp(-2 * 64 / 32))
    assert theory.binomial_tail_ge(4, 0.5, 2) == pytest.approx(11 / 16)


@pytest.mark.slow
def test_empirical_recall_bound_with_rotation():
    """Over rebuilds with independent rotations, the rate at which the true
    nearest neighbour reaches tau collisions is at least the bound evaluated
    at its measured per-subspace collision rate (minus sampling slack)."""
    w = synth.WORKLOADS["d4096"].scaled(n=1500, d=64, m=8, k_half=4, n_comp=10)
    x = synth.rows(w, w.seed_data, 0, w.n)
    qs = synth.rows(w, 777, 0, 10)
    gt, _ = brute.knn(x, qs, 1)
    tau, alpha, reps = 3, 0.05, 16
    hits = np.zeros((qs.shape[0], reps), dtype=bool)
    rate = np.zeros(qs.shape[0])
    for rep in range(reps):
        g = synth.gaussian_matrix(5000 + rep, w.d)
        idx = build.build_index_for(w, x, g=g, force_rotation=True)
        for qi in range(qs.shape[0]):
            _, _, tr = query.search_one(idx, qs[qi], 1, mode=0, alpha=alpha, tau=tau, trace=True)
            s = int(tr["scores"][gt[qi, 0]])
            hits[qi, rep] = s >= tau
            rate[qi] += s / (w.m * reps)
    for qi in range(qs.shape[0]):
        lb = theory.recall_lower_bound(w.m, rate[qi], tau)
        slack = 3.0 * math.sqrt(0.25 / reps)
        assert hits[qi].mean() >= lb - slack
