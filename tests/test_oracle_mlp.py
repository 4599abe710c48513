"""Pins of the learned-budget reference (CPU): analytic gradients against
central finite differences, Adam against its closed-form first step, bf16
rounding against bit-level cases, features against their definitions."""
import math

import numpy as np
import pytest

import synth
from oracle import build, mlp, query


def _params(f, seed=3):
    p = mlp.init_params(f, seed)
    rng = np.random.default_rng(seed)
    p["b1"] = rng.standard_normal(mlp.HIDDEN).astype(np.float32) * 0.1
    p["b2"] = np.array([0.3], np.float32)
    return p


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    f = 11
    x = rng.standard_normal((17, f))
    t = rng.standard_normal(17)
    p = {k: v.astype(np.float64) for k, v in _params(f).items()}
    g = mlp.backward(p, x, t)
    h = 1e-6
    for key in ("w1", "b1", "w2", "b2"):
        flat = p[key].reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(p, x, t)
            flat[idx] = old - h
            lm = mlp.loss(p, x, t)
            flat[idx] = old
            num = (lp - lm) / (2 * h)
            ana = g[key].reshape(-1)[idx]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana)), (key, idx, num, ana)


def test_adam_first_step_is_signed_learning_rate():
    """After one step from zero moments, Adam moves each weight by -lr*sign(g)
    (up to eps)."""
    p = {"w": np.array([1.0, -2.0, 0.5], np.float32)}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    out = mlp.adam_step(p, g, {}, 1, lr=0.01, eps=1e-12)
    assert np.allclose(out["w"], p["w"] - 0.01 * np.sign(g["w"]), atol=1e-6)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.140625, 0.0], np.float32)
    got = mlp.to_bf16(vals)
    assert got.tolist() == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -3.140625, 0.0]


def test_features_follow_their_definitions():
    w = synth.WORKLOADS["d128"].scaled(n=2000, d=64, m=4, k_half=5)
    x = synth.rows(w, w.seed_data, 0, w.n)
    idx = build.build_index_for(w, x)
    q = synth.rows(w, 55, 0, 3)
    for qi in range(3):
        _, _, tr = query.search_one(idx, q[qi], 5, mode=1, alpha=0.05, tau=3, trace=True)
        f = mlp.features(idx, tr, 5)
        assert f.shape == (mlp.n_features(4),)
        assert f[0] == np.float32(math.log1p(tr["candidates"].size))
        v = tr["scores"]
        assert f[1] == np.float32(math.log1p(int((v == 8).sum())))
        # subspace 0 from a brute-force sort of all cells
        d1, d2 = tr["half_dist"][0]
        costs = sorted(d1[i] + d2[j] for i in range(5) for j in range(5))
        assert f[17] == np.float32((costs[1] - costs[0]) / costs[0])
        hm = tr["hamming"]
        assert f[17 + 3 * 4] == np.float32(hm[0] / 64)
        assert f[17 + 3 * 4 + 3] == np.float32(hm[min(8, hm.size) - 1] / 64)
        assert f[-1] == np.float32(hm[(hm.size + 1) // 2 - 1] / 64)


def test_limits_from_clamps_to_k_and_candidates():
    """L = clamp(ceil(exp(y + delta)), k, |C|); no candidates gives 0."""
    y = np.log(np.array([4.4, 0.01, 4.4, 1e6, 4.4, 2.2]))
    ncand = np.array([100, 100, 3, 50, 0, 100])
    got = mlp.limits_from(y, 0.0, 2, ncand)
    assert got.tolist() == [5, 2, 3, 50, 0, 3]
    got = mlp.limits_from(y, float(np.log(2.0)), 2, ncand)
    assert got.tolist() == [9, 2, 3, 50, 0, 5]
