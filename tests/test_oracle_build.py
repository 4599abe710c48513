"""Pins of the oracle index build against the paper, closed forms and brute force (CPU)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import build

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_csr_worked_example():
    """Section 4.2: {2,4,7,9,15,22} in C_i and {3,8,12,20} in C_j lay out as the golden order."""
    with open(os.path.join(GOLD, "csr_example.json")) as f:
        ex = json.load(f)
    n = 23
    ci, cj, other = 5, 2, 7            # j < i, other points in a later cell
    cells = np.full(n, other)
    cells[ex["cell_i_points"]] = ci
    cells[ex["cell_j_points"]] = cj
    off, ids = build.build_csr(cells, 9)
    lay = ids[off[cj]:off[ci + 1]].tolist()
    assert lay == ex["layout"]
    assert off.size == 9 + 1 and off[0] == 0 and off[-1] == n
    assert ids[off[cj]:off[cj + 1]].tolist() == ex["cell_j_points"]


def test_csr_invariants_random():
    rng = np.random.default_rng(0)
    cells = rng.integers(0, 37, size=5000)
    cells[cells == 11] = 12            # an empty cell
    off, ids = build.build_csr(cells, 40)
    assert off[0] == 0 and off[-1] == 5000 and np.all(np.diff(off) >= 0)
    assert np.array_equal(np.sort(ids), np.arange(5000))
    for c in range(40):
        seg = ids[off[c]:off[c + 1]]
        assert np.all(cells[seg] == c)
        assert np.all(np.diff(seg) > 0)
    assert off[12] == off[11]


def test_cev_closed_form_diagonal():
    """X = Z diag(sigma): the CEV is the share of the top floor(0.2 D) sigma^2."""
    rng = np.random.default_rng(1)
    d = 50
    sig = np.linspace(3.0, 0.2, d)
    z = rng.standard_normal((200_000, d))
    cev = build.cumulative_explained_variance(z * sig)
    top = int(math.floor(0.2 * d))
    expect = (sig[:top] ** 2).sum() / (sig ** 2).sum()
    assert abs(cev - expect) < 5e-3


def test_cev_isotropic_and_low_rank_decisions():
    rng = np.random.default_rng(2)
    iso = rng.standard_normal((20_000, 100))
    c_iso = build.cumulative_explained_variance(iso)
    assert 0.2 < c_iso < 0.3 and not build.needs_rotation(c_iso)
    low = rng.standard_normal((20_000, 8)) @ rng.standard_normal((8, 100)) + 0.01 * rng.standard_normal((20_000, 100))
    c_low = build.cumulative_explained_variance(low)
    assert c_low > 0.99 and build.needs_rotation(c_low)
    assert not build.needs_rotation(0.85) and build.needs_rotation(0.8500001)


def test_rotation_orthogonal_and_preserves_distance():
    g = synth.gaussian_matrix(9, 64)
    r = build.rotation_from_gaussian(g).astype(np.float64)
    assert np.abs(r.T @ r - np.eye(64)).max() < 1e-6
    q64, _ = np.linalg.qr(g)
    assert np.abs(q64.T @ q64 - np.eye(64)).max() < 1e-12
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, 64)).astype(np.float32)
    rot = build.rotate_rows(np.stack([x, y]), r.astype(np.float32)).astype(np.float64)
    d0 = np.linalg.norm(x.astype(np.float64) - y)
    assert abs(np.linalg.norm(rot[0] - rot[1]) - d0) / d0 < 1e-6


def test_rotation_is_row_times_matrix():
    """q' = q R (row vector on the left), not R q: a plane rotation pins the side."""
    c, s = np.float32(0.6), np.float32(0.8)
    r = np.array([[c, s], [-s, c]], dtype=np.float32)
    q = np.array([[1.0, 0.0]], dtype=np.float32)
    assert build.rotate_rows(q, r).tolist() == [[0.6000000238418579, 0.800000011920929]]


def test_rotate_rows_against_exact_sum():
    """Each output is within the float64 recursive-summation bound of the exact value,
    and within one float32 ulp of the correctly rounded result."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 40)).astype(np.float32)
    r = rng.standard_normal((40, 5)).astype(np.float32)
    got = build.rotate_rows(x, r)
    for a in range(3):
        for b in range(5):
            exact = sum(Fraction(float(x[a, i])) * Fraction(float(r[i, b])) for i in range(40))
            mag = sum(abs(Fraction(float(x[a, i])) * Fraction(float(r[i, b]))) for i in range(40))
            ref32 = np.float32(float(exact))
            assert abs(float(got[a, b]) - float(ref32)) <= float(np.spacing(np.abs(ref32)))
            assert abs(float(got[a, b]) - float(exact)) <= float(np.spacing(np.abs(ref32))) + 40 * 2.0 ** -53 * float(mag)


def test_half_distances_exact_bound():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((4, 16)).astype(np.float32)
    c = rng.standard_normal((6, 16)).astype(np.float32)
    got = build.half_distances(a, c)
    for i in range(4):
        for j in range(6):
            ex = sum((Fraction(float(a[i, t])) - Fraction(float(c[j, t]))) ** 2 for t in range(16))
            assert abs(Fraction(got[i, j]) - ex) <= Fraction(2 * 16) * Fraction(2.0 ** -53) * ex


def test_add_at_is_sequential():
    """k-means sums rely on numpy applying np.add.at in index order."""
    rng = np.random.default_rng(6)
    vals = (rng.standard_normal(20_000) * 10.0 ** rng.integers(-8, 8, 20_000)).astype(np.float64)
    lab = rng.integers(0, 5, 20_000)
    got = np.zeros(5)
    np.add.at(got, lab, vals)
    ref = [0.0] * 5
    for v, l in zip(vals.tolist(), lab.tolist()):
        ref[l] = ref[l] + v
    assert got.tolist() == ref


def test_kmeans_assignment_is_argmin_and_inertia_decreases():
    rng = np.random.default_rng(7)
    a = (rng.standard_normal((3000, 8)) + rng.integers(0, 4, (3000, 1)) * 3.0).astype(np.float32)
    init = np.arange(6)
    inert = []
    for it in (1, 2, 5, 10, 25):
        cen = build.kmeans(a, init, iters=it)
        lab = build.nearest_centroid(a, cen)
        d = ((a[:, None, :].astype(np.float64) - cen[None].astype(np.float64)) ** 2).sum(-1)
        best = d.min(axis=1)
        assert np.all(d[np.arange(3000), lab] <= best * (1 + 1e-12))
        inert.append(best.sum())
    assert all(inert[i + 1] <= inert[i] * (1 + 1e-6) for i in range(len(inert) - 1))


def test_sign_codes_match_signs():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((20, 192)).astype(np.float32)
    x[0, 5] = 0.0
    codes = build.sign_codes(x)
    for i in range(20):
        for dim in range(192):
            bit = (int(codes[i, dim // 64]) >> (dim % 64)) & 1
            assert bit == (1 if x[i, dim] > 0 else 0)


def test_build_index_structure_d128_small():
    w = synth.WORKLOADS["d128"].scaled(n=3000, d=64, m=4, k_half=6)
    x = synth.rows(w, w.seed_data, 0, w.n)
    idx = build.build_index_for(w, x)
    assert idx["rotation"] is None
    h = w.d // (2 * w.m)
    for sub in range(w.m):
        off, ids = idx["offsets"][sub], idx["ids"][sub]
        assert off[0] == 0 and off[-1] == w.n
        assert np.array_equal(np.sort(ids), np.arange(w.n))
        # stored cell = pair of brute-force nearest half-centroids
        for s, factor in ((0, w.k_half), (1, 1)):
            part = x[:, sub * 2 * h + s * h: sub * 2 * h + (s + 1) * h].astype(np.float64)
            cen = idx["centroids"][sub, s].astype(np.float64)
            dd = ((part[:, None, :] - cen[None]) ** 2).sum(-1)
            lab = (idx["assign"][sub] // w.k_half) if s == 0 else (idx["assign"][sub] % w.k_half)
            assert np.all(dd[np.arange(w.n), lab] <= dd.min(axis=1) * (1 + 1e-12))


def test_build_index_rotation_fires_on_correlated_data():
    w = synth.WORKLOADS["d4096"].scaled(n=2000, d=128, m=4, k_half=5, rank=8)
    x = synth.rows(w, w.seed_data, 0, w.n)
    idx = build.build_index_for(w, x)
    assert idx["cev"] > 0.85 and idx["rotation"] is not None
    assert np.array_equal(idx["base"], build.rotate_rows(x, idx["rotation"]))
