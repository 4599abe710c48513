"""Pins of the shared synthetic-input generator (CPU)."""
import json
import os

import numpy as np

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox4x32_kat.json")) as f:
        kat = json.load(f)
    for case in kat["cases"]:
        c = [np.array([int(v, 16)], dtype=np.uint64) for v in case["ctr"]]
        k = [int(v, 16) for v in case["key"]]
        out = synth.philox4x32(*c, *k)
        assert [int(o[0]) for o in out] == [int(v, 16) for v in case["out"]]


def test_normals_moments_and_exactness():
    z = synth.normals(7, 1, np.arange(200_000, dtype=np.uint64))
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert z.min() >= -6.0 and z.max() <= 6.0
    # every value is an exact multiple of 2^-32
    scaled = (z + 6.0) * 2.0 ** 32
    assert np.all(scaled == np.round(scaled))


def test_rows_are_random_access():
    w = synth.WORKLOADS["d128"].scaled(n=300, d=64)
    p = synth.mixture_params(w)
    full = synth.rows(w, w.seed_data, 0, 300, p)
    part = synth.rows(w, w.seed_data, 123, 177, p)
    assert np.array_equal(full[123:177], part)
    wg = synth.WORKLOADS["d4096"].scaled(n=100, d=128)
    pg = synth.mixture_params(wg)
    assert np.array_equal(synth.rows(wg, 5, 0, 50, pg)[10:20], synth.rows(wg, 5, 10, 20, pg))


def test_sample_indices_distinct_sorted():
    s = synth.sample_indices(3, synth.TAG["cev_sample"], 1000, 100)
    assert s.size == 100 and np.unique(s).size == 100
    assert np.all(np.diff(s) > 0) and s.min() >= 0 and s.max() < 1000
    assert np.array_equal(synth.sample_indices(3, 8, 10, 50), np.arange(10))


def test_batch_sizes_cover_total():
    b = synth.batch_sizes(5005, 20_000)
    assert sum(b) == 20_000 and min(b) >= 1 and max(b) <= 4096


def test_center_scale_scales_the_centres_exactly():
    """The component centres of a global mixture are center_scale x the same
    normals: power-of-two scales give exact multiples, and the default (2)
    reproduces the draw every other workload was generated with."""
    import numpy as np
    import synth
    w = synth.WORKLOADS["d1024mix"].scaled(n=100, d=128, n_query=4)
    p_half = synth.mixture_params(w)
    p_two = synth.mixture_params(w.scaled(center_scale=2.0))
    assert w.center_scale == 0.5
    assert np.array_equal(p_half["nu"] * np.float32(4.0), p_two["nu"])
    assert np.array_equal(p_half["b"], p_two["b"])
    d4096 = synth.WORKLOADS["d4096"].scaled(n=100, d=128)
    assert d4096.center_scale == 2.0
    ref = (2.0 * synth.normals(d4096.seed_data, synth.TAG["center"],
                               np.arange(d4096.n_comp * d4096.rank))).astype(np.float32)
    assert np.array_equal(synth.mixture_params(d4096)["nu"].reshape(-1), ref)
