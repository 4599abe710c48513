"""GPU twin of the input generator and GPU index build vs their CPU counterparts."""
import numpy as np
import pytest
import torch

import synth
from oracle import build as obuild
from parity_util import compare

pytestmark = pytest.mark.gpu


def test_synth_gpu_twin_matches_numpy():
    import synth.gpu as sg
    for name, kw in (("d128", dict(n=3000)), ("d4096", dict(n=500, d=512, rank=64)),
                     ("d960", dict(n=200, d=192, rank=32)), ("d1024mix", dict(n=500, d=256, rank=64))):
        w = synth.WORKLOADS[name].scaled(**kw)
        p = synth.mixture_params(w)
        pg = sg.mixture_params(w)
        for key in p:
            assert np.array_equal(pg[key].cpu().numpy().view(np.uint32), p[key].view(np.uint32)), (name, key)
        xg = sg.rows(w, w.seed_data, 0, w.n, pg).cpu().numpy()
        x = synth.rows(w, w.seed_data, 0, w.n, p)
        assert np.array_equal(xg.view(np.uint32), x.view(np.uint32)), name
        part = sg.rows(w, 77, 41, 97, pg).cpu().numpy()
        assert np.array_equal(part.view(np.uint32), synth.rows(w, 77, 41, 97, p).view(np.uint32))
    g = sg.gaussian_matrix(4003, 64)
    assert np.array_equal(g.view(np.uint64), synth.gaussian_matrix(4003, 64).view(np.uint64))


def test_synth_full_size_rows_sampled():
    """The N = 1M, D = 4096 data set on the device: sampled rows equal the CPU twin."""
    import synth.gpu as sg
    w = synth.WORKLOADS["d4096"]
    pg = sg.mixture_params(w)
    p = synth.mixture_params(w)
    x = sg.rows(w, w.seed_data, 0, w.n, pg)
    torch.cuda.synchronize()
    for r in (0, 1, 65535, 65536, 523_777, w.n - 1):
        ref = synth.rows(w, w.seed_data, r, r + 1, p)[0]
        assert np.array_equal(x[r].cpu().numpy().view(np.uint32), ref.view(np.uint32)), r
    del x


def _build_both(w, x, **kw):
    from paper_2603_05180_amd import engine
    n = x.shape[0]
    cev_rows = synth.sample_indices(w.seed_index, synth.TAG["cev_sample"], n, obuild.cev_sample_size(n))
    km_rows = synth.sample_indices(w.seed_index, synth.TAG["kmeans_sample"], n, min(n, obuild.KMEANS_SAMPLE_CAP))
    km_init = synth.permutation_prefix(w.seed_index, synth.TAG["kmeans_init"], np.arange(km_rows.size), w.k_half)
    ref = obuild.build_index(x, w.m, w.k_half, g=lambda: synth.gaussian_matrix(w.seed_index, w.d),
                             cev_rows=cev_rows, km_rows=km_rows, km_init=km_init, **kw)
    xd = torch.from_numpy(x).cuda()
    got = engine.build_index(xd, w.m, w.k_half, g=lambda: synth.gaussian_matrix(w.seed_index, w.d),
                             cev_rows=cev_rows, km_rows=km_rows, km_init=km_init, **kw)
    torch.cuda.synchronize()
    return ref, got


def _assert_same_index(ref, got):
    assert abs(ref["cev"] - got["cev"]) < 1e-9
    assert (ref["rotation"] is None) == (got["rotation"] is None)
    if ref["rotation"] is not None:
        assert np.array_equal(got["rotation"].cpu().numpy().view(np.uint32), ref["rotation"].view(np.uint32))
    assert np.array_equal(got["base"].cpu().numpy().view(np.uint32), ref["base"].view(np.uint32))
    assert np.array_equal(got["centroids"].cpu().numpy().view(np.uint32), ref["centroids"].view(np.uint32))
    assert np.array_equal(got["offsets"].cpu().numpy(), ref["offsets"])
    assert np.array_equal(got["ids"].cpu().numpy(), ref["ids"])
    assert np.array_equal(got["codes"].cpu().numpy().view(np.uint64), ref["codes"])


def test_gpu_build_equals_oracle_build_unrotated():
    w = synth.WORKLOADS["d128"]
    x = synth.rows(w, w.seed_data, 0, w.n)
    ref, got = _build_both(w, x)
    assert ref["rotation"] is None
    _assert_same_index(ref, got)


def test_gpu_build_equals_oracle_build_rotated():
    w = synth.WORKLOADS["d4096"].scaled(n=4000, d=256, m=8, k_half=6, rank=16)
    x = synth.rows(w, w.seed_data, 0, w.n)
    ref, got = _build_both(w, x)
    assert ref["rotation"] is not None
    _assert_same_index(ref, got)


def test_search_on_gpu_built_index_matches_oracle():
    """End to end: the GPU-built index, searched on the GPU, equals the oracle
    searching its own build (the two builds are identical)."""
    w = synth.WORKLOADS["d4096"].scaled(n=5000, d=256, m=8, k_half=8, rank=16, n_query=20)
    x = synth.rows(w, w.seed_data, 0, w.n)
    q = synth.rows(w, w.seed_query, 0, w.n_query)
    ref, got = _build_both(w, x)
    from paper_2603_05180_amd import engine
    gidx = engine.Index(got)
    for mode in (0, 1):
        compare(ref, q, 10, mode=mode, alpha=0.03, tau=3, gpu=gidx)


def test_sign_codes_of_every_row_at_full_size():
    """N = 2M, D = 3072: 96M code words, more wave-threads than one dispatch
    holds, so the kernel strides; sampled rows across the whole range
    (including the last) equal the signs of the rows."""
    import ctypes
    import synth.gpu as sg
    from paper_2603_05180_amd._lib import check, lib
    w = synth.WORKLOADS["d3072"]
    x = sg.rows(w, w.seed_data, 0, w.n, sg.mixture_params(w))
    words = w.d // 64
    codes = torch.empty(w.n, words, dtype=torch.int64, device="cuda")
    check(lib.crisp_build_codes(ctypes.c_void_p(x.data_ptr()), w.n, w.d, ctypes.c_void_p(codes.data_ptr()), None))
    torch.cuda.synchronize()
    sh = torch.arange(64, device="cuda", dtype=torch.int64)
    for r in (0, 1, 1_398_101, 1_398_102, 1_500_000, w.n - 2, w.n - 1):
        bits = ((codes[r].view(words, 1) >> sh) & 1).bool().view(-1)
        assert torch.equal(bits, x[r] > 0), r
    del x, codes
    torch.cuda.empty_cache()


@pytest.mark.parametrize("rows,d,offset", [
    (16500, 192, 0),   # 128x128 direct-to-LDS tiles: half-filled last column tile, ragged rows
    (4100, 1024, 0),   # direct-to-LDS tiles, ragged rows
    (16500, 192, 1),   # rows not 16-byte aligned: small-tile kernel
    (300, 192, 0),     # too few tiles to fill the chip: small-tile kernel
])
def test_rotation_kernels_equal_oracle(rows, d, offset):
    """x R through the C ABI on both rotation kernels equals the oracle's
    ascending-i float64 sum rounded to float32, bit for bit (Section 3)."""
    from paper_2603_05180_amd import engine
    rng = np.random.default_rng(rows * 7 + d + offset)
    x = (rng.standard_normal((rows, d)) * np.exp2(rng.integers(-6, 7, (rows, 1)))).astype(np.float32)
    r = obuild.rotation_from_gaussian(rng.standard_normal((d, d)))
    ref = obuild.rotate_rows(x, r)
    buf = torch.zeros(rows * d + offset, dtype=torch.float32, device="cuda")
    buf[offset:] = torch.from_numpy(x.reshape(-1)).cuda()
    xt = buf[offset:].view(rows, d)
    print(f"rotation rows={rows} d={d} offset={offset}", flush=True)
    got = engine.rotate_rows(xt, torch.from_numpy(r).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), ref.view(np.uint32))
