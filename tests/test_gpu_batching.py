"""Uneven batches on the GPU (needs an MI355X): the batch executor's captured
graphs must return exactly what a direct search returns, for every batch
size of a bucket, replay after replay with other GPU work in between; and
results must not depend on the id tile or the query chunk."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from parity_util import gpu_index, make_workload, oracle_index

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 7, 16, 33, 64, 65, 100, 5, 1, 100, 47]


@pytest.fixture(scope="module")
def d128():
    w, x, q = make_workload("d128", n_query=300)
    idx = oracle_index(w, x)
    g = gpu_index(idx)
    g.enable_bf16()
    return w, x, torch.from_numpy(q).cuda(), idx, g


def _same(a, b):
    ia, da = a
    ib, db = b
    torch.cuda.synchronize()
    assert torch.equal(ia, ib)
    assert torch.equal(da.view(torch.int32), db.view(torch.int32))


@pytest.mark.parametrize("mode,precision,k", [(0, 0, 10), (0, 1, 1), (1, 0, 10), (1, 1, 100)])
def test_plan_replays_match_direct_search(d128, mode, precision, k):
    from paper_2603_05180_amd import engine
    w, x, q, idx, g = d128
    kw = dict(mode=mode, alpha=0.05, tau=4, precision=precision)
    plan = engine.Plan(g, 100, k, **kw)
    o = 0
    for rep in range(2):
        for nb in SIZES:
            print(f"plan mode={mode} precision={precision} k={k} batch={nb} rep={rep}", flush=True)
            qb = q[o:o + nb].contiguous()
            o = (o + nb) % 200
            got = plan.search(qb)
            ref = g.search(qb, k, **kw)           # eager work between replays
            _same(got, ref)
    plan.free()


def test_plan_several_chunks_per_bucket(d128):
    from paper_2603_05180_amd import engine
    w, x, q, idx, g = d128
    kw = dict(mode=1, alpha=0.05, tau=4, max_chunk=16)
    plan = engine.Plan(g, 100, 10, **kw)
    for nb in (100, 17, 64, 99, 33):
        print(f"chunked plan batch={nb}", flush=True)
        qb = q[:nb].contiguous()
        _same(plan.search(qb), g.search(qb, 10, **kw))


def test_plan_with_learned_budget(d128):
    from paper_2603_05180_amd import engine
    w, x, q, idx, g = d128
    f = g.n_features
    p = omlp.init_params(f, 3)
    p["b2"] = np.array([3.5], np.float32)
    flat = np.concatenate([p["w1"].reshape(-1), p["b1"], p["w2"], p["b2"]]).astype(np.float32)
    g.set_budget_model(torch.from_numpy(flat).cuda(), torch.zeros(f, device="cuda"), torch.ones(f, device="cuda"),
                       0.5)
    kw = dict(mode=1, alpha=0.05, tau=4, budget_source=1, precision=1)
    plan = engine.Plan(g, 64, 10, **kw)
    for nb in (64, 3, 40, 1):
        print(f"learned plan batch={nb}", flush=True)
        qb = q[100:100 + nb].contiguous()
        _same(plan.search(qb), g.search(qb, 10, **kw))
    g.set_budget_model(None)


def test_plan_follows_budget_model_and_bf16_changes(d128):
    """A plan captured under one budget model (or bfloat16 copy) must not
    replay stale state after it changes: the bucket is captured anew."""
    from paper_2603_05180_amd import engine
    w, x, q, idx, g = d128
    f = g.n_features
    p = omlp.init_params(f, 5)
    p["b2"] = np.array([3.0], np.float32)
    flat = np.concatenate([p["w1"].reshape(-1), p["b1"], p["w2"], p["b2"]]).astype(np.float32)
    params = torch.from_numpy(flat).cuda()
    mean, std = torch.zeros(f, device="cuda"), torch.ones(f, device="cuda")
    kw = dict(mode=1, alpha=0.05, tau=4, budget_source=1, precision=1)
    qb = q[:50].contiguous()
    g.set_budget_model(params, mean, std, -2.0)
    plan = engine.Plan(g, 64, 10, **kw)
    first = plan.search(qb)
    _same(first, g.search(qb, 10, **kw))
    g.set_budget_model(params, mean, std, 1.5)        # another margin: other limits
    second = plan.search(qb)
    _same(second, g.search(qb, 10, **kw))
    torch.cuda.synchronize()
    assert not torch.equal(first[0], second[0])        # the change is visible
    g.enable_bf16()                                     # new copy, new pointers
    _same(plan.search(qb), g.search(qb, 10, **kw))
    g.set_budget_model(None)
    with pytest.raises(engine.CrispError):              # the model is gone
        plan.search(qb)
    plan.free()


@pytest.mark.parametrize("mode", [0, 1])
def test_results_do_not_depend_on_tiles_or_chunks(d128, mode):
    from paper_2603_05180_amd import engine
    w, x, q, idx, g = d128
    kw = dict(mode=mode, alpha=0.05, tau=4)
    ref = g.search(q, 10, **kw)
    for tile in (4096, 8192, 65536):
        print(f"tile={tile} mode={mode}", flush=True)
        gt = engine.Index(g.arrays | {"n": g.n, "d": g.d, "m": g.m, "k_half": g.k_half}, tile_ids=tile)
        for chunk in (0, 7, 64):
            _same(gt.search(q, 10, max_chunk=chunk, **kw), ref)
        if tile == 4096:
            # three tiles: counted one, two or three per block
            for ct in (1, 2, 3, 5):
                _same(gt.search(q, 10, count_tiles=ct, **kw), ref)
            # every cell activated: each tile's sub-slices overflow the
            # block's list and are counted in several batches
            wide = dict(kw, alpha=1.0, tau=8)
            ref1 = g.search(q[:8].contiguous(), 10, **wide)
            for ct in (1, 3):
                _same(gt.search(q[:8].contiguous(), 10, count_tiles=ct, **wide), ref1)
        gt.free()


@pytest.mark.parametrize("mode,precision", [(0, 1), (1, 0), (1, 1)])
def test_persistent_rerank_matches(d128, mode, precision):
    w, x, q, idx, g = d128
    kw = dict(mode=mode, alpha=0.05, tau=4, precision=precision)
    print(f"persistent mode={mode} precision={precision}", flush=True)
    for k in (1, 10):
        _same(g.search(q, k, persistent=1, **kw), g.search(q, k, **kw))
        _same(g.search(q[:5].contiguous(), k, persistent=1, max_chunk=2, **kw), g.search(q[:5].contiguous(), k, **kw))


def test_tuned_runner_serves_uneven_batches(d128, tmp_path):
    """The tuner picks a setting per (k, bucket); every batch served through
    it equals the direct search."""
    import synth
    from paper_2603_05180_amd import autotune
    w, x, q, idx, g = d128
    params = dict(mode=1, alpha=0.05, tau=4, precision=1)
    srv = autotune.Server(None, g, params, max_batch=64, ks=(1, 10), tiles=(4096, 16384), chunks=(16, 64),
                          count_tiles=(0, 2))
    cache = str(tmp_path / "tune.json")
    choice = srv.tune(q, [1, 2, 4, 8, 16, 32, 64], reps=1, cache=cache)
    assert len(choice) == 14
    sizes = synth.batch_sizes(5, 250, max_batch=64)
    ks = synth.batch_ks(5, len(sizes), choices=(1, 10))
    lat, outs = srv.run(q, sizes, ks)
    assert len(lat) == len(sizes) and all(v > 0 for v in lat)
    o = 0
    for (ids, d), nq, k in zip(outs, sizes, ks):
        print(f"runner batch={nq} k={k}", flush=True)
        _same((ids, d), g.search(q[o:o + nq].contiguous(), k, **params))
        o += nq
    # the cache is reused
    srv2 = autotune.Server(None, g, params, max_batch=64, ks=(1, 10), tiles=(4096, 16384), chunks=(16, 64),
                           count_tiles=(0, 2))
    assert srv2.tune(q, [1, 2, 4, 8, 16, 32, 64], cache=cache) == choice
    srv.free()
    srv2.free()


@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 1)])
def test_two_chunk_pipelines_match(d128, mode, precision):
    """overlap = 1 runs odd chunks on the index's second stream with their own
    workspace; results equal the single-stream search, also inside a plan."""
    from paper_2603_05180_amd import engine
    w, x, q, idx, g = d128
    kw = dict(mode=mode, alpha=0.05, tau=4, precision=precision)
    print(f"overlap mode={mode} precision={precision}", flush=True)
    for chunk in (7, 64, 0):
        _same(g.search(q, 10, overlap=1, max_chunk=chunk, **kw), g.search(q, 10, max_chunk=chunk, **kw))
    plan = engine.Plan(g, 100, 10, overlap=1, max_chunk=16, **kw)
    for nb in (100, 17, 3, 64):
        qb = q[:nb].contiguous()
        _same(plan.search(qb), g.search(qb, 10, **kw))
    plan.free()


@pytest.mark.parametrize("mode", [0, 1])
def test_query_run_order_does_not_change_results(d128, mode):
    """Chunks of up to 4096 queries run their candidate-reading stages in a
    sorted query order, larger chunks in index order: both, and chunks that
    straddle the limit, give the same ids and distances."""
    w, x, q, idx, g = d128
    kw = dict(mode=mode, alpha=0.05, tau=4, precision=1)
    qq = q.repeat(15, 1).contiguous()                     # 4,500 queries
    ref = g.search(qq, 10, max_chunk=4500, **kw)          # one chunk, index order
    _same(g.search(qq, 10, max_chunk=4096, **kw), ref)    # 4,096 sorted + 404 sorted
    _same(g.search(qq, 10, max_chunk=1000, overlap=1, **kw), ref)
    ids = ref[0].cpu().numpy()
    assert np.array_equal(ids[:300], ids[4200:])          # repeated queries, repeated answers


def test_stage_profile_intervals(d128):
    """The per-stage timers: one counting interval (the first pass alone) per
    chunk, two candidate-list intervals per chunk, positive times."""
    w, x, q, idx, g = d128
    g.profile_begin(1024)
    g.search(q, 10, mode=1, alpha=0.05, tau=4, max_chunk=100)    # 300 queries: three chunks
    torch.cuda.synchronize()
    st = g.profile_end()
    assert st["dropped"] == 0
    for name in ("rotate", "select", "count", "hamming_dist", "hamming_place", "rerank"):
        assert st[name]["intervals"] == 3 and st[name]["ms"] > 0, (name, st[name])
    assert st["candidates"]["intervals"] == 6 and st["candidates"]["ms"] > 0
    assert st["budget"]["intervals"] == 0


@pytest.mark.parametrize("mode,precision", [(0, 1), (1, 0), (1, 1)])
def test_capped_candidate_lists_match(d128, mode, precision):
    """max_candidates caps each query's candidate-indexed buffers; queries
    with more candidates are searched again uncapped after the batch.  Ids,
    distances and every stage tap equal the uncapped search, with chunks and
    two pipelines, through a plan's graph replays and through the static
    scratch; the capped workspace is smaller."""
    import ctypes
    from paper_2603_05180_amd import engine
    from paper_2603_05180_amd._lib import check, lib
    w, x, q, idx, g = d128
    kw = dict(mode=mode, alpha=0.05, tau=4, precision=precision)
    nq = q.shape[0]
    t0 = g.alloc_taps(nq, mode)
    ref = g.search(q, 10, taps=t0, **kw)
    torch.cuda.synchronize()
    nc = t0["n_cand"].cpu().numpy()
    cap = int(np.percentile(nc, 60))           # about 40% of the queries overflow
    assert 0 < cap < nc.max() and (nc > cap).sum() > 0
    print(f"cap {cap}, {(nc > cap).sum()} of {nq} queries above it", flush=True)
    for extra in (dict(), dict(max_chunk=37), dict(max_chunk=64, overlap=1)):
        t1 = g.alloc_taps(nq, mode)
        _same(g.search(q, 10, taps=t1, max_candidates=cap, **kw, **extra), ref)
        for key in t0:
            if key == "limits":                  # written only with a budget model
                continue
            a, b = t0[key].cpu().numpy(), t1[key].cpu().numpy()
            if key in ("cand", "cand_score", "order", "hamming"):
                for qi in range(nq):
                    assert np.array_equal(a[qi, :nc[qi]], b[qi, :nc[qi]]), (key, qi, extra)
            elif key == "cells":                 # each subspace's activated cells only
                ncl = t0["n_cells"].cpu().numpy()
                for qi in range(nq):
                    for sub in range(ncl.shape[1]):
                        assert np.array_equal(a[qi, sub, :ncl[qi, sub]], b[qi, sub, :ncl[qi, sub]]), (key, qi, extra)
            else:
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (key, extra)
    # a cap above every candidate list changes nothing either
    _same(g.search(q, 10, max_candidates=int(nc.max()) + 1, **kw), ref)
    # the workspace shrinks: 21 bytes fewer per entry and query
    sizes = []
    for c in (0, cap):
        b = ctypes.c_size_t(0)
        p = g.params(max_candidates=c, max_chunk=256, **kw)
        check(lib.crisp_search_workspace_bytes(g._h, 256, 10, ctypes.byref(p), ctypes.byref(b)))
        sizes.append(b.value)
    assert sizes[1] < sizes[0]
    # plan replays (the overflowing queries redone after each replay)
    pl = engine.Plan(g, 300, 10, max_candidates=cap, **kw)
    for rep in range(2):
        _same(pl.search(q), ref)
        sub = q[:70].contiguous()
        _same(pl.search(sub), g.search(sub, 10, **kw))
    pl.free()
    # the static scratch
    _same(g.search_static(q, 10, max_candidates=cap, **kw), ref)
