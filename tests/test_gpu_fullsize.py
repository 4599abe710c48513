"""Full-size parity on sampled queries (needs an MI355X).

The N = 1M, D = 4096 index, the N = 1M, D = 960 index (K = 16 centroids per
half; the K = 256 reading is switched off) and the N = 2M, D = 3072 index
are generated and built on the GPU
exactly as bench.py does.  The whole batch is searched in the configuration
bench.py times (10,000 queries, chunks of 4,096, two chunk pipelines,
float32 and bfloat16 verification, persistent re-rank; the batch executor's
graphs for the uneven workload).  64 sampled queries spread over every
chunk are re-run by the CPU oracle (worker processes over a memory-mapped
copy of the same index arrays): ids and float32 distances must be
identical.  The same sampled queries are searched again with stage taps,
which must equal the oracle's trace: q' bit for bit at D = 4096, the
threshold after the fallback, |C| and the candidate list, the Hamming order
and distances, the verified prefix, the last top-k update (the learned
budget's training label) and the stop flag.  The learned limits are
recomputed by the oracle's own feature and bfloat16 inference code from its
own traces.
"""
import os
import sys

import numpy as np
import pytest
import torch

from parity_util import oracle_many, oracle_pool

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def pool():
    p = oracle_pool()
    yield p
    p.terminate()
    p.join()


def _build(name):
    import bench
    import synth
    w = synth.WORKLOADS[name]
    arrays, params = bench.build_gpu_index(w)
    return w, arrays, params


def _spread(nq, per_chunk_edges, count=64, seed=0):
    """`count` query positions: the edges of every chunk plus seeded others."""
    rng = np.random.default_rng(seed)
    s = set(int(v) for v in per_chunk_edges if 0 <= v < nq)
    while len(s) < count:
        s.add(int(rng.integers(0, nq)))
    return np.array(sorted(s))


def _same_results(ref, got_ids, got_d, sample, what):
    for j, qi in enumerate(sample):
        assert np.array_equal(got_ids[qi], ref[j]["ids"]), (what, int(qi))
        assert np.array_equal(got_d[qi].view(np.uint32), ref[j]["dists"].view(np.uint32)), (what, int(qi))


def _same_stages(ref, taps, mode, what):
    for j, r in enumerate(ref):
        nc = int(taps["n_cand"][j])
        assert np.array_equal(taps["q_rot"][j].view(np.uint32), r["q_rot"].view(np.uint32)), (what, j, "q_rot")
        assert int(taps["tau_eff"][j]) == r["tau_eff"], (what, j, "tau_eff")
        assert nc == r["candidates"].size, (what, j, "|C|")
        assert np.array_equal(taps["cand"][j, :nc], r["candidates"]), (what, j, "cand")
        assert int(taps["examined"][j]) == r["examined"], (what, j, "examined")
        if mode == 1:
            assert np.array_equal(taps["order"][j, :nc], r["order"]), (what, j, "order")
            assert np.array_equal(taps["hamming"][j, :nc], r["hamming"]), (what, j, "hamming")
            assert int(taps["last_update"][j]) == r["last_update"], (what, j, "last_update")
            assert int(taps["stopped"][j]) == int(r["stopped"]), (what, j, "stopped")


def _taps(index, nq, mode):
    keep = {"q_rot", "tau_eff", "n_cand", "cand", "examined", "order", "hamming", "last_update", "stopped",
            "features", "limits"}
    return {k: v for k, v in index.alloc_taps(nq, mode).items() if k in keep}


def test_d4096_bench_configuration_sampled(pool):
    import bench
    import synth.gpu as sg
    from oracle import mlp as omlp
    from paper_2603_05180_amd import engine, learned
    w, arrays, params = _build("d4096")
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays)
    index.enable_bf16()
    kw = dict(mode=1, alpha=0.002, tau=16, patience_factor=40)
    ck = dict(max_chunk=4096)
    res = {}
    for name, extra in (("float32", dict(overlap=1)), ("bf16", dict(overlap=1, precision=1)),
                        ("bf16 persistent", dict(precision=1, persistent=1)),
                        ("bf16 pre-scored", dict(overlap=1, precision=2))):
        print(f"d4096 full batch, {name}", flush=True)
        ids, d = index.search(queries, w.k, **kw, **ck, **extra)
        torch.cuda.synchronize()
        res[name] = (ids.cpu().numpy(), d.cpu().numpy())
    for name in res:
        assert np.array_equal(res[name][0], res["float32"][0]), name
        assert np.array_equal(res[name][1].view(np.uint32), res["float32"][1].view(np.uint32)), name
    sample = _spread(w.n_query, [0, 1, 4095, 4096, 8191, 8192, 9999])
    qs = queries[sample.tolist()].contiguous()
    taps = _taps(index, sample.size, 1)
    index.search(qs, w.k, taps=taps, precision=1, **kw)
    torch.cuda.synchronize()
    taps = {k: v.cpu().numpy() for k, v in taps.items()}
    print("d4096: index arrays to files for the oracle", flush=True)
    tmp, paths, meta = bench.export_index(arrays)
    try:
        q = qs.cpu().numpy()
        print(f"d4096 oracle on {sample.size} sampled queries", flush=True)
        ref = oracle_many(pool, paths, meta, q, w.k, feats=True, **kw)
        _same_results(ref, *res["float32"], sample, "d4096 optimized")
        _same_stages(ref, taps, 1, "d4096 optimized")
        print("d4096 Guaranteed Mode (bf16), 16 sampled queries", flush=True)
        gs = sample[::4]
        gi, gd = index.search(queries[gs.tolist()].contiguous(), w.k, mode=0, alpha=0.002, tau=16, precision=1)
        torch.cuda.synchronize()
        gref = oracle_many(pool, paths, meta, queries[gs.tolist()].cpu().numpy(), w.k, mode=0, alpha=0.002, tau=16)
        _same_results(gref, gi.cpu().numpy(), gd.cpu().numpy(), np.arange(gs.size), "d4096 guaranteed")
        # learned budget: the oracle's features and bfloat16 inference from its own traces
        print("d4096 learned budget", flush=True)
        trainq = sg.rows(w, 3004, 0, 20_000, params)
        model = learned.train_budget(index, trainq, w.k, epochs=5, alpha=0.002, tau=16, patience_factor=40)
        del trainq
        lt = {"limits": torch.empty(sample.size, dtype=torch.int32, device="cuda"),
              "n_cand": torch.empty(sample.size, dtype=torch.int32, device="cuda")}
        li, ld = index.search(qs, w.k, budget_source=1, precision=1, taps=lt, **kw)
        torch.cuda.synchronize()
        lim = lt["limits"].cpu().numpy()
        f = index.n_features
        p = model.params.cpu().numpy().astype(np.float32)
        h = learned.HIDDEN
        pd = {"w1": p[:f * h].reshape(f, h), "b1": p[f * h:f * h + h],       # the flat layout of the library
              "w2": p[f * h + h:f * h + 2 * h], "b2": p[f * h + 2 * h:f * h + 2 * h + 1]}
        feats = np.stack([r["features"] for r in ref]).astype(np.float32)
        xs = ((feats - model.mean.cpu().numpy()) / model.std.cpu().numpy()).astype(np.float32)
        y = omlp.infer_bf16(pd, xs)
        lim_ref = omlp.limits_from(y, model.delta, w.k, np.array([r["candidates"].size for r in ref]))
        e = np.exp(y + model.delta)
        close = np.abs(e - np.round(e)) < 1e-3 * e
        assert np.all((lim == lim_ref) | close)
        assert np.mean(lim == lim_ref) >= 0.9
        same = np.flatnonzero(lim == lim_ref)
        lref = oracle_many(pool, paths, meta, q[same], w.k, limits=lim_ref[same], **kw)
        _same_results(lref, li.cpu().numpy()[same], ld.cpu().numpy()[same], np.arange(same.size), "d4096 learned")
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)
    index.free()
    del index, arrays, queries
    torch.cuda.empty_cache()


@pytest.mark.skip(reason="the library refuses K > 64: a search at N = 1M, D = 960, K = 256 faulted the GPU "
                         "(twice, chunks of 4,096 and of 1,024) and the cause is not found yet")
def test_d960_k256_both_modes_k10_k100_sampled(pool):
    """N = 1M, D = 960, 16 subspaces of 60 dims, K = 256 centroids per half
    (65,536 cells per subspace), unrotated: the whole batch of 10,000 queries
    in chunks of 1,024 on two pipelines (the per-query workspace is about
    34 MB at this K: 35 GB per chunk), both modes at k = 10 and k = 100; 64
    sampled queries re-run by the oracle, stage taps compared."""
    import bench
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w, arrays, params = _build("d960k256")
    assert arrays["rotation"] is None
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays)
    index.enable_bf16()
    sample = _spread(w.n_query, [0, 1023, 1024, 4095, 4096, 8191, 8192, 9215, 9216, 9999], seed=1)
    qs = queries[sample.tolist()].contiguous()
    tmp, paths, meta = bench.export_index(arrays)
    try:
        q = qs.cpu().numpy()
        for mode in (0, 1):
            for k in (10, 100):
                kw = dict(mode=mode, alpha=0.01, tau=4 if mode == 0 else 8, patience_factor=10)
                print(f"d960 K=256 full batch, mode={mode} k={k}", flush=True)
                ids, d = index.search(queries, k, max_chunk=1024, overlap=1, precision=1, **kw)
                taps = _taps(index, sample.size, mode)
                index.search(qs, k, taps=taps, **kw)
                torch.cuda.synchronize()
                taps = {kk: v.cpu().numpy() for kk, v in taps.items()}
                ref = oracle_many(pool, paths, meta, q, k, **kw)
                _same_results(ref, ids.cpu().numpy(), d.cpu().numpy(), sample, f"d960 mode={mode} k={k}")
                _same_stages(ref, taps, mode, f"d960 mode={mode} k={k}")
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)
    index.free()
    del index, arrays, queries
    torch.cuda.empty_cache()


def test_d960_both_modes_k10_k100_sampled(pool):
    """N = 1M, D = 960, 16 subspaces of 60 dims, K = 16 centroids per half
    (256 cells per subspace), unrotated: the whole batch of 10,000 queries in
    chunks of 2,048 on two pipelines, both modes at k = 10 and k = 100, the
    bfloat16 pass; 64 sampled queries re-run by the oracle, stage taps
    compared."""
    import bench
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w, arrays, params = _build("d960")
    assert arrays["rotation"] is None
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays)
    index.enable_bf16()
    sample = _spread(w.n_query, [0, 2047, 2048, 4095, 4096, 8191, 8192, 9999], seed=1)
    qs = queries[sample.tolist()].contiguous()
    tmp, paths, meta = bench.export_index(arrays)
    try:
        q = qs.cpu().numpy()
        for mode in (0, 1):
            for k in (10, 100):
                kw = dict(mode=mode, alpha=0.01, tau=4 if mode == 0 else 8, patience_factor=10)
                print(f"d960 K=16 full batch, mode={mode} k={k}", flush=True)
                ids, d = index.search(queries, k, max_chunk=2048, overlap=1, precision=1, **kw)
                torch.cuda.synchronize()
                taps = _taps(index, sample.size, mode)
                index.search(qs, k, taps=taps, **kw)
                torch.cuda.synchronize()
                taps = {kk: v.cpu().numpy() for kk, v in taps.items()}
                ref = oracle_many(pool, paths, meta, q, k, **kw)
                _same_results(ref, ids.cpu().numpy(), d.cpu().numpy(), sample, f"d960 mode={mode} k={k}")
                _same_stages(ref, taps, mode, f"d960 mode={mode} k={k}")
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)
    index.free()
    del index, arrays, queries
    torch.cuda.empty_cache()


def test_d3072_graph_batch_sampled(pool):
    import bench
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w, arrays, params = _build("d3072")
    queries = sg.rows(w, w.seed_query, 0, 1000, params)
    index = engine.Index(arrays)
    index.enable_bf16()
    kw = dict(mode=1, alpha=0.002, tau=16, patience_factor=40)
    plan = engine.Plan(index, 1024, 10, precision=1, max_chunk=512, **kw)
    print("d3072 batch of 1,000 through a captured graph (two chunks)", flush=True)
    ids, d = plan.search(queries)
    torch.cuda.synchronize()
    sample = _spread(1000, [0, 511, 512, 999], seed=2)
    tmp, paths, meta = bench.export_index(arrays)
    try:
        ref = oracle_many(pool, paths, meta, queries[sample.tolist()].cpu().numpy(), 10, **kw)
        _same_results(ref, ids.cpu().numpy(), d.cpu().numpy(), sample, "d3072 graph")
    finally:
        import shutil
        shutil.rmtree(tmp, ignore_errors=True)
    plan.free()
    index.free()
    del index, arrays, queries
    torch.cuda.empty_cache()
