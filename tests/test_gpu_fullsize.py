"""Full-size parity on sampled queries (needs an MI355X).

The N = 1M, D = 4096 index, the N = 1M, D = 960 index and the N = 2M,
D = 3072 index are generated and built on the GPU exactly as bench.py does; the whole batch is searched in
the configuration bench.py times (10,000 queries, chunks of 4,096, two chunk
pipelines, float32 and bfloat16 verification; the batch executor's graphs
for the uneven workload), and sampled queries, spread over the chunks, are
re-run one by one by the CPU oracle on a host copy of the same index arrays:
ids and float32 distances must be identical.
"""
import os
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _host(arrays):
    return {"n": arrays["n"], "d": arrays["d"], "m": arrays["m"], "k_half": arrays["k_half"],
            "rotation": None if arrays["rotation"] is None else arrays["rotation"].cpu().numpy(),
            "centroids": arrays["centroids"].cpu().numpy(), "offsets": arrays["offsets"].cpu().numpy(),
            "ids": arrays["ids"].cpu().numpy(), "base": arrays["base"].cpu().numpy(),
            "codes": arrays["codes"].cpu().numpy().view(np.uint64)}


def _build(name):
    sys.path.insert(0, ROOT)
    import bench
    import synth
    import synth.gpu as sg
    w = synth.WORKLOADS[name]
    arrays, params = bench.build_gpu_index(w)
    return w, arrays, params


def _check(host, q, sample, got_ids, got_d, k, **kw):
    from oracle import query as oquery
    oi, od, _ = oquery.search(host, q[sample], k, **kw)
    gi = got_ids[sample]
    gd = got_d[sample]
    assert np.array_equal(gi, oi), (kw, sample)
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), (kw, sample)


def test_d4096_bench_configuration_sampled():
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w, arrays, params = _build("d4096")
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays)
    index.enable_bf16()
    kw = dict(mode=1, alpha=0.002, tau=16, patience_factor=40)
    ck = dict(max_chunk=4096)
    res = {}
    for name, extra in (("float32", dict(overlap=1)), ("bf16", dict(overlap=1, precision=1)),
                        ("bf16 persistent", dict(precision=1, persistent=1))):
        print(f"d4096 full batch, {name}", flush=True)
        ids, d = index.search(queries, w.k, **kw, **ck, **extra)
        torch.cuda.synchronize()
        res[name] = (ids.cpu().numpy(), d.cpu().numpy())
    for name in res:
        assert np.array_equal(res[name][0], res["float32"][0]), name
        assert np.array_equal(res[name][1].view(np.uint32), res["float32"][1].view(np.uint32)), name
    print("d4096 Guaranteed Mode, bf16", flush=True)
    gsample = np.array([3, 4321])
    gi, gd = index.search(queries[gsample.tolist()].contiguous(), w.k, mode=0, alpha=0.002, tau=16, precision=1)
    torch.cuda.synchronize()
    host = _host(arrays)
    q = queries.cpu().numpy()
    sample = np.array([0, 1, 2047, 4095, 4096, 5000, 8191, 8192, 9999])
    print("d4096 oracle on sampled queries", flush=True)
    _check(host, q, sample, *res["float32"], w.k, **kw)
    from oracle import query as oquery
    oi, od, _ = oquery.search(host, q[gsample], w.k, mode=0, alpha=0.002, tau=16)
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), od.view(np.uint32))
    # learned budget: the engine's limits (bf16 MFMA inference) given to the oracle
    from paper_2603_05180_amd import learned
    print("d4096 learned budget", flush=True)
    trainq = sg.rows(w, 3004, 0, 20_000, params)
    learned.train_budget(index, trainq, w.k, epochs=5, alpha=0.002, tau=16, patience_factor=40)
    taps = {"limits": torch.empty(w.n_query, dtype=torch.int32, device="cuda")}
    li, ld = index.search(queries, w.k, budget_source=1, precision=1, overlap=1, taps=taps, **kw, **ck)
    torch.cuda.synchronize()
    lim = taps["limits"].cpu().numpy()
    oi, od, _ = oquery.search(host, q[sample], w.k, limits=lim[sample], **kw)
    assert np.array_equal(li.cpu().numpy()[sample], oi)
    assert np.array_equal(ld.cpu().numpy()[sample].view(np.uint32), od.view(np.uint32))
    del host, index, arrays, queries
    torch.cuda.empty_cache()


def test_d960_both_modes_k10_k100_sampled():
    """N = 1M, D = 960 (16 subspaces of 60 dims, 256 cells each, unrotated):
    the whole batch of 10,000 queries in chunks of 4,096, both modes at
    k = 10 and k = 100; sampled queries of every chunk re-run by the oracle."""
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w, arrays, params = _build("d960")
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays)
    host = _host(arrays)
    q = queries.cpu().numpy()
    sample = np.array([0, 4095, 4096, 9999])
    for mode in (0, 1):
        for k in (10, 100):
            kw = dict(mode=mode, alpha=0.01, tau=4)
            print(f"d960 full batch, mode={mode} k={k}", flush=True)
            ids, d = index.search(queries, k, max_chunk=4096, **kw)
            torch.cuda.synchronize()
            _check(host, q, sample, ids.cpu().numpy(), d.cpu().numpy(), k, **kw)
    del host, index, arrays, queries
    torch.cuda.empty_cache()


def test_d3072_graph_batch_sampled():
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
    host = _host(arrays)
    q = queries.cpu().numpy()
    _check(host, q, np.array([0, 511, 512, 999]), ids.cpu().numpy(), d.cpu().numpy(), 10, **kw)
    plan.free()
    del host, index, arrays, queries
    torch.cuda.empty_cache()
