"""Helpers that compare the GPU engine stage by stage with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import synth
from oracle import build as obuild
from oracle import query as oquery


def make_workload(base: str, **kw):
    w = synth.WORKLOADS[base].scaled(**kw)
    p = synth.mixture_params(w)
    x = synth.rows(w, w.seed_data, 0, w.n, p)
    q = synth.rows(w, w.seed_query, 0, w.n_query, p)
    return w, x, q


def oracle_index(w, x, **kw):
    return obuild.build_index_for(w, x, **kw)


def gpu_index(idx, tile_ids=0):
    from paper_2603_05180_amd import engine
    return engine.Index(idx, tile_ids=tile_ids)


def run_gpu(gidx, q: np.ndarray, k: int, *, mode, alpha, tau, patience_factor=40, limits=None, max_chunk=0,
            precision=0, walk_order=0, verify=0):
    qt = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float32)).to(gidx.device)
    taps = gidx.alloc_taps(q.shape[0], mode if walk_order == 0 else 0)
    lim = None
    if limits is not None:
        lim = torch.from_numpy(np.asarray(limits, dtype=np.int32)).to(gidx.device)
    ids, d = gidx.search(qt, k, mode=mode, alpha=alpha, tau=tau, patience_factor=patience_factor,
                         limits=lim, max_chunk=max_chunk, precision=precision, walk_order=walk_order,
                         verify=verify, taps=taps)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy(), {kk: v.cpu().numpy() for kk, v in taps.items()}


def compare(idx, q, k, *, mode, alpha, tau, patience_factor=40, limits=None, gpu=None, max_chunk=0,
            tile_ids=0, check_stages=True, precision=0, walk_order=0, verify=0):
    """Run both sides; assert bit-exact stages and results.  Returns a summary."""
    g = gpu if gpu is not None else gpu_index(idx, tile_ids)
    gi, gd, tp = run_gpu(g, q, k, mode=mode, alpha=alpha, tau=tau, patience_factor=patience_factor,
                         limits=limits, max_chunk=max_chunk, precision=precision, walk_order=walk_order,
                         verify=verify)
    oi, od, tr = oquery.search(idx, q, k, mode=mode, alpha=alpha, tau=tau, patience_factor=patience_factor,
                               limits=limits, trace=True, hamming=(walk_order == 0), ads=(verify == 1))
    m, kh, n = idx["m"], idx["k_half"], idx["n"]
    for qi in range(q.shape[0]):
        t = tr[qi]
        if check_stages:
            assert np.array_equal(tp["q_rot"][qi].view(np.uint32), t["q_rot"].view(np.uint32)), f"q_rot q={qi}"
            assert np.array_equal(tp["half_dist"][qi].view(np.uint64), t["half_dist"].view(np.uint64)), \
                f"half_dist q={qi}"
            for sub in range(m):
                nc = int(tp["n_cells"][qi, sub])
                got = sorted((int(v) & 0xFFFFFF, int(v) >> 24) for v in tp["cells"][qi, sub, :nc])
                ref = sorted(t["activated"][sub])
                assert got == ref, f"cells q={qi} m={sub}"
                sizes = np.diff(idx["offsets"][sub].astype(np.int64))
                assert int(tp["retrieved"][qi, sub]) == int(sum(sizes[c] for c, _ in ref))
            assert int(tp["tau_eff"][qi]) == t["tau_eff"], f"tau_eff q={qi}"
            nc = int(tp["n_cand"][qi])
            assert nc == t["candidates"].size, f"|C| q={qi}"
            assert np.array_equal(tp["cand"][qi, :nc], t["candidates"]), f"cand q={qi}"
            assert np.array_equal(tp["cand_score"][qi, :nc].astype(np.int64), t["scores"][t["candidates"]])
            floor = max(t["tau_eff"], 1)
            v = t["scores"]
            hist = np.bincount(v[v >= floor], minlength=2 * m + 1)
            assert np.array_equal(tp["hist"][qi], hist), f"hist q={qi}"
            if mode == 1:
                if walk_order == 0:
                    assert np.array_equal(tp["order"][qi, :nc], t["order"]), f"order q={qi}"
                    assert np.array_equal(tp["hamming"][qi, :nc], t["hamming"]), f"hamming q={qi}"
                assert int(tp["examined"][qi]) == t["examined"], f"examined q={qi}"
                assert int(tp["last_update"][qi]) == t["last_update"], f"last_update q={qi}"
                assert int(tp["stopped"][qi]) == (0 if t["stop"] is None else 1), f"stopped q={qi}"
    assert np.array_equal(gi, oi), "ids"
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), "dists"
    if mode == 1 and walk_order == 0:
        # without the order taps only a prefix of the Hamming order is placed
        # before the walk (order_prefix 0: automatic; 1: every walk that goes
        # past its first candidate is redone on the full order)
        qt = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float32)).to(g.device)
        lim = None if limits is None else torch.from_numpy(np.asarray(limits, dtype=np.int32)).to(g.device)
        for op in (0, 1):
            small = {"examined": torch.empty(q.shape[0], dtype=torch.int32, device=g.device),
                     "last_update": torch.empty(q.shape[0], dtype=torch.int32, device=g.device)}
            pi, pd = g.search(qt, k, mode=mode, alpha=alpha, tau=tau, patience_factor=patience_factor, limits=lim,
                              max_chunk=max_chunk, precision=precision, verify=verify, order_prefix=op, taps=small)
            torch.cuda.synchronize()
            assert np.array_equal(pi.cpu().numpy(), oi), f"ids, order prefix {op}"
            assert np.array_equal(pd.cpu().numpy().view(np.uint32), od.view(np.uint32)), f"dists, order prefix {op}"
            assert np.array_equal(small["examined"].cpu().numpy(), tp["examined"]), f"examined, order prefix {op}"
            assert np.array_equal(small["last_update"].cpu().numpy(), tp["last_update"]), f"L*, order prefix {op}"
    return {"n_cand": [t["candidates"].size for t in tr], "gpu": g, "taps": tp, "ids": gi, "dists": gd}


def key_stress_rows(d: int = 128):
    """Rows whose distance from the zero query separates the defined key (sum
    over the dimensions in ascending order) from other summation orders.

    Returns {name: row}: with q = 0 the terms are (x_i)^2.
      A  -- 1, then d-1 terms of 2^-54: every term after the first is a
            quarter of an ulp of 1 and is absorbed, so the key is exactly 1;
            an order that first adds the small terms together gives more.
      B  -- 1 + 2^-52 exactly (two terms): above A's key, below A's other sums.
      C  -- 1, 2^-24, then d-2 terms of 2^-54: the key is exactly 1 + 2^-24,
            the float32 midpoint between 1 and 1 + 2^-23, so its float32 value
            is 1 (ties to even); the small terms added first round it up.
    """
    a = np.full(d, -2.0 ** -27, dtype=np.float32)
    a[0] = -1.0
    b = np.zeros(d, dtype=np.float32)
    b[0] = -1.0
    b[1] = -2.0 ** -26
    c = np.full(d, -2.0 ** -27, dtype=np.float32)
    c[0] = -1.0
    c[1] = -2.0 ** -12
    return {"A": a, "B": b, "C": c}


# ---------------------------------------------------------------------------
# The oracle on many queries at full size: worker processes (new interpreters,
# numpy and the oracle only) over the index arrays memory-mapped from files.
# ---------------------------------------------------------------------------
def oracle_pool(n: int = 0):
    import multiprocessing as mp
    import os
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return mp.get_context("spawn").Pool(n or min(16, avail), initializer=_pool_init)


def _pool_init():
    import os
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _mapped(paths, meta):
    index = dict(meta)
    for name, path in paths.items():
        index[name] = None if path is None else np.load(path, mmap_mode="r")
    return index


def _oracle_one(task):
    from oracle import mlp as omlp
    paths, meta, q, k, okw, feats = task
    index = _mapped(paths, meta)
    ids, dists, tr = oquery.search(index, q[None, :], k, trace=True, **okw)
    t = tr[0]
    rec = {"ids": ids[0], "dists": dists[0], "q_rot": t["q_rot"], "tau_eff": t["tau_eff"],
           "candidates": np.asarray(t["candidates"]), "examined": t["examined"]}
    if okw["mode"] == 1:
        rec.update(order=np.asarray(t["order"]), last_update=t["last_update"], stopped=t["stop"] is not None)
        if t.get("hamming") is not None:
            rec["hamming"] = np.asarray(t["hamming"])
        if feats:
            rec["features"] = omlp.features(index, t, k)
    return rec


def oracle_many(pool, paths, meta, q: np.ndarray, k: int, feats=False, limits=None, **okw):
    """oracle traces of every row of q (one task per query)."""
    tasks = []
    for i in range(q.shape[0]):
        kw = dict(okw)
        if limits is not None and int(limits[i]) >= 1:
            kw["limits"] = np.array([int(limits[i])])
        tasks.append((paths, meta, q[i], k, kw, feats))
    return pool.map(_oracle_one, tasks, chunksize=1)
