#!/usr/bin/env python3
"""Throughput of the CRISP query engine on one MI355X.

Workload (default): N = 1,000,000 float32 points, D = 4096, strongly
correlated Gaussian mixture (global rank-64 covariance + 0.05 I noise, 100
components; the correlation check fires and the index is rotated), M = 32
subspaces, K = 50 centroids per half, 10,000 queries per batch, k = 10.
Data, queries and index are generated and built on the GPU (seeded); the
timed region starts with everything resident in HBM.

A step is one search over the whole 10,000-query batch (every stage of the
hot path).  Three forms are timed: plain (float32 rows), bf16 (certified
bfloat16 first pass; identical results) and, in Optimized Mode, learned_bf16
(the learned verification budget trained beforehand on 200,000 separate
queries, plus the bfloat16 pass).  The headline value is the fastest form
whose recall@10 is at least 0.90; every form is listed under "forms".
Prints one JSON line; see ``--help`` for the knobs.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/s at recall@10>=0.90 (N=1M, D=4096), plain vs learned/BF16; HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="d4096")
    ap.add_argument("--n", type=int, default=0, help="override N (smaller dry runs)")
    ap.add_argument("--nq", type=int, default=0, help="override the batch size")
    ap.add_argument("--mode", type=int, default=1, help="0 Guaranteed, 1 Optimized")
    ap.add_argument("--alpha", type=float, default=0.002)
    ap.add_argument("--tau", type=int, default=16)
    ap.add_argument("--patience", type=int, default=40)
    ap.add_argument("--max-chunk", type=int, default=4096,
                    help="queries per chunk (4096: two pipelines of N-sized per-query buffers fill most of HBM)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--guaranteed", type=int, default=1, help="also time Guaranteed Mode (plain and bf16)")
    ap.add_argument("--scoring", type=int, default=1,
                    help="also time the tuned form with certified bfloat16 matrix-core pre-scoring (precision 2)")
    ap.add_argument("--tuned-patience", type=int, default=10,
                    help="also time the bf16 form at this patience factor (0 = skip)")
    ap.add_argument("--overlap", type=int, default=1,
                    help="two chunk pipelines on two streams (the per-kernel roofline pass always runs with one)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-oracle time budget (0 = skip)")
    ap.add_argument("--train-queries", type=int, default=200_000,
                    help="queries the learned budget is trained on (0 = no learned form)")
    ap.add_argument("--train-seed", type=int, default=3004)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--uneven-workload", default="d3072",
                    help="workload of the uneven-batch section ('' = skip)")
    ap.add_argument("--uneven-queries", type=int, default=50_000)
    ap.add_argument("--autotune-cache", default="",
                    help="JSON file the uneven-batch tuner reuses and extends ('' = tune afresh, keep nothing)")
    ap.add_argument("--floor", type=float, default=0.998,
                    help="fraction of the plain top-k the learned budget must keep on held-out queries")
    return ap.parse_args()


def ground_truth(base, qrot, k, chunk=256, pool=64):
    """Exact k nearest neighbours of the rotated queries among the stored rows
    (measurement only): float32 GEMM shortlist of `pool` ids per query,
    re-scored in float64 and ordered by (distance, id)."""
    import torch
    xn = torch.empty(base.shape[0], dtype=torch.float64, device=base.device)
    for r0 in range(0, base.shape[0], 1 << 16):
        xn[r0:r0 + (1 << 16)] = (base[r0:r0 + (1 << 16)].double() ** 2).sum(1)
    xn32 = xn.float()
    out = torch.empty(qrot.shape[0], k, dtype=torch.int64, device=base.device)
    for q0 in range(0, qrot.shape[0], chunk):
        q = qrot[q0:q0 + chunk]
        approx = xn32[None, :] - 2.0 * (q @ base.T)
        cand = torch.topk(approx, pool, dim=1, largest=False).indices
        cand = torch.sort(cand, dim=1).values                      # ascending id
        exact = ((base[cand].double() - q.double()[:, None, :]) ** 2).sum(-1)
        order = torch.sort(exact, dim=1, stable=True).indices      # (distance, id)
        out[q0:q0 + chunk] = cand.gather(1, order)[:, :k]
    return out


def recall(found, truth):
    import torch
    k = truth.shape[1]
    hit = (found[:, :, None] == truth[:, None, :]).any(-1).sum().item()
    return hit / float(truth.shape[0] * k)


COPY_PROBE_BYTES = 1 << 30


def copy_probe():
    """One plain device-to-device copy of 1 GiB (outside the timed region):
    the reference a hardware-counter run scales FETCH_SIZE / WRITE_SIZE by."""
    import ctypes
    import torch
    from paper_2603_05180_amd._lib import check, lib
    src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    check(lib.crisp_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), COPY_PROBE_BYTES,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    del src, dst


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when it was taken on other kernel sources or another kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    ent = t.get(kernel)
    from paper_2603_05180_amd.provenance import source_hash
    if not ent or ent.get("source_hash") != source_hash() or ent.get("workload") != workload:
        return None
    return round(ent["fetch_bytes_per_launch"] + ent["write_bytes_per_launch"], 1)


def timed(index, queries, k, kw, steps, ids, dists, profile=False):
    """K searches of the whole batch between two HIP events on the current stream."""
    import torch
    if profile:
        index.profile_begin(16384)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        index.search(queries, k, out=(ids, dists), **kw)
    ev1.record()
    torch.cuda.synchronize()
    stages = index.profile_end() if profile else None
    return ev0.elapsed_time(ev1) / steps, stages


def counts(index, queries, k, kw):
    """Per-step totals of the work the search did (identical in every run)."""
    import torch
    nq, m = queries.shape[0], index.m
    dev = queries.device
    taps = {"examined": torch.empty(nq, dtype=torch.int32, device=dev),
            "refined": torch.empty(nq, dtype=torch.int32, device=dev),
            "n_cand": torch.empty(nq, dtype=torch.int32, device=dev),
            "retrieved": torch.empty(nq, m, dtype=torch.int32, device=dev)}
    index.search(queries, k, taps=taps, **kw)
    torch.cuda.synchronize()
    return {key: int(v.long().sum()) for key, v in taps.items()}


def fp64_error(base, qrot, ids, dists):
    """max |d_returned - d_fp64| / d_fp64 over every returned result."""
    import torch
    worst = 0.0
    for q0 in range(0, ids.shape[0], 512):
        i = ids[q0:q0 + 512]
        ok = i >= 0
        rows = base[i.clamp(min=0)].double()
        d64 = ((rows - qrot[q0:q0 + 512].double()[:, None, :]) ** 2).sum(-1)
        rel = ((dists[q0:q0 + 512].double() - d64).abs() / d64.clamp(min=1e-300))[ok]
        if rel.numel():
            worst = max(worst, float(rel.max()))
    return worst


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the engine shards by query batch; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import synth.gpu as sg
    from paper_2603_05180_amd import engine, learned

    w = synth.WORKLOADS[args.workload]
    if args.n:
        w = w.scaled(n=args.n)
    if args.nq:
        w = w.scaled(n_query=args.nq)
    dev = torch.device("cuda:0")
    t = time.time()
    arrays, params = build_gpu_index(w)
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    torch.cuda.synchronize()
    log(f"data {w.n}x{w.d} generated and indexed on the GPU in {time.time() - t:.1f}s (CEV {arrays['cev']:.3f}, "
        f"rotated={arrays['rotation'] is not None})")
    index = engine.Index(arrays, tile_ids=args.tile)
    index.enable_bf16()
    k = w.k
    base_kw = dict(mode=args.mode, alpha=args.alpha, tau=args.tau, patience_factor=args.patience,
                   max_chunk=args.max_chunk, overlap=args.overlap)

    # Rotated queries (same kernel as the search) for the exact ground truth.
    qrot = engine.rotate_rows(queries, arrays["rotation"]) if arrays["rotation"] is not None else queries
    t = time.time()
    truth = ground_truth(arrays["base"], qrot, k)
    torch.cuda.synchronize()
    log(f"ground truth in {time.time() - t:.1f}s")

    # Learned verification budget (Optimized Mode): trained on separate
    # queries of the same mixture with the engine's own kernels, before timing.
    model = None
    if args.mode == 1 and args.train_queries > 0:
        t = time.time()
        trainq = sg.rows(w, args.train_seed, 0, args.train_queries, params)
        model = learned.train_budget(index, trainq, k, alpha=args.alpha, tau=args.tau,
                                     patience_factor=args.patience, epochs=args.epochs, floor=args.floor)
        del trainq
        torch.cuda.synchronize()
        log(f"budget model trained on {args.train_queries} queries in {time.time() - t:.1f}s "
            f"(delta {model.delta:.3f})")

    forms = {"plain": dict(precision=0), "bf16": dict(precision=1)}
    if model is not None:
        forms["learned_bf16"] = dict(precision=1, budget_source=1)
    if args.mode == 1 and args.tuned_patience > 0:
        # a tuned operating point: the same engine with a shorter patience
        forms[f"bf16_pf{args.tuned_patience}"] = dict(precision=1, patience_factor=args.tuned_patience)
        if args.scoring:
            # and with the half distances pre-scored on bfloat16 matrix cores (same results)
            forms[f"bf16_scored_pf{args.tuned_patience}"] = dict(precision=2, patience_factor=args.tuned_patience)
    if args.mode == 1 and args.guaranteed:
        # Guaranteed Mode (every candidate verified) at the same alpha and tau
        forms["guaranteed"] = dict(mode=0, precision=0)
        forms["guaranteed_bf16"] = dict(mode=0, precision=1)
    ids = torch.empty(w.n_query, k, dtype=torch.int64, device=dev)
    dists = torch.empty(w.n_query, k, dtype=torch.float32, device=dev)
    plain_ids = None
    results = {}
    for name, extra in forms.items():
        kw = dict(base_kw, **extra)
        for _ in range(args.warmup):
            index.search(queries, k, out=(ids, dists), **kw)
        torch.cuda.synchronize()
        rec = recall(ids, truth)
        if plain_ids is None:
            plain_ids = ids.clone()
        same = float((ids[:, :, None] == plain_ids[:, None, :]).any(-1).float().mean())
        ms, _ = timed(index, queries, k, kw, args.steps, ids, dists)
        c = counts(index, queries, k, dict(kw, overlap=0))
        # re-rank gather rate of this form: one single-pipeline step, stage-timed
        _, st1 = timed(index, queries, k, dict(kw, overlap=0), 1, ids, dists, profile=True)
        rr_bytes = (((2.0 * w.d + 4.0) * c["examined"] + 4.0 * w.d * c["refined"]) if kw.get("precision", 0) >= 1
                    else 4.0 * w.d * c["examined"])
        results[name] = {"queries_per_s": round(w.n_query / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                         "recall_at_10": round(rec, 4), "plain_ids_kept": round(same, 5),
                         "mean_verified": round(c["examined"] / w.n_query, 1),
                         "mean_float32_rows": round(c["refined"] / w.n_query, 1),
                         "rerank_gb_s": round(rr_bytes / 1e9 / (st1["rerank"]["ms"] / 1e3), 1),
                         "max_rel_err_vs_fp64": fp64_error(arrays["base"], qrot, ids, dists),
                         "_kw": kw, "_counts": c}
        log(f"form {name}: {results[name]['queries_per_s']} q/s, recall {rec:.4f}, "
            f"verified {results[name]['mean_verified']}, float32 rows {results[name]['mean_float32_rows']}, "
            f"re-rank {results[name]['rerank_gb_s']} GB/s")

    # Headline: the fastest form at recall@10 >= 0.90.
    ok = [f for f in results if results[f]["recall_at_10"] >= 0.90] or list(results)
    head = max(ok, key=lambda f: results[f]["queries_per_s"])
    kw, c = results[head]["_kw"], results[head]["_counts"]
    ms_step = results[head]["ms_per_step"]
    qps = results[head]["queries_per_s"]
    # Per-kernel roofline: the same form timed stage by stage with one chunk
    # pipeline, so that no other kernel shares the GPU during a launch.
    copy_probe()
    _, stages = timed(index, queries, k, dict(kw, overlap=0), args.steps, ids, dists, profile=True)

    # ---- roofline of each stage (algorithmic bytes / flops per step) --------
    d = w.d
    bf16 = kw.get("precision", 0) >= 1
    rerank_bytes = ((2.0 * d + 4.0) * c["examined"] + 4.0 * d * c["refined"]) if bf16 else 4.0 * d * c["examined"]
    per_step = {
        "rotate": ("mfma", 2.0 * d * d * w.n_query / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"),
        # first counting pass: every retrieved id read once, every candidate (id, score) written once
        "count": ("hbm", (4.0 * c["retrieved"] + 5.0 * c["n_cand"]) / 1e9, HBM_PEAK_GBS, "GB/s"),
        "hamming_dist": ("hbm", (d / 8.0 + 8.0) * c["n_cand"] / 1e9, HBM_PEAK_GBS, "GB/s"),
        "rerank": ("hbm", rerank_bytes / 1e9, HBM_PEAK_GBS, "GB/s"),
    }
    stage_out = {}
    for name, rec_s in stages.items():
        if name == "dropped" or rec_s["intervals"] == 0:
            continue
        ms = rec_s["ms"] / args.steps
        ent = {"ms_per_step": round(ms, 4), "launches_per_step": rec_s["intervals"] / args.steps}
        if name in per_step:
            bound, amount, peak, unit = per_step[name]
            ach = amount / (ms / 1e3)
            ent.update(bound=bound, achieved=round(ach, 2), peak=peak, unit=unit, frac=round(ach / peak, 4))
        stage_out[name] = ent
    dom = max((s for s in stage_out if s in per_step), key=lambda s: stage_out[s]["ms_per_step"])
    launches = stage_out[dom]["launches_per_step"]
    kernel_of = {"rerank": "k_rerank", "count": "k_count<0>", "rotate": "k_rotate_rows",
                 "hamming_dist": "k_hamming_dist"}
    roof = {"kernel": kernel_of[dom],
            "bound": per_step[dom][0], "achieved": stage_out[dom]["achieved"], "peak": per_step[dom][2],
            "unit": per_step[dom][3], "frac": stage_out[dom]["frac"],
            "traffic": measured_traffic(kernel_of[dom], w.name),
            "avg_launch_ms": round(stage_out[dom]["ms_per_step"] / launches, 4),
            "algorithmic_per_launch": round(per_step[dom][1] / launches, 4)}
    if "rerank" in stage_out:
        roof["rerank_gather"] = {k_: stage_out["rerank"][k_] for k_ in ("achieved", "peak", "unit", "frac")}

    # ---- CPU oracle baseline on a bounded sample of the same workload --------
    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(arrays, queries, k, base_kw, args.cpu_seconds)

    for f in results.values():
        f.pop("_kw"); f.pop("_counts")
    rotated = arrays["rotation"] is not None
    line = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+bf16" if bf16 else "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.n} D={w.d} correlated Gaussian mixture ({w.kind} rank {w.rank}, "
                               f"{w.n_comp} comps), M={w.m} K={w.k_half}, {w.n_query} queries/batch, k={k}",
                   "mode": "optimized" if kw.get("mode", args.mode) == 1 else "guaranteed",
                   "alpha": args.alpha, "tau": args.tau,
                   "patience_factor": kw.get("patience_factor", args.patience),
                   "recall_at_10": results[head]["recall_at_10"],
                   "overlap": args.overlap, "queries_per_chunk": base_kw["max_chunk"],
                   "rotated": rotated,
                   "mean_candidates": round(c["n_cand"] / w.n_query, 1),
                   "mean_verified": round(c["examined"] / w.n_query, 1), "form": head,
                   "learned_delta": None if model is None else round(model.delta, 4),
                   "learned_train_queries": args.train_queries if model is not None else 0},
        "forms": results,
        "roofline": roof,
        "stages": stage_out,
        "cpu_baseline": cpu,
    }

    # ---- uneven batches (served through the tuned batch executor) ------------
    if args.uneven_workload:
        del index, arrays, queries, qrot, truth, ids, dists, plain_ids, model
        torch.cuda.empty_cache()
        line["uneven_batching"] = uneven_batches(args)
    print(json.dumps(line), flush=True)


def build_gpu_index(w):
    """Seeded data of workload w generated and indexed on the GPU."""
    import numpy as np
    import synth
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    params = sg.mixture_params(w)
    x = sg.rows(w, w.seed_data, 0, w.n, params)
    n = w.n
    cev_rows = synth.sample_indices(w.seed_index, synth.TAG["cev_sample"], n, max(2, min(n // 10, 100_000)))
    km_rows = synth.sample_indices(w.seed_index, synth.TAG["kmeans_sample"], n, min(n, 100_000))
    km_init = synth.permutation_prefix(w.seed_index, synth.TAG["kmeans_init"], np.arange(km_rows.size), w.k_half)
    arrays = engine.build_index(x, w.m, w.k_half, g=lambda: sg.gaussian_matrix(w.seed_index, w.d),
                                cev_rows=cev_rows, km_rows=km_rows, km_init=km_init, keep_input=False)
    return arrays, params


def uneven_batches(args):
    """Seeded batches of 1..4096 queries (log-uniform), k in {1, 10, 100},
    served by the batch executor with the learned budget and the bfloat16
    pass; the tuner picks tile, chunk and re-rank grid per (k, bucket)
    first.  Reports per-batch GPU latency percentiles and throughput."""
    import numpy as np
    import torch
    import synth
    import synth.gpu as sg
    from paper_2603_05180_amd import autotune, engine, learned

    w = synth.WORKLOADS[args.uneven_workload]
    t = time.time()
    arrays, params = build_gpu_index(w)
    torch.cuda.synchronize()
    log(f"uneven: {w.name} index N={w.n} D={w.d} built in {time.time() - t:.1f}s")
    index = engine.Index(arrays)
    index.enable_bf16()
    kw = dict(alpha=args.alpha, tau=args.tau, patience_factor=args.patience)
    model = None
    if args.train_queries > 0:
        trainq = sg.rows(w, args.train_seed, 0, args.train_queries, params)
        model = learned.train_budget(index, trainq, 10, epochs=args.epochs, floor=args.floor, **kw)
        del trainq
        torch.cuda.empty_cache()
    queries = sg.rows(w, w.seed_query, 0, args.uneven_queries, params)
    sizes = synth.batch_sizes(w.seed_query, args.uneven_queries, max_batch=4096)
    ks = synth.batch_ks(w.seed_query, len(sizes))
    sp = dict(kw, mode=1, precision=1, budget_source=1 if model is not None else 0)
    t = time.time()
    srv = autotune.Server(None, index, sp, max_batch=4096, ks=(1, 10, 100), tiles=(16384, 65536),
                          chunks=(512, 1024))
    choice = srv.tune(queries, [1 << i for i in range(13)], reps=2, cache=args.autotune_cache or None)
    torch.cuda.synchronize()
    log(f"uneven: tuned {len(choice)} (k, bucket) pairs in {time.time() - t:.1f}s")
    srv.run(queries, sizes[:8], ks[:8])                   # first replays of the common buckets
    torch.cuda.synchronize()
    t0 = time.time()
    lat, outs = srv.run(queries, sizes, ks)
    wall = time.time() - t0
    lat = np.asarray(lat)
    # recall@10 on the batches with k >= 10, a sample of them
    qrot = engine.rotate_rows(queries[:5000], arrays["rotation"]) if arrays["rotation"] is not None \
        else queries[:5000]
    truth = ground_truth(arrays["base"], qrot, 10)
    hit = tot = 0
    o = 0
    for (ids, _), nq, k in zip(outs, sizes, ks):
        if k >= 10 and o < 5000:
            m = min(nq, 5000 - o)
            found = ids[:m, :10]
            hit += int((found[:, :, None] == truth[o:o + m, None, :]).any(-1).sum())
            tot += m * 10
        o += nq
    tuned = {}
    for (k, b), (tile, chunk, pers) in sorted(choice.items()):
        tuned[f"k{k}_b{b}"] = [tile, chunk, pers]
    out = {"workload": f"{w.name}: N={w.n} D={w.d} correlated Gaussian mixture ({w.kind} rank {w.rank}, "
                       f"{w.n_comp} comps), M={w.m} K={w.k_half}",
           "queries": int(sum(sizes)), "batches": len(sizes), "batch_sizes": "log-uniform in [1, 4096]",
           "k": "uniform over {1, 10, 100}", "form": "learned_bf16" if model is not None else "bf16",
           "queries_per_s": round(sum(sizes) / (lat.sum() / 1e3), 1),
           "queries_per_s_wall": round(sum(sizes) / wall, 1),
           "p50_batch_ms": round(float(np.percentile(lat, 50)), 4),
           "p99_batch_ms": round(float(np.percentile(lat, 99)), 4),
           "max_batch_ms": round(float(lat.max()), 4),
           "recall_at_10_sample": round(hit / max(1, tot), 4),
           "tuned_tile_chunk_persistent": tuned}
    log(f"uneven: {out['queries_per_s']} q/s, p50 {out['p50_batch_ms']} ms, p99 {out['p99_batch_ms']} ms")
    srv.free()
    index.free()
    return out


def cpu_baseline(arrays, queries, k, kw, budget_s):
    """The CPU oracle's query engine, timed on the host cores on the first S
    queries of the batch against the same index arrays (timing only)."""
    import numpy as np
    import torch
    from oracle import query as oquery

    t = time.time()
    host = {"n": arrays["n"], "d": arrays["d"], "m": arrays["m"], "k_half": arrays["k_half"],
            "rotation": None if arrays["rotation"] is None else arrays["rotation"].cpu().numpy(),
            "centroids": arrays["centroids"].cpu().numpy(), "offsets": arrays["offsets"].cpu().numpy(),
            "ids": arrays["ids"].cpu().numpy(), "base": arrays["base"].cpu().numpy(),
            "codes": arrays["codes"].cpu().numpy().view(np.uint64)}
    qh = queries[:512].cpu().numpy()
    log(f"host copy of the index for the CPU baseline in {time.time() - t:.1f}s")
    okw = dict(mode=kw["mode"], alpha=kw["alpha"], tau=kw["tau"], patience_factor=kw["patience_factor"])
    t0 = time.time()
    oquery.search(host, qh[:1], k, **okw)
    per_q = max(1e-3, time.time() - t0)
    s = int(max(2, min(qh.shape[0], budget_s / per_q)))
    t0 = time.time()
    oquery.search(host, qh[:s], k, **okw)
    el = time.time() - t0
    log(f"CPU oracle: {s} queries in {el:.1f}s")
    return {"value": round(s / el, 3), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"first {s} queries of the batch through the oracle query engine (oracle/query.py, "
                      f"one process, numpy) against the same index arrays"}


if __name__ == "__main__":
    main()
