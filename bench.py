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

Also measured (each section can be switched off): a patience-factor sweep of
the bf16 form, which places the learned form against the plain walk at
matched recall; the ablations of Section 6.4 on this workload (Optimized
Mode without the Hamming order; the correlation-check threshold, i.e. the
index with and without its rotation); an alpha x tau operating-point grid;
the N = 1M, D = 960 workload (K = 16 centroids per half) in both modes at
k = 10 and 100; uneven batches on N = 2M, D = 3072; and the CPU oracle on
the host cores, timed in worker processes forked before this process first
touches the GPU.
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
    ap.add_argument("--max-candidates", type=int, default=0,
                    help="candidate-list capacity per query (0: N); queries with more are searched again uncapped")
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
    ap.add_argument("--patience-sweep", default="5,20,30,60",
                    help="extra patience factors of the bf16 form ('' = none; 10 and 40 are always timed)")
    ap.add_argument("--ads", type=int, default=1, help="also time ADSampling verification (Optimized Mode)")
    ap.add_argument("--ablations", type=int, default=1,
                    help="Section 6.4 ablations: Hamming order off, correlation-check threshold")
    ap.add_argument("--grid", type=int, default=1, help="alpha x tau operating-point grid of the head form")
    ap.add_argument("--d960", type=int, default=1, help="time the N=1M, D=960 (K=16) workload, both modes")
    ap.add_argument("--overlap-grid", type=int, default=1,
                    help="alpha x tau grid on the N=1M, D=1024 mixture with overlapping components")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="CPU oracle worker processes (0 = the host cores, at most 16)")
    ap.add_argument("--label-check", type=int, default=32,
                    help="training queries whose learned-budget labels are checked against the oracle's trace")
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
            "retrieved": torch.empty(nq, m, dtype=torch.int32, device=dev),
            "row_bytes": torch.empty(nq, dtype=torch.int64, device=dev)}
    if kw.get("precision", 0) >= 2:
        # subspaces whose centroid scores could not be certified (exact path)
        taps["score_fallback"] = torch.empty(nq, dtype=torch.int32, device=dev)
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


def stage_rates(stages, steps, per_step, workload):
    """Per-stage time and rate.  A byte-bound stage whose algorithmic bytes
    arrive faster than HBM can deliver them is served from L2 / the
    last-level cache: it is labelled so, with no HBM fraction from the
    algorithmic bytes; its HBM fraction then comes only from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE per launch), when that summary
    was taken on the current kernel sources."""
    kernel_of = {"rerank": "k_rerank", "count": "k_count<0>", "rotate": "k_rotate_rows",
                 "hamming_dist": "k_hamming_dist"}
    out = {}
    for name, rec_s in stages.items():
        if name == "dropped" or rec_s["intervals"] == 0:
            continue
        ms = rec_s["ms"] / steps
        launches = rec_s["intervals"] / steps
        ent = {"ms_per_step": round(ms, 4), "launches_per_step": launches}
        if name in per_step:
            bound, amount, peak, unit = per_step[name]
            ach = amount / (ms / 1e3)
            ent.update(bound=bound, achieved=round(ach, 2), peak=peak, unit=unit, frac=round(ach / peak, 4),
                       algorithmic_per_launch=round(amount / launches, 4))
            if bound == "hbm":
                traffic = measured_traffic(kernel_of[name], workload)
                if traffic is not None:
                    ent["hbm_bytes_per_launch"] = traffic
                    ent["hbm_frac_measured"] = round(traffic / ((ms / launches) / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                if ach > peak:
                    ent["bound"] = "l2/mall"
                    ent["frac"] = None
                    ent["note"] = ("algorithmic bytes above what HBM delivers: served from cache; "
                                   "HBM share only from counters")
        out[name] = ent
    return out, kernel_of


def rerank_bytes_of(kw, c, d):
    """Algorithmic bytes of stored rows the verification needs per step:
    the verified prefix in float32, or in bfloat16 (+ a 4-byte bound) plus
    the float32 rows the bounds kept; with ADSampling the rows as far as the
    kernel read them (its row-byte count: each pruned row to the end of the
    256-dimension block pair where the test fired)."""
    if kw.get("verify", 0) == 1:
        return float(c["row_bytes"])
    if kw.get("precision", 0) >= 1:
        return (2.0 * d + 4.0) * c["examined"] + 4.0 * d * c["refined"]
    return 4.0 * d * c["examined"]


def run_form(index, queries, truth, k, kw, args, ids, dists, plain_ids, base, qrot, d):
    """Warm up, time, count and stage-profile one form; returns its record."""
    import torch
    for _ in range(args.warmup):
        index.search(queries, k, out=(ids, dists), **kw)
    torch.cuda.synchronize()
    rec = recall(ids, truth)
    same = None
    if plain_ids is not None:
        same = round(float((ids[:, :, None] == plain_ids[:, None, :]).any(-1).float().mean()), 5)
    ms, _ = timed(index, queries, k, kw, args.steps, ids, dists)
    c = counts(index, queries, k, dict(kw, overlap=0))
    _, st1 = timed(index, queries, k, dict(kw, overlap=0), 1, ids, dists, profile=True)
    rr_bytes = rerank_bytes_of(kw, c, d)
    nq = queries.shape[0]
    return {"queries_per_s": round(nq / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
            "recall_at_k": round(rec, 4), "plain_ids_kept": same,
            "mean_verified": round(c["examined"] / nq, 1),
            "mean_float32_rows": round(c["refined"] / nq, 1),
            "mean_candidates": round(c["n_cand"] / nq, 1),
            "mean_row_bytes_read": round(c["row_bytes"] / nq, 1),
            "rerank_algorithmic_gb_s": round(rr_bytes / 1e9 / (st1["rerank"]["ms"] / 1e3), 1),
            "max_rel_err_vs_fp64": fp64_error(base, qrot, ids, dists),
            **({"exact_scoring_subspace_frac": round(c["score_fallback"] / (nq * index.m), 5)}
               if "score_fallback" in c else {}),
            "_kw": kw, "_counts": c}


def matched_recall(results, learned="learned_bf16"):
    """The learned form against the plain bf16 walk at the learned form's
    recall: the plain patience sweep's queries/s interpolated (linearly in
    recall) between the two sweep points around that recall."""
    if learned not in results:
        return None
    sweep = sorted(((r["_kw"]["patience_factor"], r) for f, r in results.items()
                    if f.startswith("bf16_pf") or f == "bf16"), key=lambda t: t[0])
    pts = sorted({(r["recall_at_k"], r["queries_per_s"], pf) for pf, r in sweep})
    lr, lq = results[learned]["recall_at_k"], results[learned]["queries_per_s"]
    above = [p for p in pts if p[0] >= lr]
    below = [p for p in pts if p[0] < lr]
    out = {"learned": {"recall_at_10": lr, "queries_per_s": lq,
                       "mean_verified": results[learned]["mean_verified"]},
           "plain_sweep": [{"patience_factor": pf, "recall_at_10": r["recall_at_k"],
                            "queries_per_s": r["queries_per_s"], "mean_verified": r["mean_verified"]}
                           for pf, r in sweep]}
    if not above:
        out["outcome"] = "the plain sweep does not reach the learned form's recall"
        return out
    hi = min(above, key=lambda p: p[0])
    if below:
        lo = max(below, key=lambda p: p[0])
        t = (lr - lo[0]) / (hi[0] - lo[0]) if hi[0] > lo[0] else 1.0
        q_plain = lo[1] + t * (hi[1] - lo[1])
    else:
        q_plain = hi[1]
    gain = lq / q_plain - 1.0
    out["plain_queries_per_s_at_learned_recall"] = round(q_plain, 1)
    out["learned_gain"] = round(gain, 4)
    out["outcome"] = ("learned beats the plain walk at matched recall" if gain > 0.01 else
                      "no gain: the plain walk with a tuned patience is as fast at this recall")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the engine shards by query batch; see the design notes)", file=sys.stderr)
        sys.exit(2)
    # The CPU oracle's workers are forked now, before anything touches the GPU.
    pool = start_cpu_pool(args.cpu_workers) if args.cpu_seconds > 0 else None
    try:
        line = measure(args, pool)
    finally:
        if pool is not None:
            pool.terminate()
            pool.join()
    print(json.dumps(line), flush=True)


def measure(args, pool):
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
                   max_chunk=args.max_chunk, overlap=args.overlap, max_candidates=args.max_candidates)

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
            # and on FP8 (e4m3) matrix cores, two-term split (same results; more exact-path subspaces)
            forms[f"fp8_scored_pf{args.tuned_patience}"] = dict(precision=3, patience_factor=args.tuned_patience)
    if args.mode == 1 and args.ads:
        # ADSampling verification (float32 rows read only as far as Eq. (2) needs)
        forms["ads"] = dict(precision=0, verify=1)
        if args.tuned_patience > 0:
            forms[f"ads_pf{args.tuned_patience}"] = dict(precision=0, verify=1, patience_factor=args.tuned_patience)
    if args.mode == 1:
        for pf in [int(v) for v in args.patience_sweep.split(",") if v.strip()]:
            forms.setdefault(f"bf16_pf{pf}", dict(precision=1, patience_factor=pf))
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
        results[name] = run_form(index, queries, truth, k, kw, args, ids, dists, plain_ids, arrays["base"], qrot,
                                 w.d)
        if plain_ids is None:
            plain_ids = ids.clone()
            results[name]["plain_ids_kept"] = 1.0
        r = results[name]
        log(f"form {name}: {r['queries_per_s']} q/s, recall {r['recall_at_k']:.4f}, verified {r['mean_verified']}, "
            f"float32 rows {r['mean_float32_rows']}, re-rank {r['rerank_algorithmic_gb_s']} GB/s algorithmic")

    # Headline: the fastest form at recall@10 >= 0.90.
    ok = [f for f in results if results[f]["recall_at_k"] >= 0.90] or list(results)
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
    rerank_bytes = rerank_bytes_of(kw, c, d)
    per_step = {
        "rotate": ("mfma", 2.0 * d * d * w.n_query / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"),
        # first counting pass: every retrieved posting entry read once (its
        # 2-byte counter position), every candidate (id, score) written once
        "count": ("hbm", (2.0 * c["retrieved"] + 5.0 * c["n_cand"]) / 1e9, HBM_PEAK_GBS, "GB/s"),
        "hamming_dist": ("hbm", (d / 8.0 + 8.0) * c["n_cand"] / 1e9, HBM_PEAK_GBS, "GB/s"),
        "rerank": ("hbm", rerank_bytes / 1e9, HBM_PEAK_GBS, "GB/s"),
    }
    if arrays["rotation"] is None:
        per_step.pop("rotate")
    stage_out, kernel_of = stage_rates(stages, args.steps, per_step, w.name)
    cands = [s_ for s_ in stage_out if s_ in per_step and stage_out[s_].get("frac") is not None]
    dom = max(cands, key=lambda s_: stage_out[s_]["ms_per_step"])
    launches = stage_out[dom]["launches_per_step"]
    roof = {"kernel": kernel_of[dom],
            "bound": per_step[dom][0], "achieved": stage_out[dom]["achieved"], "peak": per_step[dom][2],
            "unit": per_step[dom][3], "frac": stage_out[dom]["frac"],
            "traffic": measured_traffic(kernel_of[dom], w.name),
            "avg_launch_ms": round(stage_out[dom]["ms_per_step"] / launches, 4),
            "algorithmic_per_launch": round(per_step[dom][1] / launches, 4)}
    if "rerank" in stage_out:
        rr = stage_out["rerank"]
        roof["rerank_gather"] = {"achieved_algorithmic": rr["achieved"], "peak": rr["peak"], "unit": rr["unit"],
                                 "frac_algorithmic": rr["frac"],
                                 "hbm_frac_measured": rr.get("hbm_frac_measured")}

    # ---- the learned form against the plain walk at matched recall --------
    mr = matched_recall(results)

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
                   "recall_at_10": results[head]["recall_at_k"],
                   "overlap": args.overlap, "queries_per_chunk": base_kw["max_chunk"],
                   "rotated": rotated,
                   "mean_candidates": round(c["n_cand"] / w.n_query, 1),
                   "mean_verified": round(c["examined"] / w.n_query, 1), "form": head,
                   "learned_delta": None if model is None else round(model.delta, 4),
                   "learned_train_queries": args.train_queries if model is not None else 0},
        "forms": results,
        "learned_vs_plain_at_matched_recall": mr,
        "roofline": roof,
        "stages": stage_out,
    }

    # ---- Section 6.4 ablation: Optimized Mode without the Hamming order -----
    if args.ablations and args.mode == 1:
        abl = {}
        for pf in sorted({args.tuned_patience or args.patience, args.patience}):
            kwx = dict(base_kw, precision=1, patience_factor=pf)
            r_on = next((results[f] for f in results if results[f]["_kw"] == kwx), None)
            r_off = run_form(index, queries, truth, k, dict(kwx, walk_order=1), args, ids, dists, None,
                             arrays["base"], qrot, d)
            ent = {"patience_factor": pf,
                   "hamming_order": None if r_on is None else {x_: r_on[x_] for x_ in
                                                               ("queries_per_s", "recall_at_k", "mean_verified")},
                   "id_order": {x_: r_off[x_] for x_ in ("queries_per_s", "recall_at_k", "mean_verified")}}
            if r_on is not None:
                ent["throughput_without_hamming_rel"] = round(r_off["queries_per_s"] / r_on["queries_per_s"], 4)
            abl[f"pf{pf}"] = ent
            log(f"ablation hamming off pf{pf}: {r_off['queries_per_s']} q/s, recall {r_off['recall_at_k']:.4f}")
        line["ablation_hamming_order"] = abl

    # ---- operating-point grid: alpha x tau (tau = ceil(beta M)) -------------
    if args.grid:
        grid = []
        for alpha in (0.002, 0.005, 0.01, 0.02, 0.04, 0.06):
            for beta in (0.1, 0.2, 0.3, 0.4, 0.5, 0.6):
                tau = int(math.ceil(beta * w.m))
                kwg = dict(kw, alpha=alpha, tau=tau)
                for _ in range(1):
                    index.search(queries, k, out=(ids, dists), **kwg)
                torch.cuda.synchronize()
                rec = recall(ids, truth)
                ms, _ = timed(index, queries, k, kwg, 2, ids, dists)
                grid.append({"alpha": alpha, "beta": beta, "tau": tau, "queries_per_s": round(w.n_query / ms * 1e3, 1),
                             "recall_at_10": round(rec, 4)})
        best = max((g_ for g_ in grid if g_["recall_at_10"] >= 0.90), key=lambda g_: g_["queries_per_s"],
                   default=None)
        line["operating_grid"] = {"form": head, "points": grid, "best_at_recall_0.90": best}
        log(f"grid: best {best}")

    # ---- CPU oracle: baseline on a bounded sample, learned-label check -------
    cpu = None
    if pool is not None:
        import shutil
        t = time.time()
        tmp, paths, meta = export_index(arrays)
        log(f"CPU oracle: index arrays written to {tmp} in {time.time() - t:.1f}s")
        try:
            okw = dict(mode=kw["mode"], alpha=kw["alpha"], tau=kw["tau"], patience_factor=kw["patience_factor"],
                       hamming=kw.get("walk_order", 0) == 0)
            cpu = cpu_baseline(pool, paths, meta, queries, k, okw, args.cpu_seconds)
            if model is not None and args.label_check > 0:
                sample = sg.rows(w, args.train_seed, 0, args.label_check, params)
                eng = learned.collect(index, sample, k, alpha=args.alpha, tau=args.tau,
                                      patience_factor=args.patience)
                lk = dict(mode=1, alpha=args.alpha, tau=args.tau, patience_factor=args.patience)
                line["learned_label_check"] = check_labels(pool, paths, meta, sample,
                                                           {x_: eng[x_].cpu() for x_ in
                                                            ("last_update", "examined", "n_cand")}, k, lk)
                log(f"learned labels vs oracle: {line['learned_label_check']}")
        finally:
            shutil.rmtree(tmp, ignore_errors=True)
    line["cpu_baseline"] = cpu

    for f in results.values():
        f.pop("_kw"); f.pop("_counts")
    cev = float(arrays["cev"])
    head_kw = dict(kw)
    index.free()
    del index, arrays, queries, qrot, truth, ids, dists, plain_ids, model
    torch.cuda.empty_cache()

    # ---- Section 6.4 ablation: the correlation-check threshold --------------
    if args.ablations:
        line["ablation_cev_threshold"] = cev_ablation(w, head_kw, cev, head, results[head], args)

    # ---- the N = 1M, D = 960 workload, both modes, k = 10 and 100 -----------
    if args.d960:
        torch.cuda.empty_cache()
        line["d960"] = d960_section(args)

    # ---- alpha x tau on overlapping components (selectivity) ---------------
    if args.overlap_grid:
        torch.cuda.empty_cache()
        line["overlap_grid"] = overlap_grid_section(args)

    # ---- uneven batches (served through the tuned batch executor) ------------
    if args.uneven_workload:
        torch.cuda.empty_cache()
        line["uneven_batching"] = uneven_batches(args)
    return line


def cev_ablation(w, kw, cev, head, head_rec, args):
    """The index built with the rotation decision reversed (Section 6.4:
    the threshold tau_CEV on the correlation check decides whether the data
    are rotated): the head form timed on it.  Every threshold below the
    measured CEV rotates, every threshold at or above it does not."""
    import torch
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    t = time.time()
    rotated = cev > engine.TAU_CEV
    arrays, params = build_gpu_index(w, force_rotation=not rotated)
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays, tile_ids=args.tile)
    index.enable_bf16()
    qrot = engine.rotate_rows(queries, arrays["rotation"]) if arrays["rotation"] is not None else queries
    truth = ground_truth(arrays["base"], qrot, w.k)
    log(f"ablation: index with rotated={arrays['rotation'] is not None} built in {time.time() - t:.1f}s")
    ids = torch.empty(w.n_query, w.k, dtype=torch.int64, device="cuda")
    dists = torch.empty_like(ids, dtype=torch.float32)
    r = run_form(index, queries, truth, w.k, kw, args, ids, dists, None, arrays["base"], qrot, w.d)
    other = {x_: r[x_] for x_ in ("queries_per_s", "recall_at_k", "mean_candidates", "mean_verified")}
    mine = {x_: head_rec[x_] for x_ in ("queries_per_s", "recall_at_k", "mean_verified")}
    variants = {"rotated" if rotated else "not_rotated": dict(mine, form=head),
                "not_rotated" if rotated else "rotated": dict(other, form=head)}
    sweep = [{"tau_cev": tc, "rotated": bool(cev > tc)} for tc in (0.5, 0.7, 0.8, 0.85, 0.9, 0.95, 0.99, 0.999)]
    del index, arrays, queries, qrot, truth
    torch.cuda.empty_cache()
    return {"cev": round(cev, 4), "variants": variants, "threshold_sweep": sweep}


def d960_section(args):
    """The N = 1M, D = 960 workload (100 local rank-32 components, 16
    subspaces of 60 dims, K = 16 centroids per half; the correlation check
    does not fire): both modes at k = 10 and k = 100, 10,000 queries."""
    import torch
    import synth
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w = synth.WORKLOADS["d960"]
    t = time.time()
    arrays, params = build_gpu_index(w)
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays, tile_ids=args.tile)
    index.enable_bf16()
    log(f"d960: index built in {time.time() - t:.1f}s (CEV {arrays['cev']:.3f})")
    out = {"workload": f"{w.name}: N={w.n} D={w.d} local rank {w.rank}, {w.n_comp} comps, M={w.m} K={w.k_half}",
           "rotated": arrays["rotation"] is not None}
    truth100 = ground_truth(arrays["base"], queries, 100, pool=192)
    for k in (10, 100):
        truth = truth100[:, :k].contiguous()
        ids = torch.empty(w.n_query, k, dtype=torch.int64, device="cuda")
        dists = torch.empty(w.n_query, k, dtype=torch.float32, device="cuda")
        for mode, name in ((0, "guaranteed"), (1, "optimized")):
            # operating point: the fastest of a small alpha x tau grid (one
            # timed search each) whose recall@k reaches 0.90
            base = dict(mode=mode, patience_factor=10, precision=1, max_chunk=2048, overlap=1)
            pick, pick_q = None, -1.0
            for alpha in (0.005, 0.01, 0.02, 0.05):
                for tau in ((4, 8, 12) if mode == 0 else (8, 16, 24)):
                    kwg = dict(base, alpha=alpha, tau=tau)
                    index.search(queries, k, out=(ids, dists), **kwg)
                    torch.cuda.synchronize()
                    rec = recall(ids, truth)
                    ms, _ = timed(index, queries, k, kwg, 1, ids, dists)
                    if rec >= 0.90 and w.n_query / ms > pick_q:
                        pick, pick_q = kwg, w.n_query / ms
            kw = pick or dict(base, alpha=0.05, tau=4 if mode == 0 else 8)
            r = run_form(index, queries, truth, k, kw, args, ids, dists, None, arrays["base"], queries, w.d)
            r.pop("_counts")
            r["operating_point"] = {x_: kw[x_] for x_ in ("alpha", "tau", "patience_factor", "precision")}
            r.pop("_kw")
            out[f"{name}_k{k}"] = r
            log(f"d960 {name} k={k}: {r['queries_per_s']} q/s, recall@{k} {r['recall_at_k']:.4f}")
    index.free()
    del index, arrays, queries, truth100
    torch.cuda.empty_cache()
    return out


def overlap_grid_section(args):
    """The N = 1M, D = 1024 mixture whose 100 components overlap (centres at
    scale 0.5 against unit spread in the 64-dim latent space; M = 16,
    K = 50): there the candidate set C (Eq. (1), Section 4.3.2 Stage 1)
    depends on the retrieval budget alpha and the threshold tau, so this
    grid shows the selectivity trade-off that the clustered d4096 data hide.
    Optimized Mode, bfloat16 pass, the paper's default patience 40 k,
    10,000 queries."""
    import torch
    import synth
    import synth.gpu as sg
    from paper_2603_05180_amd import engine
    w = synth.WORKLOADS["d1024mix"]
    t = time.time()
    arrays, params = build_gpu_index(w)
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    index = engine.Index(arrays, tile_ids=args.tile)
    index.enable_bf16()
    qrot = engine.rotate_rows(queries, arrays["rotation"]) if arrays["rotation"] is not None else queries
    truth = ground_truth(arrays["base"], qrot, w.k)
    log(f"overlap grid: {w.name} index built in {time.time() - t:.1f}s (CEV {arrays['cev']:.3f})")
    ids = torch.empty(w.n_query, w.k, dtype=torch.int64, device="cuda")
    dists = torch.empty(w.n_query, w.k, dtype=torch.float32, device="cuda")
    base = dict(mode=1, patience_factor=40, precision=1, max_chunk=2048, overlap=1)
    pts = []
    for alpha in (0.002, 0.005, 0.01, 0.02, 0.05, 0.1):
        for tau in (2, 3, 4, 6, 8, 12):
            kwg = dict(base, alpha=alpha, tau=tau)
            index.search(queries, w.k, out=(ids, dists), **kwg)
            torch.cuda.synchronize()
            rec = recall(ids, truth)
            ms, _ = timed(index, queries, w.k, kwg, 1, ids, dists)
            c = counts(index, queries, w.k, kwg)
            pts.append({"alpha": alpha, "tau": tau, "queries_per_s": round(w.n_query / ms * 1e3, 1),
                        "recall_at_10": round(rec, 4), "mean_candidates": round(c["n_cand"] / w.n_query, 1),
                        "mean_verified": round(c["examined"] / w.n_query, 1)})
    best = max((p_ for p_ in pts if p_["recall_at_10"] >= 0.90), key=lambda p_: p_["queries_per_s"], default=None)
    log(f"overlap grid: best at recall >= 0.90 {best}")
    index.free()
    del index, arrays, queries, qrot, truth
    torch.cuda.empty_cache()
    return {"workload": f"{w.name}: N={w.n} D={w.d} global rank {w.rank}, {w.n_comp} comps at centre scale "
                        f"{w.center_scale}, M={w.m} K={w.k_half}",
            "form": "bf16, patience 40k", "points": pts, "best_at_recall_0.90": best}


def build_gpu_index(w, force_rotation=None):
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
                                cev_rows=cev_rows, km_rows=km_rows, km_init=km_init, keep_input=False,
                                force_rotation=force_rotation)
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
    # candidate lists capped at 65,536 per query (queries with more are
    # searched again uncapped, same results): 11.4 MB of workspace per query
    # instead of 52 MB, so chunks of 2,048 fit with two pipelines
    sp = dict(kw, mode=1, precision=1, budget_source=1 if model is not None else 0, max_candidates=65536)
    t = time.time()
    srv = autotune.Server(None, index, sp, max_batch=4096, ks=(1, 10, 100), tiles=(16384, 65536),
                          chunks=(512, 1024, 2048), count_tiles=(1, 4))
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
    for (k, b), setting in sorted(choice.items()):
        tuned[f"k{k}_b{b}"] = list(setting)
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
           "max_candidates": 65536,
           "tuned_tile_chunk_persistent_counttiles": tuned}
    log(f"uneven: {out['queries_per_s']} q/s, p50 {out['p50_batch_ms']} ms, p99 {out['p99_batch_ms']} ms")
    srv.free()
    index.free()
    return out


def start_cpu_pool(n_workers=0):
    """Worker processes for the CPU oracle, forked before the GPU is first
    touched; they import numpy and the oracle only, one BLAS thread each."""
    import multiprocessing as mp
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    n = n_workers or min(16, avail)
    return mp.get_context("fork").Pool(n, initializer=_cpu_worker_init)


def _cpu_worker_init():
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _cpu_worker(task):
    """One worker's share: the oracle's query engine over its queries, on
    the index arrays memory-mapped from files."""
    import numpy as np
    from oracle import query as oquery
    paths, meta, q, k, okw = task
    index = dict(meta)
    for name, path in paths.items():
        index[name] = None if path is None else np.load(path, mmap_mode="r")
    t0 = time.perf_counter()
    oquery.search(index, q, k, **okw)
    return time.perf_counter() - t0, int(q.shape[0])


def _cpu_info():
    model, flags = "", ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name") and not model:
                    model = ln.split(":", 1)[1].strip()
                if ln.startswith("flags") and not flags:
                    flags = ln.split(":", 1)[1]
    except OSError:
        pass
    avx512 = sorted({t for t in flags.split() if t.startswith("avx512")})
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model,
            "avx512": avx512[:8]}


def export_index(arrays):
    """The index arrays written once to .npy files (in /dev/shm when it has
    room) that the CPU workers memory-map.  Returns (folder, paths, meta)."""
    import shutil
    import tempfile
    import numpy as np
    need = sum(v.numel() * v.element_size() for v in arrays.values() if hasattr(v, "numel"))
    try:
        root = "/dev/shm" if shutil.disk_usage("/dev/shm").free > 1.5 * need else tempfile.gettempdir()
    except OSError:
        root = tempfile.gettempdir()
    tmp = tempfile.mkdtemp(prefix="crisp_cpu_", dir=root)
    paths = {}
    for name in ("rotation", "centroids", "offsets", "ids", "base", "codes"):
        v = arrays[name]
        if v is None:
            paths[name] = None
            continue
        path = os.path.join(tmp, name + ".npy")
        dt = np.uint64 if name == "codes" else v[:0].cpu().numpy().dtype
        mm = np.lib.format.open_memmap(path, mode="w+", dtype=dt, shape=tuple(v.shape))
        step = max(1, (1 << 28) // max(1, v[0].numel() * v.element_size())) if v.dim() > 1 else v.shape[0]
        for r0 in range(0, v.shape[0], step):
            chunk = v[r0:r0 + step].cpu().numpy()
            mm[r0:r0 + step] = chunk.view(np.uint64) if name == "codes" else chunk
        mm.flush()
        del mm
        paths[name] = path
    meta = {"n": int(arrays["n"]), "d": int(arrays["d"]), "m": int(arrays["m"]), "k_half": int(arrays["k_half"])}
    return tmp, paths, meta


def _cpu_labels(task):
    """Oracle trace of one query: the plain walk's last update and prefix."""
    import numpy as np
    from oracle import query as oquery
    paths, meta, q, k, okw = task
    index = dict(meta)
    for name, path in paths.items():
        index[name] = None if path is None else np.load(path, mmap_mode="r")
    _, _, tr = oquery.search(index, q, k, trace=True, **okw)
    return [(int(t["last_update"]), int(t["examined"]), int(t["candidates"].size)) for t in tr]


def check_labels(pool, paths, meta, queries, engine_out, k, okw):
    """The learned budget's training labels (the engine's plain walk: last
    update L*, verified prefix, |C|) against the oracle's trace on a sample
    of the training queries."""
    qh = queries.cpu().numpy()
    res = pool.map(_cpu_labels, [(paths, meta, qh[i:i + 1], k, okw) for i in range(qh.shape[0])], chunksize=1)
    got = list(zip(engine_out["last_update"].tolist(), engine_out["examined"].tolist(),
                   engine_out["n_cand"].tolist()))
    ref = [r[0] for r in res]
    return {"sample": len(ref), "equal": sum(1 for a_, b_ in zip(got, ref) if tuple(a_) == tuple(b_)),
            "compared": "L* (last top-k update), verified prefix and |C| of the plain walk"}


def cpu_baseline(pool, paths, meta, queries, k, okw, budget_s):
    """The CPU oracle's query engine (the plain numpy one of the parity
    tests, untuned), timed on the host cores at the headline form's operating
    point: each worker process searches its own slice of the batch's first
    queries against the memory-mapped index arrays."""
    qh = queries[:4096].cpu().numpy()
    nw = pool._processes
    # one query on one worker sizes the shares
    el, _ = pool.apply(_cpu_worker, ((paths, meta, qh[:1], k, okw),))
    per = int(max(1, min(qh.shape[0] // nw, budget_s / max(el, 1e-3))))
    tasks = [(paths, meta, qh[i * per:(i + 1) * per], k, okw) for i in range(nw)]
    t0 = time.time()
    res = pool.map(_cpu_worker, tasks, chunksize=1)
    wall = time.time() - t0
    total = sum(n_ for _, n_ in res)
    single = sum(n_ / e_ for e_, n_ in res) / len(res)
    log(f"CPU oracle: {total} queries on {nw} processes in {wall:.1f}s")
    return {"value": round(total / wall, 3), "unit": "queries/s", "cores": nw, "kind": "oracle",
            "single_core_queries_per_s": round(single, 4),
            "host": _cpu_info(),
            "operating_point": {x_: okw[x_] for x_ in ("mode", "alpha", "tau", "patience_factor")},
            "sample": f"the batch's first {total} queries, {per} per process, through the oracle query engine "
                      f"(oracle/query.py, numpy, one BLAS thread per process) on {nw} worker processes against "
                      f"the same index arrays (memory-mapped), at the headline form's operating point"}


if __name__ == "__main__":
    main()
