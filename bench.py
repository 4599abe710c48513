#!/usr/bin/env python3
"""Throughput of the CRISP query engine on one MI355X.

Workload (default): N = 1,000,000 float32 points, D = 4096, strongly
correlated Gaussian mixture (global rank-64 covariance + 0.05 I noise, 100
components; the correlation check fires and the index is rotated), M = 32
subspaces, K = 50 centroids per half, 10,000 queries per batch, k = 10.
Data, queries and index are generated and built on the GPU (seeded); the
timed region starts with everything resident in HBM.

A step is one search over the whole 10,000-query batch (every stage of the
hot path).  Prints one JSON line; see ``--help`` for the knobs.
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
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--n", type=int, default=0, help="override N (smaller dry runs)")
    ap.add_argument("--nq", type=int, default=0, help="override the batch size")
    ap.add_argument("--mode", type=int, default=1, help="0 Guaranteed, 1 Optimized")
    ap.add_argument("--alpha", type=float, default=0.002)
    ap.add_argument("--tau", type=int, default=16)
    ap.add_argument("--patience", type=int, default=40)
    ap.add_argument("--max-chunk", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-oracle time budget (0 = skip)")
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
    from paper_2603_05180_amd import engine

    w = synth.WORKLOADS[args.workload]
    if args.n:
        w = w.scaled(n=args.n)
    if args.nq:
        w = w.scaled(n_query=args.nq)
    dev = torch.device("cuda:0")
    t_setup = time.time()
    params = sg.mixture_params(w)
    x = sg.rows(w, w.seed_data, 0, w.n, params)
    queries = sg.rows(w, w.seed_query, 0, w.n_query, params)
    torch.cuda.synchronize()
    log(f"data {w.n}x{w.d} + {w.n_query} queries generated in {time.time() - t_setup:.1f}s")
    t = time.time()
    n = w.n
    cev_rows = synth.sample_indices(w.seed_index, synth.TAG["cev_sample"], n, max(2, min(n // 10, 100_000)))
    km_rows = synth.sample_indices(w.seed_index, synth.TAG["kmeans_sample"], n, min(n, 100_000))
    km_init = synth.permutation_prefix(w.seed_index, synth.TAG["kmeans_init"], np.arange(km_rows.size), w.k_half)
    arrays = engine.build_index(x, w.m, w.k_half, g=lambda: sg.gaussian_matrix(w.seed_index, w.d),
                                cev_rows=cev_rows, km_rows=km_rows, km_init=km_init, keep_input=False)
    torch.cuda.synchronize()
    log(f"index built on the GPU in {time.time() - t:.1f}s (CEV {arrays['cev']:.3f}, "
        f"rotated={arrays['rotation'] is not None})")
    index = engine.Index(arrays, tile_ids=args.tile)
    del x
    k = w.k
    kw = dict(mode=args.mode, alpha=args.alpha, tau=args.tau, patience_factor=args.patience,
              max_chunk=args.max_chunk)

    # Rotated queries (same kernel as the search) for the exact ground truth.
    qrot = engine.rotate_rows(queries, arrays["rotation"]) if arrays["rotation"] is not None else queries
    t = time.time()
    truth = ground_truth(arrays["base"], qrot, k)
    torch.cuda.synchronize()
    log(f"ground truth in {time.time() - t:.1f}s")

    ids = torch.empty(w.n_query, k, dtype=torch.int64, device=dev)
    dists = torch.empty(w.n_query, k, dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        index.search(queries, k, out=(ids, dists), **kw)
    torch.cuda.synchronize()
    rec = recall(ids, truth)
    # Verified prefix per query (identical in every run) for the algorithmic bytes.
    taps = {"examined": torch.empty(w.n_query, dtype=torch.int32, device=dev),
            "n_cand": torch.empty(w.n_query, dtype=torch.int32, device=dev),
            "retrieved": torch.empty(w.n_query, w.m, dtype=torch.int32, device=dev)}
    index.search(queries, k, taps=taps, **kw)
    torch.cuda.synchronize()
    examined = int(taps["examined"].long().sum())
    ncand = int(taps["n_cand"].long().sum())
    retrieved = int(taps["retrieved"].long().sum())

    # ---- timed region ----------------------------------------------------
    index.profile_begin(16384)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        index.search(queries, k, out=(ids, dists), **kw)
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    stages = index.profile_end()
    ms_step = total_ms / args.steps
    qps = w.n_query / (ms_step / 1e3)

    # ---- roofline of each stage (algorithmic bytes / flops per step) --------
    d = w.d
    per_step = {
        "rotate": ("alu", 2.0 * d * d * w.n_query / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"),
        "count": ("hbm", (4.0 * retrieved + 5.0 * ncand * 2) / 1e9, HBM_PEAK_GBS, "GB/s"),
        "hamming_order": ("hbm", (d / 8.0 * ncand + 12.0 * ncand) / 1e9, HBM_PEAK_GBS, "GB/s"),
        "rerank": ("hbm", (4.0 * d * examined) / 1e9, HBM_PEAK_GBS, "GB/s"),
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
    roof = {"kernel": {"rerank": "k_rerank", "count": "k_count", "rotate": "k_rotate_rows",
                       "hamming_order": "k_hamming_order"}[dom],
            "bound": per_step[dom][0], "achieved": stage_out[dom]["achieved"], "peak": per_step[dom][2],
            "unit": per_step[dom][3], "frac": stage_out[dom]["frac"], "traffic": None,
            "avg_launch_ms": round(stage_out[dom]["ms_per_step"] / launches, 4),
            "algorithmic_per_launch": round(per_step[dom][1] / launches, 4)}

    # ---- CPU oracle baseline on a bounded sample of the same workload --------
    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(arrays, queries, k, kw, args.cpu_seconds)

    line = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.n} D={w.d} correlated Gaussian mixture ({w.kind} rank {w.rank}, "
                               f"{w.n_comp} comps), M={w.m} K={w.k_half}, {w.n_query} queries/batch, k={k}",
                   "mode": "optimized" if args.mode == 1 else "guaranteed", "alpha": args.alpha, "tau": args.tau,
                   "patience_factor": args.patience, "recall_at_10": round(rec, 4),
                   "rotated": arrays["rotation"] is not None,
                   "mean_candidates": round(ncand / w.n_query, 1), "mean_verified": round(examined / w.n_query, 1),
                   "form": "plain"},
        "roofline": roof,
        "stages": stage_out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


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
