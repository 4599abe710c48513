"""Launch-shape tuner and uneven-batch runner for the batch executor.

The tuner times the batch executor (crisp_plan_*) over candidate settings
for each (k, batch-size bucket) on synthetic queries of the index's own
distribution and keeps the fastest:

  tile_ids   -- ids per collision-counting tile (an index-level choice: one
                derived cell x tile table per value; small tiles spread a
                small batch over more workgroups)
  max_chunk  -- queries per internal chunk (bounded by workspace memory)
  persistent -- re-rank with one block per query, or a persistent grid
                pulling queries from a device-side counter
  count_tiles -- id tiles counted in turn by one collision-counting block
                (0: the library's choice)

Every candidate returns identical results (results do not depend on tiles,
chunks or the re-rank grid), so the choice only affects time.  Results are
cached in a JSON file keyed by the index shape, k, bucket and the search
parameters.

The runner serves a stream of uneven batches: each batch goes to the plan
tuned for its (k, bucket); all plans share one device buffer (their batches
are ordered on one stream), and each batch's latency is measured with HIP
events on that stream.
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

from . import engine
from ._lib import check, lib


def bucket_of(nq: int) -> int:
    b = 1
    while b < nq:
        b *= 2
    return b


def _key(index: engine.Index, k: int, bucket: int, params: dict) -> str:
    pk = ",".join(f"{a}={params[a]}" for a in sorted(params))
    return f"D{index.d}_M{index.m}_K{index.k_half}_N{index.n}_k{k}_b{bucket}_{pk}"


class Server:
    """Indexes per tile over the same arrays, plans per setting, one shared buffer."""

    def __init__(self, arrays: dict, base: engine.Index, params: dict, max_batch: int, ks, tiles, chunks,
                 count_tiles=(0,)):
        self.arrays = {name: base.arrays[name] for name in base.arrays} | {
            "n": base.n, "d": base.d, "m": base.m, "k_half": base.k_half}
        self.base, self.params, self.max_batch = base, dict(params), int(max_batch)
        self.ks, self.tiles, self.chunks = list(ks), list(tiles), list(chunks)
        self.count_tiles = list(count_tiles)
        self.indexes = {}
        self.plans = {}
        self.choice = {}
        # one buffer, large enough for the largest plan
        need = 0
        for tile in self.tiles:
            ix = self.index(tile)
            for k in self.ks:
                for c in self.chunks:
                    p = ix.params(**(self.params | {"max_chunk": c}))
                    nb = ctypes.c_size_t(0)
                    check(lib.crisp_plan_bytes(ix._h, self.max_batch, int(k), ctypes.byref(p), ctypes.byref(nb)))
                    need = max(need, nb.value)
        self.buf = torch.empty(need, dtype=torch.uint8, device=base.device)

    def index(self, tile: int) -> engine.Index:
        if tile not in self.indexes:
            ix = engine.Index(self.arrays, tile_ids=tile)
            if getattr(self.base, "_bf16", None) is not None:
                ix.enable_bf16(buffer=self.base._bf16)
            if getattr(self.base, "_model", None) is not None and self.base._model[0] is not None:
                ix.set_budget_model(*self.base._model, delta=self.base._delta)
            self.indexes[tile] = ix
        return self.indexes[tile]

    def plan(self, k: int, tile: int, chunk: int, persistent: int, count_tiles: int = 0):
        key = (k, tile, chunk, persistent, count_tiles)
        if key not in self.plans:
            ix = self.index(tile)
            pl = engine.Plan.__new__(engine.Plan)
            pl._p = ix.params(**(self.params | {"max_chunk": chunk, "persistent": persistent,
                                                "count_tiles": count_tiles}))
            h = ctypes.c_void_p(0)
            check(lib.crisp_plan_create(ix._h, self.max_batch, int(k), ctypes.byref(pl._p), engine._ptr(self.buf),
                                        self.buf.numel(), ctypes.byref(h)))
            pl._h, pl._buf, pl.index, pl.max_batch, pl.k = h, self.buf, ix, self.max_batch, int(k)
            self.plans[key] = pl
        return self.plans[key]

    def candidates(self, bucket: int):
        for tile in self.tiles:
            for chunk in self.chunks:
                if chunk > max(bucket, min(self.chunks)) and chunk != min(self.chunks):
                    continue
                for persistent in (0, 1):
                    for ct in self.count_tiles:
                        yield tile, chunk, persistent, ct

    def tune(self, queries: torch.Tensor, buckets, reps: int = 3, cache: str | None = None, log=None):
        """Fastest setting per (k, bucket); reuses and extends the JSON cache."""
        saved = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                saved = json.load(f)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for k in self.ks:
            for b in buckets:
                key = _key(self.base, k, b, self.params)
                if key in saved:
                    self.choice[(k, b)] = tuple(saved[key]["setting"])
                    continue
                nq = min(b, self.max_batch)
                qb = queries[:nq].contiguous()
                best = None
                for cand in self.candidates(b):
                    pl = self.plan(k, *cand)
                    pl.search(qb)                      # captures the bucket's graph
                    torch.cuda.synchronize()
                    ev0.record()
                    for _ in range(reps):
                        pl.search(qb)
                    ev1.record()
                    torch.cuda.synchronize()
                    ms = ev0.elapsed_time(ev1) / reps
                    if best is None or ms < best[0]:
                        best = (ms, cand)
                self.choice[(k, b)] = best[1]
                saved[key] = {"setting": list(best[1]), "ms": round(best[0], 4),
                              "fields": ["tile_ids", "max_chunk", "persistent", "count_tiles"]}
                if log:
                    log(f"tuned k={k} bucket={b}: tile={best[1][0]} chunk={best[1][1]} "
                        f"persistent={best[1][2]} count_tiles={best[1][3]} {best[0]:.3f} ms")
        if cache:
            with open(cache, "w") as f:
                json.dump(saved, f, indent=1, sort_keys=True)
        return self.choice

    def run(self, queries: torch.Tensor, sizes, ks):
        """Serve the batches in order; returns per-batch GPU latency (ms) and the results."""
        events = []
        outs = []
        o = 0
        for nq, k in zip(sizes, ks):
            b = bucket_of(nq)
            pl = self.plan(k, *self.choice[(k, b)])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ids, d = pl.search(queries[o:o + nq])
            e1.record()
            events.append((e0, e1))
            outs.append((ids, d))
            o += nq
        torch.cuda.synchronize()
        lat = [a.elapsed_time(b) for a, b in events]
        return lat, outs

    def free(self):
        for pl in self.plans.values():
            pl.free()
        self.plans.clear()
        for ix in self.indexes.values():
            ix.free()
        self.indexes.clear()
