"""Python binding of the CRISP engine.

Marshals torch device tensors into the C ABI of ``libcrisp.so`` and runs
every step on the GPU: the query path (rotation, half distances, cell
selection, collision counting, candidate selection, Hamming order, re-rank)
and the index build's data-sized steps (sample covariance, row rotation,
k-means assignment and update, CSR counting sort, sign codes).  The build
performs two D x D dense factorisations on the host with numpy -- the
eigenvalues of the sample covariance for the correlation check (Section 4.1)
and the QR factor of the Gaussian matrix that becomes the rotation
(Section 3) -- which involve no data-sized arrays.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import CrispError, IndexDesc, SearchParams, Taps, check, lib

__all__ = ["Index", "build_index", "CrispError", "budget_for", "TAU_CEV"]

TAU_CEV = 0.85
KMEANS_ITERS = 25
CEV_SAMPLE_CAP = 100_000
KMEANS_SAMPLE_CAP = 100_000


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_out(name: str, t, dtype, shape, device):
    """A caller-provided output must be exactly what the C side writes."""
    if (not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous()
            or tuple(t.shape) != tuple(shape)):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {list(shape)} on {device}")


def _check_queries(queries, d: int, device):
    if (not isinstance(queries, torch.Tensor) or queries.device != device or queries.dtype != torch.float32
            or not queries.is_contiguous()):
        raise ValueError("queries must be a contiguous float32 tensor on the index device")
    if queries.dim() != 2 or queries.shape[1] != d:
        raise ValueError(f"queries must have shape [nq, {d}]")


def _outputs(out, nq: int, k: int, device):
    if out is None:
        return (torch.empty(nq, k, dtype=torch.int64, device=device),
                torch.empty(nq, k, dtype=torch.float32, device=device))
    if not isinstance(out, (tuple, list)) or len(out) != 2:
        raise ValueError("out must be a tuple (ids, dists)")
    ids, dists = out
    _check_out("out ids", ids, torch.int64, (nq, k), device)
    _check_out("out dists", dists, torch.float32, (nq, k), device)
    return ids, dists


# Device memory left free after any buffer the binding allocates: kernels'
# private scratch, kernel arguments and library allocations come from it.
DEVICE_MEMORY_RESERVE = 4 << 30


def ensure_device_memory(nbytes: int, device) -> None:
    """Refuse (MemoryError, nothing allocated) a buffer that would leave less
    than DEVICE_MEMORY_RESERVE bytes of device memory free; the allocator's
    cached blocks are released first."""
    free, total = torch.cuda.mem_get_info(device)
    cached = torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)
    if nbytes + DEVICE_MEMORY_RESERVE <= free + cached:
        return
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info(device)
    if nbytes + DEVICE_MEMORY_RESERVE > free:
        raise MemoryError(f"a buffer of {nbytes / 2**30:.1f} GiB would leave less than "
                          f"{DEVICE_MEMORY_RESERVE / 2**30:.0f} GiB of the {free / 2**30:.1f} GiB free on {device}; "
                          f"use a smaller max_chunk or overlap=0")


def budget_for(alpha: float, n: int) -> int:
    return max(1, int(math.ceil(float(alpha) * float(n))))


class Index:
    """A CRISP index resident on the GPU (the arrays of Section 4.2).

    ``arrays`` maps the names of ``crisp_index_desc`` to tensors (device or
    host; host arrays are copied to ``device``).  The index keeps them alive.
    """

    def __init__(self, arrays: dict, *, tile_ids: int = 0, device: str = "cuda:0", stream=None):
        self.device = torch.device(device)
        dev = {}
        for name in ("rotation", "centroids", "offsets", "ids", "base", "codes"):
            v = arrays.get(name)
            if v is None:
                dev[name] = None
                continue
            if isinstance(v, np.ndarray):
                if name == "codes":
                    v = torch.from_numpy(np.ascontiguousarray(v).view(np.int64))
                else:
                    v = torch.from_numpy(np.ascontiguousarray(v))
            dev[name] = v.to(self.device).contiguous()
        self.arrays = dev
        self.n = int(arrays["n"])
        self.d = int(arrays["d"])
        self.m = int(arrays["m"])
        self.k_half = int(arrays["k_half"])
        self.rotated = dev["rotation"] is not None
        self._desc = IndexDesc(self.n, self.d, self.m, self.k_half, _ptr(dev["rotation"]),
                               _ptr(dev["centroids"]), _ptr(dev["offsets"]), _ptr(dev["ids"]),
                               _ptr(dev["base"]), _ptr(dev["codes"]))
        nbytes = ctypes.c_size_t(0)
        check(lib.crisp_index_derived_bytes(ctypes.byref(self._desc), int(tile_ids), ctypes.byref(nbytes)))
        self._derived = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p(0)
        check(lib.crisp_index_load(ctypes.byref(self._desc), int(tile_ids), _ptr(self._derived),
                                   nbytes.value, _stream(stream), ctypes.byref(h)))
        self._h = h
        self._ws = {}     # one workspace per stream (searches on two streams must not share one)

    # ------------------------------------------------------------------
    def free(self):
        if self._h is not None and self._h.value:
            lib.crisp_index_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def profile_begin(self, max_intervals: int = 4096):
        check(lib.crisp_profile_begin(self._h, int(max_intervals)))

    def profile_end(self) -> dict:
        """Per-stage GPU milliseconds and interval counts since profile_begin."""
        pr = _lib.Profile()
        check(lib.crisp_profile_end(self._h, ctypes.byref(pr)))
        return {name: {"ms": pr.ms[i], "intervals": pr.intervals[i]} for i, name in enumerate(_lib.STAGES)} | \
            {"dropped": pr.dropped}

    def params(self, *, mode=0, alpha=0.01, tau=1, patience_factor=40, limits=None, max_chunk=0, budget_source=0,
               precision=0, persistent=0, overlap=0, walk_order=0, verify=0, order_prefix=0, count_tiles=0,
               max_candidates=0):
        return SearchParams(int(mode), float(alpha), int(tau), int(patience_factor), _ptr(limits), int(max_chunk),
                            int(budget_source), int(precision), int(persistent), int(overlap), int(walk_order),
                            int(verify), int(order_prefix), int(count_tiles), int(max_candidates))

    def enable_bf16(self, stream=None, buffer: torch.Tensor | None = None) -> torch.Tensor:
        """bfloat16 copy of the rows + per-row error bounds for precision=1
        (the buffer is kept alive by the index; another index over the same
        rows may pass its buffer to share it)."""
        b = ctypes.c_size_t(0)
        check(lib.crisp_index_bf16_bytes(self._h, ctypes.byref(b)))
        buf = buffer if buffer is not None else torch.empty(b.value, dtype=torch.uint8, device=self.device)
        if buf.numel() < b.value:
            raise ValueError("bfloat16 buffer too small")
        check(lib.crisp_index_enable_bf16(self._h, _ptr(buf), b.value, _stream(stream)))
        self._bf16 = buf
        return buf

    def bf16_rows(self) -> tuple[torch.Tensor, torch.Tensor]:
        """Views of the bfloat16 copy [N, D] and the row error bounds [N]."""
        n, d = self.n, self.d
        off = (n * d * 2 + 255) // 256 * 256
        rows = self._bf16[: n * d * 2].view(torch.bfloat16).view(n, d)
        err = self._bf16[off: off + 4 * n].view(torch.float32)
        return rows, err

    @property
    def n_features(self) -> int:
        return int(lib.crisp_feature_count(self.m))

    def set_budget_model(self, params: torch.Tensor | None, mean: torch.Tensor | None = None,
                         std: torch.Tensor | None = None, delta: float = 0.0):
        """Learned verification budget for budget_source=1 (tensors are kept alive here)."""
        self._model = (params, mean, std)
        self._delta = float(delta)
        check(lib.crisp_set_budget_model(self._h, _ptr(params), self.n_features, _ptr(mean), _ptr(std),
                                         float(delta)))

    def workspace_bytes(self, nq: int, k: int, params: SearchParams) -> int:
        b = ctypes.c_size_t(0)
        check(lib.crisp_search_workspace_bytes(self._h, int(nq), int(k), ctypes.byref(params), ctypes.byref(b)))
        return b.value

    def workspace(self, nq: int, k: int, params: SearchParams, stream=None) -> torch.Tensor:
        """The search workspace for `stream` (kept per stream and grown on
        demand; allocated on that stream so the caching allocator never hands
        it to another stream while a search may still run there)."""
        need = self.workspace_bytes(nq, k, params)
        key = _stream(stream).value
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            self._ws.pop(key, None)
            ws = None
            ensure_device_memory(need, self.device)
            if isinstance(stream, torch.cuda.Stream):
                with torch.cuda.stream(stream):
                    ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            else:
                ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def tap_specs(self, nq: int) -> dict:
        """(dtype, shape) of every stage tap crisp_search can fill."""
        n, m, kh, d = self.n, self.m, self.k_half, self.d
        return {
            "q_rot": (torch.float32, (nq, d)),
            "half_dist": (torch.float64, (nq, m, 2, kh)),
            "n_cells": (torch.int32, (nq, m)),
            "cells": (torch.int32, (nq, m, kh * kh)),
            "retrieved": (torch.int32, (nq, m)),
            "hist": (torch.int32, (nq, 2 * m + 1)),
            "tau_eff": (torch.int32, (nq,)),
            "n_cand": (torch.int32, (nq,)),
            "cand": (torch.int32, (nq, n)),
            "cand_score": (torch.uint8, (nq, n)),
            "examined": (torch.int32, (nq,)),
            "last_update": (torch.int32, (nq,)),
            "stopped": (torch.int32, (nq,)),
            "refined": (torch.int32, (nq,)),
            "order": (torch.int32, (nq, n)),
            "hamming": (torch.int32, (nq, n)),
            "features": (torch.float32, (nq, self.n_features)),
            "limits": (torch.int32, (nq,)),
            "score_lb": (torch.float32, (nq, m, 2, kh)),
            "score_ub": (torch.float32, (nq, m, 2, kh)),
            "row_bytes": (torch.int64, (nq,)),
            "score_fallback": (torch.int32, (nq,)),
        }

    def alloc_taps(self, nq: int, mode: int) -> dict:
        only1 = {"order", "hamming", "features", "limits"}
        skip = {"score_lb", "score_ub", "score_fallback"}
        return {name: torch.empty(shape, dtype=dt, device=self.device)
                for name, (dt, shape) in self.tap_specs(nq).items()
                if name not in skip and (mode == 1 or name not in only1)}

    def search(self, queries: torch.Tensor, k: int, *, mode: int = 0, alpha: float = 0.01, tau: int = 1,
               patience_factor: int = 40, limits: torch.Tensor | None = None, max_chunk: int = 0,
               budget_source: int = 0, precision: int = 0, persistent: int = 0, overlap: int = 0,
               walk_order: int = 0, verify: int = 0, order_prefix: int = 0, count_tiles: int = 0,
               max_candidates: int = 0, taps: dict | None = None,
               out: tuple | None = None, stream=None):
        """Algorithm 1 for a batch; returns (ids int64 [nq, k], dists f32 [nq, k])."""
        _check_queries(queries, self.d, self.device)
        if limits is not None and (limits.dtype != torch.int32 or limits.device != self.device
                                   or limits.numel() != queries.shape[0]):
            raise ValueError("limits must be an int32 device tensor with one entry per query")
        nq = int(queries.shape[0])
        p = self.params(mode=mode, alpha=alpha, tau=tau, patience_factor=patience_factor,
                        limits=limits, max_chunk=max_chunk, budget_source=budget_source, precision=precision,
                        persistent=persistent, overlap=overlap, walk_order=walk_order, verify=verify,
                        order_prefix=order_prefix, count_tiles=count_tiles, max_candidates=max_candidates)
        ids, dists = _outputs(out, nq, int(k), self.device)
        tp = None
        if taps is not None:
            specs = self.tap_specs(nq)
            for name, t in taps.items():
                if name not in specs:
                    raise ValueError(f"unknown tap {name!r}")
                _check_out(f"tap {name}", t, specs[name][0], specs[name][1], self.device)
            tp = Taps(*[_ptr(taps.get(f)) for f in _lib.TAP_FIELDS])
        ws = self.workspace(nq, k, p, stream)
        check(lib.crisp_search(self._h, _ptr(queries), nq, int(k), ctypes.byref(p), _ptr(ids), _ptr(dists),
                               _ptr(ws), ws.numel(), ctypes.byref(tp) if tp is not None else None,
                               _stream(stream)))
        return ids, dists

    def search_static(self, queries: torch.Tensor, k: int, *, out: tuple | None = None, stream=None, **params):
        """crisp_search_static: as search() (no taps, one pipeline), with the
        library's static per-GPU scratch instead of a workspace."""
        _check_queries(queries, self.d, self.device)
        nq = int(queries.shape[0])
        if params.get("limits") is not None:
            lim = params["limits"]
            if lim.dtype != torch.int32 or lim.device != self.device or lim.numel() != nq:
                raise ValueError("limits must be an int32 device tensor with one entry per query")
        p = self.params(**params)
        ids, dists = _outputs(out, nq, int(k), self.device)
        check(lib.crisp_search_static(self._h, _ptr(queries), nq, int(k), ctypes.byref(p), _ptr(ids), _ptr(dists),
                                      _stream(stream)))
        return ids, dists


class Plan:
    """Batch executor for uneven batches (crisp_plan_*): one captured HIP
    graph per power-of-two batch-size bucket, replayed for every batch of
    that bucket.  Results equal Index.search with the same parameters."""

    def __init__(self, index: Index, max_batch: int, k: int, **params):
        if params.get("limits") is not None:
            raise ValueError("plans take no per-query limits")
        self._p = index.params(**params)
        b = ctypes.c_size_t(0)
        check(lib.crisp_plan_bytes(index._h, int(max_batch), int(k), ctypes.byref(self._p), ctypes.byref(b)))
        ensure_device_memory(b.value, index.device)
        self._buf = torch.empty(b.value, dtype=torch.uint8, device=index.device)
        h = ctypes.c_void_p(0)
        check(lib.crisp_plan_create(index._h, int(max_batch), int(k), ctypes.byref(self._p), _ptr(self._buf),
                                    b.value, ctypes.byref(h)))
        self._h = h
        self.index, self.max_batch, self.k = index, int(max_batch), int(k)

    def search(self, queries: torch.Tensor, out: tuple | None = None, stream=None):
        _check_queries(queries, self.index.d, self.index.device)
        nq = int(queries.shape[0])
        if nq > self.max_batch:
            raise ValueError(f"a batch holds at most {self.max_batch} queries")
        ids, dists = _outputs(out, nq, self.k, self.index.device)
        check(lib.crisp_plan_search(self._h, _ptr(queries), nq, _ptr(ids), _ptr(dists), _stream(stream)))
        return ids, dists

    def free(self):
        if self._h is not None and self._h.value:
            lib.crisp_plan_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# Index build on the GPU
# ----------------------------------------------------------------------------
def rotate_rows(x: torch.Tensor, r: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """x' = x R (float64 ascending accumulation per output), in chunks of rows."""
    if out is None:
        out = torch.empty_like(x)
    rows, d = x.shape
    step = 64 * 65535
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        check(lib.crisp_rotate_rows(ctypes.c_void_p(x[r0:r1].data_ptr()), r1 - r0, d, _ptr(r),
                                    ctypes.c_void_p(out[r0:r1].data_ptr()), _stream(stream)))
    return out


def sample_cev(x: torch.Tensor, rows: np.ndarray, stream=None) -> float:
    """Correlation check of Section 4.1 on the sampled rows."""
    n, d = x.shape
    rows_t = torch.from_numpy(np.ascontiguousarray(rows, dtype=np.int64)).to(x.device)
    cov = torch.empty(d * d + d, dtype=torch.float64, device=x.device)
    check(lib.crisp_build_covariance(_ptr(x), n, d, _ptr(rows_t), rows_t.numel(), _ptr(cov), _stream(stream)))
    c = cov[: d * d].reshape(d, d).cpu().numpy()
    lam = np.linalg.eigvalsh(c)[::-1]
    top = int(math.floor(0.2 * d))
    return float(lam[:top].sum() / lam.sum())


BUILD_STREAMS = 8  # side streams for the half-codebook k-means of the index build


def _csr(cell_of: torch.Tensor, cells: int, stream=None):
    n = cell_of.numel()
    off = torch.empty(cells + 1, dtype=torch.int32, device=cell_of.device)
    ids = torch.empty(n, dtype=torch.int32, device=cell_of.device)
    scratch = torch.empty(int(lib.crisp_build_csr_scratch(n, cells)), dtype=torch.int32, device=cell_of.device)
    check(lib.crisp_build_csr(_ptr(cell_of), n, cells, _ptr(off), _ptr(ids), _ptr(scratch), _stream(stream)))
    return off, ids


def _kmeans_half(x, col0, h, rows_t, init_pos, k, iters, stream=None):
    """Lloyd's k-means on the sampled rows of one half; returns f32 [k, h]."""
    n, d = x.shape
    s = rows_t.numel()
    dev = x.device
    cent = torch.empty(k, h, dtype=torch.float32, device=dev)
    # Initial centroids = the sampled rows at init_pos, via a one-member update.
    init_off = torch.arange(k + 1, dtype=torch.int32, device=dev)
    init_mem = torch.from_numpy(np.ascontiguousarray(init_pos, dtype=np.int32)).to(dev)
    check(lib.crisp_build_update(_ptr(x), n, d, col0, h, _ptr(rows_t), _ptr(init_off), _ptr(init_mem), k,
                                 _ptr(cent), _stream(stream)))
    label = torch.empty(s, dtype=torch.int32, device=dev)
    for _ in range(iters):
        check(lib.crisp_build_assign(_ptr(x), n, d, col0, h, _ptr(rows_t), s, _ptr(cent), k, _ptr(label),
                                     _stream(stream)))
        moff, mem = _csr(label, k, stream)
        check(lib.crisp_build_update(_ptr(x), n, d, col0, h, _ptr(rows_t), _ptr(moff), _ptr(mem), k,
                                     _ptr(cent), _stream(stream)))
    return cent


def build_index(x: torch.Tensor, m: int, k_half: int, *, g, cev_rows: np.ndarray, km_rows: np.ndarray,
                km_init: np.ndarray, force_rotation: bool | None = None, iters: int = KMEANS_ITERS,
                keep_input: bool = True, stream=None) -> dict:
    """Build a CRISP index from device data ``x`` (float32 [N, D]).

    g        -- the D x D Gaussian matrix (numpy, or a callable returning it),
                used only if the rotation fires
    cev_rows, km_rows, km_init -- sampled rows / initial centroid positions
    keep_input -- when False and the rotation fires, ``x`` is overwritten by
                the rotated rows in chunks (peak device memory ~ N D floats)
    Returns the arrays of crisp_index_desc as device tensors plus "cev".
    """
    n, d = x.shape
    dev = x.device
    if d % (2 * m) or d % 64:
        raise ValueError("D must be a multiple of 2M and of 64")
    h = d // (2 * m)
    cev = sample_cev(x, cev_rows, stream)
    rotate = (cev > TAU_CEV) if force_rotation is None else bool(force_rotation)
    rot = None
    base = x
    if rotate:
        gm = g() if callable(g) else g
        q, _ = np.linalg.qr(np.asarray(gm, dtype=np.float64))
        rot = torch.from_numpy(q.astype(np.float32)).to(dev)
        if keep_input:
            base = rotate_rows(x, rot, stream=stream)
        else:
            step = 1 << 16
            buf = torch.empty(min(step, n), d, dtype=torch.float32, device=dev)
            for r0 in range(0, n, step):
                r1 = min(n, r0 + step)
                rotate_rows(x[r0:r1], rot, out=buf[: r1 - r0], stream=stream)
                x[r0:r1].copy_(buf[: r1 - r0])
            base = x
    rows_t = torch.from_numpy(np.ascontiguousarray(km_rows, dtype=np.int64)).to(dev)
    cent = torch.empty(m, 2, k_half, h, dtype=torch.float32, device=dev)
    offsets = torch.empty(m, k_half * k_half + 1, dtype=torch.int32, device=dev)
    ids = torch.empty(m, n, dtype=torch.int32, device=dev)
    lab = torch.empty(m, 2, n, dtype=torch.int32, device=dev)
    cell = torch.empty(n, dtype=torch.int32, device=dev)
    # The 2M half codebooks are independent and each one's launches are
    # small, so they run on BUILD_STREAMS side streams (default priority),
    # joined before the cells are formed; every kernel and input is the
    # same as on one stream.
    main = stream if stream is not None else torch.cuda.current_stream(dev)
    side = [torch.cuda.Stream(device=dev) for _ in range(min(BUILD_STREAMS, 2 * m))]
    for st in side:
        st.wait_stream(main)
    for j in range(2 * m):
        sub, s = divmod(j, 2)
        st = side[j % len(side)]
        with torch.cuda.stream(st):
            col0 = sub * 2 * h + s * h
            c = _kmeans_half(base, col0, h, rows_t, km_init, k_half, iters, st)
            cent[sub, s].copy_(c)
            check(lib.crisp_build_assign(_ptr(base), n, d, col0, h, None, n, _ptr(cent[sub, s]), k_half,
                                         _ptr(lab[sub, s]), _stream(st)))
    for st in side:
        main.wait_stream(st)
    for sub in range(m):
        check(lib.crisp_build_combine(_ptr(lab[sub, 0]), _ptr(lab[sub, 1]), n, k_half, _ptr(cell), _stream(stream)))
        off_s, ids_s = _csr(cell, k_half * k_half, stream)
        offsets[sub].copy_(off_s)
        ids[sub].copy_(ids_s)
    codes = torch.empty(n, d // 64, dtype=torch.int64, device=dev)
    check(lib.crisp_build_codes(_ptr(base), n, d, _ptr(codes), _stream(stream)))
    return {"n": n, "d": d, "m": m, "k_half": k_half, "cev": cev, "rotation": rot, "centroids": cent,
            "offsets": offsets, "ids": ids, "base": base, "codes": codes}
