"""GPU twin of the synthetic-input generator (same values as the numpy twin).

Used to materialise full-size workloads directly in device memory; any row
can be reproduced on the CPU with ``synth.rows`` for checks.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import TAG, Workload

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
if not os.path.exists(_PATH):
    raise ImportError(f"{_PATH} missing: run synth/csrc/build.sh")
_lib = ctypes.CDLL(_PATH)
_u64, _i64, _u32, _i32, _f32, _f64, _vp = (ctypes.c_uint64, ctypes.c_longlong, ctypes.c_uint32, ctypes.c_int,
                                           ctypes.c_float, ctypes.c_double, ctypes.c_void_p)
_lib.synth_normals_f64.argtypes = [_u64, _u32, _u64, _i64, _vp, _vp]
_lib.synth_normals_f32.argtypes = [_u64, _u32, _u64, _i64, _f64, _vp, _vp]
_lib.synth_rows.argtypes = [_i32, _u64, _i32, _i32, _i32, _f32, _u64, _i64, _vp, _vp, _vp, _vp, _vp]
for _f in (_lib.synth_normals_f64, _lib.synth_normals_f32, _lib.synth_rows):
    _f.restype = _i32


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def normals_f32(seed: int, tag: int, count: int, scale: float = 1.0, device="cuda") -> torch.Tensor:
    out = torch.empty(count, dtype=torch.float32, device=device)
    if _lib.synth_normals_f32(seed, tag, 0, count, scale, _p(out), _stream()) != 0:
        raise RuntimeError("synth_normals_f32 failed")
    return out


def normals_f64(seed: int, tag: int, count: int, device="cuda") -> torch.Tensor:
    out = torch.empty(count, dtype=torch.float64, device=device)
    if _lib.synth_normals_f64(seed, tag, 0, count, _p(out), _stream()) != 0:
        raise RuntimeError("synth_normals_f64 failed")
    return out


def mixture_params(w: Workload, device="cuda") -> dict:
    s = w.seed_data
    if w.kind == "local":
        return {"mu": normals_f32(s, TAG["mean"], w.n_comp * w.d, 2.0, device).reshape(w.n_comp, w.d),
                "a": normals_f32(s, TAG["factor"], w.n_comp * w.d * w.rank, 1.0, device)
                .reshape(w.n_comp, w.d, w.rank)}
    return {"b": normals_f32(s, TAG["factor"], w.d * w.rank, 0.125, device).reshape(w.d, w.rank),
            "nu": normals_f32(s, TAG["center"], w.n_comp * w.rank, float(w.center_scale), device)
            .reshape(w.n_comp, w.rank)}


def rows(w: Workload, seed: int, start: int, stop: int, params: dict, out: torch.Tensor | None = None):
    n = stop - start
    if out is None:
        out = torch.empty(n, w.d, dtype=torch.float32, device=next(iter(params.values())).device)
    kind = 0 if w.kind == "local" else 1
    fac = params["a"] if kind == 0 else params["b"]
    rc = _lib.synth_rows(kind, seed, w.n_comp, w.rank, w.d, float(w.sigma32), start, n,
                         _p(params.get("mu")), _p(fac), _p(params.get("nu")), _p(out), _stream())
    if rc != 0:
        raise RuntimeError("synth_rows failed")
    return out


def gaussian_matrix(seed: int, d: int) -> np.ndarray:
    """The D x D rotation draw, generated on the device and returned as numpy."""
    return normals_f64(seed, TAG["rotation"], d * d).reshape(d, d).cpu().numpy()
