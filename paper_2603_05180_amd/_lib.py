"""ctypes declarations of the C ABI in include/crisp.h (argument marshalling only).

The shared library must have been built (``__graft_entry__.build()`` or
``csrc/build.sh``); importing this module without it raises ImportError so a
missing GPU engine can never go unnoticed.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrisp.so")

c_int32, c_int64, c_double, c_size_t, c_void_p = (
    ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p)

STATUS = {0: "CRISP_OK", -1: "CRISP_E_INVALID", -2: "CRISP_E_WORKSPACE", -3: "CRISP_E_HIP",
          -4: "CRISP_E_FORMAT", -5: "CRISP_E_UNSUPPORTED"}


class CrispError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class IndexDesc(ctypes.Structure):
    _fields_ = [("n", c_int64), ("d", c_int32), ("m", c_int32), ("k_half", c_int32),
                ("rotation", c_void_p), ("centroids", c_void_p), ("offsets", c_void_p),
                ("ids", c_void_p), ("base", c_void_p), ("codes", c_void_p)]


class SearchParams(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("alpha", c_double), ("tau", c_int32),
                ("patience_factor", c_int32), ("limits", c_void_p), ("max_chunk", c_int32),
                ("budget_source", c_int32), ("precision", c_int32), ("persistent", c_int32),
                ("overlap", c_int32), ("walk_order", c_int32), ("verify", c_int32), ("order_prefix", c_int32),
                ("count_tiles", c_int32), ("max_candidates", c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("intervals", c_int64 * 8), ("dropped", c_int64)]


STAGES = ["rotate", "hamming_place", "select", "count", "hamming_dist", "rerank", "budget", "candidates"]

TAP_FIELDS = ["q_rot", "half_dist", "n_cells", "cells", "retrieved", "hist", "tau_eff", "n_cand",
              "cand", "cand_score", "order", "hamming", "examined", "last_update", "stopped", "features",
              "limits", "refined", "score_lb", "score_ub", "row_bytes", "score_fallback"]


class Taps(ctypes.Structure):
    _fields_ = [(f, c_void_p) for f in TAP_FIELDS]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"CRISP HIP library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build() or paper_2603_05180_amd/csrc/build.sh)")

lib = ctypes.CDLL(LIB_PATH)

_SIGS = {
    "crisp_last_error": (ctypes.c_char_p, []),
    "crisp_version": (ctypes.c_char_p, []),
    "crisp_index_derived_bytes": (c_int32, [ctypes.POINTER(IndexDesc), c_int32, ctypes.POINTER(c_size_t)]),
    "crisp_index_load": (c_int32, [ctypes.POINTER(IndexDesc), c_int32, c_void_p, c_size_t, c_void_p,
                                   ctypes.POINTER(c_void_p)]),
    "crisp_index_free": (c_int32, [c_void_p]),
    "crisp_index_bf16_bytes": (c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    "crisp_index_enable_bf16": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "crisp_search_workspace_bytes": (c_int32, [c_void_p, c_int64, c_int32, ctypes.POINTER(SearchParams),
                                               ctypes.POINTER(c_size_t)]),
    "crisp_search": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, ctypes.POINTER(SearchParams), c_void_p,
                               c_void_p, c_void_p, c_size_t, ctypes.POINTER(Taps), c_void_p]),
    "crisp_search_static": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, ctypes.POINTER(SearchParams),
                                      c_void_p, c_void_p, c_void_p]),
    "crisp_plan_bytes": (c_int32, [c_void_p, c_int32, c_int32, ctypes.POINTER(SearchParams),
                                   ctypes.POINTER(c_size_t)]),
    "crisp_plan_create": (c_int32, [c_void_p, c_int32, c_int32, ctypes.POINTER(SearchParams), c_void_p, c_size_t,
                                    ctypes.POINTER(c_void_p)]),
    "crisp_plan_search": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "crisp_plan_free": (c_int32, [c_void_p]),
    "crisp_rotate_rows": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p]),
    "crisp_build_covariance": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_int64, c_void_p, c_void_p]),
    "crisp_build_assign": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p, c_int64, c_void_p,
                                     c_int32, c_void_p, c_void_p]),
    "crisp_build_update": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                     c_int32, c_void_p, c_void_p]),
    "crisp_build_csr_scratch": (c_int64, [c_int64, c_int32]),
    "crisp_build_csr": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "crisp_build_combine": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    "crisp_build_codes": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    "crisp_profile_begin": (c_int32, [c_void_p, c_int32]),
    "crisp_copy_probe": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "crisp_feature_count": (c_int32, [c_int32]),
    "crisp_mlp_param_count": (c_int32, [c_int32]),
    "crisp_set_budget_model": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_double]),
    "crisp_mlp_forward": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "crisp_mlp_backward": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p]),
    "crisp_mlp_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, ctypes.c_float,
                                 c_void_p]),
    "crisp_profile_end": (c_int32, [c_void_p, ctypes.POINTER(Profile)]),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = sorted(_SIGS)

# CRISP_STATIC_SCRATCH_BYTES of crisp.h: the static scratch of crisp_search_static
STATIC_SCRATCH_BYTES = 256 << 20


def check(status: int) -> None:
    if status != 0:
        raise CrispError(status, lib.crisp_last_error().decode(errors="replace"))
