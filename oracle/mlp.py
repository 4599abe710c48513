"""Learned candidate budget: features and a 2-layer MLP (test infrastructure only).

An addition on top of the paper's Optimized Mode (Section 4.3.2, Stage 3):
instead of always walking until the patience rule fires, a small network
predicts, per query, how many candidates of the Hamming order must be
verified.  The plain patience walk stays the fallback: the walk stops at the
earlier of the patience stop and the predicted prefix.

Label: L* = 1-based position of the last top-k update in the plain walk (the
shortest prefix that reproduces the plain result).  Target y = log(L*).

Features (float32, F = 1 + 16 + 3M + 13), from the query's own intermediates:
  * log1p(|C|)
  * log1p of the number of points at each of the 16 highest score levels
    2M, 2M-1, ..., 2M-15 (only levels >= max(tau_eff, 1) are counted)
  * per subspace m: (c2 - c1) / c1, (c_cut - c1) / c1 and log1p(size of the
    cheapest cell), where c1, c2 are the two smallest cell costs and c_cut the
    cost of the last activated cell (c1 floored at 1e-30 in the divisions)
  * the Hamming distances at positions 1, 2, 4, ..., 2048 (each clamped to
    |C|) and at position ceil(|C| / 2) of the Hamming order, divided by D
    (0 when |C| = 0): how sharply the sign codes separate the front of the
    order from the bulk

Network: y = w2 . relu(W1^T f + b1) + b2, 64 hidden units.  Training is plain
mean squared error on log L* with Adam (Kingma & Ba); inference rounds f and
W1 to bfloat16 (round to nearest even).
"""
from __future__ import annotations

import math

import numpy as np

HIDDEN = 64


HAMMING_POSITIONS = [1 << i for i in range(12)]


def n_features(m: int) -> int:
    return 1 + 16 + 3 * m + len(HAMMING_POSITIONS) + 1


def subspace_stats(index: dict, hd: np.ndarray, activated: list) -> np.ndarray:
    """(M, 4) float64: c1, c2, c_cut, size of the cheapest cell."""
    m, kh = index["m"], index["k_half"]
    out = np.zeros((m, 4))
    for sub in range(m):
        d1, d2 = hd[sub, 0], hd[sub, 1]
        o1, o2 = np.argsort(d1, kind="stable"), np.argsort(d2, kind="stable")
        d1s, d2s = d1[o1], d2[o2]
        c1 = d1s[0] + d2s[0]
        c2 = min(d1s[0] + d2s[1], d1s[1] + d2s[0]) if kh > 1 else c1
        inv1 = {int(o1[i]): i for i in range(kh)}
        inv2 = {int(o2[j]): j for j in range(kh)}
        ccut = max(d1s[inv1[c // kh]] + d2s[inv2[c % kh]] for c, _ in activated[sub])
        off = index["offsets"][sub]
        cell0 = int(o1[0]) * kh + int(o2[0])
        out[sub] = (c1, c2, ccut, off[cell0 + 1] - off[cell0])
    return out


def features(index: dict, trace: dict, k: int) -> np.ndarray:
    """Feature vector of one query from its oracle trace (Optimized Mode)."""
    m, d = index["m"], index["d"]
    f = np.zeros(n_features(m), dtype=np.float64)
    cand = trace["candidates"]
    f[0] = math.log1p(cand.size)
    v = trace["scores"]
    floor = max(trace["tau_eff"], 1)
    for j in range(16):
        s = 2 * m - j
        f[1 + j] = math.log1p(int(np.count_nonzero(v == s))) if s >= floor else 0.0
    st = subspace_stats(index, trace["half_dist"], trace["activated"])
    for sub in range(m):
        c1, c2, ccut, size1 = st[sub]
        den = max(c1, 1e-30)
        f[17 + 3 * sub] = (c2 - c1) / den
        f[18 + 3 * sub] = (ccut - c1) / den
        f[19 + 3 * sub] = math.log1p(size1)
    hm = trace.get("hamming")
    base = 17 + 3 * m
    if hm is not None and hm.size > 0:
        n = hm.size
        for j, pos in enumerate(HAMMING_POSITIONS):
            f[base + j] = hm[min(pos, n) - 1] / d
        f[base + len(HAMMING_POSITIONS)] = hm[(n + 1) // 2 - 1] / d
    return f.astype(np.float32)


def init_params(f: int, seed: int = 0):
    """He-style initial weights from the shared generator (float32)."""
    import synth
    n1 = f * HIDDEN
    z = synth.normals(seed, synth.TAG["mlp_init"], np.arange(n1 + HIDDEN, dtype=np.uint64))
    w1 = (z[:n1] * math.sqrt(2.0 / f)).reshape(f, HIDDEN)
    w2 = z[n1:] * math.sqrt(1.0 / HIDDEN)
    return {"w1": w1.astype(np.float32), "b1": np.zeros(HIDDEN, np.float32),
            "w2": w2.astype(np.float32), "b2": np.zeros(1, np.float32)}


def forward(p: dict, x: np.ndarray):
    """float64 forward; returns (y, pre-activation, hidden)."""
    x = np.asarray(x, dtype=np.float64)
    pre = x @ p["w1"].astype(np.float64) + p["b1"].astype(np.float64)
    hid = np.maximum(pre, 0.0)
    y = hid @ p["w2"].astype(np.float64) + float(p["b2"][0])
    return y, pre, hid


def loss(p: dict, x: np.ndarray, t: np.ndarray) -> float:
    y, _, _ = forward(p, x)
    return float(np.mean((y - t) ** 2))


def backward(p: dict, x: np.ndarray, t: np.ndarray) -> dict:
    """Analytic gradient of the mean squared error (float64)."""
    x = np.asarray(x, dtype=np.float64)
    y, pre, hid = forward(p, x)
    b = x.shape[0]
    dy = 2.0 * (y - t) / b
    g = {"w2": hid.T @ dy, "b2": np.array([dy.sum()])}
    dh = np.outer(dy, p["w2"].astype(np.float64)) * (pre > 0)
    g["w1"] = x.T @ dh
    g["b1"] = dh.sum(axis=0)
    return g


def adam_step(p: dict, g: dict, state: dict, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in float64, parameters rounded back to float32."""
    out = {}
    for k in p:
        mk, vk = state.setdefault(k, (np.zeros_like(g[k]), np.zeros_like(g[k])))
        mk = b1 * mk + (1 - b1) * g[k]
        vk = b2 * vk + (1 - b2) * g[k] ** 2
        state[k] = (mk, vk)
        mhat = mk / (1 - b1 ** step)
        vhat = vk / (1 - b2 ** step)
        out[k] = (p[k].astype(np.float64) - lr * mhat / (np.sqrt(vhat) + eps)).astype(np.float32)
    return out


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (nearest even), returned as float32 values."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32)


def infer_bf16(p: dict, x: np.ndarray) -> np.ndarray:
    """Inference with bfloat16 features and first-layer weights (float64 sums)."""
    q = {"w1": to_bf16(p["w1"]), "b1": p["b1"], "w2": p["w2"], "b2": p["b2"]}
    y, _, _ = forward(q, to_bf16(x))
    return y


def limits_from(y: np.ndarray, delta: float, k: int, ncand: np.ndarray) -> np.ndarray:
    """Predicted prefix L = clamp(ceil(exp(y + delta)), k, |C|) (|C| = 0 -> 0)."""
    lim = np.ceil(np.exp(np.asarray(y, dtype=np.float64) + delta))
    lim = np.minimum(np.maximum(lim, k), np.asarray(ncand, dtype=np.float64))
    return lim.astype(np.int64)
