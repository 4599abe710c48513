"""Learned verification budget for Optimized Mode: trace collection, training
with the engine's float32 kernels, and calibration of the safety margin.

The label of a query is L*, the 1-based position of the last top-k update of
the plain patience walk (read from the engine's `last_update` tap); the
network predicts log L* from the features the engine computes during the
same search.  At search time the walk stops at the earlier of the patience
stop and clamp(ceil(exp(y + delta)), k, |C|).  The margin delta is the
smallest value (found by bisection) at which held-out queries keep a given
fraction of their plain top-k: the plain result is the reference.  A prefix
never loses a plain result it contains, so that fraction is non-decreasing
in delta and bisection finds the threshold.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import engine
from ._lib import check, lib

HIDDEN = 64


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _st():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def collect(index: engine.Index, queries: torch.Tensor, k: int, *, alpha: float, tau: int, patience_factor: int = 40,
            batch: int = 8192):
    """Plain Optimized-Mode searches with taps: features, L*, verified prefix,
    |C| and the plain top-k ids."""
    nq = queries.shape[0]
    dev = queries.device
    f = index.n_features
    out = {"features": torch.empty(nq, f, dtype=torch.float32, device=dev),
           "last_update": torch.empty(nq, dtype=torch.int32, device=dev),
           "examined": torch.empty(nq, dtype=torch.int32, device=dev),
           "n_cand": torch.empty(nq, dtype=torch.int32, device=dev),
           "ids": torch.empty(nq, k, dtype=torch.int64, device=dev)}
    dists = torch.empty(nq, k, dtype=torch.float32, device=dev)
    for q0 in range(0, nq, batch):
        q1 = min(nq, q0 + batch)
        taps = {key: v[q0:q1] for key, v in out.items() if key != "ids"}
        index.search(queries[q0:q1], k, mode=1, alpha=alpha, tau=tau, patience_factor=patience_factor, taps=taps,
                     out=(out["ids"][q0:q1], dists[q0:q1]))
    torch.cuda.synchronize()
    return out


class BudgetModel:
    """The 2-layer MLP and its standardisation (device float32 tensors)."""

    def __init__(self, n_features: int, device="cuda", seed: int = 0):
        import synth
        self.f = n_features
        self.np = int(lib.crisp_mlp_param_count(n_features))
        n1 = n_features * HIDDEN
        z = synth.normals(seed, synth.TAG["mlp_init"], np.arange(n1 + HIDDEN, dtype=np.uint64))
        p = np.zeros(self.np, np.float32)
        p[:n1] = z[:n1] * math.sqrt(2.0 / n_features)
        p[n1 + HIDDEN:n1 + 2 * HIDDEN] = z[n1:] * math.sqrt(1.0 / HIDDEN)
        self.params = torch.from_numpy(p).to(device)
        self.mean = torch.zeros(n_features, dtype=torch.float32, device=device)
        self.std = torch.ones(n_features, dtype=torch.float32, device=device)
        self.delta = 0.0

    def fit_standardisation(self, feats: torch.Tensor):
        x = feats.double().cpu().numpy()
        mu = x.mean(axis=0)
        sd = x.std(axis=0)
        sd[sd < 1e-6] = 1.0
        self.mean = torch.from_numpy(mu.astype(np.float32)).to(feats.device)
        self.std = torch.from_numpy(sd.astype(np.float32)).to(feats.device)

    def standardise(self, feats: torch.Tensor) -> torch.Tensor:
        return ((feats - self.mean) / self.std).contiguous()

    def forward(self, x: torch.Tensor):
        b = x.shape[0]
        pre = torch.empty(b, HIDDEN, dtype=torch.float32, device=x.device)
        y = torch.empty(b, dtype=torch.float32, device=x.device)
        check(lib.crisp_mlp_forward(_p(x), b, self.f, _p(self.params), _p(pre), _p(y), _st()))
        return y, pre

    def train(self, x: torch.Tensor, t: torch.Tensor, *, epochs: int = 30, batch: int = 1024, lr: float = 1e-3,
              seed: int = 0, log=None):
        """Adam on mean squared error, minibatches in a seeded shuffled order."""
        import synth
        n = x.shape[0]
        m1 = torch.zeros_like(self.params)
        m2 = torch.zeros_like(self.params)
        grad = torch.empty_like(self.params)
        step = 0
        for ep in range(epochs):
            perm = synth.permutation_prefix(seed + ep, synth.TAG["mlp_shuffle"], np.arange(n), n)
            perm_t = torch.from_numpy(perm).to(x.device)
            for b0 in range(0, n - batch + 1, batch):
                idx = perm_t[b0:b0 + batch]
                xb = x.index_select(0, idx).contiguous()
                tb = t.index_select(0, idx).contiguous()
                y, pre = self.forward(xb)
                check(lib.crisp_mlp_backward(_p(xb), _p(tb), batch, self.f, _p(self.params), _p(pre), _p(y),
                                             _p(grad), _st()))
                step += 1
                check(lib.crisp_mlp_adam(_p(self.params), _p(grad), _p(m1), _p(m2), self.f, step, float(lr), _st()))
            if log is not None:
                y, _ = self.forward(x[: min(n, 65536)])
                mse = float(((y - t[: y.shape[0]]) ** 2).mean())
                log(f"epoch {ep + 1}/{epochs}: mse {mse:.4f}")
        return self

    def calibrate(self, index: engine.Index, queries: torch.Tensor, plain_ids: torch.Tensor, k: int, *,
                  floor: float = 0.998, lo: float = -2.0, hi: float = 6.0, iters: int = 14, batch: int = 8192,
                  **search_kw) -> float:
        """Smallest delta in [lo, hi] (to within (hi - lo) / 2^iters) at which
        the learned searches of `queries` keep at least `floor` of the plain
        top-k ids `plain_ids`; `hi` if none does."""
        def kept(delta):
            self.delta = delta
            self.install(index)
            hit = 0.0
            for q0 in range(0, queries.shape[0], batch):
                q1 = min(queries.shape[0], q0 + batch)
                ids, _ = index.search(queries[q0:q1], k, mode=1, budget_source=1, **search_kw)
                hit += float((ids[:, :, None] == plain_ids[q0:q1, None, :]).any(-1).sum())
            return hit / max(1, plain_ids.numel())

        if kept(lo) >= floor:
            return self.delta
        if kept(hi) < floor:
            return self.delta
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if kept(mid) >= floor:
                hi = mid
            else:
                lo = mid
        self.delta = hi
        self.install(index)
        return self.delta

    def install(self, index: engine.Index):
        index.set_budget_model(self.params, self.mean, self.std, self.delta)


def train_budget(index: engine.Index, train_queries: torch.Tensor, k: int, *, alpha: float, tau: int,
                 patience_factor: int = 40, epochs: int = 30, holdout: float = 0.1, floor: float = 0.998,
                 seed: int = 0, log=None) -> BudgetModel:
    """Collect plain traces, train on all but the first `holdout` fraction of
    the queries, calibrate delta on that held-out part, install."""
    kw = dict(alpha=alpha, tau=tau, patience_factor=patience_factor)
    tr = collect(index, train_queries, k, **kw)
    nq = train_queries.shape[0]
    nval = max(1, int(nq * holdout))
    keep = (tr["last_update"][nval:] >= 1).nonzero().squeeze(1) + nval
    feats = tr["features"].index_select(0, keep)
    lstar = tr["last_update"].index_select(0, keep)
    model = BudgetModel(index.n_features, device=feats.device, seed=seed)
    model.fit_standardisation(feats)
    model.train(model.standardise(feats), torch.log(lstar.float()), epochs=epochs, seed=seed, log=log)
    model.calibrate(index, train_queries[:nval], tr["ids"][:nval], k, floor=floor, **kw)
    if log is not None:
        log(f"delta {model.delta:.4f} (floor {floor} of the plain top-{k} on {nval} held-out queries)")
    return model
