"""Learned verification budget for Optimized Mode: trace collection, training
with the engine's float32 kernels, and calibration of the safety margin.

The label of a query is L*, the 1-based position of the last top-k update of
the plain patience walk (read from the engine's `last_update` tap); the
network predicts log L* from the features the engine computes during the
same search.  At search time the walk stops at the earlier of the patience
stop and clamp(ceil(exp(y + delta)), k, |C|); delta is chosen on held-out
queries so that a target fraction of them keeps a prefix >= L* (for those
the result equals the plain result exactly).
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
    """Plain Optimized-Mode searches with taps: features, L*, verified prefix, |C|."""
    nq = queries.shape[0]
    dev = queries.device
    f = index.n_features
    out = {"features": torch.empty(nq, f, dtype=torch.float32, device=dev),
           "last_update": torch.empty(nq, dtype=torch.int32, device=dev),
           "examined": torch.empty(nq, dtype=torch.int32, device=dev),
           "n_cand": torch.empty(nq, dtype=torch.int32, device=dev)}
    for q0 in range(0, nq, batch):
        q1 = min(nq, q0 + batch)
        taps = {key: v[q0:q1] for key, v in out.items()}
        index.search(queries[q0:q1], k, mode=1, alpha=alpha, tau=tau, patience_factor=patience_factor, taps=taps)
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

    def calibrate(self, x: torch.Tensor, l_star: torch.Tensor, target: float = 0.99) -> float:
        """delta = the `target` quantile of log L* - y over held-out queries."""
        y, _ = self.forward(x)
        gap = (torch.log(l_star.double().clamp(min=1.0)) - y.double()).cpu().numpy()
        self.delta = float(np.quantile(gap, target)) if gap.size else 0.0
        return self.delta

    def install(self, index: engine.Index):
        index.set_budget_model(self.params, self.mean, self.std, self.delta)


def train_budget(index: engine.Index, train_queries: torch.Tensor, k: int, *, alpha: float, tau: int,
                 patience_factor: int = 40, epochs: int = 30, holdout: float = 0.1, target: float = 0.99,
                 seed: int = 0, log=None) -> BudgetModel:
    """Collect plain traces, train, calibrate on a held-out split, install."""
    tr = collect(index, train_queries, k, alpha=alpha, tau=tau, patience_factor=patience_factor)
    keep = (tr["last_update"] >= 1).nonzero().squeeze(1)
    feats = tr["features"].index_select(0, keep)
    lstar = tr["last_update"].index_select(0, keep)
    n = feats.shape[0]
    nval = max(1, int(n * holdout))
    model = BudgetModel(index.n_features, device=feats.device, seed=seed)
    model.fit_standardisation(feats[nval:])
    x = model.standardise(feats)
    t = torch.log(lstar.float())
    model.train(x[nval:], t[nval:], epochs=epochs, seed=seed, log=log)
    model.calibrate(x[:nval], lstar[:nval], target)
    model.install(index)
    return model
