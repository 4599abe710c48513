"""Learned verification budget on the GPU vs the oracle (needs an MI355X)."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import build as obuild
from oracle import mlp as omlp
from oracle import query as oquery
from parity_util import compare, gpu_index, make_workload, oracle_index

pytestmark = pytest.mark.gpu


def _flat(p):
    return np.concatenate([p["w1"].reshape(-1), p["b1"], p["w2"], p["b2"]]).astype(np.float32)


def _unflat(v, f):
    h = omlp.HIDDEN
    return {"w1": v[:f * h].reshape(f, h), "b1": v[f * h:f * h + h], "w2": v[f * h + h:f * h + 2 * h],
            "b2": v[f * h + 2 * h:f * h + 2 * h + 1]}


def test_training_kernels_match_reference():
    from paper_2603_05180_amd import _lib
    f, b = 116, 257
    rng = np.random.default_rng(0)
    p = omlp.init_params(f, 5)
    p["b1"] = (rng.standard_normal(64) * 0.1).astype(np.float32)
    p["b2"] = np.array([0.2], np.float32)
    x = rng.standard_normal((b, f)).astype(np.float32)
    t = rng.standard_normal(b).astype(np.float32)
    dev = torch.device("cuda")
    pt = torch.from_numpy(_flat(p)).to(dev)
    xt, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    pre = torch.empty(b, 64, device=dev)
    y = torch.empty(b, device=dev)
    grad = torch.empty_like(pt)
    P = lambda a: ctypes.c_void_p(a.data_ptr())
    _lib.check(_lib.lib.crisp_mlp_forward(P(xt), b, f, P(pt), P(pre), P(y), None))
    _lib.check(_lib.lib.crisp_mlp_backward(P(xt), P(tt), b, f, P(pt), P(pre), P(y), P(grad), None))
    torch.cuda.synchronize()
    y_ref, pre_ref, _ = omlp.forward(p, x)
    assert np.allclose(y.cpu().numpy(), y_ref, rtol=1e-5, atol=1e-5)
    assert np.allclose(pre.cpu().numpy(), pre_ref, rtol=1e-5, atol=1e-5)
    g_ref = omlp.backward(p, x, t)
    g = _unflat(grad.cpu().numpy(), f)
    for key in ("w1", "b1", "w2", "b2"):
        scale = np.abs(g_ref[key]).max()
        assert np.abs(g[key] - g_ref[key]).max() <= 1e-4 * max(scale, 1e-3), key
    # one Adam step
    m1 = torch.zeros_like(pt)
    m2 = torch.zeros_like(pt)
    _lib.check(_lib.lib.crisp_mlp_adam(P(pt), P(grad), P(m1), P(m2), f, 1, ctypes.c_float(1e-3), None))
    torch.cuda.synchronize()
    ref = omlp.adam_step(p, {k_: g[k_].astype(np.float64) for k_ in g}, {}, 1, lr=1e-3)
    assert np.allclose(pt.cpu().numpy(), _flat(ref), rtol=1e-6, atol=1e-7)


@pytest.fixture(scope="module")
def small():
    w, x, q = make_workload("d4096", n=6000, d=256, m=8, k_half=8, rank=16, n_query=48)
    idx = oracle_index(w, x)
    return w, x, q, idx


def test_features_match_oracle(small):
    w, x, q, idx = small
    g = gpu_index(idx)
    taps = g.alloc_taps(q.shape[0], 1)
    g.search(torch.from_numpy(q).cuda(), 10, mode=1, alpha=0.03, tau=4, taps=taps)
    torch.cuda.synchronize()
    got = taps["features"].cpu().numpy()
    for qi in range(q.shape[0]):
        _, _, tr = oquery.search_one(idx, q[qi], 10, mode=1, alpha=0.03, tau=4, trace=True)
        ref = omlp.features(idx, tr, 10)
        assert np.allclose(got[qi], ref, rtol=2e-7, atol=0), qi


def test_bf16_mfma_inference_and_learned_search(small):
    """Limits from the engine's bfloat16 MFMA inference equal the oracle's
    (bfloat16-rounded inputs, float64 sums) except where exp(y + delta) sits
    within float32 rounding of an integer; where they are equal, the searches
    with those limits return identical ids."""
    w, x, q, idx = small
    g = gpu_index(idx)
    f = g.n_features
    rng = np.random.default_rng(1)
    p = omlp.init_params(f, 9)
    p["b2"] = np.array([4.0], np.float32)
    feats = np.stack([omlp.features(idx, oquery.search_one(idx, q[i], 10, mode=1, alpha=0.03, tau=4,
                                                            trace=True)[2], 10) for i in range(q.shape[0])])
    mean = feats.mean(0).astype(np.float32)
    sd = feats.std(0).astype(np.float32)
    sd[sd < 1e-6] = 1.0
    delta = 0.25
    dev = torch.device("cuda")
    pt = torch.from_numpy(_flat(p)).to(dev)
    g.set_budget_model(pt, torch.from_numpy(mean).to(dev), torch.from_numpy(sd).to(dev), delta)
    taps = g.alloc_taps(q.shape[0], 1)
    ids, dists = g.search(torch.from_numpy(q).to(dev), 10, mode=1, alpha=0.03, tau=4, budget_source=1, taps=taps)
    torch.cuda.synchronize()
    xs = ((feats - mean) / sd).astype(np.float32)
    y_ref = omlp.infer_bf16(p, xs)
    ncand = taps["n_cand"].cpu().numpy()
    lim_ref = omlp.limits_from(y_ref, delta, 10, ncand)
    lim = taps["limits"].cpu().numpy()
    close = np.abs(np.exp(y_ref + delta) - np.round(np.exp(y_ref + delta))) < 1e-3 * np.exp(y_ref + delta)
    assert np.all((lim == lim_ref) | close)
    assert np.mean(lim == lim_ref) >= 0.9
    same = np.flatnonzero(lim == lim_ref)
    oi, od, _ = oquery.search(idx, q[same], 10, mode=1, alpha=0.03, tau=4, limits=lim_ref[same])
    assert np.array_equal(ids.cpu().numpy()[same], oi)
    assert np.array_equal(dists.cpu().numpy()[same].view(np.uint32), od.view(np.uint32))


def test_learned_budget_verifies_fewer_candidates():
    """Trained on plain-walk traces, the learned budget verifies fewer
    candidates than the patience rule alone, at recall within 0.005 of it."""
    import synth.gpu as sg
    from paper_2603_05180_amd import engine, learned
    w = synth.WORKLOADS["d4096"].scaled(n=200_000, d=1024, m=16, k_half=32, rank=64)
    params = sg.mixture_params(w)
    x = sg.rows(w, w.seed_data, 0, w.n, params)
    n = w.n
    from oracle.build import cev_sample_size
    cev_rows = synth.sample_indices(w.seed_index, synth.TAG["cev_sample"], n, cev_sample_size(n))
    km_rows = synth.sample_indices(w.seed_index, synth.TAG["kmeans_sample"], n, min(n, 100_000))
    km_init = synth.permutation_prefix(w.seed_index, synth.TAG["kmeans_init"], np.arange(km_rows.size), w.k_half)
    arr = engine.build_index(x, w.m, w.k_half, g=lambda: sg.gaussian_matrix(w.seed_index, w.d), cev_rows=cev_rows,
                             km_rows=km_rows, km_init=km_init, keep_input=False)
    index = engine.Index(arr)
    trainq = sg.rows(w, 3004, 0, 20_000, params)
    evalq = sg.rows(w, w.seed_query, 0, 2000, params)
    kw = dict(alpha=0.002, tau=8, patience_factor=40)
    model = learned.train_budget(index, trainq, 10, epochs=15, **kw)
    plain_t = {"examined": torch.empty(2000, dtype=torch.int32, device="cuda")}
    ids_p, _ = index.search(evalq, 10, mode=1, taps=plain_t, **kw)
    lt = {"examined": torch.empty(2000, dtype=torch.int32, device="cuda")}
    ids_l, _ = index.search(evalq, 10, mode=1, budget_source=1, taps=lt, **kw)
    torch.cuda.synchronize()
    overlap = (ids_l[:, :, None] == ids_p[:, None, :]).any(-1).float().mean().item()
    ex_p = plain_t["examined"].float().mean().item()
    ex_l = lt["examined"].float().mean().item()
    print(f"plain verified {ex_p:.1f}, learned {ex_l:.1f}, overlap with plain {overlap:.4f}, delta {model.delta:.3f}")
    assert ex_l < ex_p
    assert overlap >= 0.995
