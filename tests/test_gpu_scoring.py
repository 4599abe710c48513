"""Certified matrix-core pre-scoring of the half distances (needs an
MI355X): bfloat16 (precision 2) and FP8 e4m3 (precision 3).  The scoring
kernel's bounds must contain the exact float64 half distances; and a search
with precision 2 or 3 must return exactly what precision 0 and the oracle
return, with the same activated cells, candidates and walk, both when the
cell walk stays inside the certified ranks and when it needs the exact path
(hundreds of cells per subspace)."""
import numpy as np
import pytest
import torch

from oracle import query as oquery
from parity_util import gpu_index, make_workload, oracle_index, run_gpu

pytestmark = pytest.mark.gpu

CASES = {
    # K = 8: every rank certified outright
    "K8": (("d128", dict()), dict(mode=1, alpha=0.05, tau=4)),
    # K = 32 and 64 over 4,000 points
    "K32": (("d128", dict(n=4000, m=4, k_half=32, n_query=24)), dict(mode=1, alpha=0.03, tau=2)),
    "K64": (("d128", dict(n=4000, m=4, k_half=64, n_query=24)), dict(mode=0, alpha=0.03, tau=2)),
    # K = 50 with h = 64 coordinates per half, the large workload's codebook shape
    "K50h64": (("d4096", dict(n=6000, d=256, m=2, k_half=50, rank=16, n_query=24)), dict(mode=1, alpha=0.01, tau=1)),
    # half the points as the budget: hundreds of cells, beyond the certified ranks
    "K32wide": (("d128", dict(n=3000, m=4, k_half=32, n_query=12)), dict(mode=0, alpha=0.5, tau=3)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    (base, wkw), kw = CASES[request.param]
    w, x, q = make_workload(base, **wkw)
    idx = oracle_index(w, x)
    g = gpu_index(idx)
    g.enable_bf16()
    return request.param, w, q, idx, g, kw


@pytest.mark.parametrize("precision", [2, 3])
def test_bounds_contain_the_exact_half_distances(case, precision):
    name, w, q, idx, g, kw = case
    nq, m, kh = q.shape[0], idx["m"], idx["k_half"]
    z = dict(device=g.device)
    taps = {"half_dist": torch.empty(nq, m, 2, kh, dtype=torch.float64, **z),
            "score_lb": torch.empty(nq, m, 2, kh, dtype=torch.float32, **z),
            "score_ub": torch.empty(nq, m, 2, kh, dtype=torch.float32, **z)}
    qt = torch.from_numpy(np.ascontiguousarray(q)).to(g.device)
    print(f"{name}: bounds, precision {precision}", flush=True)
    g.search(qt, 10, precision=precision, taps=taps, **kw)
    torch.cuda.synchronize()
    hd = taps["half_dist"].cpu().numpy()
    lb = taps["score_lb"].cpu().numpy().astype(np.float64)
    ub = taps["score_ub"].cpu().numpy().astype(np.float64)
    assert np.all(lb >= 0)
    assert np.all(lb <= hd), (name, float((lb - hd).max()))
    assert np.all(hd <= ub), (name, float((hd - ub).max()))
    # the bounds are tight enough to certify (reported, not asserted)
    print(f"{name}: precision {precision}, median relative width "
          f"{float(np.median((ub - lb) / np.maximum(hd, 1e-30))):.2e}")


@pytest.mark.parametrize("precision", [2, 3])
def test_results_equal_precision_0_and_the_oracle(case, precision):
    name, w, q, idx, g, kw = case
    k = 10
    print(f"{name}: precision 0 vs {precision}", flush=True)
    i0, d0, t0 = run_gpu(g, q, k, precision=0, **kw)
    taps = g.alloc_taps(q.shape[0], kw["mode"])
    del taps["half_dist"]            # with it the selection takes the exact path
    qt = torch.from_numpy(np.ascontiguousarray(q)).to(g.device)
    taps["score_fallback"] = torch.empty(q.shape[0], dtype=torch.int32, device=g.device)
    ids, d = g.search(qt, k, precision=precision, taps=taps, **kw)
    torch.cuda.synchronize()
    i2, d2 = ids.cpu().numpy(), d.cpu().numpy()
    t2 = {key: v.cpu().numpy() for key, v in taps.items()}
    fb = t2["score_fallback"]
    assert np.all((fb >= 0) & (fb <= idx["m"]))
    print(f"{name}: precision {precision}, exact-path subspaces {int(fb.sum())} of {fb.size * idx['m']}")
    assert np.array_equal(i2, i0)
    assert np.array_equal(d2.view(np.uint32), d0.view(np.uint32))
    keys = ["n_cells", "retrieved", "hist", "tau_eff", "n_cand", "examined", "last_update", "stopped"]
    if kw["mode"] == 1:
        keys.append("features")       # built from the selection's statistics
    for key in keys:
        assert np.array_equal(t2[key].view(np.uint32) if key == "features" else t2[key],
                              t0[key].view(np.uint32) if key == "features" else t0[key]), key
    for qi in range(q.shape[0]):
        nc = int(t0["n_cand"][qi])
        assert np.array_equal(t2["cand"][qi, :nc], t0["cand"][qi, :nc])
        if kw["mode"] == 1:
            assert np.array_equal(t2["order"][qi, :nc], t0["order"][qi, :nc])
        for sub in range(idx["m"]):
            n = int(t0["n_cells"][qi, sub])
            assert sorted(t2["cells"][qi, sub, :n].tolist()) == sorted(t0["cells"][qi, sub, :n].tolist())
    oi, od, _ = oquery.search(idx, q, k, **kw)
    assert np.array_equal(i2, oi)
    assert np.array_equal(d2.view(np.uint32), od.view(np.uint32))
