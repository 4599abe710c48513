"""Mixed-precision verification on the GPU vs the oracle (needs an MI355X).

With precision 1 every verified row is first read from a bfloat16 copy to
bound its distance and read in float32 only where the bound cannot exclude
it; every comparison that decides a result still uses the exact float64
key, so ids and distances must equal the oracle's (and the float32 path's)
bit for bit, including on inputs built to stress the bounds: duplicate
rows, rows closer to each other than bfloat16 can resolve, and queries
that coincide with data points.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from parity_util import compare, gpu_index, make_workload, oracle_index, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def d128():
    w, x, q = make_workload("d128")
    idx = oracle_index(w, x)
    g = gpu_index(idx)
    g.enable_bf16()
    return w, x, q, idx, g


def test_bf16_copy_and_row_error_bounds(d128):
    w, x, q, idx, g = d128
    rows, err = g.bf16_rows()
    torch.cuda.synchronize()
    got = rows.cpu().view(torch.int16).numpy().view(np.uint16)
    base = idx["base"]
    ref = omlp.to_bf16(base).view(np.uint32) >> np.uint32(16)
    assert np.array_equal(got, ref.astype(np.uint16))
    xt = (ref.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    true = np.sqrt(((base.astype(np.float64) - xt) ** 2).sum(1))
    e = err.cpu().numpy().astype(np.float64)
    assert np.all(e >= true)
    assert np.all(e <= true * (1 + 1e-6) + 1e-30)


def _both(idx, g, q, k, **kw):
    """precision 0 and 1 through the engine, then precision 1 against the oracle."""
    i0, d0, t0 = run_gpu(g, q, k, precision=0, **kw)
    s = compare(idx, q, k, gpu=g, precision=1, check_stages=False, **kw)
    t1 = s["taps"]
    assert np.array_equal(i0, s["ids"])
    assert np.array_equal(d0.view(np.uint32), s["dists"].view(np.uint32))
    for key in ("examined", "last_update", "stopped"):
        assert np.array_equal(t0[key], t1[key]), key
    assert np.array_equal(t0["refined"], t0["examined"])
    assert np.all(t1["refined"] <= t1["examined"])
    return t0, t1


@pytest.mark.parametrize("mode,alpha,tau,k", [(0, 0.05, 4, 10), (0, 0.02, 6, 1), (0, 0.05, 2, 100),
                                              (1, 0.05, 4, 10), (1, 0.1, 6, 1), (1, 0.05, 2, 100)])
def test_d128_bf16_equals_oracle(d128, mode, alpha, tau, k):
    w, x, q, idx, g = d128
    print(f"d128 bf16 mode={mode} alpha={alpha} tau={tau} k={k}", flush=True)
    t0, t1 = _both(idx, g, q, k, mode=mode, alpha=alpha, tau=tau)
    frac = t1["refined"].sum() / max(1, t1["examined"].sum())
    print(f"  float32 rows read: {frac:.3f} of the verified rows", flush=True)
    if mode == 0 and k == 10:
        assert frac < 0.5


def test_ragged_width_and_rotation():
    """D = 192 (bfloat16 row groups do not fill the wave) on a rotated index."""
    w, x, q = make_workload("d4096", n=3000, d=192, m=4, k_half=6, rank=8, n_query=24)
    idx = oracle_index(w, x)
    assert idx["rotation"] is not None
    g = gpu_index(idx)
    g.enable_bf16()
    print("D=192 rotated bf16", flush=True)
    for mode in (0, 1):
        _both(idx, g, q, 10, mode=mode, alpha=0.05, tau=3)


def test_ties_near_duplicates_and_exact_hits():
    w, x, q = make_workload("d128", n=4000, d=128, m=8, k_half=8, n_query=40)
    x = x.copy()
    x[1::4] = x[0::4]                                     # exact duplicates (ties broken by id)
    x[2::4] = x[0::4] + np.float32(1e-5) * np.sign(x[0::4])  # closer than bfloat16 resolves
    q = q.copy()
    q[::2] = x[:q.shape[0] * 4:8]                         # queries on data points (distance 0)
    idx = oracle_index(w, x)
    g = gpu_index(idx)
    g.enable_bf16()
    for mode in (0, 1):
        for k in (1, 3, 10):
            print(f"ties mode={mode} k={k}", flush=True)
            _both(idx, g, q, k, mode=mode, alpha=0.05, tau=4)


def test_precision_needs_the_bf16_copy():
    from paper_2603_05180_amd._lib import CrispError
    w, x, q = make_workload("d128", n=800, d=64, m=2, k_half=4, n_query=3)
    idx = oracle_index(w, x)
    g = gpu_index(idx)
    with pytest.raises(CrispError):
        g.search(torch.from_numpy(q).cuda(), 5, mode=0, alpha=0.1, tau=1, precision=1)
    with pytest.raises(CrispError):
        g.search(torch.from_numpy(q).cuda(), 5, mode=0, alpha=0.1, tau=1, precision=2)
