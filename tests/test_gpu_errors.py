"""Error handling of the C ABI on the GPU: bad parameters, corrupt indexes,
undersized workspace.  Every failing call is rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from parity_util import make_workload, oracle_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    w, x, q = make_workload("d128", n=2000, d=64, m=4, k_half=4, n_query=4)
    return w, x, q, oracle_index(w, x)


def test_bad_parameters(small):
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    g = engine.Index(idx)
    qt = torch.from_numpy(q).cuda()
    for kw in ({"mode": 2}, {"alpha": 0.0}, {"alpha": 1.5}, {"tau": -1}, {"tau": 9}):
        args = dict(mode=0, alpha=0.1, tau=2)
        args.update(kw)
        with pytest.raises(engine.CrispError) as e:
            g.search(qt, 5, **args)
        assert e.value.status == -1
    with pytest.raises(engine.CrispError):
        g.search(qt, 0, mode=0, alpha=0.1, tau=2)
    with pytest.raises(engine.CrispError):
        g.search(qt, 2001, mode=0, alpha=0.1, tau=2)


def test_workspace_too_small(small):
    from paper_2603_05180_amd import engine, _lib
    w, x, q, idx = small
    g = engine.Index(idx)
    qt = torch.from_numpy(q).cuda()
    p = g.params(mode=0, alpha=0.1, tau=2)
    need = g.workspace_bytes(4, 5, p)
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    ids = torch.empty(4, 5, dtype=torch.int64, device="cuda")
    d = torch.empty(4, 5, dtype=torch.float32, device="cuda")
    st = _lib.lib.crisp_search(g._h, ctypes.c_void_p(qt.data_ptr()), 4, 5, ctypes.byref(p),
                               ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, None)
    assert st == -2


def test_corrupt_csr_is_rejected(small):
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    bad = dict(idx)
    off = idx["offsets"].copy()
    off[1, 3] = off[1, 4] + 1          # non-monotone offsets
    bad["offsets"] = off
    with pytest.raises(engine.CrispError) as e:
        engine.Index(bad)
    assert e.value.status == -4
    bad = dict(idx)
    ids = idx["ids"].copy()
    ids[0, 0] = w.n + 5                 # id out of range
    bad["ids"] = ids
    with pytest.raises(engine.CrispError) as e:
        engine.Index(bad)
    assert e.value.status == -4


def test_optimized_mode_needs_codes(small):
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    nocodes = dict(idx)
    nocodes["codes"] = None
    g = engine.Index(nocodes)
    with pytest.raises(engine.CrispError) as e:
        g.search(torch.from_numpy(q).cuda(), 5, mode=1, alpha=0.1, tau=2)
    assert e.value.status == -5
    ids, d = g.search(torch.from_numpy(q).cuda(), 5, mode=0, alpha=0.1, tau=2)
    torch.cuda.synchronize()
    assert ids.shape == (4, 5)


def test_empty_batch_is_a_noop(small):
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    g = engine.Index(idx)
    ids, d = g.search(torch.empty(0, w.d, dtype=torch.float32, device="cuda"), 5, mode=0, alpha=0.1, tau=2)
    torch.cuda.synchronize()
    assert ids.shape == (0, 5)


def test_bad_options_and_plan_limits(small):
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    g = engine.Index(idx)
    qt = torch.from_numpy(q).cuda()
    for kw in ({"persistent": 2}, {"overlap": 2}, {"precision": 1}, {"precision": 3}, {"budget_source": 1}):
        with pytest.raises(engine.CrispError) as e:
            g.search(qt, 5, mode=1, alpha=0.1, tau=2, **kw)
        assert e.value.status == -1
    plan = engine.Plan(g, 4, 5, mode=1, alpha=0.1, tau=2)
    q8 = torch.from_numpy(np.concatenate([q, q])).cuda()
    with pytest.raises(ValueError):                                        # the binding: 8 > max_batch
        plan.search(q8)
    from paper_2603_05180_amd import _lib
    o_i = torch.empty(8, 5, dtype=torch.int64, device="cuda")
    o_d = torch.empty(8, 5, dtype=torch.float32, device="cuda")
    st = _lib.lib.crisp_plan_search(plan._h, ctypes.c_void_p(q8.data_ptr()), 8, ctypes.c_void_p(o_i.data_ptr()),
                                    ctypes.c_void_p(o_d.data_ptr()), None)
    assert st == -1                                                        # and the library itself
    plan.free()
    with pytest.raises(ValueError):
        engine.Plan(g, 4, 5, mode=1, alpha=0.1, tau=2, limits=torch.ones(4, dtype=torch.int32, device="cuda"))


def test_overlap_needs_the_doubled_workspace(small):
    from paper_2603_05180_amd import engine, _lib
    w, x, q, idx = small
    g = engine.Index(idx)
    qt = torch.from_numpy(np.concatenate([q] * 4)).cuda()
    p1 = g.params(mode=1, alpha=0.1, tau=2, max_chunk=4, overlap=0)
    p2 = g.params(mode=1, alpha=0.1, tau=2, max_chunk=4, overlap=1)
    b1, b2 = g.workspace_bytes(16, 5, p1), g.workspace_bytes(16, 5, p2)
    # a second chunk pipeline's workspace (the batch's overflow list is shared)
    assert b1 < b2 <= 2 * b1 and b2 - b1 > b1 // 2
    ws = torch.empty(b1, dtype=torch.uint8, device="cuda")
    ids = torch.empty(16, 5, dtype=torch.int64, device="cuda")
    d = torch.empty(16, 5, dtype=torch.float32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    st = _lib.lib.crisp_search(g._h, P(qt), 16, 5, ctypes.byref(p2), P(ids), P(d), P(ws), b1, None, None)
    assert st == -2


def test_mis_shaped_tensors_are_rejected_before_launch(small):
    """Outputs, taps and queries that do not match what the C side writes or
    reads raise ValueError in the binding (no launch)."""
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    g = engine.Index(idx)
    qt = torch.from_numpy(q).cuda()
    nq, k = qt.shape[0], 3
    good = (torch.empty(nq, k, dtype=torch.int64, device="cuda"), torch.empty(nq, k, dtype=torch.float32, device="cuda"))
    bad_outs = [
        (torch.empty(nq, k + 1, dtype=torch.int64, device="cuda"), good[1]),
        (good[0], torch.empty(nq, k, dtype=torch.float64, device="cuda")),
        (torch.empty(nq, k, dtype=torch.int32, device="cuda"), good[1]),
        (good[0], torch.empty(k, nq, dtype=torch.float32, device="cuda").t()),
        (torch.empty(nq, k, dtype=torch.int64), good[1]),
    ]
    for out in bad_outs:
        with pytest.raises(ValueError):
            g.search(qt, k, mode=0, alpha=0.1, tau=2, out=out)
        with pytest.raises(ValueError):
            g.search_static(qt, k, mode=0, alpha=0.1, tau=2, out=out)
    taps = g.alloc_taps(nq, 1)
    taps["cand"] = torch.empty(nq, g.n - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        g.search(qt, k, mode=1, alpha=0.1, tau=2, taps=taps)
    with pytest.raises(ValueError):
        g.search(qt, k, mode=0, alpha=0.1, tau=2, taps={"nonsense": good[0]})
    plan = engine.Plan(g, 8, k, mode=0, alpha=0.1, tau=2)
    with pytest.raises(ValueError):
        plan.search(qt[:, : g.d // 2].contiguous())
    with pytest.raises(ValueError):
        plan.search(qt.reshape(-1))
    with pytest.raises(ValueError):
        plan.search(torch.zeros(9, g.d, device="cuda"))
    with pytest.raises(ValueError):
        plan.search(qt, out=bad_outs[0])
    ids, d = g.search(qt, k, mode=0, alpha=0.1, tau=2, out=good)
    torch.cuda.synchronize()
    assert ids.data_ptr() == good[0].data_ptr()
    plan.free()


def test_searches_on_two_streams_use_two_workspaces(small):
    from paper_2603_05180_amd import engine
    w, x, q, idx = small
    g = engine.Index(idx)
    qt = torch.from_numpy(q).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    a = g.search(qt, 3, mode=0, alpha=0.1, tau=2, stream=s1)
    b = g.search(qt, 3, mode=0, alpha=0.1, tau=2, stream=s2)
    torch.cuda.synchronize()
    assert len(g._ws) >= 2
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
