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
    with pytest.raises(engine.CrispError):
        plan.search(torch.from_numpy(np.concatenate([q, q])).cuda())       # 8 > max_batch
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
    assert b2 == 2 * b1
    ws = torch.empty(b1, dtype=torch.uint8, device="cuda")
    ids = torch.empty(16, 5, dtype=torch.int64, device="cuda")
    d = torch.empty(16, 5, dtype=torch.float32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    st = _lib.lib.crisp_search(g._h, P(qt), 16, 5, ctypes.byref(p2), P(ids), P(d), P(ws), b1, None, None)
    assert st == -2
