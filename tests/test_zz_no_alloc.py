"""crisp_search_static (the entry point that allocates nothing) against
crisp_search, through the C ABI (needs an MI355X).

Two calls in a row, the second with fewer queries, in both modes; the first
batch needs more workspace than the static scratch holds in one chunk, so
the entry point also has to cut it into smaller chunks.  Results must equal
crisp_search's bit for bit.
"""
import ctypes

import numpy as np
import pytest
import torch

from parity_util import gpu_index, make_workload, oracle_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    w, x, q = make_workload("d128", n_query=1400)
    idx = oracle_index(w, x)
    g = gpu_index(idx)
    g.enable_bf16()
    return w, q, g


def _static(g, qt, k, p):
    from paper_2603_05180_amd import _lib
    nq = int(qt.shape[0])
    ids = torch.full((nq, k), -7, dtype=torch.int64, device=g.device)
    dists = torch.full((nq, k), -7.0, dtype=torch.float32, device=g.device)
    st = _lib.lib.crisp_search_static(g._h, ctypes.c_void_p(qt.data_ptr()), nq, int(k), ctypes.byref(p),
                                      ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dists.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream(g.device).cuda_stream))
    assert st == 0, _lib.lib.crisp_last_error()
    return ids, dists


@pytest.mark.parametrize("mode,precision,persistent", [(0, 0, 0), (1, 0, 0), (1, 1, 1), (0, 1, 1)])
def test_static_scratch_equals_workspace_search(setup, mode, precision, persistent):
    from paper_2603_05180_amd import _lib
    w, q, g = setup
    kw = dict(mode=mode, alpha=0.05, tau=4, precision=precision, persistent=persistent)
    p = g.params(**kw)
    one = g.workspace_bytes(1, w.k, p)
    assert one * q.shape[0] > _lib.STATIC_SCRATCH_BYTES   # the first batch needs several chunks
    for nq in (q.shape[0], 301):
        print(f"static mode={mode} precision={precision} persistent={persistent} nq={nq}", flush=True)
        qt = torch.from_numpy(np.ascontiguousarray(q[:nq])).to(g.device)
        si, sd = _static(g, qt, w.k, p)
        ri, rd = g.search(qt, w.k, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(si.cpu().numpy(), ri.cpu().numpy())
        assert np.array_equal(sd.cpu().numpy().view(np.uint32), rd.cpu().numpy().view(np.uint32))
