"""The distance key on rows where summation order matters (needs an MI355X).

The key is the squared L2 distance summed in float64 over the dimensions in
ascending order (Section 4.3.2, Stage 3).  The engine adds the terms
lane-parallel and falls back to that definition whenever the two orders
could disagree on a comparison or on the returned float32 value.  The rows
of ``key_stress_rows`` are built so that they do disagree: ordering by the
lane-parallel value would rank B before A and return 1 + 2^-23 for C, where
the definition ranks A (and its duplicate) first and returns 1.0 for C.
"""
import numpy as np
import pytest

from parity_util import compare, gpu_index, key_stress_rows, make_workload, oracle_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stress():
    w, x, q = make_workload("d128", n=3000, n_query=8)
    x = x.copy()
    rows = key_stress_rows(w.d)
    x[5] = rows["B"]
    x[17] = rows["A"]
    x[18] = rows["A"]        # duplicate: the tie goes to the smaller id
    x[40] = rows["C"]
    q = q.copy()
    q[0] = 0.0
    q[3] = 0.0
    idx = oracle_index(w, x, force_rotation=False)
    g = gpu_index(idx)
    g.enable_bf16()
    return w, x, q, idx, g


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 10])
def test_defined_key_decides(stress, mode, precision, k):
    w, x, q, idx, g = stress
    print(f"key stress mode={mode} precision={precision} k={k}", flush=True)
    r = compare(idx, q, k, mode=mode, alpha=1.0, tau=1, gpu=g, precision=precision, check_stages=(k == 4))
    want = [17, 18, 5, 40][:k]
    assert list(r["ids"][0, :len(want)]) == want
    if k >= 4:
        assert r["dists"][0, 3] == np.float32(1.0)
