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


def test_adsampling_decision_on_a_rounding_tie():
    """Row B's running sum after 32 dimensions is exactly 1 by the definition
    (31 terms of 2^-54 absorbed) and 1 + 7 2^-52 when added lane-parallel;
    row A's key r puts the ADSampling threshold fl(r f_32) at 1 + 2 2^-52,
    between the two.  The definition does not prune B (1 <= threshold), so B
    (key 1) replaces A as the nearest neighbour; a decision taken on the
    lane-parallel sum would prune it."""
    from oracle import query as oquery
    from parity_util import compare
    w, x, q = make_workload("d128", n=3000, n_query=4)
    a, b, c = np.float32(1.4585433), np.float32(0.00051286776), np.float32(2.107314e-07)
    r = (np.float64(a) * np.float64(a) + np.float64(b) * np.float64(b)) + np.float64(c) * np.float64(c)
    f = oquery.ads_factors(w.d)
    assert r * f[0] == 1.0 + 2.0 ** -51                 # the threshold at t = 32
    x = x.copy()
    x[20] = 0.0
    x[20, :3] = [-a, -b, -c]
    x[30] = 0.0
    x[30, 0] = -1.0
    x[30, 1:32] = -2.0 ** -27
    q = q.copy()
    q[0] = 0.0
    idx = oracle_index(w, x, force_rotation=False)
    key, pre = oquery.sqdist_with_prefixes(q[0], x[[20, 30]])
    assert key[0] == r and pre[1, 0] == 1.0
    g = gpu_index(idx)
    for k in (1, 2):
        res = compare(idx, q, k, mode=1, alpha=1.0, tau=1, gpu=g, verify=1)
        assert res["ids"][0, 0] == 30 and res["dists"][0, 0] == np.float32(1.0)
