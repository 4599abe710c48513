"""GPU engine vs oracle, element by element, through the C ABI (needs an MI355X).

Indexes are built by the oracle (CPU) and loaded by the engine as data, so
the two sides search the same index.  Every stage is compared bit for bit:
rotated queries, half distances, activated cells and weights, candidate
lists and scores, threshold after the fallback, Hamming order, verified
prefix, and the final ids and float32 distances.
"""
import numpy as np
import pytest

from parity_util import compare, gpu_index, make_workload, oracle_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def d128():
    w, x, q = make_workload("d128")
    idx = oracle_index(w, x)
    return w, x, q, idx


@pytest.mark.parametrize("mode,alpha,tau", [(0, 0.05, 4), (0, 0.02, 6), (1, 0.05, 4), (1, 0.1, 6)])
def test_d128_full(d128, mode, alpha, tau):
    """Plain Guaranteed / Optimized Mode at the CPU-fast size (N=10k, D=128, 100 queries)."""
    w, x, q, idx = d128
    print(f"d128 mode={mode} alpha={alpha} tau={tau}", flush=True)
    compare(idx, q, w.k, mode=mode, alpha=alpha, tau=tau)


def test_d128_ragged_tiles_and_chunks(d128):
    """4096-id tiles (N=10k: 3 tiles, ragged tail) and 7-query chunks."""
    w, x, q, idx = d128
    print("d128 tiles=4096 chunk=7", flush=True)
    compare(idx, q[:30], w.k, mode=1, alpha=0.05, tau=4, tile_ids=4096, max_chunk=7)
    compare(idx, q[:30], w.k, mode=0, alpha=0.05, tau=4, tile_ids=4096, max_chunk=7)


def test_fallback_and_degenerate_thresholds(d128):
    w, x, q, idx = d128
    g = gpu_index(idx)
    print("fallback tau=16", flush=True)
    s = compare(idx, q[:20], w.k, mode=0, alpha=0.002, tau=16, gpu=g)          # forces the fallback
    assert min(s["n_cand"]) >= w.k
    print("tau=0", flush=True)
    compare(idx, q[:5], w.k, mode=0, alpha=0.01, tau=0, gpu=g)                 # every point a candidate
    print("alpha=1", flush=True)
    compare(idx, q[:5], w.k, mode=1, alpha=1.0, tau=8, gpu=g)                  # every cell activated
    print("k=1", flush=True)
    compare(idx, q[:10], 1, mode=1, alpha=0.02, tau=3, gpu=g)
    print("k=100", flush=True)
    compare(idx, q[:10], 100, mode=0, alpha=0.02, tau=3, gpu=g)
    print("single query", flush=True)
    compare(idx, q[:1], w.k, mode=1, alpha=0.03, tau=2, gpu=g, patience_factor=1)


def test_padding_when_too_few_points_collide():
    w, x, q = make_workload("d128", n=600, d=64, m=2, k_half=4, n_query=6)
    idx = oracle_index(w, x)
    print("padding", flush=True)
    compare(idx, q, 50, mode=0, alpha=0.001, tau=2)


def test_learned_prefix_limits(d128):
    w, x, q, idx = d128
    lim = np.array([1, 5, 17, 0, 200, 3] * 5, dtype=np.int32)
    print("limits", flush=True)
    compare(idx, q[:30], w.k, mode=1, alpha=0.05, tau=4, limits=lim)


K_ABOVE_64_OFF = ("the library refuses K > 64: its selection path for K > 64 faulted the GPU in a search "
                  "at N = 1M, D = 960, K = 256 and the cause is not found yet")


@pytest.mark.parametrize("k_half", [1, 64, pytest.param(80, marks=pytest.mark.skip(reason=K_ABOVE_64_OFF))])
def test_codebook_sizes(k_half):
    """K = 1 (one cell), K = 64 (4096 cells), K = 80 (prefix tables in device memory)."""
    w, x, q = make_workload("d128", n=4000, d=128, m=4, k_half=k_half, n_query=12)
    idx = oracle_index(w, x)
    print(f"K={k_half}", flush=True)
    for mode in (0, 1):
        compare(idx, q, 10, mode=mode, alpha=0.03, tau=2)


def test_tied_half_distances():
    """Centroids 0 and 1 of every half made equal (and 2 equal to 3 in half
    1): every query has tied half distances, which the (distance, index)
    order breaks by index; the selection must rank them as the oracle does."""
    w, x, q = make_workload("d128", n=4000, d=128, m=4, k_half=8, n_query=10)
    idx = oracle_index(w, x)
    cent = idx["centroids"].copy()
    cent[:, :, 1] = cent[:, :, 0]
    cent[:, 1, 3] = cent[:, 1, 2]
    idx = dict(idx, centroids=cent)
    for mode in (0, 1):
        compare(idx, q, 10, mode=mode, alpha=0.03, tau=2)


def test_cell_selection_beyond_direct_pops():
    """K = 32 (1,024 cells of about three ids) with half the points as the
    budget: several hundred cells per subspace, more than the direct
    enumeration pops, so the selection takes its bisection path (prefix
    sums of cell sizes summed from the offsets)."""
    w, x, q = make_workload("d128", n=3000, d=128, m=4, k_half=32, n_query=8)
    idx = oracle_index(w, x)
    print("K=32 alpha=0.5", flush=True)
    for mode in (0, 1):
        s = compare(idx, q, 10, mode=mode, alpha=0.5, tau=3)
        assert int(s["taps"]["n_cells"].min()) > 256


def test_rotated_index():
    """Correlated data: the rotation fires, queries are rotated on the GPU."""
    w, x, q = make_workload("d4096", n=3000, d=256, m=8, k_half=6, rank=16, n_query=16)
    idx = oracle_index(w, x)
    assert idx["rotation"] is not None
    print("rotated", flush=True)
    for mode in (0, 1):
        compare(idx, q, 10, mode=mode, alpha=0.05, tau=3)


def test_wide_rows_several_tiles():
    """D = 1024 (float4 path), 5 tiles of 4096 with a ragged tail."""
    w, x, q = make_workload("d4096", n=18000, d=1024, m=16, k_half=8, rank=32, n_query=10)
    idx = oracle_index(w, x)
    print("D=1024", flush=True)
    for mode in (0, 1):
        compare(idx, q, 10, mode=mode, alpha=0.02, tau=4, tile_ids=4096)


@pytest.mark.parametrize("d,m,cases", [
    (256, 64, [(1, 0.5, 128), (1, 0.5, 108), (0, 0.3, 32)]),
    (192, 96, [(1, 0.5, 130), (1, 0.5, 172), (0, 0.3, 48)]),
])
def test_many_subspaces_scores_above_127(d, m, cases):
    """M = 64 and 96: Optimized-Mode scores reach 2M = 128 and 192, so the
    counting scan takes its 16-bit-field test; thresholds near the top force
    the fallback passes (tau 128 = 2M at M = 64 drops to tau_eff of about 120)."""
    w, x, q = make_workload("d128", n=3000, d=d, m=m, k_half=4, n_query=6)
    idx = oracle_index(w, x)
    for tile in (0, 4096):
        g = gpu_index(idx, tile)
        for mode, alpha, tau in cases:
            print(f"M={m} tile={tile} mode={mode} alpha={alpha} tau={tau}", flush=True)
            compare(idx, q, 10, mode=mode, alpha=alpha, tau=tau, gpu=g)


@pytest.mark.parametrize("d,m", [(192, 4), (320, 5), (448, 7)])
def test_code_widths_not_a_power_of_two(d, m):
    """3, 5 and 7 sign-code words per row: the Hamming kernel's lanes per row
    must still cover every word exactly once."""
    w, x, q = make_workload("d4096", n=2500, d=d, m=m, k_half=6, rank=8, n_query=12)
    idx = oracle_index(w, x)
    print(f"D={d} M={m}", flush=True)
    for mode in (0, 1):
        compare(idx, q, 10, mode=mode, alpha=0.05, tau=3)


def test_hamming_order_wide_ranges():
    """Every point a candidate (alpha = 1, tau = 1) at D = 1024: each query's
    Hamming distances span several hundred values, and the (h, id) order must
    still equal the oracle's."""
    from oracle import query as oquery
    w, x, q = make_workload("d4096", n=3000, d=1024, m=8, k_half=6, rank=16, n_query=6)
    idx = oracle_index(w, x)
    spans = []
    for qi in range(q.shape[0]):
        _, _, tr = oquery.search_one(idx, q[qi], 10, mode=1, alpha=1.0, tau=1, trace=True)
        spans.append(int(tr["hamming"].max() - tr["hamming"].min()))
    print("D=1024 alpha=1 spans", spans, flush=True)
    assert min(spans) >= 256, spans
    compare(idx, q, 10, mode=1, alpha=1.0, tau=1)


@pytest.mark.parametrize("pf", [40, 300])
def test_hamming_order_placed_span_above_1024(pf):
    """D = 2048, every point a candidate, base rows among the queries (a
    Hamming distance of 0 to themselves): the placed bins of those queries
    span more than 1,024 distances (the placement by one wave) while the
    others span fewer (the placement by all waves of the block); with patience
    300 * k every candidate is placed, with 40 * k a prefix."""
    from oracle import query as oquery
    w, x, q = make_workload("d128", n=3000, d=2048, m=8, k_half=6, n_query=3)
    q = np.ascontiguousarray(np.concatenate([x[[0, 7, 1500]], q]), dtype=np.float32)
    idx = oracle_index(w, x, force_rotation=False)
    spans = []
    for qi in range(q.shape[0]):
        _, _, tr = oquery.search_one(idx, q[qi], 10, mode=1, alpha=1.0, tau=1, trace=True)
        h = np.sort(tr["hamming"])
        plen = min(h.size, 2 * pf * 10 + 1024)
        spans.append(int(h[plen - 1] - h[0]))
    print(f"D=2048 patience={pf} placed spans", spans, flush=True)
    if pf == 300:
        assert max(spans) > 1024 and min(spans) <= 1024, spans
    compare(idx, q, 10, mode=1, alpha=1.0, tau=1, patience_factor=pf)


@pytest.mark.parametrize("precision", [0, 1])
def test_walk_in_id_order(d128, precision):
    """Optimized Mode without the Hamming order (the Section 6.4 ablation):
    candidates verified in ascending id order, patience as usual."""
    w, x, q, idx = d128[:4]
    g = gpu_index(idx)
    if precision:
        g.enable_bf16()
    for pf in (2, 40):
        print(f"id-order walk precision={precision} patience={pf}", flush=True)
        compare(idx, q, w.k, mode=1, alpha=0.05, tau=4, patience_factor=pf, gpu=g, precision=precision,
                walk_order=1)


@pytest.fixture(scope="module")
def d128_rotated():
    w, x, q = make_workload("d128", n_query=60)
    idx = oracle_index(w, x, force_rotation=True)
    return w, x, q, idx


@pytest.mark.parametrize("k,pf", [(1, 40), (10, 2), (10, 40), (100, 5)])
def test_adsampling_walk(d128_rotated, k, pf):
    """Optimized Mode with ADSampling (Eq. (2)) on a rotated index: the
    verified prefix, last update, stop flag, ids and distances equal the
    oracle's sequential walk."""
    w, x, q, idx = d128_rotated
    g = gpu_index(idx)
    print(f"adsampling k={k} patience={pf}", flush=True)
    r = compare(idx, q, k, mode=1, alpha=0.05, tau=4, patience_factor=pf, gpu=g, verify=1)
    assert sum(r["n_cand"]) > 0


def test_adsampling_unrotated_chunks_and_limits(d128):
    """Unrotated data (the test still runs; only its statistics change),
    7-query chunks, learned-style prefix limits."""
    w, x, q, idx = d128[:4]
    g = gpu_index(idx)
    lim = np.array([0, 1, 5, 17, 40, 300] * 17)[: q.shape[0]]
    compare(idx, q, 10, mode=1, alpha=0.05, tau=4, patience_factor=3, gpu=g, verify=1, max_chunk=7, limits=lim)


def test_adsampling_rejects_guaranteed_and_bf16(d128):
    import torch
    from paper_2603_05180_amd import engine
    w, x, q, idx = d128[:4]
    g = gpu_index(idx)
    g.enable_bf16()
    qt = torch.from_numpy(q).cuda()
    for kw in (dict(mode=0), dict(mode=1, precision=1), dict(mode=1, verify=2)):
        args = dict(alpha=0.05, tau=4, verify=1)
        args.update(kw)
        with pytest.raises(engine.CrispError):
            g.search(qt, 10, **args)
