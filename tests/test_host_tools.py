"""Host-side measurement tools, on the CPU: the rocprofv3 CSV summaries, the
scaling of hardware byte counters by the copy probe, the gate that reports
HBM traffic only for the kernel sources it was measured on, and bench.py's
one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2603_05180_amd import rocprof_summary as rs
from paper_2603_05180_amd.provenance import source_hash

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)
    return str(path)


def test_kernel_names_match_one_instantiation_or_all():
    assert rs._matches("void crisp::k_count<0>(int const*, int const*, int)", "k_count<0>")
    assert not rs._matches("void crisp::k_count<1>(int const*, int const*, int)", "k_count<0>")
    assert rs._matches("void crisp::k_rerank<1, true>(float const*, int)", "k_rerank")
    assert rs._matches("void crisp::k_rerank<0, false>(float const*, int)", "k_rerank")
    assert rs._matches("void crisp::k_hamming_dist<2>(float const*, int)", "k_hamming_dist")
    assert not rs._matches("void crisp::k_hamming_place(int, int const*)", "k_hamming_dist")
    assert rs._matches("crisp::k_rotate_rows(float const*, long long, int)", "k_rotate_rows")


def _counter_rows(counter, values):
    """Counter rows as rocprofv3 writes them: one row per dispatch and
    hardware instance, summed per dispatch by the reader."""
    rows = []
    for did, (name, v) in enumerate(values, start=1):
        rows.append([did, name, counter, v / 2])
        rows.append([did, name, counter, v / 2])
    return rows


def test_traffic_scales_each_counter_by_the_copy_probe(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    cnt = "void crisp::k_count<0>(int const*)"
    # the copy probe moves 1 GiB each way: FETCH_SIZE reads half of that in
    # KiB (factor 2), WRITE_SIZE all of it (factor 1)
    fetch = _csv(tmp_path / "f.csv", hdr, _counter_rows("FETCH_SIZE", [
        ("void crisp::k_copy_probe(uint4 const*, uint4*, long long)", 524288.0),
        (cnt, 100.0), (cnt, 200.0), ("void crisp::k_count<1>(int const*)", 999.0), (cnt, 300.0), (cnt, 400.0)]))
    write = _csv(tmp_path / "w.csv", hdr, _counter_rows("WRITE_SIZE", [
        ("void crisp::k_copy_probe(uint4 const*, uint4*, long long)", 1048576.0),
        (cnt, 10.0), (cnt, 20.0), ("void crisp::k_count<1>(int const*)", 999.0), (cnt, 30.0), (cnt, 40.0)]))
    out = tmp_path / "traffic.json"
    ent = rs.traffic(fetch, write, "k_count<0>", "d4096", str(out), last=3)
    assert ent["counters"]["FETCH_SIZE"]["factor"] == pytest.approx(2.0)
    assert ent["counters"]["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    assert ent["counters"]["FETCH_SIZE"]["launches"] == 3
    assert ent["fetch_bytes_per_launch"] == pytest.approx(300.0 * 1024 * 2.0)    # mean of the last three
    assert ent["write_bytes_per_launch"] == pytest.approx(30.0 * 1024 * 1.0)
    saved = json.load(open(out))
    assert saved["k_count<0>"]["source_hash"] == source_hash()
    assert saved["k_count<0>"]["workload"] == "d4096"
    # every dispatch when `last` is 0
    ent = rs.traffic(fetch, write, "k_count<0>", "d4096", str(out))
    assert ent["fetch_bytes_per_launch"] == pytest.approx(250.0 * 1024 * 2.0)
    # a stage that dispatches the kernel twice per launch: the last four
    # dispatches are two launches
    ent = rs.traffic(fetch, write, "k_count<0>", "d4096", str(out), last=4, launches=2)
    assert ent["counters"]["FETCH_SIZE"]["launches"] == 2
    assert ent["counters"]["FETCH_SIZE"]["dispatches"] == 4
    assert ent["fetch_bytes_per_launch"] == pytest.approx(500.0 * 1024 * 2.0)


def test_traffic_needs_exactly_one_copy_probe(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    f = _csv(tmp_path / "f.csv", hdr, _counter_rows("FETCH_SIZE", [("void crisp::k_rerank<1, true>(int)", 5.0)]))
    with pytest.raises(SystemExit):
        rs.traffic(f, f, "k_rerank", "d4096", str(tmp_path / "t.json"))


def test_dispatches_group_by_grid_and_average_the_last(tmp_path):
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z",
           "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z"]
    k = "void crisp::k_rotate_rows(float const*, long long, int)"
    rows = [  # listed out of time order on purpose
        [k, 5000, 8000, 64 * 256, 15, 1, 256, 1, 1],           # 3 us, grid 64 x 15
        [k, 0, 2000, 64 * 256, 32, 1, 256, 1, 1],              # 2 us, grid 64 x 32
        ["void crisp::k_fill<int>(int*, long long, int)", 2500, 2600, 64, 1, 1, 64, 1, 1],
        [k, 3000, 4000, 64 * 256, 32, 1, 256, 1, 1],           # 1 us
    ]
    text = rs.dispatches(_csv(tmp_path / "t.csv", hdr, rows), "k_rotate_rows", last=2)
    assert "| 64 x 32 x 1 | 2 | 1.5 | 1.0 | 2.0 |" in text
    assert "| 64 x 15 x 1 | 1 | 3.0 | 3.0 | 3.0 |" in text
    assert "The last 2 dispatches (in time order): avg 2.0 us, min 1.0 us, max 3.0 us." in text
    assert "k_fill" not in text


def test_stats_table_orders_kernels_by_total_time(tmp_path):
    hdr = ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"]
    rows = [["void crisp::k_fill<int>(int*)", 10, 1e6, 1e5, 9e4, 2e5],
            ["void crisp::k_rotate_rows(float const*)", 3, 3e6, 1e6, 9e5, 1.1e6]]
    text = rs.stats(_csv(tmp_path / "s.csv", hdr, rows), "title", "cmd")
    lines = [l for l in text.splitlines() if l.startswith("| `")]
    assert lines[0].startswith("| `crisp::k_rotate_rows` | 3 | 3.00 | 1000.0 |")
    assert lines[0].endswith("| 75.00 |") and lines[1].endswith("| 25.00 |")


def test_bench_reports_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_rotate_rows", "d4096") is None          # no summary at all
    (tmp_path / "profiles").mkdir()
    ent = {"workload": "d4096", "source_hash": source_hash(),
           "fetch_bytes_per_launch": 1.5e9, "write_bytes_per_launch": 0.25e9}
    with open(tmp_path / "profiles" / "traffic.json", "w") as f:
        json.dump({"k_rotate_rows": ent, "k_rerank": dict(ent, source_hash="0" * 16)}, f)
    assert bench.measured_traffic("k_rotate_rows", "d4096") == pytest.approx(1.75e9)
    assert bench.measured_traffic("k_rotate_rows", "d3072") is None          # another workload
    assert bench.measured_traffic("k_rerank", "d4096") is None               # other kernel sources
    assert bench.measured_traffic("k_count<0>", "d4096") is None             # never measured


def test_bench_measures_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bench_matched_recall_and_cache_served_stages():
    """bench.py's learned-vs-plain comparison interpolates the plain sweep at
    the learned recall, and a byte-bound stage faster than HBM is labelled
    cache-served with no HBM fraction from algorithmic bytes."""
    import bench
    def form(pf, rec, qps, **kw):
        return {"_kw": dict(patience_factor=pf, **kw), "recall_at_k": rec, "queries_per_s": qps,
                "mean_verified": pf * 10.0}
    res = {"bf16": form(40, 0.999, 400.0), "bf16_pf10": form(10, 0.98, 500.0), "bf16_pf20": form(20, 0.995, 460.0),
           "learned_bf16": form(40, 0.9975, 450.0, budget_source=1)}
    mr = bench.matched_recall(res)
    # between pf20 (0.995, 460) and pf40 (0.999, 400): 460 - 0.625 * 60 = 422.5
    assert abs(mr["plain_queries_per_s_at_learned_recall"] - 422.5) < 1e-6
    assert mr["learned_gain"] > 0 and mr["outcome"].startswith("learned beats")
    res["learned_bf16"]["queries_per_s"] = 420.0
    assert bench.matched_recall(res)["outcome"].startswith("no gain")
    stages = {"rerank": {"ms": 10.0, "intervals": 5}, "hamming_dist": {"ms": 1.0, "intervals": 5},
              "dropped": 0}
    per_step = {"rerank": ("hbm", 10.0, 8000.0, "GB/s"), "hamming_dist": ("hbm", 50.0, 8000.0, "GB/s")}
    out, _ = bench.stage_rates(stages, 5, per_step, "none")
    assert out["rerank"]["bound"] == "hbm" and abs(out["rerank"]["frac"] - 5000.0 / 8000.0) < 1e-9
    assert out["hamming_dist"]["bound"] == "l2/mall" and out["hamming_dist"]["frac"] is None
