"""Short text summaries of rocprofv3 output (CSV), for the profiles folder.

  python -m paper_2603_05180_amd.rocprof_summary stats <kernel_stats.csv> <title> <command>
      per-kernel dispatch durations from `rocprofv3 --kernel-trace --stats`
  python -m paper_2603_05180_amd.rocprof_summary dispatches <kernel_trace.csv> <kernel> [last]
      one kernel's dispatch durations grouped by grid size (from --kernel-trace),
      and the average of its last `last` dispatches
  python -m paper_2603_05180_amd.rocprof_summary traffic <fetch.csv> <write.csv> <kernel> <workload> <out.json> [last] [launches]
      HBM bytes per launch of <kernel> from two `--pmc FETCH_SIZE` / `--pmc
      WRITE_SIZE` runs, each scaled by what the same counter reads for the
      run's k_copy_probe dispatch (a plain copy: 1 GiB read, 1 GiB written);
      with `last`, over the kernel's last `last` dispatches only; with
      `launches`, their total divided by that many launches (a stage that
      dispatches the kernel more than once per launch)
"""
from __future__ import annotations

import collections
import csv
import json
import os
import sys


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")[:90]


def stats(path: str, title: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp):", "", "```", command, "```", "",
           "Per-kernel dispatch durations (`rocprofv3 --kernel-trace --stats`, kernel_stats.csv).", "",
           "| kernel | calls | total ms | avg us | min us | max us | % GPU time |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:24]:
        t = float(r["TotalDurationNs"])
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {t / 1e6:.2f} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {100 * t / tot:.2f} |")
    return "\n".join(out) + "\n"


def _matches(name: str, kernel: str) -> bool:
    """kernel 'k_count<0>' names one instantiation; 'k_rerank' every one."""
    short = _short(name)
    return short.endswith(kernel) if "<" in kernel else short.split("<")[0].endswith(kernel)


def dispatches(path: str, kernel: str, last: int = 0) -> str:
    groups = collections.defaultdict(list)
    seq = []
    for r in sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"])):
        if _matches(r["Kernel_Name"], kernel):
            grid = tuple(int(r[f"Grid_Size_{a}"]) // int(r[f"Workgroup_Size_{a}"]) for a in "XYZ")
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            groups[grid].append(us)
            seq.append(us)
    out = [f"Dispatches of `{kernel}` by grid (workgroups x, y, z), from the kernel trace:", "",
           "| grid | dispatches | avg us | min us | max us |", "|---|---:|---:|---:|---:|"]
    for grid, v in sorted(groups.items(), key=lambda kv: -len(kv[1])):
        out.append(f"| {grid[0]} x {grid[1]} x {grid[2]} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | "
                   f"{max(v):.1f} |")
    if last and len(seq) >= last:
        v = seq[-last:]
        out += ["", f"The last {last} dispatches (in time order): avg {sum(v) / len(v):.1f} us, "
                    f"min {min(v):.1f} us, max {max(v):.1f} us."]
    return "\n".join(out) + "\n"


def _per_dispatch(path: str, counter: str):
    acc = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        acc[r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = r["Kernel_Name"]
    return acc, names


def traffic(fetch_csv: str, write_csv: str, kernel: str, workload: str, out_json: str, last: int = 0,
            copy_bytes=1 << 30, launches: int = 0):
    """HBM bytes per launch of `kernel`: over its last `last` dispatches (in
    dispatch order; 0 = all of them), their total divided by `launches`
    (0 = one launch per dispatch)."""
    from .provenance import source_hash
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        acc, names = _per_dispatch(path, counter)
        copies = [v for d, v in acc.items() if "k_copy_probe" in names[d]]
        if len(copies) != 1:
            raise SystemExit(f"expected one k_copy_probe dispatch in {path}, found {len(copies)}")
        ref_kib = copies[0]
        factor = copy_bytes / (ref_kib * 1024.0)
        ks = [acc[d] for d in sorted(acc, key=int) if _matches(names[d], kernel)]
        if last:
            ks = ks[-last:]
        if not ks:
            raise SystemExit(f"no {kernel} dispatch in {path}")
        nl = launches if launches else len(ks)
        res[counter] = {"kib_per_launch": sum(ks) / nl, "launches": nl, "dispatches": len(ks), "copy_kib": ref_kib,
                        "factor": factor}
    t = json.load(open(out_json)) if os.path.exists(out_json) else {}
    t[kernel] = {"workload": workload, "source_hash": source_hash(),
                 "fetch_bytes_per_launch": res["FETCH_SIZE"]["kib_per_launch"] * 1024 * res["FETCH_SIZE"]["factor"],
                 "write_bytes_per_launch": res["WRITE_SIZE"]["kib_per_launch"] * 1024 * res["WRITE_SIZE"]["factor"],
                 "counters": res}
    with open(out_json, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    return t[kernel]


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        sys.stdout.write(stats(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "dispatches":
        sys.stdout.write(dispatches(sys.argv[2], sys.argv[3], int(sys.argv[4]) if len(sys.argv) > 4 else 0))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:7], last=int(sys.argv[7]) if len(sys.argv) > 7 else 0,
                                 launches=int(sys.argv[8]) if len(sys.argv) > 8 else 0), indent=1))
    else:
        raise SystemExit(__doc__)
