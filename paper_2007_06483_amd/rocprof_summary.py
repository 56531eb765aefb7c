"""Summaries of rocprofv3 output for the measurement notes in profiles/.

Reads the CSV files rocprofv3 writes with ``--output-format csv`` (kernel
traces and counter collections, found anywhere under the given directory) and
prints short Markdown tables; with ``--json`` the counter summary is also
written as the traffic file bench.py reads.  Host-side text processing only.

    python -m paper_2007_06483_amd.rocprof_summary trace DIR [--first k_zero]
    python -m paper_2007_06483_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR --workload NAME [--json FILE]
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2007_06483_amd", "csrc", f) for f in ("mtb_kernels.hip", "mtb_internal.h")]


def short_name(name: str) -> str:
    """Kernel name without namespaces, template and argument lists
    ("void ns::(anonymous namespace)::k<4>(ns::Args)" -> "k")."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    if n.endswith(")") and "(" in n:
        depth = 0
        for i in range(len(n) - 1, -1, -1):  # the argument list's opening parenthesis
            depth += n[i] == ")"
            depth -= n[i] == "("
            if depth == 0:
                n = n[:i]
                break
    n = n.split("<")[0]
    return n.split("::")[-1].strip() or name


def _rows(root: str, suffix: str):
    files = sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {root}")
    for path in files:
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def _grid(r: dict) -> str:
    if "Grid_Size_X" in r:
        dims = [r.get(f"Grid_Size_{a}", "1") for a in "XYZ"]
        while len(dims) > 1 and dims[-1] == "1":
            dims.pop()
        return "x".join(dims)
    return r.get("Grid_Size", "?")


def kernel_dispatches(root: str):
    """[(start_ns, end_ns, short name, grid)] of every kernel dispatch, by start time."""
    out = []
    for r in _rows(root, "kernel_trace.csv"):
        out.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]), _grid(r)))
    out.sort()
    return out


def trace_tables(root: str, first: str = "k_zero", last_names=("k_search_fine",)) -> str:
    d = kernel_dispatches(root)
    by = {}
    for s, e, n, _ in d:
        by.setdefault(n, []).append((e - s) / 1e3)
    total = sum(sum(v) for v in by.values())
    lines = ["| kernel | calls | average us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for n, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {n} | {len(v)} | {statistics.mean(v):.2f} | {min(v):.2f} | {max(v):.2f} | "
                     f"{100 * sum(v) / total:.1f}% |")
    # Steps: from each dispatch of `first` to the dispatch before the next one.
    starts = [i for i, x in enumerate(d) if x[2] == first]
    steps = []
    for a, b in zip(starts, starts[1:] + [len(d)]):
        seq = [x for x in d[a:b] if x[2].startswith("k_")]
        if not seq:
            continue
        span = (max(x[1] for x in seq) - seq[0][0]) / 1e3
        steps.append((span, seq))
    if steps:
        steps_sorted = sorted(steps, key=lambda t: t[0])
        span, seq = steps_sorted[len(steps_sorted) // 2]
        t0 = seq[0][0]
        lines += ["", f"Median step of {len(steps)} by span ({span:.1f} us from the start of {first} "
                      "to the end of its last kernel):", "",
                  "| kernel | grid (threads) | start us | duration us |", "|---|---|---|---|"]
        for s, e, n, g in seq:
            lines.append(f"| {n} | {g} | {(s - t0) / 1e3:.1f} | {(e - s) / 1e3:.1f} |")
    return "\n".join(lines)


def counter_means(root: str, counter: str):
    """{(short name, grid): mean value per dispatch} of one counter."""
    acc = {}
    for r in _rows(root, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (short_name(r["Kernel_Name"]), r.get("Grid_Size", "?"))
        acc.setdefault(key, []).append(float(r["Counter_Value"]))
    return {k: statistics.mean(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic(fetch_root: str, write_root: str, workload: str, copy_kernel: str = "__amd_rocclr_copyBuffer",
            copy_bytes: int = 1 << 30):
    """Per-dispatch HBM bytes of every kernel: FETCH_SIZE and WRITE_SIZE (KiB)
    scaled by what the same counters read for a device copy of copy_bytes
    (read and written), taken in the same runs."""
    fetch, n_f = counter_means(fetch_root, "FETCH_SIZE")
    write, _ = counter_means(write_root, "WRITE_SIZE")
    cf = [v for (n, _), v in fetch.items() if n == copy_kernel and v > 0.4 * copy_bytes / 1024]
    cw = [v for (n, _), v in write.items() if n == copy_kernel and v > 0.4 * copy_bytes / 1024]
    if not cf or not cw:
        raise SystemExit(f"no {copy_kernel} dispatch of {copy_bytes} bytes for calibration")
    f_factor = round(copy_bytes / 1024 / max(cf), 2)
    w_factor = round(copy_bytes / 1024 / max(cw), 2)
    kernels = {}
    for key in sorted(set(fetch) | set(write)):
        name, grid = key
        if not name.startswith("k_"):
            continue
        fk, wk = fetch.get(key, 0.0), write.get(key, 0.0)
        label = name if sum(1 for k in fetch if k[0] == name) <= 1 else f"{name}[{grid}]"
        kernels[label] = {"grid": grid, "dispatches": n_f.get(key, 0), "fetch_size_kib": round(fk, 1),
                          "write_size_kib": round(wk, 1), "read_bytes": int(fk * 1024 * f_factor),
                          "written_bytes": int(wk * 1024 * w_factor),
                          "traffic_bytes_per_launch": int(fk * 1024 * f_factor + wk * 1024 * w_factor)}
    return {"workload": workload, "kernel_source_sha256": kernel_source_sha256(), "fetch_factor": f_factor,
            "write_factor": w_factor, "kernels": kernels}


def traffic_table(t: dict) -> str:
    lines = [f"Calibration: bytes = FETCH_SIZE x {t['fetch_factor']} KiB + WRITE_SIZE x {t['write_factor']} KiB "
             "(from the 1 GiB device copy in the same runs).", "",
             "| kernel | grid | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB |",
             "|---|---|---|---|---|---|---|"]
    for k, v in t["kernels"].items():
        lines.append(f"| {k} | {v['grid']} | {v['dispatches']} | {v['fetch_size_kib']:.1f} | {v['write_size_kib']:.1f} | "
                     f"{v['read_bytes'] / 1e6:.1f} | {v['written_bytes'] / 1e6:.1f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--first", default="k_zero")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--workload", required=True)
    c.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_tables(a.dir, a.first))
    else:
        tr = traffic(a.fetch_dir, a.write_dir, a.workload)
        print(traffic_table(tr))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(tr, f, indent=1)
                f.write("\n")


if __name__ == "__main__":
    sys.exit(main())
