"""Short text summaries of rocprofv3 CSV output for the kernels of this library.

    python -m paper_1110_2921_amd.rocprof_summary trace  TRACE_DIR  [--command CMD]
    python -m paper_1110_2921_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR --workload NAME [--command CMD]
    python -m paper_1110_2921_amd.rocprof_summary counters PMC_DIR [--command CMD] [--top N]

``trace`` reads ``*_kernel_stats.csv`` and ``*_kernel_trace.csv`` of a
``rocprofv3 --kernel-trace --stats --output-format csv`` run and prints the
per-kernel table (calls, average and total time) plus the per-launch-shape
durations of the translation and near-field kernels.

``traffic`` reads the counter CSVs of two ``rocprofv3 --pmc`` runs of the same
command (``FETCH_SIZE``, then ``WRITE_SIZE``), calibrates both counters against
the largest device-to-device copy in the run (a copy of known size; bench.py
makes a 1 GiB one with ``--copy-calibration``) and prints, as one JSON object,
the HBM bytes per launch of the tree, expansion, M2L, P2P and Gaussian-sum
kernels, together with a SHA-256
of the library's kernel sources, so that a reader can tell whether the
figures still describe the code.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CALIBRATION_BYTES = 1 << 30


# the sources the profiled kernels (tree, expansions, translations, near field)
# and their launch configurations are built from
MEASURED_SOURCES = ("kernels.h", "device_harmonics.h", "kernels_tree.hip", "kernels_fmm.hip", "kernels_p2p.hip",
                    "kernels_m2l_sym.hip", "operators.h", "operators.cpp", "vmfmm.cpp")


def sources_sha256() -> str:
    """Hash of the sources of the measured kernels."""
    h = hashlib.sha256()
    for name in MEASURED_SOURCES:
        h.update(name.encode())
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    m = re.search(r"(k_\w+)(<[^>]*>)?\(", name)
    if m:
        return m.group(1) + (m.group(2) or "").replace(" ", "")
    return name.split("(")[0][:60]


def _one(d, pattern):
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits[0]


def trace_summary(d: str, command: str | None) -> str:
    stats = list(csv.DictReader(open(_one(d, "*kernel_stats.csv"))))
    trace = list(csv.DictReader(open(_one(d, "*kernel_trace.csv"))))
    out = []
    if command:
        out.append(f"command: {command}")
    out.append(f"{'kernel':48s} {'calls':>6s} {'avg ms':>10s} {'total ms':>10s} {'%':>6s}")
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        out.append(f"{short_name(r['Name']):48s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.3f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    shapes = collections.defaultdict(list)
    for r in trace:
        n = short_name(r["Kernel_Name"])
        if n.startswith(("k_m2l_os", "k_m2l_sym", "k_translate", "k_p2p", "k_split_reduce", "k_gauss")):
            key = (n, int(r["Grid_Size_X"]), int(r.get("Grid_Size_Y", 1) or 1))
            shapes[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    out.append("")
    out.append("per launch shape (grid x, grid y): launches, average ms")
    for (n, gx, gy), v in sorted(shapes.items()):
        out.append(f"  {n:40s} {gx:>9d} {gy:>4d} {len(v):5d} {sum(v) / len(v):10.3f}")
    return "\n".join(out)


def _counters(d: str, counter: str):
    """Per kernel name and per (name, grid size) launch shape: the counter's
    value of every dispatch; plus the values of the copy kernels."""
    rows = list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    per = collections.defaultdict(list)
    shape = collections.defaultdict(list)
    copies = []
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        n = short_name(r["Kernel_Name"])
        per[n].append(v)
        shape[(n, int(r["Grid_Size"]))].append(v)
        if "copyBuffer" in r["Kernel_Name"]:
            copies.append(v)
    return per, shape, copies


def traffic_summary(fetch_dir: str, write_dir: str, workload: str, command: str | None) -> dict:
    """Calibrated HBM bytes of each kernel: per dispatch averaged over all its
    dispatches, per evaluation (all its dispatches over the number of
    evaluations, counted by the key kernel, which runs once per evaluation:
    meaningful when the profiled command runs evaluations only) and per
    launch shape (grid size), so that one level's launch of a kernel that runs
    at every level can be read on its own."""
    fetch, fshape, fcopies = _counters(fetch_dir, "FETCH_SIZE")
    write, wshape, wcopies = _counters(write_dir, "WRITE_SIZE")
    if not wcopies:
        raise SystemExit("no copy kernel in the run: profile a command with --copy-calibration")
    # the calibration copy is the copy that writes the most
    i = max(range(len(wcopies)), key=lambda k: wcopies[k])
    w_kib = wcopies[i]
    f_kib = fcopies[max(range(len(fcopies)), key=lambda k: fcopies[k])]
    known_kib = CALIBRATION_BYTES / 1024.0
    ff, wf = known_kib / f_kib, known_kib / w_kib
    kernels = {}
    evals = len(fetch.get("k_keys", []))
    for name in sorted(set(fetch) | set(write)):
        if not name.startswith(("k_m2l_os", "k_m2l_sym", "k_sym_pack", "k_translate", "k_p2p", "k_split_reduce",
                                "k_permute",
                                "k_radix", "k_keys", "k_iota", "k_scan", "k_ranges", "k_p2m", "k_l2p",
                                "k_gauss", "k_pack", "k_multidot", "k_multiaxpy", "k_gather3", "k_scatter3")):
            continue
        fv, wv = fetch.get(name, []), write.get(name, [])
        if not fv or not wv:
            continue
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        shapes = []
        for (nm, grid) in sorted(k for k in fshape if k[0] == name):
            a, b = fshape[(nm, grid)], wshape.get((nm, grid), [])
            if not b:
                continue
            shapes.append({"grid_size": grid, "dispatches": len(a),
                           "hbm_bytes_per_dispatch": 1024.0 * (sum(a) / len(a) * ff + sum(b) / len(b) * wf)})
        kernels[name] = {"dispatches": len(fv), "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
                         "hbm_bytes_per_launch": 1024.0 * (fk * ff + wk * wf),
                         "hbm_bytes_per_evaluation": (1024.0 * (sum(fv) * ff + sum(wv) * wf) / evals
                                                      if evals else None),
                         "shapes": shapes}
    return {"workload": workload, "command": command, "evaluations": evals,
            "calibration": {"copy_bytes": CALIBRATION_BYTES, "fetch_kib": f_kib, "write_kib": w_kib,
                            "fetch_factor": ff, "write_factor": wf},
            "sources_sha256": sources_sha256(), "kernels": kernels}


def counters_summary(d: str, command: str | None, top: int = 8) -> str:
    """Average of every collected counter per dispatch, for the `top` library kernel
    launch shapes with the largest counts."""
    rows = list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        n = short_name(r["Kernel_Name"])
        if not n.startswith("k_"):
            continue
        per[(n, int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = [f"command: {command}"] if command else []
    for (n, g), cs in sorted(per.items(), key=lambda kv: -max(sum(v) for v in kv[1].values()))[:top]:
        first = next(iter(cs.values()))
        out.append(f"{n} grid {g} ({len(first)} dispatches)")
        for c, v in sorted(cs.items()):
            out.append(f"    {c:32s} {sum(v) / len(v):.4e}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--command")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("--workload", required=True)
    f.add_argument("--command")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--command")
    c.add_argument("--top", type=int, default=8)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        print(trace_summary(a.dir, a.command))
    elif a.mode == "counters":
        print(counters_summary(a.dir, a.command, a.top))
    else:
        print(json.dumps(traffic_summary(a.fetch_dir, a.write_dir, a.workload, a.command), indent=1))


if __name__ == "__main__":
    sys.exit(main())
