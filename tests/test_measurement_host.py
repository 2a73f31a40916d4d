"""Host logic of the measurement (no GPU): the work counts bench.py divides
by, and the rocprofv3 summaries its roofline fields are read from.

* M2L translations over the levels of a uniform tree and near-field pairs of
  a leaf population: brute force over cells and offsets.
* rocprof_summary on small synthetic CSV files in rocprofv3's column layout:
  the copy calibration (FETCH_SIZE of a 1 GiB copy reads half its bytes),
  per-dispatch, per-evaluation and per-launch-shape bytes, kernel names, the
  per-shape trace durations.
* bench.py takes the committed traffic summary only while the sources hash
  it records matches the sources.
"""
import csv
import itertools
import json
import os

import numpy as np
import pytest

import bench
from paper_1110_2921_amd import rocprof_summary as R


def _spread(c, level):
    k = 0
    for b in range(level):
        k |= ((c >> b) & 1) << (3 * b)
    return k


def _brute_m2l(level, periodic):
    total = 0
    for l in range((1 if periodic else 2), level + 1):
        side = 1 << l
        for c in itertools.product(range(side), repeat=3):
            par = [ci >> 1 for ci in c]
            for dq in itertools.product((-1, 0, 1), repeat=3):
                q = [par[a] + dq[a] for a in range(3)]
                if not periodic and any(v < 0 or v >= side // 2 for v in q):
                    continue
                for ch in itertools.product((0, 1), repeat=3):
                    s = [2 * q[a] + ch[a] for a in range(3)]
                    if max(abs(s[a] - c[a]) for a in range(3)) > 1:
                        total += 1
    return total


@pytest.mark.parametrize("level,periodic", [(2, 0), (3, 0), (4, 0), (2, 1), (3, 1)])
def test_m2l_translation_count(level, periodic):
    assert bench.m2l_translations(level, periodic) == _brute_m2l(level, periodic)


@pytest.mark.parametrize("level,periodic", [(1, 0), (1, 1), (2, 0), (2, 1), (3, 1)])
def test_near_pair_count(level, periodic):
    side = 1 << level
    rng = np.random.default_rng(level + 10 * periodic)
    counts = rng.integers(0, 9, size=side ** 3)          # by Morton key
    start = np.concatenate([[0], np.cumsum(counts)])
    want = 0
    for c in itertools.product(range(side), repeat=3):
        kt = _spread(c[0], level) | (_spread(c[1], level) << 1) | (_spread(c[2], level) << 2)
        for d in itertools.product((-1, 0, 1), repeat=3):
            s = [c[a] + d[a] for a in range(3)]
            if periodic:
                s = [v % side for v in s]
            elif any(v < 0 or v >= side for v in s):
                continue
            ks = _spread(s[0], level) | (_spread(s[1], level) << 1) | (_spread(s[2], level) << 2)
            want += int(counts[kt]) * int(counts[ks])
    assert bench.near_pairs(start, level, periodic) == want


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _pmc_rows(counter, per_kernel):
    return [{"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v, "Grid_Size": g}
            for name, g, v in per_kernel]


def test_traffic_summary_calibrates_and_splits_by_shape(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = float(1 << 20)
    fetch = [(copy, 1 << 20, gib_kib / 2),                       # FETCH_SIZE sees half the copy
             ("void vmfmm::k_keys(int, double const*)", 4096, 100.0),
             ("void vmfmm::k_keys(int, double const*)", 4096, 100.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 3145728, 4000.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 393216, 500.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 3145728, 4200.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 393216, 520.0),
             ("void other_lib_kernel(int)", 64, 9.0)]
    write = [(copy, 1 << 20, gib_kib),
             ("void vmfmm::k_keys(int, double const*)", 4096, 50.0),
             ("void vmfmm::k_keys(int, double const*)", 4096, 50.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 3145728, 300.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 393216, 40.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 3145728, 300.0),
             ("void vmfmm::k_m2l_sym<10>(int, int)", 393216, 40.0),
             ("void other_lib_kernel(int)", 64, 9.0)]
    _write_csv(str(tmp_path / "f" / "run_counter_collection.csv"), _pmc_rows("FETCH_SIZE", fetch))
    _write_csv(str(tmp_path / "w" / "run_counter_collection.csv"), _pmc_rows("WRITE_SIZE", write))
    d = R.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "toy", "cmd")
    cal = d["calibration"]
    assert cal["fetch_factor"] == pytest.approx(2.0) and cal["write_factor"] == pytest.approx(1.0)
    assert d["evaluations"] == 2 and d["sources_sha256"] == R.sources_sha256()
    assert "other_lib_kernel" not in json.dumps(d["kernels"])
    k = d["kernels"]["k_m2l_sym<10>"]
    assert k["dispatches"] == 4
    f_avg, w_avg = (4000 + 500 + 4200 + 520) / 4, (300 + 40 + 300 + 40) / 4
    assert k["hbm_bytes_per_launch"] == pytest.approx(1024 * (2 * f_avg + w_avg))
    assert k["hbm_bytes_per_evaluation"] == pytest.approx(1024 * (2 * 9220 + 680) / 2)
    sh = {s["grid_size"]: s for s in k["shapes"]}
    assert sh[3145728]["dispatches"] == 2 and sh[393216]["dispatches"] == 2
    assert sh[3145728]["hbm_bytes_per_dispatch"] == pytest.approx(1024 * (2 * 4100 + 300))
    assert sh[393216]["hbm_bytes_per_dispatch"] == pytest.approx(1024 * (2 * 510 + 40))


def test_trace_summary_per_kernel_and_per_shape(tmp_path):
    name = "void vmfmm::(anonymous namespace)::k_p2p32(vmfmm::P2PArgs, vmfmm::Part32 const*)"
    _write_csv(str(tmp_path / "run_kernel_stats.csv"),
               [{"Name": name, "Calls": 2, "TotalDurationNs": 6e6, "AverageNs": 3e6, "Percentage": 100.0}])
    _write_csv(str(tmp_path / "run_kernel_trace.csv"),
               [{"Kernel_Name": name, "Grid_Size_X": 64, "Grid_Size_Y": 1, "Start_Timestamp": 0,
                 "End_Timestamp": 2_000_000},
                {"Kernel_Name": name, "Grid_Size_X": 64, "Grid_Size_Y": 1, "Start_Timestamp": 5_000_000,
                 "End_Timestamp": 9_000_000}])
    text = R.trace_summary(str(tmp_path), "cmd")
    lines = text.splitlines()
    assert lines[0] == "command: cmd"
    row = next(l for l in lines if l.startswith("k_p2p32 "))
    assert row.split()[1:4] == ["2", "3.000", "6.000"]
    shape = next(l for l in lines if l.strip().startswith("k_p2p32") and l is not row)
    assert shape.split()[1:] == ["64", "1", "2", "3.000"]


def test_kernel_names():
    assert R.short_name("void vmfmm::(anonymous namespace)::k_p2p32(vmfmm::P2PArgs, float)") == "k_p2p32"
    assert R.short_name("void vmfmm::(anonymous namespace)::k_m2l_sym<10>(int, int)") == "k_m2l_sym<10>"
    assert R.short_name("void vmfmm::k_l2p<float>(float const*)") == "k_l2p<float>"


def test_bench_reads_the_traffic_summary_only_for_the_profiled_sources(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    path = tmp_path / "profiles" / "hbm_traffic_toy_mixed.txt"
    body = {"kernels": {"k_p2p32": {"dispatches": 1, "hbm_bytes_per_launch": 5.0, "hbm_bytes_per_evaluation": 5.0,
                                    "shapes": [{"grid_size": 64, "hbm_bytes_per_dispatch": 5.0}]}}}
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    path.write_text(json.dumps(dict(body, sources_sha256="0" * 64)))
    assert bench.measured_traffic("toy", "mixed", "k_p2p32") is None
    path.write_text(json.dumps(dict(body, sources_sha256=R.sources_sha256())))
    assert bench.measured_traffic("toy", "mixed", "k_p2p32") == 5.0
    assert bench.measured_finest_launch("toy", "mixed", "k_p2p32") == (64, 5.0)
