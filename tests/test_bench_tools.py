"""Host logic of bench.py's measurement tools: kernel symbols to kernel kinds, and the
rocprofv3 summary (kernel statistics, FETCH_SIZE / WRITE_SIZE calibrated by the run's last
device copy) on synthetic CSV files shaped like rocprofv3's."""
import csv
import json
import os

import pytest

import bench


@pytest.mark.parametrize("name,kind", [
    ("void lamg::(anonymous namespace)::k_csr<float, 0, 1>(long, long, int const*)", ("gs_color", "fp32")),
    ("k_csr_vec<double, 1, 1, 2>(long)", ("residual", "fp64")),
    ("k_csr_mixed_vec<float, 3, 0, 4>(long)", ("cheb", "fp32")),
    ("k_csr_mixed<double, 2, 0>(long)", ("restrict", "fp64")),
    ("k_csr_long<float, 0, 0, 1024>(long)", ("gs_color", "fp32")),
    ("void lamg::(anonymous namespace)::k_tail<float, false>(lamg::TailArgs)", ("tail", "fp32")),
    ("k_red_partial<double, 5>(long, int)", ("reduce", "fp64")),
    ("lamg::k_rcf_update(long, int)", ("reduce", "fp64")),
    ("k_prolong_mu<float>(long)", ("prolong", "fp32")),
    ("void lamg::k_from_cols<float>", ("vector", "fp32")),
    ("void lamg::(anonymous namespace)::k_bjgs<double>(long, int, int, lamg::BjArgs<double>)",
     ("bjgs", "fp64")),
    ("__amd_rocclr_copyBuffer", (None, None)),
    ("k_tv_sweep_long(long, int const*)", (None, None)),
])
def test_kernel_kind(name, kind):
    assert bench.kernel_kind(name) == kind


def _write(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_profile_groups_and_calibrates(tmp_path, monkeypatch, capsys):
    d = tmp_path / "prof"
    d.mkdir()
    _write(d / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs"], [
        dict(Name="k_csr<float, 0, 0>(long)", Calls=10, TotalDurationNs=40000),
        dict(Name="k_csr_vec<float, 0, 1, 4>(long)", Calls=2, TotalDurationNs=200000),
        dict(Name="k_tail<float, false>(x)", Calls=4, TotalDurationNs=400000),
        dict(Name="__amd_rocclr_copyBuffer", Calls=3, TotalDurationNs=9000),
    ])
    rows = []
    # two GS dispatches, the solver's own large copy, then the probe (the last copy)
    for i, (name, kib) in enumerate([("k_csr<float, 0, 0>(long)", 100.0),
                                     ("k_csr<float, 0, 0>(long)", 300.0),
                                     ("__amd_rocclr_copyBuffer", 9999.0),
                                     ("__amd_rocclr_copyBuffer", 512.0)]):
        rows.append(dict(Dispatch_Id=i + 1, Kernel_Name=name, Counter_Name="FETCH_SIZE",
                         Counter_Value=kib))
    _write(d / "run_counter_collection.csv",
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_path", lambda wl, k: str(rec_path))
    # the probe moved 1 MiB each way and read as 512 KiB: factor 2
    assert bench.summarize_profile(str(d), "w", 3, 1 << 20, True) == 0
    out = capsys.readouterr().out
    import re

    # both GS symbols in one kind: 12 calls, 0.24 ms, 20 us each
    assert re.search(r"gs_color\s+fp32\s+12\s+0\.24\s+20\.000", out), out
    assert "factor 2.0" in out
    rec = json.load(open(rec_path))
    assert rec["workload"] == "w" and rec["nrhs"] == 3
    assert rec["source_hash"] == bench.kernel_source_hash()
    g = rec["kinds"]["gs_color_fp32"]
    assert g["dispatches"] == 2
    assert g["fetch_size_kib_per_dispatch"] == pytest.approx(200.0)
    assert g["fetch_size_bytes_per_dispatch"] == pytest.approx(200.0 * 1024 * 2.0)
    # traffic_of needs both counters
    assert bench.traffic_of("w", 3, "gs_color_fp32") is None
