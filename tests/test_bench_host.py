"""CPU checks of bench.py's host logic: the rocprofv3 summaries that the
committed profiles come from (kernel-trace statistics, and HBM bytes per
launch from FETCH_SIZE / WRITE_SIZE scaled by reference kernels of known
size), the source-hash guard on the stored traffic, and the one-GPU refusal.
Small sqlite databases with the tables rocprofv3 writes stand in for real
traces."""

import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

P2 = "void nys::k_gemv_n<nys::F32, 8, true, false>(nys::T2Args)"
P1 = "void nys::k_gemv_tt<nys::F32, 8, true>(nys::TTArgs)"


def _trace_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)", rows)
    con.commit()
    con.close()


def test_summarize_trace_counts_and_rates(tmp_path):
    m, n, b_A = 1000, 2000, 4                    # 8 MB per pass
    rows = [(P2, 1000)] * 3 + [(P2, 20000), (P2, 40000)] + [(P1, 16000)] * 2 + [("void nys::k_other()", 5000)]
    db = tmp_path / "t.db"
    _trace_db(str(db), rows)
    out = tmp_path / "k.md"
    bench.summarize_trace(str(db), str(out), "cmd", "w", m, n, b_A)
    text = out.read_text()
    line2 = [ln for ln in text.splitlines() if "k_gemv_n" in ln][0].split("|")
    # calls 5, avg over all 12.6 us; reads of A: the two launches above 10 us, avg 30 us
    assert line2[2].strip() == "5" and line2[3].strip() == "12.6"
    assert line2[7].strip() == "2" and line2[8].strip() == "30.0"
    assert line2[9].strip() == f"{m * n * b_A / 30e-6 / 1e9:.0f}"   # 267 GB/s
    line1 = [ln for ln in text.splitlines() if "k_gemv_tt" in ln][0].split("|")
    assert line1[9].strip() == f"{m * n * b_A / 16e-6 / 1e9:.0f}"
    other = [ln for ln in text.splitlines() if "k_other" in ln][0].split("|")
    assert other[7].strip() == ""                 # no rate for kernels that do not read A
    assert "Command: `cmd`" in text


def _pmc_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_summarize_pmc_scales_by_the_reference_kernels(tmp_path):
    m, n, b_A = 1000, 2048, 4
    read_bytes = m * n * b_A                     # multiple of 16
    # FETCH_SIZE reads half the bytes of the reference read stream (factor 2)
    fetch = [("nys::k_stream_read(...)", "FETCH_SIZE", read_bytes / 2 / 1024)] * 2
    fetch += [(P1, "FETCH_SIZE", 1.1 * read_bytes / 2 / 1024), (P2, "FETCH_SIZE", 1.0 * read_bytes / 2 / 1024),
              (P2, "FETCH_SIZE", 1.2 * read_bytes / 2 / 1024)]
    write = [("void at::native::copy_kernel(...)", "WRITE_SIZE", 2 ** 31 / 1024),
             (P1, "WRITE_SIZE", 64.0), (P2, "WRITE_SIZE", 32.0)]
    fdb, wdb = tmp_path / "f.db", tmp_path / "w.db"
    _pmc_db(str(fdb), fetch)
    _pmc_db(str(wdb), write)
    out = tmp_path / "traffic.json"
    bench.summarize_pmc(str(fdb), str(wdb), "w", m, n, b_A, "cmd", str(out))
    rec = json.loads(out.read_text())
    assert rec["FETCH_SIZE_scale"] == pytest.approx(2.0)
    assert rec["WRITE_SIZE_scale"] == pytest.approx(1.0)
    hb = rec["hbm_bytes_per_launch"]
    assert hb["normal_pass1"] == round(1.1 * read_bytes + 64 * 1024)
    assert hb["normal_pass2"] == round(1.1 * read_bytes + 32 * 1024)    # mean of 1.0 and 1.2
    assert rec["gemv_source_hash"] == bench.gemv_source_hash()


def test_stored_traffic_is_dropped_when_the_sources_change(tmp_path, monkeypatch):
    """A stored counter summary counts only for the GEMV sources it was taken
    with (the hash of gemv.hip and common.hpp)."""
    real = bench.gemv_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "gemv_source_hash", lambda: real)
    (prof / "gemv_traffic_w.json").write_text(json.dumps({"gemv_source_hash": "0" * 16,
                                                          "hbm_bytes_per_launch": {"normal_pass2": 1}}))
    assert bench.load_traffic("w") is None
    (prof / "gemv_traffic_w.json").write_text(json.dumps({"gemv_source_hash": real,
                                                          "hbm_bytes_per_launch": {"normal_pass2": 1}}))
    assert bench.load_traffic("w")["hbm_bytes_per_launch"]["normal_pass2"] == 1
    assert bench.load_traffic("missing") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_split_cores_keeps_two_for_the_gpu_thread():
    assert bench.split_cores({5, 0, 3, 1, 2, 4}) == ([2, 3, 4, 5], [0, 1])
    assert bench.split_cores({0, 1, 2}) == ([0, 1, 2], [0, 1, 2])
    assert bench.cpu_model() != ""


def test_oracle_child_and_its_record(tmp_path):
    """The oracle child's full solve of a small configuration and its two
    measured pieces on a handed-over instance; the cpu_baseline record
    extrapolates initial point + K iterations."""
    import numpy as np
    from instances import make_instance
    inst = make_instance("gauss_200x500", seed=3, m=60, n=150)
    np.save(tmp_path / "A.npy", inst.A.float().numpy())
    for v in ("b", "c", "q"):
        np.save(tmp_path / f"{v}.npy", getattr(inst, v).numpy())
    (tmp_path / "ready").write_text("1")
    bench.oracle_child(str(tmp_path), seed=0, names=("gauss_200x500",), wait_s=5.0)
    res = json.load(open(tmp_path / "result.json"))
    fs = res["full_solves"]["gauss_200x500"]
    assert fs["status"] == 0 and fs["kkt_rel"] <= 1e-6 and fs["x_rel_err_vs_planted"] < 1e-4
    bi = res["bench_instance"]
    assert bi["m"] == 60 and bi["n"] == 150 and bi["initial_point_s"] > 0 and bi["one_iteration_s"] > 0
    rec = bench.oracle_baseline_record(res, gpu_iters=12)
    assert rec["kind"] == "oracle" and rec["cores"] == res["cores"] and rec["unit"] == "s"
    assert abs(rec["value"] - round(bi["initial_point_s"] + 12 * bi["one_iteration_s"], 1)) < 1e-9
    assert "extrapolated" in rec["sample"]
    empty = bench.oracle_baseline_record({}, gpu_iters=12)
    assert empty["value"] is None
