"""Host logic of bench.py that runs without a GPU: the one-GPU refusal, the
algorithmic byte count of the projection launches, and the HBM-traffic record
(counter scaling by a plain copy, and its validity check against the kernel
sources and the workload size)."""

import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, timeout=120)
    assert r.returncode == 2 and r.stdout == b""
    assert b"one GPU" in r.stderr


def test_projection_bytes_count_each_launch():
    # column 0 reads w_0, writes q'_0; column i >= 1 reads Q_{i-1} (i columns) and
    # w_i, writes q'_i and the normalised q_{i-1}: i + 3 columns of n elements
    n, b = 1000, 4
    for m in (1, 2, 3, 7):
        by_hand = b * n * 2 + sum(b * n * (i + 3) for i in range(1, m))
        assert bench.project_bytes(n, m, b) == by_hand
    m = 512   # closed form: 2 + (m - 1) m / 2 + 3 (m - 1) columns
    assert bench.project_bytes(n, m, b) == b * n * (2 + (m - 1) * m // 2 + 3 * (m - 1))


def _counter_db(path, counter, values):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    for d, (name, v) in enumerate(values):
        con.execute("insert into counters_collection values (?, ?, ?, ?)", (d, name, counter, v))
    con.commit()
    con.close()


def test_traffic_record_scales_counters_by_the_copy(tmp_path, monkeypatch):
    n, m = 4096, 3
    kern = "rgs::" + bench.PROJECT_KERNEL + "(args)"
    fetch = [(kern, 100.0), (kern, 200.0), (kern, 300.0), ("__amd_rocclr_copyBuffer", 524288.0)]
    write = [(kern, 10.0), (kern, 20.0), (kern, 30.0), ("__amd_rocclr_copyBuffer", 1048576.0)]
    _counter_db(tmp_path / "f.db", "FETCH_SIZE", fetch)
    _counter_db(tmp_path / "w.db", "WRITE_SIZE", write)
    out = tmp_path / "rec.json"
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(out))
    bench.write_traffic_record(str(tmp_path / "f.db"), str(tmp_path / "w.db"), n=n, m=m, k=64)
    rec = json.load(open(out))
    # the 1 GiB copy reads 2^20 KiB: a fetch counter of 2^19 KiB means 0.5 counted per byte
    assert rec["copy_calibration"]["fetch_factor"] == 0.5 and rec["copy_calibration"]["write_factor"] == 1.0
    assert rec["traffic_bytes_per_launch"] == pytest.approx(200.0 * 1024 / 0.5 + 20.0 * 1024 / 1.0)
    assert rec["algorithmic_bytes_per_launch"] == pytest.approx(bench.project_bytes(n, m, 4) / m)
    assert rec["source_sha256"] == bench.sources_sha256(rec["source_files"])


def test_traffic_record_needs_every_launch_and_the_copy(tmp_path, monkeypatch):
    kern = "rgs::" + bench.PROJECT_KERNEL
    _counter_db(tmp_path / "f.db", "FETCH_SIZE", [(kern, 1.0), (kern, 1.0)])
    _counter_db(tmp_path / "w.db", "WRITE_SIZE", [(kern, 1.0), (kern, 1.0)])
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "rec.json"))
    with pytest.raises(SystemExit):
        bench.write_traffic_record(str(tmp_path / "f.db"), str(tmp_path / "w.db"), n=4096, m=2, k=64)
    assert not (tmp_path / "rec.json").exists()


def test_committed_traffic_record_is_used_only_while_it_applies(monkeypatch):
    rec = json.load(open(bench.TRAFFIC_RECORD))
    assert set(rec["source_files"]) == set(bench.TRAFFIC_SOURCES)
    t = bench.measured_traffic(1 << 22, 512, 2048)
    assert t == rec["traffic_bytes_per_launch"]
    # a few tenths of a percent above the algorithmic bytes at the headline size
    assert 1.0 <= t / rec["algorithmic_bytes_per_launch"] < 1.05
    assert bench.measured_traffic(1 << 21, 512, 2048) is None
    monkeypatch.setattr(bench, "sources_sha256", lambda files: "changed")
    assert bench.measured_traffic(1 << 22, 512, 2048) is None


def test_batched_traffic_record_takes_the_second_call(tmp_path, monkeypatch):
    """One batched call = the dispatches after the previous call's last scale
    pass up to its own last one (two shares, two scale passes per call); the
    table generation before the second call's shares counts, the first call
    (warm-up and tuning) and anything after the second call do not."""
    init, proj, scale, table = "rgs::kb_init(a)", "rgs::kb_qa(a)", "rgs::kb_scale<bf16, true>(a)", "rgs::k_theta_table(a)"
    call1 = [(table, 1e6), (init, 1.0), (init, 1.0), (proj, 1e6), (proj, 1e6), (scale, 1.0), (scale, 1.0)]
    call2 = [(table, 7.0), (init, 11.0), (proj, 13.0), (init, 17.0), (proj, 19.0), (scale, 23.0), (scale, 29.0)]
    after = [(table, 1e6), (init, 1e6), (scale, 1e6), (scale, 1e6)]
    copy = [("__amd_rocclr_copyBuffer", 524288.0)]
    _counter_db(tmp_path / "f.db", "FETCH_SIZE", call1 + call2 + after + copy)
    _counter_db(tmp_path / "w.db", "WRITE_SIZE", call1 + call2 + after + [("__amd_rocclr_copyBuffer", 1048576.0)])
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.write_batched_traffic_record(str(tmp_path / "f.db"), str(tmp_path / "w.db"), "gaussian_bf16_table", batch=4)
    rec = json.load(open(tmp_path / "profiles" / "rgs_qr_batched_2048_gaussian_bf16_table_traffic.json"))
    raw = sum(v for _, v in call2)
    assert rec["fetch_kib_raw"] == raw and rec["write_kib_raw"] == raw
    assert rec["traffic_bytes"] == pytest.approx(raw * 1024 / 0.5 + raw * 1024 / 1.0)
    assert rec["kernels"]["rgs::k_theta_table"]["dispatches"] == 1
    assert rec["kernels"]["rgs::kb_init"]["dispatches"] == 2
