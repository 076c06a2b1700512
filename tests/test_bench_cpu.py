"""Host logic of bench.py (no GPU): the counter summaries built from rocprofv3
databases, the traffic summary's source check, the algorithmic FLOP counts
and the one-GPU guard."""

import csv
import os
import re
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

EVAL = "void nnp::k_eval_pooled<10, 2, true>(nnp::Sys)"
GATHER = "nnp::k_gather_integrate(nnp::Sys, double, int, int)"


def _db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?)", rows)
    c.commit()
    c.close()


def _stats(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        for name, calls, avg in rows:
            w.writerow([name, calls, calls * avg, avg, 50.0, avg, avg, 0.0])


def test_counter_summary_rates(tmp_path, capsys):
    """MFMA rate = issued FLOP / traced duration against 2.5 PFLOP/s; HBM
    bytes = counters x calibration factor (torch.neg over 256 MiB read as
    half the bytes fetched and all the bytes written) / duration."""
    mib = 256
    kib = mib * 1024.0
    m = str(tmp_path / "m.db")
    _db(m, [(EVAL, "MfmaFlopsBF16", 4.5e9), (EVAL, "MfmaFlopsBF16", 4.5e9), (EVAL, "MfmaUtil", 3.0),
            (EVAL, "MfmaUtil", 4.0), (GATHER, "MfmaFlopsBF16", 0.0), (GATHER, "MfmaUtil", 0.0)])
    f = str(tmp_path / "f.db")
    _db(f, [("void at::native::neg_kernel", "FETCH_SIZE", kib / 2), (EVAL, "FETCH_SIZE", 1000.0),
            (GATHER, "FETCH_SIZE", 100.0)])
    w = str(tmp_path / "w.db")
    _db(w, [("void at::native::neg_kernel", "WRITE_SIZE", kib), (EVAL, "WRITE_SIZE", 500.0),
            (GATHER, "WRITE_SIZE", 50.0)])
    st = str(tmp_path / "stats.csv")
    _stats(st, [(EVAL, 2, 45000.0), (GATHER, 2, 4500.0)])
    bench.counter_summary("bf16x3:fused", st, [m, f, w], mib, "--steps 2 --warmup 0")
    out = capsys.readouterr().out
    row = next(l for l in out.splitlines() if l.startswith("| void k_eval_pooled<10, 2, true>"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    head = next(l for l in out.splitlines() if l.startswith("| kernel"))
    names = [c.strip() for c in head.strip("|").split("|")]
    v = dict(zip(names, cells))
    assert float(v["mean us (trace)"]) == pytest.approx(45.0)
    assert float(v["MfmaUtil"]) == pytest.approx(3.5)
    tflops = 4.5e9 / 45e-6 / 1e12
    assert float(v["MFMA TFLOP/s"]) == pytest.approx(tflops, abs=0.05)
    assert v["of 2500"] == "%.2f %%" % (100 * tflops / 2500.0)
    hbm = (1000.0 * 2.0 + 500.0 * 1.0) * 1024
    assert float(v["HBM bytes (scaled)"]) == pytest.approx(hbm, abs=1.0)
    assert float(v["GB/s"]) == pytest.approx(hbm / 45e-6 / 1e9, abs=1.0)
    assert "FETCH_SIZE x 2.000" in out and "WRITE_SIZE x 1.000" in out


def test_traffic_summary_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    """The committed traffic summary is used only for its own variant and
    tile configuration and only while the kernel sources hash as recorded."""
    txt = open(bench.TRAFFIC_SUMMARY).read()
    kv = dict(re.findall(r"^- (\w+): (\S+)$", txt, re.M))
    current = tmp_path / "current.md"
    current.write_text(txt.replace(kv["kernel_source_sha256"], bench.kernel_source_hash()))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(current))
    assert bench.load_traffic(kv["variant"]) == int(kv["hbm_bytes_per_launch"])
    assert bench.load_traffic(kv["variant"], tile=kv.get("tile")) == int(kv["hbm_bytes_per_launch"])
    assert bench.load_traffic(kv["variant"], tile="999") is None
    assert bench.load_traffic("fp32:plain") is None
    stale = tmp_path / "stale.md"
    stale.write_text(txt.replace(kv["kernel_source_sha256"], "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(stale))
    assert bench.load_traffic(kv["variant"]) is None


def test_algorithmic_flop_counts():
    # forward + input gradient of 384 -> 160 -> 128 -> 96 -> 1
    assert bench.FLOP_MLP_ATOM == 377216
    assert bench.FLOP_RADIAL_PAIR > 0 and bench.FLOP_ANGULAR_TRIPLE > bench.FLOP_RADIAL_PAIR


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_tile_names():
    names = ["void nnp::k_eval_pooled<13, 2, true>(nnp::Sys)"]
    assert bench.tile_of_kernels(names) == "13"
    split = ["void nnp::k_desc_pooled<5>(nnp::Sys)", "void nnp::k_mlp_wide<2, true, true>(nnp::Sys)",
             "void nnp::k_adj_pooled<5>(nnp::Sys)"]
    assert bench.tile_of_kernels(split) == "5x32"
    assert bench.tile_of_kernels(names + split) is None
    assert bench.tile_of_choice({"path": "fused", "atoms_per_tile": 13, "network_tile": 64}) == "13"
    assert bench.tile_of_choice({"path": "split", "atoms_per_tile": 5, "network_tile": 32}) == "5x32"
    assert bench.tile_of_choice(None) is None
