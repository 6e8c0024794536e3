"""Host logic of bench.py (CPU only): the one-GPU contract and the rule that HBM traffic
from committed counter runs is reported only for the kernel sources it was measured on."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_source_digest_is_stable_and_covers_the_kernel_sources(tmp_path, monkeypatch):
    d = bench.kernel_source_digest()
    assert d == bench.kernel_source_digest() and len(d) == 16
    # a copy of the sources with one byte changed gives another digest
    src = tmp_path / "paper_2402_16683_amd" / "csrc"
    src.mkdir(parents=True)
    csrc = os.path.join(ROOT, "paper_2402_16683_amd", "csrc")
    for name in os.listdir(csrc):
        with open(os.path.join(csrc, name), "rb") as f:
            (src / name).write_bytes(f.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_digest() == d
    p = src / "level0.hip"
    p.write_bytes(p.read_bytes() + b"\n")
    assert bench.kernel_source_digest() != d


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    rec = {"refine_adj_last:w:f32": {"source_digest": "abcd", "hbm_bytes_per_launch": 123.0}}
    (tmp_path / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic("refine_adj_last:w:f32", "abcd") == 123.0
    assert bench.measured_traffic("refine_adj_last:w:f32", "other") is None   # sources changed since
    assert bench.measured_traffic("refine_fwd_last:w:f32", "abcd") is None    # never measured
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "missing"))
    assert bench.measured_traffic("refine_adj_last:w:f32", "abcd") is None
