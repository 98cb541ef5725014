"""Host-side logic of bench.py (no GPU): the one-GPU guard, the canonical
flop count of a moment build, and the rule that attaches measured HBM
traffic to the roofline only for the source and workload it was taken on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_canonical_flops_counts_each_integral_once():
    """Counted step by step for each part: every distinct integral (xp|qc)
    once (2Q flops), and both moments as full products over the pair
    columns (2N flops per output element and column, two moments)."""
    N, o, v, Q = 7, 3, 4, 11
    slab = 2 * Q * (N * o * o * v + N * v * v * o)
    contraction = 2 * (2 * N * N) * (o * o * v + v * v * o)
    assert bench.canonical_flops(N, o, v, Q) == slab + contraction
    # nmo=1000, nocc=76, naux=3500: the figure the benchmark divides by
    assert bench.canonical_flops(1000, 76, 924, 3500) == 7.72464e14


def _traffic_tree(tmp_path, source_text, **rec):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "kernel.hip"
    src.write_text(source_text)
    record = {"source": "kernel.hip",
              "source_sha256": hashlib.sha256(source_text.encode()).hexdigest(),
              "bytes_per_launch": 123, "precision": "split_fp16", "workload": "large"}
    record.update(rec)
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({"moments.slab": record}))
    return src


def test_traffic_is_attached_only_to_its_own_source_and_workload(tmp_path, monkeypatch):
    src = _traffic_tree(tmp_path, "kernel text\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = bench.measured_traffic("moments.slab", "split_fp16", "large")
    assert rec is not None and rec["bytes_per_launch"] == 123
    assert bench.measured_traffic("moments.syrk", "split_fp16", "large") is None
    assert bench.measured_traffic("moments.slab", "split_bf16", "large") is None
    assert bench.measured_traffic("moments.slab", "split_fp16", "batch64") is None
    # the kernel's source changed since the counters were taken
    src.write_text("kernel text, edited\n")
    assert bench.measured_traffic("moments.slab", "split_fp16", "large") is None


def test_missing_traffic_record_gives_none(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("moments.slab", "split_fp16", "large") is None
