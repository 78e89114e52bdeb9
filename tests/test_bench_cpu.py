"""Host logic of bench.py that needs no GPU: the HBM traffic figure is taken
from the committed counter summary only while that summary names the current
evaluation source, and runs on more than one GPU are refused."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    bench = _bench_module()
    src = tmp_path / "eval.hip"
    src.write_bytes(b"// kernel source v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "traffic.md"
    summary.write_text(f"kernel source sha256: {sha}\n\n"
                       "k_pass1 HBM bytes per launch: 3.357301e+08\n"
                       "k_pass2 HBM bytes per launch: 7.373038e+08\n")
    monkeypatch.setattr(bench, "EVAL_SOURCES", [str(src)])
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    assert bench.counter_traffic("k_pass1") == 3.357301e+08
    assert bench.counter_traffic("k_pass2") == 7.373038e+08
    assert bench.counter_traffic("k_pass3") is None          # no such line
    src.write_bytes(b"// kernel source v2\n")                  # source edited since
    assert bench.counter_traffic("k_pass1") is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.counter_traffic("k_pass1") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""                                       # no JSON line


def test_result_line_takes_numpy_values():
    """The one JSON line is printed whatever numpy scalars or arrays a leg
    leaves in its results; anything else still fails loudly."""
    import json

    import numpy as np
    import pytest
    import bench
    out = {"a": np.float64(1.5), "b": np.int32(3), "c": np.arange(3), "d": [np.float32(0.25)]}
    assert json.loads(json.dumps(out, default=bench.json_value)) == \
        {"a": 1.5, "b": 3, "c": [0, 1, 2], "d": [0.25]}
    with pytest.raises(TypeError):
        json.dumps({"x": object()}, default=bench.json_value)
