"""bench.py's host-side contract (CPU only): one GPU only, and the counter
traffic reported only for the kernel sources and workload it was taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=e, timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run(["--gpus", "2"])
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""
    r = _run([], env={"WORLD_SIZE": "4"})
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_matching_kernel_and_workload(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("w") is None  # no file
    f.write_text(json.dumps({"kernel_sha": bench.kernel_sha(), "workload": "w", "hbm_bytes_per_launch": 123.0}))
    assert bench.load_traffic("w") == 123.0
    assert bench.load_traffic("other") is None
    f.write_text(json.dumps({"kernel_sha": "0" * 16, "workload": "w", "hbm_bytes_per_launch": 123.0}))
    assert bench.load_traffic("w") is None
    f.write_text("not json")
    assert bench.load_traffic("w") is None
