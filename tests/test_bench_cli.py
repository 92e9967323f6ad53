"""The benchmark's command-line contract, on the CPU: more than one GPU is refused with a JSON
message and exit status 2 before anything touches a device, and the defaults are one GPU and a
short run."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_defaults_are_one_gpu_and_a_short_run(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and 1 <= a.steps <= 5 and 0 <= a.warmup <= 2
    assert a.pipelined == 0 and not a.copy_calibration
