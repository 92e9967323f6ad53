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


def test_default_workload_is_the_mixed_batch_in_slices():
    """The headline is the 1,048,576-primary mixed workload; its K timed steps run disjoint
    consecutive id slices that together cover every primary once, and the warm-up slices lie
    beyond them."""
    sys.path.insert(0, ROOT)
    import bench
    sys_argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        assert bench.parse().workload == "c2"
    finally:
        sys.argv = sys_argv
    for N, K, W in ((1048576, 20, 5), (1048576, 3, 1), (1000, 7, 2)):
        s, timed, warm = bench.plan_steps(N, K, W, False)
        ids = [i for id0, n in timed for i in range(id0, id0 + n)] if N <= 1000 else None
        assert sum(n for _, n in timed) == N and timed[0][0] == 0
        assert all(timed[j][0] + timed[j][1] == timed[j + 1][0] for j in range(len(timed) - 1))
        assert all(id0 >= N for id0, _ in warm) and len(warm) == W
        if ids is not None:
            assert ids == list(range(N))
    s, timed, warm = bench.plan_steps(65536, 3, 1, True)
    assert s == 65536 and timed == [(0, 65536)] * 3
