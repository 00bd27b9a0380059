"""bench.py refuses more than one GPU before it touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT,
                          env={**os.environ, **(env or {})})


def test_more_than_one_gpu_is_refused():
    r = run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_distributed_launch_is_refused():
    r = run([], env={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
