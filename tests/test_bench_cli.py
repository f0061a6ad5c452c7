"""Command-line contract of bench.py that holds without a GPU: one GPU only,
at least one timed step.  Both checks run before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_zero_steps_is_refused():
    r = _run("--steps", "0")
    assert r.returncode == 2
    assert "--steps" in r.stderr
