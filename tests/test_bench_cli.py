"""bench.py argument checks that run before any GPU work (CPU only): more than one GPU
is refused, and the split-BF16 contraction choice applies to the mixed form only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_split_contractions_need_the_mixed_form():
    r = _run("--rr", "bf16x3")
    assert r.returncode == 2
    assert "--precision mixed" in r.stderr
