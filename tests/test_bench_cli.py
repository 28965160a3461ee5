"""bench.py's command-line contract, checked without a GPU: more than one GPU
is refused with a message and exit status 2 (the benchmark runs on one GPU),
and the options parse."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "single GPU" in r.stderr


def test_options_parse():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--workload", "--peaks", "--no-cpu-baseline",
                "--record-traffic"):
        assert opt in r.stdout
