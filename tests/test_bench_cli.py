"""The benchmark's command-line contract that holds without a GPU: more than
one GPU is refused with a message, and the serving process that the main run
starts exits cleanly when the main run ends before releasing it."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_serving_process_exits_on_eof():
    # no "go" line: the process must leave before it imports torch or
    # touches a GPU, and print nothing
    r = subprocess.run([sys.executable, BENCH, "--serving-only"], input="", capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 0
    assert r.stdout == ""
