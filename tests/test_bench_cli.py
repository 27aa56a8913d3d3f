"""bench.py's command line on the host: more than one GPU is refused with a
message, and an unknown configuration name is rejected before any work."""
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
    assert r.stdout == ""


def test_unknown_configuration_is_rejected():
    r = _run("--config", "C9")
    assert r.returncode == 2
    assert "invalid choice" in r.stderr
