"""bench.py's command line on the CPU: more than one GPU is refused with a message
before any device work, and the workload list parses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_help_lists_every_workload():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("er800", "ea3d", "batch512", "es", "k2000", "glass", "dense8k", "sweep", "copy", "peaks"):
        assert w in r.stdout
