"""bench.py's command line on the CPU: more than one GPU is refused with a message
before any device work, the workload list parses, and the kernel-code hash that ties a
PMC summary to the kernel it measured is well defined."""
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


def test_kernel_code_hash_identifies_one_kernel():
    """The PMC summaries are tied to a kernel's gfx950 code in the built library: the
    hash is stable, distinct between kernels, and refuses an ambiguous name."""
    sys.path.insert(0, ROOT)
    from paper_2004_03972_amd import hqa, profsum
    hqa.lib()
    a = profsum.isa_hash("k_step_batch_lds")
    assert a is not None and len(a) == 64
    assert profsum.isa_hash("k_step_batch_lds") == a
    b = profsum.isa_hash("k_energy_mv<64, 1>")
    assert b is not None and b != a
    assert profsum.isa_hash("k_energy_mv<") is None          # four instances match
    assert profsum.isa_hash("no_such_kernel_name") is None
