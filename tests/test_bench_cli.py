"""bench.py's command line on the CPU: a run on more than one GPU is refused
with a message and exit status 2, before any device is touched."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and ("--gpus %d" % n) in r.stderr
        assert r.stdout == ""


def test_bench_help_lists_the_legs():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--large", "--no-batched", "--no-warm",
                 "--no-tuned", "--no-cpu-baseline"):
        assert flag in r.stdout, flag
