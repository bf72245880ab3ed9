"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the library runs one plan on one GPU), before any GPU work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2, (p.returncode, p.stdout, p.stderr)
    assert "one GPU" in p.stdout + p.stderr
