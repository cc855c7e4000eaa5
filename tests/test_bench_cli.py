"""bench.py's command-line contract on the host (no GPU): more than one GPU
is refused with a message, and the option parser knows every workload and
switch the documentation names."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert out.returncode != 0
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_options_are_known():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                         timeout=300, cwd=ROOT)
    assert out.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--precision", "--workload", "--transfer", "--mls-alpha",
                "--subsolver", "--ilu-fill", "--coarsen", "--kernels-only", "--no-cpu-baseline", "--no-legs", "--nparts", "--physics", "--mls-clip", "--factor-only"):
        assert opt in out.stdout, opt
