"""The benchmark's command line on the CPU: more than one GPU is refused with a message and
a non-zero status before any GPU work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "8"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, cwd=ROOT, capture_output=True,
                           text=True, timeout=120, env={**os.environ, **env})
        assert r.returncode == 2, (argv, r.returncode, r.stderr[-500:])
        assert "one GPU" in r.stderr
