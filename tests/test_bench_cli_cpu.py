"""The benchmark's command line: more than one GPU is refused with a JSON error line and exit
status 2 before anything touches a device; --help lists the modes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    p = _run("--gpus", "2")
    assert p.returncode == 2
    line = [l for l in p.stdout.splitlines() if l.startswith("{")][-1]
    assert "one GPU" in json.loads(line)["error"]


def test_help_lists_the_modes():
    p = _run("--help")
    assert p.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--learned", "--c5", "--c3", "--eval-dn", "--no-cpu"):
        assert flag in p.stdout
