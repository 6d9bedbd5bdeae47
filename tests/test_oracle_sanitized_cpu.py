"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code) and
run through every entry point on small inputs (tests/csrc/oracle_sanitize_main.c): no invalid
memory access, leak, signed overflow, misaligned or out-of-range access is reported."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-mfma", "-ffp-contract=off", "-fno-fast-math",
             "-std=gnu11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc", *flags, os.path.join(HERE, "csrc", "oracle_sanitize_main.c"), "-o", exe, "-lm"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "sanitized oracle run" in out.stdout and "runtime error" not in out.stderr, out.stderr
