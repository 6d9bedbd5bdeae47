"""Exhaustive CPU check of the integer range reductions of the step kernel's normal generator.

The kernel forms the Box-Muller angle's quadrant and remainder from the Philox word, and the
logarithm's exponent / mantissa split from the bits of u, instead of by float rounding and
compares. Both must give the same bits as the float forms (which the oracle uses) for every
input; tests/csrc/reduction_identities.c runs over all 2^32 words and all positive normal
binary32 values.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_integer_reductions_match_float_forms(tmp_path):
    exe = str(tmp_path / "reduction_identities")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                    os.path.join(HERE, "csrc", "reduction_identities.c"), "-o", exe, "-lm"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "quarter-turn mismatches 0, log-split mismatches 0" in out.stdout
