"""C-ABI checks that need no GPU: the library loads, exports every entry point declared
in include/pyfpt.h, reports its result layout, and rejects invalid inputs with
PYFPT_EINVAL before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2206_11234_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2206_11234_amd import build
        build.build()
    return L


def test_every_declared_symbol_is_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "pyfpt.h")).read()
    declared = set(re.findall(r"^(?:int|const char \*)\s*(pyfpt_\w+)\s*\(", hdr, re.M))
    assert {"pyfpt_run", "pyfpt_run_batch", "pyfpt_result_layout", "pyfpt_last_error"} <= declared
    L = lib.load()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(lib.EXPORTS)


def test_result_layout(lib):
    lay = lib.pyfpt_layout()
    assert lib.load().pyfpt_result_layout(200, 16, ctypes.byref(lay)) == 0
    R, J, B = 204, 16, 200
    assert lay.count == 0 and lay.jk_count == R and lay.n_traj == R + J * R
    assert lay.n_counts == R + J * R + 2
    assert lay.lse_w == 0 and lay.lse_w2 == R and lay.jk_lse_w == 2 * R
    assert lay.log_p == 2 * R + J * R + 4 * R
    assert lay.log_p_ln == lay.log_p + 3 * B and lay.normal_p == lay.log_p + 6 * B
    assert lay.n_values == 2 * R + J * R + 4 * R + 7 * B + 6
    assert lib.load().pyfpt_result_layout(0, 16, ctypes.byref(lay)) == lib.PYFPT_EINVAL
    assert lib.load().pyfpt_result_layout(10, 1, ctypes.byref(lay)) == lib.PYFPT_EINVAL


def _instance(lib, keep, **kw):
    from paper_2206_11234_amd.api import make_instance
    import workloads as W
    inst = W.c1()
    for k, v in kw.items():
        setattr(inst, k, v)
    return make_instance(inst, 16, keep)


@pytest.mark.parametrize("field,value", [
    ("phi_in", 1.0),            # phi_in <= phi_end
    ("phi_in", math.nan),
    ("dN", 0.0),
    ("dN", -1e-3),
    ("phi_uv", 4.0),            # wall below phi_in
    ("phi_uv", math.nan),
    ("k_max", 1 << 33),
    ("m", 0.0),
    ("phi_esc", 3.0),
    ("edges", np.array([0.0, 1.0, 1.0])),
    ("edges", np.array([0.0, math.inf])),
    ("A", math.inf),
])
def test_invalid_inputs_rejected_without_device(lib, field, value):
    keep = []
    kw = {field: value}
    if field == "A":
        kw["bias"] = 1
    I = _instance(lib, keep, **kw)
    arr = (lib.pyfpt_instance * 1)(I)
    res = (lib.pyfpt_result * 1)()
    rc = lib.load().pyfpt_run_batch(arr, 1, 0, res, None)
    assert rc == lib.PYFPT_EINVAL, (field, value, rc)
    assert len(lib.load().pyfpt_last_error()) > 0


def test_mixed_kinds_unsupported(lib):
    keep = []
    a = _instance(lib, keep)
    b = _instance(lib, keep, bias=2, A=1.0, p=2)
    arr = (lib.pyfpt_instance * 2)(a, b)
    res = (lib.pyfpt_result * 2)()
    assert lib.load().pyfpt_run_batch(arr, 2, 0, res, None) == lib.PYFPT_EUNSUPPORTED


def test_build_flags_forbid_packed_fp32_and_contraction():
    from paper_2206_11234_amd import build
    f = " ".join(build.HIPCC_FLAGS)
    assert "-packed-fp32-ops" in f and "-ffp-contract=off" in f
    assert "-fhip-fp32-correctly-rounded-divide-sqrt" in f
