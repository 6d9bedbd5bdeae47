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
    assert lay.ess == lay.pearson_r + 1 and lay.lognormal_gate == lay.ess + B
    assert lay.n_values == 2 * R + J * R + 4 * R + 8 * B + 7
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
    ("t_first", (1 << 64) - 100),   # t_first + n_traj past 2^64 - 1
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


def test_batch_size_limits(lib):
    """A batch holds 1 .. 1024 instances; 0 and 1025 are rejected before any device work."""
    keep = []
    one = _instance(lib, keep)
    for n in (0, 1025):
        arr = (lib.pyfpt_instance * max(n, 1))(*([one] * max(n, 1)))
        res = (lib.pyfpt_result * max(n, 1))()
        assert lib.load().pyfpt_run_batch(arr, n, 0, res, None) == lib.PYFPT_EINVAL, n


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


def test_training_and_combine_entry_points_reject_bad_input(lib):
    """Validation happens before any device work, so these run without a GPU."""
    import workloads as W
    from paper_2206_11234_amd.api import make_instance
    L = lib.load()
    keep = [{}]
    inst = make_instance(W.c2(10)[3], 16, keep)
    opt = lib.pyfpt_options()
    t = np.arange(2, dtype=np.uint64)
    off = np.array([0, 3, 2], np.uint64)                       # not ascending
    rec = np.zeros(3, np.dtype([("a", "<u4")] * 0 + [("phi", "<f4"), ("k", "<u4"), ("H", "<f4"), ("pn", "<u4")]))
    k = np.zeros(2, np.uint32)
    lw = np.zeros(2)
    st = np.zeros(2, np.int32)
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)
    assert L.pyfpt_proposal_records(ctypes.byref(inst), 0, vp(t), 2, 3, 1, vp(off), vp(rec), vp(k), vp(lw), vp(st),
                                    ctypes.byref(opt)) == lib.PYFPT_EINVAL          # group 3
    assert L.pyfpt_proposal_records(ctypes.byref(inst), 0, vp(t), 2, 4, 0, vp(off), vp(rec), vp(k), vp(lw), vp(st),
                                    ctypes.byref(opt)) == lib.PYFPT_EINVAL          # stride 0
    assert L.pyfpt_proposal_records(ctypes.byref(inst), 0, vp(t), 2, 4, 1, vp(off), vp(rec), vp(k), vp(lw), vp(st),
                                    ctypes.byref(opt)) == lib.PYFPT_EINVAL          # offsets
    net = lib.pyfpt_mlp()
    net.hidden = 64
    theta = np.zeros(4481, np.float32)
    loss = np.zeros(1)
    grad = np.zeros(4481)
    lwt = np.zeros(2)
    off2 = np.array([0, 1, 3], np.uint64)
    rec["pn"] = [(0 << 5) | 4, (1 << 5) | 4, (5 << 5) | 4]       # path index 5 >= n_paths
    assert L.pyfpt_proposal_loss_grad(ctypes.byref(net), 196.0, 1e-3, vp(theta), vp(rec), 3, vp(off2), 2, vp(lw), 10.0,
                                      0, 1.0, 1.0, vp(loss), vp(grad), vp(lwt), ctypes.byref(opt)) == lib.PYFPT_EINVAL
    rec["pn"] = [(0 << 5) | 4, (1 << 5) | 0, (1 << 5) | 4]       # zero steps in a group
    assert L.pyfpt_proposal_loss_grad(ctypes.byref(net), 196.0, 1e-3, vp(theta), vp(rec), 3, vp(off2), 2, vp(lw), 10.0,
                                      0, 1.0, 1.0, vp(loss), vp(grad), vp(lwt), ctypes.byref(opt)) == lib.PYFPT_EINVAL
    rec["pn"] = [(0 << 5) | 4, (1 << 5) | 17, (1 << 5) | 4]      # more steps than the largest group
    assert L.pyfpt_proposal_loss_grad(ctypes.byref(net), 196.0, 1e-3, vp(theta), vp(rec), 3, vp(off2), 2, vp(lw), 10.0,
                                      0, 1.0, 1.0, vp(loss), vp(grad), vp(lwt), ctypes.byref(opt)) == lib.PYFPT_EINVAL
    rec["pn"] = [(0 << 5) | 4, (1 << 5) | 4, (1 << 5) | 4]
    assert L.pyfpt_proposal_loss_grad(ctypes.byref(net), 196.0, 1e-3, vp(theta), vp(rec), 3, vp(off2), 2, vp(lw), 10.0,
                                      2, 1.0, 1.0, vp(loss), vp(grad), vp(lwt), ctypes.byref(opt)) == lib.PYFPT_EINVAL  # objective
    assert L.pyfpt_proposal_loss_grad(ctypes.byref(net), 196.0, 1e-3, vp(theta), vp(rec), 3, vp(off2), 2, vp(lw), 10.0,
                                      1, 0.0, 1.0, vp(loss), vp(grad), vp(lwt), ctypes.byref(opt)) == lib.PYFPT_EINVAL  # temper
    assert L.pyfpt_proposal_loss_grad(ctypes.byref(net), 196.0, 1e-3, vp(theta), vp(rec), 3, vp(off2), 2, vp(lw), 10.0,
                                      0, 1.0, 4.0, vp(loss), vp(grad), vp(lwt), ctypes.byref(opt)) == lib.PYFPT_EINVAL  # strided log M2
    cfg = lib.pyfpt_train_config(10.0, 5.0, 100, 0, 1, 1, 4, 1e-3, 0.9, 0.999, 1e-8, 0, 1.0, 1, 0)   # lo > hi
    inst.bias.kind = lib.BIAS_MLP
    bf = np.zeros(4481, np.uint16)
    rep = (lib.pyfpt_train_report * 1)()
    assert L.pyfpt_train_proposal(ctypes.byref(inst), 0, ctypes.byref(cfg), vp(theta), vp(bf),
                                  ctypes.cast(rep, ctypes.c_void_p), ctypes.byref(opt)) == lib.PYFPT_EINVAL
    cfg = lib.pyfpt_train_config(5.0, 10.0, 100, 0, 1, 1, 4, 1e-3, 0.9, 0.999, 1e-8, 1, 1.0, 1, -1)   # select < 0
    assert L.pyfpt_train_proposal(ctypes.byref(inst), 0, ctypes.byref(cfg), vp(theta), vp(bf),
                                  ctypes.cast(rep, ctypes.c_void_p), ctypes.byref(opt)) == lib.PYFPT_EINVAL
    assert b"select" in L.pyfpt_last_error()
    res = (lib.pyfpt_result * 1)()
    lp = np.zeros(4)
    n_used = np.zeros(4, np.int32)
    assert L.pyfpt_combine(res, 1, 4, 16, 4, vp(lp), vp(lp), vp(n_used)) == lib.PYFPT_EINVAL      # estimator 4
    assert b"estimator" in L.pyfpt_last_error()
    assert L.pyfpt_combine(res, 0, 4, 16, 0, vp(lp), vp(lp), vp(lp)) == lib.PYFPT_EINVAL          # no results


def test_noalloc_entry_point_refuses_workspace_and_graphs(lib):
    """The allocation-free batch works in its static scratch: a caller workspace or a graph
    request is refused before any device work."""
    keep = []
    arr = (lib.pyfpt_instance * 1)(_instance(lib, keep))
    res = (lib.pyfpt_result * 1)()
    opt = lib.pyfpt_options()
    buf = np.zeros(16, np.uint8)
    opt.workspace = ctypes.c_void_p(buf.ctypes.data)
    opt.workspace_bytes = 16
    assert lib.load().pyfpt_run_batch_noalloc(arr, 1, 0, res, ctypes.byref(opt)) == lib.PYFPT_EINVAL
    assert b"workspace" in lib.load().pyfpt_last_error()
    opt = lib.pyfpt_options()
    opt.use_graph = 1
    assert lib.load().pyfpt_run_batch_noalloc(arr, 1, 0, res, ctypes.byref(opt)) == lib.PYFPT_EINVAL
    assert lib.NOALLOC_SCRATCH_BYTES == 64 << 20
    hdr = open(os.path.join(ROOT, "include", "pyfpt.h")).read()
    assert "#define PYFPT_NOALLOC_SCRATCH_BYTES (64u << 20)" in hdr
