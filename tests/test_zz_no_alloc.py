"""The allocation-free entry point (pyfpt_run_batch_noalloc) against pyfpt_run_batch.

Both run the same kernels; the allocation-free one keeps its scratch in a static device array
that every call on the device shares.  Two calls in a row, the second on a smaller batch with
host result buffers, must each agree with pyfpt_run_batch on the same inputs and launch shape:
identical counts, step totals and per-run dumps (integer and bit-for-bit work), binary64
log-sums within 1e-12 relative (only the order of the workgroup atomics differs), estimators
within the tolerances of the oracle comparisons.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import assert_histogram_matches, close_lse, to_model

pytestmark = pytest.mark.gpu

SEED = 0
CFG = dict(block=256, wg_per_cu=2, chunk=1)


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


def _print_case(label, **kw):
    print(f"[case] {label} {kw}", flush=True)


def _assert_results_agree(a, b):
    assert np.array_equal(a.counts, b.counts), "counts differ"
    for name in ("lse_w", "lse_w2", "jk_lse_w"):
        ok, bad = close_lse(getattr(a, name), getattr(b, name), 1e-12)
        assert ok, (name, bad[:5])
    for name in ("lse_w_all", "lse_w2_all", "lse_wk", "lse_wk2"):
        ok, _ = close_lse([getattr(a, name)], [getattr(b, name)], 1e-12)
        assert ok, name
    assert abs(a.sum_k2 - b.sum_k2) <= 1e-12 * abs(b.sum_k2)
    for name, rel in (("mean_lnw", 1e-9), ("log_p", 1e-12), ("log_p_ln", 1e-8), ("rel_err_jk", 1e-8),
                      ("rel_err_kish", 1e-8), ("m2_lnw", 1e-8), ("normal_p", 1e-4), ("pearson_r", 1e-9)):
        x = np.atleast_1d(np.asarray(getattr(a, name), np.float64))
        y = np.atleast_1d(np.asarray(getattr(b, name), np.float64))
        assert np.array_equal(np.isnan(x), np.isnan(y)), name
        f = np.isfinite(y)
        assert np.array_equal(np.isfinite(x), f), name
        assert np.all(np.abs(x[f] - y[f]) <= rel * np.maximum(1.0, np.abs(y[f])) + 1e-12), name


def _noalloc_host(fpt, inst, seed):
    """One instance through pyfpt_run_batch_noalloc with host result buffers (ctypes)."""
    from paper_2206_11234_amd import _lib as L
    from paper_2206_11234_amd.api import Result, layout, make_instance
    keep = [{}]
    arr = (L.pyfpt_instance * 1)(make_instance(inst, 16, keep))
    lay = layout(len(inst.edges) - 1, 16)
    counts = np.zeros(int(lay.n_counts), np.uint64)
    values = np.zeros(int(lay.n_values), np.float64)
    res = (L.pyfpt_result * 1)(L.pyfpt_result(counts.ctypes.data, values.ctypes.data, 0))
    opt = L.pyfpt_options()
    opt.block, opt.wg_per_cu, opt.chunk = CFG["block"], CFG["wg_per_cu"], CFG["chunk"]
    L.check(L.load().pyfpt_run_batch_noalloc(arr, 1, seed, res, ctypes.byref(opt)))
    return Result(np.asarray(inst.edges, np.float64), 16, counts, values, lay)


def test_noalloc_matches_run_batch_two_calls(fpt):
    # call 1: two instances (direct sampling, and the diffusion case with its wall and bias),
    # device result buffers and per-run dumps
    big = [W.with_runs(W.c1(), 3001), W.with_runs(W.c2()[3], 777)]
    _print_case("noalloc call 1", n=[i.n_traj for i in big])
    r_ref, d_ref, _ = fpt.run_batch(big, SEED, dump_n=3001, **CFG)
    r_na, d_na, _ = fpt.run_batch(big, SEED, dump_n=3001, noalloc=True, **CFG)
    for a, b, da, db, inst in zip(r_na, r_ref, d_na, d_ref, big):
        _assert_results_agree(a, b)
        for f in ("k", "status"):
            assert np.array_equal(getattr(da, f), getattr(db, f)), f
        assert np.array_equal(da.lw.view(np.uint64), db.lw.view(np.uint64))
        assert np.array_equal(da.phi.view(np.uint32), db.phi.view(np.uint32))
        # and both are the oracle's runs
        tr = O.simulate(to_model(inst), SEED, inst.n_traj)
        assert np.array_equal(da.k[:inst.n_traj].astype(np.uint64), tr.k)
        assert_histogram_matches(a, O.histogram(tr, inst.dN, inst.edges))
    # call 2: a smaller batch (one instance, fewer bins, fewer runs) with host result buffers;
    # the scratch still holds call 1's tables and queue position
    small = W.with_runs(W.c1(), 500)
    _print_case("noalloc call 2", n=small.n_traj)
    a = _noalloc_host(fpt, small, SEED + 1)
    b, _, _ = fpt.run(small, SEED + 1, **CFG)
    _assert_results_agree(a, b)
    assert a.n_traj == 500 and int(a.count.sum()) == 500


def test_noalloc_rejects_what_does_not_fit(fpt):
    """The six-instance C2 batch needs about 150 MB of tables on 512 workgroups: refused with
    the size it needs, before any work; a call that fits still runs afterwards."""
    from paper_2206_11234_amd import _lib as L
    insts = [W.with_runs(i, 100) for i in W.c2()]
    _print_case("noalloc oversize", n_inst=len(insts))
    with pytest.raises(L.PyfptError) as e:
        fpt.run_batch(insts, SEED, noalloc=True, **CFG)
    assert e.value.code == L.PYFPT_ENOMEM and "static scratch holds" in str(e.value)
    with pytest.raises(L.PyfptError) as e:
        fpt.run_batch(insts[:1], SEED, noalloc=True, use_graph=True, **CFG)
    assert e.value.code == L.PYFPT_EINVAL
    a, _, _ = fpt.run_batch(insts[:1], SEED, noalloc=True, **CFG)
    b, _, _ = fpt.run_batch(insts[:1], SEED, **CFG)
    _assert_results_agree(a[0], b[0])
