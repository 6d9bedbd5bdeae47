"""Multi-bias reconstruction (Sec. 3.2, 3.3): per-bin inverse-variance combination of the
estimates of several runs with different biases.

Oracle pins: two copies of one histogram combine to the same estimate with the error divided
by sqrt 2; a bin trusted by only one input takes that input's value; untrusted bins are left
out.  The library's host combination (pyfpt_combine, no device needed for host buffers)
matches the oracle's on histograms of simulated runs.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _hist(A, n, stream, edges, m=0.01, phi_in=5.0, dN=1e-3):
    mdl = O.Model(m=m, phi_in=phi_in, bias=O.BIAS_NOISE_SCALED if A else O.BIAS_NONE, A=A, dN=dN, stream=stream)
    return O.histogram(O.simulate(mdl, 0, n), dN, edges)


@pytest.fixture(scope="module")
def hists():
    mu, sig = W.MU_SIGMA["C1"]
    edges = np.linspace(mu - 2 * sig, mu + 14 * sig, 41)
    return [_hist(A, 6000, i, edges) for i, A in enumerate((0.0, 1.0, 2.0))]


def test_duplicates_and_single_contributors(hists):
    h = hists[1]
    for est in (0, 1):
        lp1, e1, u1 = O.combine([h], est)
        lp2, e2, u2 = O.combine([h, h], est)
        f = u1 > 0
        assert f.sum() >= 3
        assert np.allclose(lp2[f], lp1[f], rtol=0, atol=1e-13)
        assert np.allclose(e2[f], e1[f] / math.sqrt(2), rtol=1e-12)
        assert np.all(u2[f] == 2) and np.all(np.isnan(lp1[~f]))
    lp, e, u = O.combine(hists, 1)
    for j in np.nonzero(u == 1)[0]:
        single = [O.combine([g], 1) for g in hists]
        src = [s for s in single if s[2][j] == 1][0]
        assert lp[j] == src[0][j] and e[j] == src[1][j]
    # the combined estimate reaches further than the direct sampling
    direct = O.combine(hists[:1], 0)[2] > 0
    assert np.max(np.nonzero(u > 0)[0]) > np.max(np.nonzero(direct)[0])


def test_per_bin_fallback_takes_each_bins_own_estimator(hists):
    """Estimator 3: a bin that passes the normality gate takes the lognormal estimate, any other
    bin the naive one under the naive trust rule (Sec. 2.4, applied bin by bin)."""
    for h in hists:
        lp3, e3, u3 = O.combine([h], 3)
        lp1, e1, u1 = O.combine([h], 1)
        lp0, e0, u0 = O.combine([h], 0)
        assert np.array_equal(u3 > 0, (u1 > 0) | (u0 > 0))
        ln = u1 > 0
        assert np.array_equal(lp3[ln], lp1[ln]) and np.array_equal(e3[ln], e1[ln])
        nv = (u0 > 0) & ~ln
        assert np.array_equal(lp3[nv], lp0[nv]) and np.array_equal(e3[nv], e0[nv])
    # with both kinds of bins present somewhere, the union reaches at least as far as either
    lp, e, u = O.combine(hists, 3)
    assert (u > 0).sum() >= max((O.combine(hists, k)[2] > 0).sum() for k in (0, 1))


def _pack(lib, h, n_sub):
    B = len(h.edges) - 1
    R = B + 4
    lay = lib.pyfpt_layout()
    assert lib.load().pyfpt_result_layout(B, n_sub, ctypes.byref(lay)) == 0
    c = np.zeros(lay.n_counts, np.uint64)
    v = np.full(lay.n_values, np.nan)
    c[lay.count:lay.count + R] = h.count
    v[lay.m2_lnw:lay.m2_lnw + R] = h.m2_lnw
    v[lay.log_p:lay.log_p + B] = h.log_p_naive()
    v[lay.rel_err_jk:lay.rel_err_jk + B] = h.jackknife_rel_err()
    lp, lo, hi = h.lognormal()
    v[lay.log_p_ln:lay.log_p_ln + B] = lp
    v[lay.rel_err_ln_hi:lay.rel_err_ln_hi + B] = hi
    v[lay.normal_p:lay.normal_p + B] = h.normal_p[:B]
    return c, v


@pytest.mark.parametrize("estimator", [0, 1, 2, 3])
def test_library_combination_matches_oracle(hists, estimator):
    from paper_2206_11234_amd import _lib as lib
    bufs = [_pack(lib, h, 16) for h in hists]
    arr = (lib.pyfpt_result * len(bufs))(*[lib.pyfpt_result(c.ctypes.data, v.ctypes.data, 0) for c, v in bufs])
    B = len(hists[0].edges) - 1
    lp, el, nu = np.zeros(B), np.zeros(B), np.zeros(B, np.int32)
    rc = lib.load().pyfpt_combine(arr, len(bufs), B, 16, estimator, ctypes.c_void_p(lp.ctypes.data),
                                  ctypes.c_void_p(el.ctypes.data), ctypes.c_void_p(nu.ctypes.data))
    assert rc == 0
    lp_o, el_o, nu_o = O.combine(hists, estimator)
    assert np.array_equal(nu, nu_o)
    f = nu > 0
    assert np.allclose(lp[f], lp_o[f], rtol=1e-13, atol=0) and np.allclose(el[f], el_o[f], rtol=1e-13, atol=0)
    assert np.all(np.isnan(lp[~f]))
