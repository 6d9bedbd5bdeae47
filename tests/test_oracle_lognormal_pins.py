"""Pins of the oracle's lognormal estimator and normality gate (Sec. 2.4), and of the
correlation coefficient of the bias optimisation (Sec. 3.4), on hand-built runs
whose weights have a known distribution.

- ln w exactly normal with mean mu and variance s^2 in one bin: the estimator is unbiased for
  n_j exp(mu + s^2/2) / (n_total Delta) up to the O(s^4/n) bias of exp(s_hat^2/2), and the
  interval of eq. eq_log_normal_bin_pdf_reconstrcuted_error_maximum_likelihood covers the
  true value in about 68 % of replicates (a one-sigma interval of the Cox method).
- the normality test's p-values are uniform for normal ln w (about 5 % below 0.05) and
  essentially zero for a skewed sample (ln w exponential).
"""
import math

import numpy as np

import oracle as O


def _runs(lw, k_in_bin, n_out, rng):
    n_in = lw.size
    k = np.concatenate([np.full(n_in, k_in_bin), rng.integers(1, 5, n_out)]).astype(np.uint64)
    lw_all = np.concatenate([lw, np.zeros(n_out)])
    n = k.size
    return O.Trajectories(t=np.arange(n, dtype=np.uint64), k=k, lw=lw_all, phi=np.zeros(n),
                          status=np.full(n, O.ST_ENDED, np.int32))


def test_lognormal_estimator_on_exact_lognormal_weights():
    rng = np.random.default_rng(1)
    mu, sig, n_in, n_out = -20.0, 1.5, 400, 600
    dN, edges = 0.5, np.array([9.0, 10.0, 11.0])        # k = 20 -> N = 10.0, bin 0
    truth = n_in * math.exp(mu + sig * sig / 2) / ((n_in + n_out) * 1.0)
    cover, est = 0, []
    reps = 400
    for _ in range(reps):
        tr = _runs(rng.normal(mu, sig, n_in), 20, n_out, rng)
        h = O.histogram(tr, dN, edges)
        lp, lo, hi = h.lognormal()
        p = math.exp(lp[0])
        est.append(p / truth)
        cover += (p * (1 - lo[0]) <= truth <= p * (1 + hi[0]))
    est = np.array(est)
    # bias of exp(s_hat^2/2): ~ sig^4/(4 n) relative
    assert abs(est.mean() - 1.0) < 3 * est.std() / math.sqrt(reps) + sig ** 4 / (2 * n_in)
    assert abs(cover / reps - 0.683) < 0.06
    # one replicate against the equations written out directly
    x = rng.normal(mu, sig, n_in)
    h = O.histogram(_runs(x, 20, n_out, rng), dN, edges)
    lp, lo, hi = h.lognormal()
    s2 = x.var(ddof=1)
    want = math.log(n_in * math.exp(x.mean() + s2 / 2) / (n_in + n_out))
    assert abs(lp[0] - want) < 1e-12 * abs(want)
    u = math.sqrt(s2 / n_in + s2 * s2 / (2 * n_in - 2))
    assert math.isclose(hi[0], math.exp(u) - 1, rel_tol=1e-12) and math.isclose(lo[0], 1 - math.exp(-u), rel_tol=1e-12)


def test_normality_gate():
    rng = np.random.default_rng(2)
    dN, edges = 0.5, np.array([9.0, 10.0, 11.0])
    ps = []
    for _ in range(300):
        h = O.histogram(_runs(rng.normal(-5.0, 2.0, 200), 20, 10, rng), dN, edges)
        ps.append(h.normal_p[0])
    ps = np.array(ps)
    assert abs(np.mean(ps < 0.05) - 0.05) < 0.04
    assert abs(np.mean(ps) - 0.5) < 0.06
    h = O.histogram(_runs(-rng.exponential(2.0, 200), 20, 10, rng), dN, edges)
    assert h.normal_p[0] < 1e-6
    # fewer than 8 runs: undefined
    h = O.histogram(_runs(rng.normal(0, 1, 7), 20, 10, rng), dN, edges)
    assert np.isnan(h.normal_p[0])


def test_pearson_r_of_log10_w_with_N():
    """|r| = 1 when ln w is an affine function of N (sign of the slope), ~0 +- 1/sqrt(n) for
    independent values; runs that did not end are left out."""
    rng = np.random.default_rng(3)
    n = 2000
    k = rng.integers(100, 200, n).astype(np.uint64)
    for slope, want in ((0.7, 1.0), (-0.2, -1.0)):
        lw = 3.0 + slope * k.astype(float)
        tr = O.Trajectories(t=np.arange(n, dtype=np.uint64), k=k, lw=lw, phi=np.zeros(n),
                            status=np.full(n, O.ST_ENDED, np.int32))
        h = O.histogram(tr, 0.01, np.linspace(0, 3, 11))
        assert abs(h.pearson_r - want) < 1e-12
    lw = rng.normal(0, 1, n)
    st = np.full(n, O.ST_ENDED, np.int32)
    st[:100] = O.ST_CENSORED
    lw[:100] = 50.0 + k[:100]                         # would dominate r if censored runs counted
    tr = O.Trajectories(t=np.arange(n, dtype=np.uint64), k=k, lw=lw, phi=np.zeros(n), status=st)
    h = O.histogram(tr, 0.01, np.linspace(0, 3, 11))
    assert abs(h.pearson_r) < 4 / math.sqrt(n - 100)
