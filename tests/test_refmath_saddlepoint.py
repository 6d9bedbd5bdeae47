"""Pins of the saddle-point tail reference (the cumulants of N to any order and Daniels' density
built from them) against closed forms that do not come from the code under test:

- Brownian motion with a constant drift toward an absorbing end is an inverse-Gaussian first
  passage, whose cumulants are kappa_n = (2n - 3)!! mu^(2n-1) / lambda^(n-1) to every order; the
  hierarchy reproduces them to order 8;
- Daniels' formula with the inverse Gaussian's exact cumulant generating function gives the
  inverse-Gaussian density exactly (the classic case where the saddle-point density is exact);
  with the series truncated after 4, 6, 8 cumulants it converges to it, and the difference of
  the last two orders bounds the remaining error;
- with two cumulants the saddle-point density is the Gaussian, and the lattice mapping of the
  Gaussian equals the closed-form lattice Gaussian (differences of the normal CDF).
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle as O
from oracle import refmath as R


def _ig(a=1.0, A=-3.0, V0=1.0):
    """Flat potential, drift v = |A| S toward the end at distance a: IG(mu = a/v, lambda = a^2/S^2)."""
    m = O.Model(pot=O.POT_FLAT, V0=V0, phi_in=a, phi_end=0.0, bias=O.BIAS_NOISE_SCALED, A=A)
    S = math.sqrt(V0 / 3) / (2 * math.pi)
    v = abs(A) * S
    return m, a / v, a * a / (S * S)


def _ig_kappas(mu, lam, order):
    dfact = lambda k: math.prod(range(k, 0, -2)) if k > 0 else 1
    return [mu] + [dfact(2 * n - 3) * mu ** (2 * n - 1) / lam ** (n - 1) for n in range(2, order + 1)]


def _ig_logpdf(x, mu, lam):
    return 0.5 * math.log(lam / (2 * math.pi * x ** 3)) - lam * (x - mu) ** 2 / (2 * mu * mu * x)


def test_cumulant_hierarchy_matches_inverse_gaussian_to_order_8():
    m, mu, lam = _ig()
    got = R.cumulants_to(m, 8, biased=True, n_grid=200001)
    want = _ig_kappas(mu, lam, 8)
    for n, (g, w) in enumerate(zip(got, want), 1):
        assert abs(g - w) < 1e-6 * abs(w), (n, g, w)
    # the first four agree with the fixed-order routine
    c = R.cumulants(m, biased=True, n_grid=200001)
    assert np.allclose(got[:4], [c.k1, c.k2, c.k3, c.k4], rtol=1e-12, atol=0)


def test_daniels_density_is_exact_for_the_inverse_gaussian():
    _, mu, lam = _ig()
    c = lam / mu
    K = lambda s: c * (1 - math.sqrt(1 - 2 * mu * mu * s / lam))
    K1 = lambda s: mu / math.sqrt(1 - 2 * mu * mu * s / lam)
    K2 = lambda s: mu ** 3 / lam * (1 - 2 * mu * mu * s / lam) ** -1.5
    s_max = lam / (2 * mu * mu)                     # K is defined for s < s_max
    for x in (0.3 * mu, 0.8 * mu, mu, 1.7 * mu, 3 * mu, 8 * mu):
        # K' is convex and increasing, so Newton converges monotonically from above the root:
        # from s = 0 below the mean, from between the root and s_max above it
        root = s_max * (1 - mu * mu / (x * x))
        s0 = 0.0 if x < mu else root + 0.5 * (s_max - root)
        got = R.saddlepoint_logpdf_cgf(x, K, K1, K2, s0)
        assert abs(got - _ig_logpdf(x, mu, lam)) < 1e-11, (x, got, _ig_logpdf(x, mu, lam))


@pytest.mark.parametrize("a", [1.0, 2.0, 4.0], ids=["skew_0.52", "skew_0.27", "skew_0.16"])
def test_truncated_series_converges_to_the_inverse_gaussian(a):
    """The inverse Gaussian's cumulant series has a finite radius, |s| < lambda / (2 mu^2), so it
    tests the truncation the hard way.  Near the mean the truncated saddle-point density
    approaches the exact one order by order.  Wherever the last-term ratio is at most 0.35 (the
    range in which `saddlepoint_reference` states an error), twice the change from order 7 to
    order 8 covers the error left; beyond that the test only checks that the ratio rises."""
    _, mu, lam = _ig(a=a)
    kap = _ig_kappas(mu, lam, 8)
    sd = math.sqrt(kap[1])
    x = mu + 1.5 * sd
    err = {n: abs(R.saddlepoint_logpdf(x, kap[:n]) - _ig_logpdf(x, mu, lam)) for n in (4, 6, 8)}
    assert err[8] < err[6] < err[4], err
    covered = 0
    q_prev = 0.0
    for z in np.arange(0.5, 10.01, 0.5):
        x = mu + z * sd
        q = R.saddlepoint_term_ratio(x, kap)
        assert q > q_prev
        q_prev = q
        if q > 0.35:
            continue
        exact = _ig_logpdf(x, mu, lam)
        e8 = abs(R.saddlepoint_logpdf(x, kap) - exact)
        last = abs(R.saddlepoint_logpdf(x, kap) - R.saddlepoint_logpdf(x, kap[:7]))
        assert e8 <= 2 * last, (z, e8, last)
        covered += 1
    assert covered >= 3


def test_two_cumulants_give_the_gaussian_and_its_lattice():
    mu, sig, dN = 24.5, 0.094, 1e-3
    for x in (mu - 3 * sig, mu, mu + 5 * sig):
        want = -0.5 * ((x - mu) / sig) ** 2 - math.log(sig * math.sqrt(2 * math.pi))
        assert abs(R.saddlepoint_logpdf(x, [mu, sig * sig]) - want) < 1e-12
    edges = np.geomspace(mu - 6 * sig, mu + 6 * sig, 41)
    eps = 0.98e-3
    lp = R.lattice_logprobs(lambda x: R.saddlepoint_logpdf(x, [mu, sig * sig]), dN, edges, eps)
    ref = R.lattice_gaussian_probs(mu, sig, dN, edges, eps)
    ok = ref > 1e-10
    assert ok.sum() > 30
    assert np.allclose(np.exp(lp[ok]), ref[ok], rtol=1e-7, atol=0)   # the CDF differences' own rounding
    # far-tail bins stay finite in log space where the CDF differences underflow
    far = np.geomspace(mu + 20 * sig, mu + 21 * sig, 4)
    lp_far = R.lattice_logprobs(lambda x: R.saddlepoint_logpdf(x, [mu, sig * sig]), dN, far, eps)
    assert np.all(np.isfinite(lp_far)) and np.all(lp_far < -200)
    Kk = np.floor(far / dN + 1e-9)
    Kk = np.where((Kk + 1) * dN <= far, Kk + 1, Kk)
    logQ = special.log_ndtr(-(Kk * dN - eps - mu) / sig)           # log P(N_c > K dN - eps)
    exact = logQ[:-1] + np.log1p(-np.exp(logQ[1:] - logQ[:-1]))
    assert np.all(np.abs(lp_far - exact) < 1e-9 * np.abs(exact))


def test_saddlepoint_reference_normalises_and_has_the_drift_cumulants():
    """The drift-dominated workload (m = 0.01, phi_in = 10): the reference density integrates to
    one over +-12 sigma, and its cumulants are those of the target process."""
    m = O.Model(m=0.01, phi_in=10.0)
    kap = R.cumulants_to(m, 6, n_grid=200001)
    c = R.cumulants(m, n_grid=200001)
    assert np.allclose(kap[:4], [c.k1, c.k2, c.k3, c.k4], rtol=1e-12, atol=0)
    sd = math.sqrt(kap[1])
    x = np.linspace(kap[0] - 12 * sd, kap[0] + 12 * sd, 4001)
    p = np.exp([R.saddlepoint_logpdf(float(v), kap) for v in x])
    Z = np.trapezoid(p, x)
    assert abs(Z - 1.0) < 1e-4
    mean = np.trapezoid(p * x, x) / Z
    var = np.trapezoid(p * (x - mean) ** 2, x) / Z
    assert abs(mean - kap[0]) < 1e-5 * sd and abs(var / kap[1] - 1) < 1e-6
