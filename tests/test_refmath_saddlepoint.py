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


# ---------------------------------------------------------------------------------------------
# The exact cumulant generating function with a reflecting wall (Riccati form of the backward
# equation), the saddle-point reference built on it, and the Pruefer form of the pole expansion.
# ---------------------------------------------------------------------------------------------
def test_walled_cgf_matches_the_flat_well_closed_form():
    """Brownian motion from x, absorbing at 0, reflecting at L (constant V):
    E[e^{sT}] = cos(k (L - x)) / cos(k L) with k = sqrt(2 s)/S (cosh for s < 0); its logarithm
    and the first two s-derivatives (central differences of the closed form) are reproduced."""
    L, x = 1.5, 1.0
    m = O.Model(pot=O.POT_FLAT, V0=1.0, phi_in=x, phi_end=0.0, phi_uv=L)
    S = math.sqrt(1 / 3) / (2 * math.pi)

    def logM(s):
        if s > 0:
            k = math.sqrt(2 * s) / S
            return math.log(math.cos(k * (L - x)) / math.cos(k * L))
        k = math.sqrt(-2 * s) / S
        return math.log(math.cosh(k * (L - x)) / math.cosh(k * L))
    def dlogM(s):           # d/ds, with dk/ds = k/(2s) on both sides of s = 0
        if s > 0:
            k = math.sqrt(2 * s) / S
            return k / (2 * s) * (L * math.tan(k * L) - (L - x) * math.tan(k * (L - x)))
        k = math.sqrt(-2 * s) / S
        return k / (2 * s) * ((L - x) * math.tanh(k * (L - x)) - L * math.tanh(k * L))
    for s in (-0.05, -0.002, 0.0015, 0.004):
        K = R.cgf_walled(m, s, 2)
        h = 1e-6 * abs(s)
        d2 = (dlogM(s + h) - dlogM(s - h)) / (2 * h)
        assert abs(K[0] - logM(s)) < 1e-9 * max(1, abs(logM(s))), (s, K[0], logM(s))
        assert abs(K[1] - dlogM(s)) < 1e-8 * abs(dlogM(s)), (s, K[1], dlogM(s))
        assert abs(K[2] - d2) < 1e-5 * abs(d2), (s, K[2], d2)


def test_walled_cgf_derivatives_at_zero_are_the_cumulants():
    """The interim-mass case (m = 0.1, phi_in = phi_UV = sqrt 42): the s-derivatives of the exact
    generating function at s = 0 equal the cumulants from the Green's-function hierarchy, two
    independent routes through the same backward equation."""
    phi = math.sqrt(42.0)
    m = O.Model(m=0.1, phi_in=phi, phi_uv=phi)
    K = R.cgf_walled(m, 0.0, 4)
    kap = R.cumulants_to(m, 4, n_grid=200001)
    assert abs(K[0]) < 1e-12
    for n in range(4):
        assert abs(K[n + 1] - kap[n]) < 1e-6 * abs(kap[n]), (n, K[n + 1], kap[n])


@pytest.fixture(scope="module")
def diffusion_modes():
    """Pole expansion of the diffusion-dominated workload (m = 1, phi_in = 6, wall at 8) by the
    direct shooting solver (pinned against the 1F1 residues and the finite-difference solve)."""
    return R.sl_modes(O.Model(m=1.0, phi_in=6.0, phi_uv=8.0), 3, lam_max=4.0, n_scan=160)


def test_walled_saddlepoint_reference_matches_the_pole_expansion_in_the_far_tail(diffusion_modes):
    """The diffusion-dominated workload (m = 1, phi_in = 6, wall at 8): far in the tail a few poles
    describe P(N) (App. A); there the saddle-point reference with the exact generating function
    agrees with the Sturm-Liouville pole expansion (pinned by the 1F1 residues and the
    finite-difference eigen-solve) to within its stated error plus 0.5 %."""
    m = O.Model(m=1.0, phi_in=6.0, phi_uv=8.0, dN=1e-3)
    edges = np.array([80.0, 80.5, 120.0, 120.5, 180.0, 180.5, 260.0, 260.5])
    ref, err = R.saddlepoint_walled_reference(m, edges, n_s=24)
    modes = diffusion_modes
    _, tau = R.noise_free_em(m)
    eps = tau - R.classical_N(m)
    for j in (0, 2, 4, 6):
        N = np.linspace(edges[j], edges[j + 1], 65) - eps
        pole = np.trapezoid(np.sum(modes.amp[None, :] * np.exp(-modes.lam[None, :] * N[:, None]), axis=1), N) / 0.5
        assert abs(ref[j] - math.log(pole)) < err[j] + 5e-3, (edges[j], ref[j], math.log(pole), err[j])


def test_pruefer_modes_match_closed_forms_and_the_shooting_solver(diffusion_modes):
    """The Pruefer form of the Sturm-Liouville problem reproduces the flat well's sine series
    (Lambda_n = (2n+1)^2 pi^2 S^2 / (8 L^2), a_n = Lambda_n 4/((2n+1) pi) sin((2n+1) pi x/(2L)))
    and the direct shooting of the diffusion-dominated case, amplitudes included."""
    mf = O.Model(pot=O.POT_FLAT, V0=1.0, phi_in=1.0, phi_end=0.0, phi_uv=1.5)
    S = math.sqrt(1 / 3) / (2 * math.pi)
    md = R.sl_modes_prufer(mf, 3, 0.001, 0.12, n_scan=12)
    for n in range(3):
        lam = (2 * n + 1) ** 2 * math.pi ** 2 * S ** 2 / (8 * 1.5 ** 2)
        amp = lam * 4 / ((2 * n + 1) * math.pi) * math.sin((2 * n + 1) * math.pi / 3)
        assert abs(md.lam[n] / lam - 1) < 1e-9 and abs(md.amp[n] - amp) < 1e-8 * max(1e-3, abs(amp))
    m = O.Model(m=1.0, phi_in=6.0, phi_uv=8.0)
    a, b = R.sl_modes_prufer(m, 3, 0.05, 1.2, n_scan=12), diffusion_modes
    assert np.allclose(a.lam, b.lam, rtol=1e-9) and np.allclose(a.amp, b.amp, rtol=1e-6)
