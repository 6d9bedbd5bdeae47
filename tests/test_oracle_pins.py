"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage (or the mathematical fact) it checks.  None of
them compares the oracle with itself: the references are published
known-answer vectors, closed forms, the quadrature of the paper's double
integral (itself pinned in test_refmath_pins.py), and statistical identities.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import refmath as R
from conftest import read_golden


# ---------------------------------------------------------------- noise ----
def test_philox_known_answers():
    """Philox4x32-10 reproduces the published known-answer vectors (SC'11)."""
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for row in rows:
        lhs, rhs = row.split(":")
        w = [int(x, 16) for x in lhs.split()]
        want = [int(x, 16) for x in rhs.split()]
        got = O.philox(w[:4], w[4:6])
        assert list(map(int, got)) == want


def test_uniform24_exact_and_open():
    """u = (2 (x >> 9) + 1) 2^-24: exact odd multiples of 2^-24 inside (0, 1)."""
    L = O.lib()
    for x, want in [(0, 2.0 ** -24), (0xFFFFFFFF, 1 - 2.0 ** -24), (0x80000000, 0.5 + 2.0 ** -24),
                    (511, 2.0 ** -24), (512, 3 * 2.0 ** -24)]:
        assert L.oracle_uniform24(x) == want


def _uniform_grid():
    i = np.arange(1 << 23, dtype=np.float64)
    u64 = (2 * i + 1) * 2.0 ** -24
    u = u64.astype(np.float32)
    assert np.all(u.astype(np.float64) == u64)
    return u


def test_log_f32_exhaustive_on_uniforms():
    """The binary32 log is within 2.5 ulp of ln over every uniform the generator can emit
    (the quotient (f-1)/(f+1) is a product with the Newton reciprocal: two roundings)."""
    u = _uniform_grid()
    y = O.log_f32(u).astype(np.float64)
    ref = np.log(u.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(y - ref) / ulp) < 2.5
    assert np.max(np.abs(y - ref) / np.abs(ref)) < 3e-7
    # and on a spread of other normal inputs
    x = np.float32(2.0) ** np.random.default_rng(1).uniform(-120, 120, 200000).astype(np.float32)
    y = O.log_f32(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(y - ref) / np.maximum(ulp, 1e-300)) < 2.5


def test_sincos2pi_exhaustive_on_uniforms():
    """cos(2 pi u), sin(2 pi u) within 1.5 * 2^-24 absolute over every uniform."""
    u = _uniform_grid()
    c, s = O.sincos2pi_f32(u)
    ang = 2 * np.pi * u.astype(np.float64)
    assert np.max(np.abs(c - np.cos(ang))) < 1.5 * 2.0 ** -24
    assert np.max(np.abs(s - np.sin(ang))) < 1.5 * 2.0 ** -24
    # unit circle
    assert np.max(np.abs(c.astype(np.float64) ** 2 + s.astype(np.float64) ** 2 - 1)) < 4e-7


def test_recip_f32_exhaustive_over_mantissas():
    """The binary32 Newton reciprocal is within 0.51 ulp of 1/x for every mantissa, at
    several exponents (it reaches the binary32 rounding level)."""
    m = np.arange(1 << 23, dtype=np.uint32)
    for e in (-20, 0, 1, 3, 40):
        x = (m | np.uint32((127 + e) << 23)).view(np.float32)
        y = O.recip_f32(x).astype(np.float64)
        ref = 1.0 / x.astype(np.float64)
        ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
        assert np.max(np.abs(y - ref) / ulp) < 0.51
        assert np.mean(y == ref.astype(np.float32)) > 0.999


def test_sqrt_f32_exhaustive_over_mantissas():
    """The binary32 square root (Newton reciprocal square root times x) is within 2 ulp of
    sqrt x over two binades of mantissas and over the range of -2 ln u (three roundings
    after the last Newton step: y*y inside it, then x*y)."""
    m = np.arange(1 << 23, dtype=np.uint32)
    for e in (0, 1, -24, 5):
        x = (m | np.uint32((127 + e) << 23)).view(np.float32)
        y = O.sqrt_f32(x).astype(np.float64)
        ref = np.sqrt(x.astype(np.float64))
        ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
        assert np.max(np.abs(y - ref) / ulp) < 2.0


def test_exp_f32_accuracy():
    x = -np.random.default_rng(2).uniform(0, 80, 1_000_000).astype(np.float32)
    x[:3] = [0.0, -1e-30, -80.0]
    y = O.exp_f32(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(y - ref) / ulp) < 1.5
    assert O.exp_f32(np.array([-81.0], np.float32))[0] == 0.0


def test_normals_are_standard_normal():
    """Box-Muller on the Philox stream gives N(0, 1) draws (Sec. 2.1: xi_m drawn from a
    normal distribution with unit variance), independent across lanes of the counter."""
    z = np.concatenate([O.normals_f32(0, 0, t, 0, 2500) for t in range(100)]).astype(np.float64)
    n = z.size
    assert n == 1_000_000
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(stats.skew(z)) < 5 * math.sqrt(6 / n)
    assert abs(stats.kurtosis(z)) < 5 * math.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # lag-1 correlation within a trajectory's stream
    assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / math.sqrt(n)
    # resolution cap of 24-bit uniforms: |xi| <= sqrt(-2 ln 2^-24)
    assert np.max(np.abs(z)) <= math.sqrt(-2 * math.log(2.0 ** -24)) + 1e-5


def test_normals_f32_match_f64_reference():
    z32 = O.normals_f32(7, 3, 12345, 10, 50000).astype(np.float64)
    z64 = O.normals_f64(7, 3, 12345, 10, 50000)
    assert np.max(np.abs(z32 - z64)) < 2e-6


# ----------------------------------------------------- direct sampling ----
def test_direct_sampling_has_unit_weights():
    """Bias 0: every run has w = 1 and the weighted estimator reduces to the count estimator
    (Sec. 2.2: B = 0 recovers eq. eq_bin_pdf_reconstrcuted)."""
    m = O.Model(m=0.01, phi_in=5.0, dN=1e-3)
    tr = O.simulate(m, 0, 2000)
    assert np.all(tr.lw == 0.0)
    assert np.all(tr.status == O.ST_ENDED)
    mu, sig = 5.750008188, 0.01171994848
    edges = np.linspace(mu - 6 * sig, mu + 6 * sig, 101)
    h = O.histogram(tr, m.dN, edges)
    nz = h.count > 0
    assert np.allclose(h.lse_w[nz], np.log(h.count[nz]), rtol=0, atol=1e-12)
    B = 100
    p_count = h.count[:B] / (np.diff(edges) * 2000)
    with np.errstate(divide="ignore"):
        assert np.allclose(np.exp(h.log_p_naive()), p_count, rtol=1e-12, atol=0)


def test_c1_mean_and_variance_match_delta_N_closed_forms():
    """Config C1 (m = 0.01, phi_in = 5, 1e4 runs): sample mean and variance of N against the
    double integral of eq. eq:meanN:S:gen and its variance companion, on the simulation's
    lattice: the discrete drift is slower than the continuum by eps (noise-free EM) and the
    crossing step rounds up by dN/2 on average; variance gains dN^2/12 (Sheppard)."""
    m = O.Model(m=0.01, phi_in=5.0, dN=1e-3)
    n = 10_000
    tr = O.simulate(m, 0, n)
    N = tr.k * m.dN
    mo = R.moments(m)
    _, tau = R.noise_free_em(m)
    eps = tau - R.classical_N(m)
    want_mean = mo.mean + eps + 0.5 * m.dN
    se = mo.std / math.sqrt(n)
    assert abs(N.mean() - want_mean) < 4 * se + 0.1 * m.dN
    want_var = mo.var + m.dN ** 2 / 12
    assert abs(N.var() - want_var) < 4 * want_var * math.sqrt(2 / n)


def test_c1_histogram_matches_lattice_gaussian():
    """Drift-dominated limit: P(N) is the Gaussian of App. B (gamma = kappa = 0), checked bin by
    bin on the lattice with a chi-square over bins holding >= 20 expected runs."""
    m = O.Model(m=0.01, phi_in=5.0, dN=1e-3)
    n = 10_000
    tr = O.simulate(m, 0, n)
    mo = R.moments(m)
    _, tau = R.noise_free_em(m)
    eps = tau - R.classical_N(m)
    edges = np.linspace(mo.mean - 6 * mo.std, mo.mean + 6 * mo.std, 101)
    h = O.histogram(tr, m.dN, edges)
    p = R.lattice_gaussian_probs(mo.mean, mo.std, m.dN, edges, eps)
    expct = n * p
    sel = expct >= 20
    chi2 = np.sum((h.count[:100][sel] - expct[sel]) ** 2 / expct[sel])
    dof = int(sel.sum())
    assert stats.chi2.sf(chi2, dof) > 1e-3


# ----------------------------------------------------- quantum well -------
def _flat(A=0.0, wall=True, dN=1e-3, x=1.0, L=1.5):
    V0 = 3.0 * (2 * math.pi) ** 2          # S = sqrt(V0/3)/(2 pi) = 1
    return O.Model(pot=O.POT_FLAT, V0=V0, phi_in=x, phi_end=0.0, phi_uv=L if wall else math.inf,
                   bias=O.BIAS_NOISE_SCALED if A else O.BIAS_NONE, A=A, dN=dN)


def test_quantum_well_mean_and_variance():
    """Constant V (the quantum well of Sec. 3): Brownian motion with an absorbing end and a
    reflecting wall.  Discrete monitoring of the end is accounted for by moving it out by
    beta S sqrt(dN), beta = -zeta(1/2)/sqrt(2 pi) (Broadie-Glasserman-Kou)."""
    m = _flat()
    n = 100_000
    tr = O.simulate(m, 0, n)
    N = tr.k * m.dN
    shift = R.BGK_BETA * 1.0 * math.sqrt(m.dN)
    want = R.brownian_mean(1.0 + shift, 0.0, 1.5 + shift, 1.0)
    var = R.brownian_var(1.0 + shift, 0.0, 1.5 + shift, 1.0)
    assert abs(N.mean() - want) < 4 * math.sqrt(var / n)
    # without the shift the discrete bias would be detected
    assert abs(N.mean() - R.brownian_mean(1.0, 0.0, 1.5, 1.0)) > 4 * math.sqrt(var / n)
    assert abs(N.var() - var) < 5 * var * math.sqrt(2 / n) * 2


def test_girsanov_weights_have_unit_mean():
    """E_S[w] = 1: the weight is the likelihood ratio p_T/p_S of the two path densities
    (eqs. eq_importance_sampling_probability_of_target_path / ..._sample_path).  The sign of
    the exponent in eq. eq_importance_sampling_bias_w as printed would give E[w] >> 1."""
    m = _flat(A=0.5)
    n = 100_000
    tr = O.simulate(m, 0, n)
    assert np.all(tr.status == O.ST_ENDED)
    h = O.histogram(tr, m.dN, np.linspace(0, 50, 51))
    mean_w = math.exp(h.lse_w_all) / n
    ess = math.exp(2 * h.lse_w_all - h.lse_w2_all)
    assert abs(mean_w - 1) < 5 / math.sqrt(ess)
    # for a constant bias the exponent is -A^2 k dN/2 - A sqrt(dN) sum xi  ->  with the
    # printed sign the weights would average far from one
    assert math.exp(O._lse(-tr.lw)) / n > 3


def test_quantum_well_density_with_wall():
    """Direct sampling of the quantum well with a reflecting wall reproduces the exact
    first-passage density (sine eigen-series of the absorbing/reflecting interval), bin by bin."""
    m = _flat()
    n = 100_000
    tr = O.simulate(m, 0, n)
    edges = np.linspace(0.0, 12.0, 61)
    h = O.histogram(tr, m.dN, edges)
    shift = R.BGK_BETA * math.sqrt(m.dN)
    surv = R.brownian_survival_wall(edges, 1.0 + shift, 0.0, 1.5 + shift, 1.0)
    surv[0] = 1.0
    expct = n * -np.diff(surv)
    sel = expct >= 20
    chi2 = np.sum((h.count[:60][sel] - expct[sel]) ** 2 / expct[sel])
    assert stats.chi2.sf(chi2, int(sel.sum())) > 1e-3


def test_weighted_far_tail_matches_levy_density():
    """Importance sampling reaches the far tail: for the quantum well without a wall the
    target first-passage density is Levy's x/(S sqrt(2 pi T^3)) exp(-x^2/(2 S^2 T)).  A bias
    B = A S with A = -30 drives runs to the end early, where P(N) is 1e-12 .. 1e-3; the
    weighted estimator (eq. eq_bin_pdf_reconstrcuted_weighted_naive) must reproduce the
    density bin by bin within its jackknife error (Sec. 2.1).  For a constant bias on a flat
    potential ln w is nearly a function of N, so the weights are well behaved."""
    dN = 1e-5
    V0 = 3.0 * (2 * math.pi) ** 2
    m = O.Model(pot=O.POT_FLAT, V0=V0, phi_in=1.0, phi_end=0.0, bias=O.BIAS_NOISE_SCALED, A=-30.0,
                dN=dN, phi_esc=5.0)
    n = 100_000
    tr = O.simulate(m, 0, n)
    assert np.all(tr.status == O.ST_ENDED)
    edges = np.linspace(0.015, 0.06, 31)
    h = O.histogram(tr, dN, edges)
    x = 1.0 + R.BGK_BETA * math.sqrt(dN)
    from scipy import integrate
    ref = np.array([integrate.quad(lambda T: R.levy_density(T, x, 0.0, 1.0), edges[i], edges[i + 1],
                                   epsrel=1e-12)[0] for i in range(30)]) / np.diff(edges)
    ok = h.count[:30] >= 30
    assert ref[ok].min() < 1e-10
    p = np.exp(h.log_p_naive()[ok])
    rel = h.jackknife_rel_err()[ok]
    z = (p - ref[ok]) / (rel * p)
    assert np.mean(np.abs(z) < 3) >= 0.9
    assert np.max(np.abs(z)) < 5
    # the printed sign of the weight exponent would miss by tens of decades
    assert np.all(np.abs(np.log(p / ref[ok])) < 0.5)


# ------------------------------------------- quadratic, importance sampled --
def test_diffusion_case_weighted_mean_matches_target():
    """Diffusion-dominated quadratic case (m = 1, phi_in = 6, reflecting wall at 8): under a
    bias A = 0.5 the unweighted mean of N follows the sample process and the weighted mean
    follows the target process, both as given by eq. eq:meanN:S:gen (absorbing end moved out
    by beta S(phi_end) sqrt(dN) for the discrete monitoring)."""
    dN = 1e-3
    m = O.Model(m=1.0, phi_in=6.0, phi_uv=8.0, bias=O.BIAS_NOISE_SCALED, A=0.5, dN=dN)
    n = 20_000
    tr = O.simulate(m, 0, n)
    assert np.all(tr.status == O.ST_ENDED)
    S_end = m.m * m.phi_end / (2 * math.pi * math.sqrt(6))
    m_ref = O.Model(m=1.0, phi_in=6.0, phi_uv=8.0, bias=O.BIAS_NOISE_SCALED, A=0.5, dN=dN,
                    phi_end=m.phi_end - R.BGK_BETA * S_end * math.sqrt(dN))
    N = tr.k * dN
    ms = R.moments(m_ref, biased=True, n_grid=100001)
    assert abs(N.mean() - ms.mean) < 4 * ms.std / math.sqrt(n)
    w = np.exp(tr.lw)
    mt = R.moments(m_ref, biased=False, n_grid=100001)
    wmean = np.sum(w * N) / np.sum(w)
    # delta-method standard error of the self-normalised weighted mean
    se = math.sqrt(np.sum(w ** 2 * (N - wmean) ** 2)) / np.sum(w)
    assert abs(wmean - mt.mean) < 4 * se
    assert abs(np.sum(w) / n - 1) < 4 * math.sqrt(np.sum(w ** 2)) / n


def test_f32_and_f64_modes_agree():
    """The binary32 mirror and the binary64 reference share the noise; their step counts
    agree for almost every run and their statistics agree."""
    m = O.Model(m=0.01, phi_in=5.0, dN=1e-3)
    a = O.simulate(m, 0, 4000, mode=O.MODE_F32)
    b = O.simulate(m, 0, 4000, mode=O.MODE_F64)
    assert np.mean(a.k == b.k) > 0.95
    assert np.max(np.abs(a.k.astype(np.int64) - b.k.astype(np.int64))) <= 3
    m2 = O.Model(m=1.0, phi_in=6.0, phi_uv=8.0, bias=O.BIAS_NOISE_SCALED, A=1.0, dN=1e-3)
    a = O.simulate(m2, 0, 300, mode=O.MODE_F32)
    b = O.simulate(m2, 0, 300, mode=O.MODE_F64)
    same = a.k == b.k
    assert np.mean(same) > 0.5
    assert np.max(np.abs(a.lw[same] - b.lw[same]) / np.maximum(1, np.abs(b.lw[same]))) < 1e-3


def test_censoring_and_escape_rows():
    """Runs stopped by the step cap or by the escape level land in their own rows with their
    weights; nothing is dropped (every launched run is counted)."""
    m = O.Model(m=1.0, phi_in=6.0, phi_uv=8.0, bias=O.BIAS_NOISE_SCALED, A=1.0, dN=1e-3, k_max=2000)
    tr = O.simulate(m, 0, 500)
    assert set(np.unique(tr.status)) <= {O.ST_ENDED, O.ST_CENSORED}
    assert np.all(tr.k[tr.status == O.ST_CENSORED] == 2000)
    h = O.histogram(tr, m.dN, np.linspace(0, 3, 31))
    assert h.count.sum() == 500
    assert h.count[30 + 2] == np.sum(tr.status == O.ST_CENSORED)
    me = O.Model(m=1.0, phi_in=3.0, bias=O.BIAS_NOISE_SCALED, A=4.0, dN=1e-3, phi_esc=4.0)
    tr = O.simulate(me, 0, 300)
    esc = tr.status == O.ST_ESCAPED
    assert esc.sum() > 0
    assert np.all(tr.phi[esc] > 4.0)
