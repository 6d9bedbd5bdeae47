"""Further pins of the oracle: the Gaussian bump potential of the C5 workload against its
classical slow-roll integral, the power-law bias (Sec. 3.4, eq.
eq_importance_sampling_amplitude_power_law) against the target moments, and the histogram
estimators (Sec. 2.1, eqs. eq_bin_pdf_reconstrcuted and
eq_bin_pdf_reconstrcuted_weighted_naive) against their linear-space definitions on
hand-built runs."""
import math

import numpy as np
from scipy.integrate import quad

import oracle as O
import oracle.refmath as R


def _bump_V(m, a, p0, w):
    V = lambda f: 0.5 * m * m * f * f * (1 + a * math.exp(-(f - p0) ** 2 / (2 * w * w)))
    dV = lambda f: (m * m * f * (1 + a * math.exp(-(f - p0) ** 2 / (2 * w * w)))
                    - 0.5 * m * m * f * f * a * math.exp(-(f - p0) ** 2 / (2 * w * w)) * (f - p0) / (w * w))
    return V, dV


def test_bump_potential_follows_classical_integral():
    """Drift-dominated (m = 0.05): N_cl = int V/V' dphi (Sec. 1, delta N with H^2 = V/3).  With the
    same noise, the bump minus the plain quadratic potential shifts every run by the
    difference of the classical integrals (0.0396 e-folds), far beyond the noise of the shift."""
    m, a, p0, w, phi_in, dN = 0.05, 0.02, 4.0, 0.1, 8.0, 1e-3
    phi_end = math.sqrt(2.0)
    V, dV = _bump_V(m, a, p0, w)
    n_bump = quad(lambda f: V(f) / dV(f), phi_end, phi_in, points=[p0 - 0.3, p0, p0 + 0.3],
                  epsabs=1e-13, epsrel=1e-13)[0]
    n_quad = (phi_in ** 2 - phi_end ** 2) / 4.0
    n = 4000
    mb = O.Model(pot=O.POT_QUADRATIC_BUMP, m=m, a=a, phi0=p0, w=w, phi_in=phi_in, dN=dN)
    mq = O.Model(pot=O.POT_QUADRATIC, m=m, phi_in=phi_in, dN=dN)
    tb = O.simulate(mb, 0, n)
    tq = O.simulate(mq, 0, n)
    assert np.all(tb.status == O.ST_ENDED) and np.all(tq.status == O.ST_ENDED)
    d = (tb.k.astype(np.float64) - tq.k.astype(np.float64)) * dN
    assert abs(d.mean() - (n_bump - n_quad)) < 4 * d.std() / math.sqrt(n) + 2e-4
    assert abs(n_bump - n_quad) > 0.035
    # absolute mean: classical value, O(m^2) stochastic correction (~1.4e-3) and one EM step
    Nb = tb.k * dN
    assert abs(Nb.mean() - n_bump) < 4 * Nb.std() / math.sqrt(n) + 2.5e-3


def test_power_law_bias_weighted_mean_matches_target():
    """Bias B = A phi^p (p = 2) in the diffusion-dominated case: the unweighted mean of N
    follows the biased process and the weighted mean the unbiased one (eq. eq:meanN:S:gen),
    with the absorbing end moved by beta S sqrt(dN) for the discrete monitoring."""
    dN = 1e-3
    kw = dict(m=1.0, phi_in=6.0, phi_uv=8.0, bias=O.BIAS_POWER, A=0.005, p=2, dN=dN)
    mdl = O.Model(**kw)
    n = 20_000
    tr = O.simulate(mdl, 0, n)
    assert np.all(tr.status == O.ST_ENDED)
    S_end = mdl.m * mdl.phi_end / (2 * math.pi * math.sqrt(6))
    m_ref = O.Model(**{**kw, "phi_end": mdl.phi_end - R.BGK_BETA * S_end * math.sqrt(dN)})
    N = tr.k * dN
    ms = R.moments(m_ref, biased=True, n_grid=100001)
    mt = R.moments(m_ref, biased=False, n_grid=100001)
    assert abs(N.mean() - ms.mean) < 4 * ms.std / math.sqrt(n)
    assert abs(ms.mean - mt.mean) > 10 * ms.std / math.sqrt(n)      # the bias matters
    w = np.exp(tr.lw)
    wmean = np.sum(w * N) / np.sum(w)
    se = math.sqrt(np.sum(w ** 2 * (N - wmean) ** 2)) / np.sum(w)
    assert abs(wmean - mt.mean) < 4 * se
    assert abs(np.sum(w) / n - 1) < 4 * math.sqrt(np.sum(w ** 2)) / n


def test_histogram_estimators_on_hand_built_runs():
    """Bins are right-closed (e_j, e_{j+1}]; n_total counts every launched run; P_hat_j =
    sum_{i in j} w_i / (n_total Delta_j); the subset error is the standard deviation of the
    n_sub subset estimates divided by sqrt(n_sub); the Kish relative variance is
    sum w^2/(sum w)^2 - 1/n_total.  Computed here directly in linear space."""
    rng = np.random.default_rng(5)
    dN = 0.5
    edges = np.array([0.0, 1.0, 2.0, 3.5, 5.0])
    n = 400
    k = rng.integers(1, 12, n).astype(np.uint64)           # N = k/2 in [0.5, 5.5], edge values hit
    lw = rng.normal(-1.0, 0.7, n)
    status = np.full(n, O.ST_ENDED, np.int32)
    status[rng.choice(n, 7, replace=False)] = O.ST_CENSORED
    tr = O.Trajectories(t=np.arange(n, dtype=np.uint64), k=k, lw=lw, phi=np.zeros(n), status=status)
    J = 8
    h = O.histogram(tr, dN, edges, n_sub=J)
    B = len(edges) - 1
    N = k * dN
    w = np.exp(lw)
    for j in range(B):
        sel = (N > edges[j]) & (N <= edges[j + 1]) & (status == O.ST_ENDED)
        width = edges[j + 1] - edges[j]
        assert h.count[j] == sel.sum()
        P = w[sel].sum() / (n * width)
        assert math.isclose(math.exp(h.log_p_naive()[j]), P, rel_tol=1e-13)
        subs = []
        for s in range(J):
            ins = (np.arange(n) % J) == s
            subs.append(w[sel & ins].sum() / (ins.sum() * width))
        jk = np.std(subs, ddof=1) / math.sqrt(J) / P
        assert math.isclose(h.jackknife_rel_err()[j], jk, rel_tol=1e-10)
        kish = (w[sel] ** 2).sum() / w[sel].sum() ** 2 - 1.0 / n
        assert math.isclose(h.kish_rel_err2()[j], kish, rel_tol=1e-10)
    # N exactly on an edge belongs to the bin below it; N <= e_0 and N > e_B go to their rows
    assert h.count[B] == np.sum((N <= edges[0]) & (status == O.ST_ENDED))
    assert h.count[B + 1] == np.sum((N > edges[-1]) & (status == O.ST_ENDED))
    assert h.count[B + 2] == 7
    assert h.count[:B + 4].sum() == n
