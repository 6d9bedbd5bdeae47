"""Shared test helpers: instance -> oracle model, and result comparisons."""
import math

import numpy as np

import oracle as O


def to_model(inst) -> O.Model:
    return O.Model.from_instance(inst)


def close_lse(a, b, rel=1e-12):
    """Log-sums agree: both -inf, or |a - b| <= rel * max(1, |b|)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    both_inf = np.isneginf(a) & np.isneginf(b)
    with np.errstate(invalid="ignore"):
        ok = both_inf | (np.abs(a - b) <= rel * np.maximum(1.0, np.abs(b)))
    return bool(np.all(ok)), np.nonzero(~ok)[0]


def assert_histogram_matches(res, h, rel=1e-12):
    """GPU result vs the oracle's plain-definition histogram of the same runs."""
    B = res.n_bins
    assert np.array_equal(res.count.astype(np.int64), h.count), (res.count, h.count)
    assert np.array_equal(res.jk_count.astype(np.int64), h.jk_count)
    if h.n_traj == 0:
        assert np.all(np.isneginf(res.lse_w)) and np.all(np.isneginf(res.jk_lse_w))
        assert res.total_steps == 0 and res.n_traj == 0
        return
    ok, bad = close_lse(res.lse_w, h.lse_w, rel)
    assert ok, ("lse_w", bad, res.lse_w[bad], h.lse_w[bad])
    ok, bad = close_lse(res.lse_w2, h.lse_w2, rel)
    assert ok, ("lse_w2", bad)
    ok, bad = close_lse(res.jk_lse_w, h.jk_lse_w, rel)
    assert ok, ("jk_lse_w", bad)
    assert res.total_steps == h.total_steps
    assert res.n_traj == h.n_traj
    for name in ("lse_w_all", "lse_w2_all", "lse_wk", "lse_wk2"):
        ok, _ = close_lse([getattr(res, name)], [getattr(h, name)], rel)
        assert ok, (name, getattr(res, name), getattr(h, name))
    assert abs(res.sum_k2 - h.sum_k2) <= 1e-12 * h.sum_k2
    if np.isnan(h.pearson_r):
        assert np.isnan(res.pearson_r)
    else:
        assert abs(res.pearson_r - h.pearson_r) <= 1e-9, (res.pearson_r, h.pearson_r)
    # moments of ln w per row (population central moments)
    nz = h.count > 0
    assert np.all(np.isnan(res.mean_lnw[~nz]))
    sd = np.sqrt(np.maximum(h.m2_lnw[nz], 0))
    scale = np.maximum(1.0, np.abs(h.mean_lnw[nz]))
    assert np.all(np.abs(res.mean_lnw[nz] - h.mean_lnw[nz]) <= 1e-9 * scale)
    assert np.all(np.abs(res.m2_lnw[nz] - h.m2_lnw[nz]) <= 1e-9 * scale ** 2 + 1e-9 * h.m2_lnw[nz])
    assert np.all(np.abs(res.m3_lnw[nz] - h.m3_lnw[nz]) <= 1e-7 * (sd + 1e-3 * scale) ** 3 + 1e-12)
    assert np.all(np.abs(res.m4_lnw[nz] - h.m4_lnw[nz]) <= 1e-7 * (sd + 1e-3 * scale) ** 4 + 1e-12)
    # estimators
    lp = h.log_p_naive()
    fin = np.isfinite(lp)
    assert np.array_equal(np.isfinite(res.log_p), fin)
    assert np.all(np.abs(res.log_p[fin] - lp[fin]) <= rel * np.maximum(1, np.abs(lp[fin])))
    jk = h.jackknife_rel_err()
    f2 = np.isfinite(jk) & fin
    bad = np.nonzero(~(np.abs(res.rel_err_jk[f2] - jk[f2]) <= 1e-8 * np.maximum(1e-3, jk[f2])))[0]
    assert bad.size == 0, ("rel_err_jk", np.nonzero(f2)[0][bad][:5], res.rel_err_jk[f2][bad][:5], jk[f2][bad][:5],
                           res.count[:B][f2][bad][:5], res.lse_w[:B][f2][bad][:5])
    kish = np.sqrt(np.maximum(h.kish_rel_err2(), 0))
    f3 = np.isfinite(kish) & (h.count[:B] > 0)
    assert np.all(np.abs(res.rel_err_kish[f3] - kish[f3]) <= 1e-8 * np.maximum(1e-3, kish[f3]) + 1e-7)
    # lognormal estimator and normality gate (Sec. 2.4); the GPU takes them from the merged
    # shifted power sums, the oracle from the runs themselves
    lp_ln, lo, hi = h.lognormal()
    f4 = np.isfinite(lp_ln)
    assert np.array_equal(np.isfinite(res.log_p_ln), f4)
    assert np.all(np.abs(res.log_p_ln[f4] - lp_ln[f4]) <= 1e-8 * np.maximum(1, np.abs(lp_ln[f4])))
    # the upper error overflows to +inf on both sides when s^2 is large for few runs
    # (u = sqrt(s^2/n + s^4/(2n - 2)) above ~709); equal values match, infinities included
    for got, want in ((res.rel_err_ln_hi[f4], hi[f4]), (res.rel_err_ln_lo[f4], lo[f4])):
        with np.errstate(invalid="ignore"):
            assert np.all((got == want) | (np.abs(got - want) <= 1e-7 * want + 1e-12))
    # Kish ESS per bin and the whole-result normality gate, as the library reports them
    ess_ref = h.ess()
    f6 = h.count[:B] > 0
    assert np.all(res.ess()[~f6] == 0.0)
    assert np.all(np.abs(res.ess()[f6] - ess_ref[f6]) <= 1e-9 * ess_ref[f6])
    pv = h.normal_p[:B]
    f5 = np.isfinite(pv)
    assert np.array_equal(np.isfinite(res.normal_p), f5), (np.nonzero(np.isfinite(res.normal_p) != f5)[0][:5])
    # the p-value depends on the third and fourth moments (agreeing to ~1e-7 relative)
    bad = np.nonzero(~(np.abs(res.normal_p[f5] - pv[f5]) <= 1e-4 * pv[f5] + 1e-9))[0]
    assert bad.size == 0, ("normal_p", res.normal_p[f5][bad][:5], pv[f5][bad][:5])
    # the gate as the paper states it, from the oracle's p-values (decided identically unless a
    # p-value lies within the comparison's tolerance of 0.005)
    near = np.abs(pv[f5] - 0.005) <= 1e-4 * 0.005 + 1e-9
    if not np.any(near):
        assert res.lognormal_accepted() == (not np.any(pv[f5] < 0.005))


def assert_dump_matches(dump, tr):
    """Per-trajectory parity: identical step count, status, final field (bit for bit)
    and log-weight (bit for bit: both accumulate the same binary32 increments in order)."""
    n = len(tr.k)
    k = dump.k[:n].astype(np.uint64)
    bad = np.nonzero(k != tr.k)[0]
    assert bad.size == 0, ("k differs", bad[:10], k[bad[:10]], tr.k[bad[:10]])
    assert np.array_equal(dump.status[:n], tr.status)
    assert np.array_equal(dump.phi[:n].astype(np.float32).view(np.uint32),
                          tr.phi.astype(np.float32).view(np.uint32))
    lw_ok = np.abs(dump.lw[:n] - tr.lw) <= 1e-5 * np.maximum(1.0, np.abs(tr.lw))
    assert np.all(lw_ok), ("lw beyond 1e-5", np.nonzero(~lw_ok)[0][:10])
    assert np.array_equal(dump.lw[:n], tr.lw), "lw not bit-identical"


def check_z(z, dof=None, label="", p_min=1e-3):
    """Agreement of estimates with a reference, given z = (estimate - reference) / error per bin.

    dof: degrees of freedom of the errors when they are estimated from few groups (jackknife
    over J subsets: J - 1); each z is then mapped to a standard normal deviate through Student's
    t distribution before the checks.  Passes when
      (1) at most 1 % of the bins lie beyond 3 sigma -- or, for sets under 100 bins, no more
          than Gaussian errors give with probability 1 - p_min (binomial tail at the rate
          2 Phi(-3) = 0.27 %), and
      (2) chi^2 = sum z^2 has a p-value of at least p_min under n degrees of freedom.
    Returns the summary it prints."""
    from scipy import stats
    z = np.asarray(z, np.float64)
    assert z.size > 0 and np.all(np.isfinite(z)), (label, z)
    if dof is not None:
        z = stats.norm.ppf(np.clip(stats.t.cdf(z, dof), 1e-300, 1.0 - 1e-16))
    n = z.size
    beyond = int(np.sum(np.abs(z) > 3.0))
    rate = 2.0 * stats.norm.sf(3.0)
    p_beyond = float(stats.binom.sf(beyond - 1, n, rate)) if beyond else 1.0
    chi2 = float(np.sum(z * z))
    p_chi2 = float(stats.chi2.sf(chi2, n))
    s = dict(label=label, n=n, beyond_3sigma=beyond, frac_beyond=beyond / n, p_beyond=p_beyond,
             chi2_per_bin=chi2 / n, p_chi2=p_chi2, max_abs=float(np.max(np.abs(z))), mean=float(np.mean(z)))
    print("[z] " + " ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}" for k, v in s.items()), flush=True)
    assert beyond <= 0.01 * n or (n < 100 and p_beyond >= p_min), s
    assert p_chi2 >= p_min, s
    return s


def z_two_sided(d, err_lo, err_hi):
    """z of a log-space difference d = log(estimate) - log(reference) with asymmetric errors:
    the upper error where the estimate lies above the reference, the lower one below."""
    return np.where(d > 0, d / err_lo, d / err_hi)
