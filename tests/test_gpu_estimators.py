"""The estimators of Sec. 2.4 and Sec. 3 on the GPU against what the paper reports.

* Lognormal estimator and normality gate (Sec. 2.4): in the drift-dominated case the
  D'Agostino-Pearson p-values of ln w pass the 0.5 % gate and the lognormal estimate agrees
  with the naive one where both are trusted.
* Interim case (Sec. 3.2: m = 0.1, phi_in = phi_UV = sqrt 42, A = 1.5, 2e5 runs): the gate
  passes and the lognormal estimate agrees with the Edgeworth expansion (App. B, cumulants
  from the backward equation) in the near tail, where the paper finds agreement.
* Multi-bias reconstruction (Sec. 3.2, 3.3): A = 0, 1, 2, 3 in one batched launch combined bin
  by bin; every contributing estimate is consistent with the combination, and the combination
  reaches far below direct sampling.
* Power-law bias (Sec. 3.4, m = 0.001): with A_p tuned to put the classical sample mean 8
  standard deviations above the target mean, |r| of log10 w with N grows from p = 1 and peaks
  near p = 3, where the paper finds the optimum.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import optimize

import oracle as O
from oracle import refmath as R
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


def test_lognormal_gate_and_estimator_drift_case(fpt):
    insts = W.c2()[:3]
    print("[case] C2 drift, A = 1, 2, 4", flush=True)
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    compared = 0
    for inst, r in zip(insts, results):
        B = r.n_bins
        n = r.count[:B].astype(float)
        pv = r.normal_p
        pop = (n >= 400) & np.isfinite(pv)
        with np.errstate(all="ignore"):
            trusted = pop & (n > np.exp(r.m2_lnw[:B]))
            err = np.sqrt(r.rel_err_jk ** 2 + (0.5 * (r.rel_err_ln_hi + r.rel_err_ln_lo)) ** 2)
            z = (np.exp(r.log_p_ln - r.log_p) - 1) / err
            mz = np.median(np.abs(z[trusted])) if trusted.any() else float("nan")
        print(f"{inst.name}: populated bins {pop.sum()}, gate failures {np.sum(pv[pop] < 0.005)}, "
              f"median p {np.median(pv[pop]):.3f}, trusted {trusted.sum()}, median |z| {mz:.2f}")
        assert pop.sum() >= 20
        assert np.mean(pv[pop] < 0.005) <= 0.05
        assert np.median(pv[pop]) > 0.1
        assert r.lognormal_accepted() or np.sum(pv[pop] < 0.005) <= 2
        # the naive estimate is trusted only where n_j > exp(sigma^2_lnw) (none for A >= 2 here)
        if trusted.sum() >= 10:
            assert np.mean(np.abs(z[trusted]) < 3) >= 0.9
        compared += trusted.sum()
    assert compared >= 20


def _interim(A, n, stream, edges, dN=1e-3):
    phi = math.sqrt(42.0)
    return W.Instance(f"interim_A{A}", m=0.1, phi_in=phi, phi_uv=phi,
                      bias=W.BIAS_NOISE_SCALED if A else W.BIAS_NONE, A=A, dN=dN, n_traj=n, stream=stream,
                      edges=edges)


@pytest.fixture(scope="module")
def interim(fpt):
    edges = np.round(np.arange(9.2, 15.0 + 1e-9, 0.02), 10)
    mdl = O.Model(m=0.1, phi_in=math.sqrt(42.0), phi_uv=math.sqrt(42.0))
    mu, sig, gam, kap = R.edgeworth_for(mdl, n_grid=200001)
    dN = 1e-3

    def edgeworth_bins(e):
        out = []
        for a, b in zip(e[:-1], e[1:]):
            x = np.linspace(a, b, 65)
            out.append(np.trapezoid(R.edgeworth_pdf(x - dN, mu, sig, gam, kap), x) / (b - a))
        return np.array(out)
    return edges, (mu, sig, gam, kap), edgeworth_bins(edges)


def test_interim_case_lognormal_matches_edgeworth(fpt, interim):
    edges, (mu, sig, gam, kap), ref = interim
    print(f"[case] interim A = 1.5: Edgeworth mu {mu:.5f} sigma {sig:.5f} gamma {gam:.4f} kappa {kap:.4f}", flush=True)
    r, _, _ = fpt.run(_interim(1.5, 200_000, 0, edges), 0, block=512, wg_per_cu=2, chunk=1)
    B = r.n_bins
    n = r.count[:B].astype(float)
    pv = r.normal_p
    c = 0.5 * (edges[:-1] + edges[1:])
    use = (n >= 100) & np.isfinite(r.log_p_ln) & (c <= mu + 3.5 * sig)
    err = 0.5 * (r.rel_err_ln_hi + r.rel_err_ln_lo)
    z = (np.exp(r.log_p_ln[use]) / ref[use] - 1) / err[use]
    reach = np.exp(r.log_p_ln[np.isfinite(r.log_p_ln) & (n >= 100)]).min()
    print(f"bins compared {use.sum()}, median |z| {np.median(np.abs(z)):.2f}, max |z| {np.max(np.abs(z)):.2f}; "
          f"gate failures {np.sum(pv[n >= 8] < 0.005)} of {np.sum(np.isfinite(pv))}; reach P {reach:.2e}")
    assert use.sum() >= 20
    assert np.mean(np.abs(z) < 3) >= 0.9
    assert np.mean(pv[np.isfinite(pv)] < 0.005) <= 0.05
    assert reach < 1e-8


def test_multi_bias_reconstruction_interim_case(fpt, interim):
    edges, (mu, sig, gam, kap), ref = interim
    insts = [_interim(A, 250_000, i, edges) for i, A in enumerate((0.0, 1.0, 2.0, 3.0))]
    print("[case] interim multi-bias A = 0, 1, 2, 3", flush=True)
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    lp, el, nu = fpt.combine(results, 2)
    ok = nu > 0
    print(f"combined bins {ok.sum()}, reach P {np.exp(lp[ok]).min():.2e}, direct-sampling reach "
          f"{np.exp(results[0].log_p[results[0].count[:results[0].n_bins] > 400]).min():.2e}")
    # every contributing estimate is consistent with the combination
    zs = []
    for r in results:
        single_lp, single_el, single_nu = fpt.combine([r], 2)
        both = ok & (single_nu > 0)
        zs.append((single_lp[both] - lp[both]) / single_el[both])
    zs = np.concatenate(zs)
    print(f"consistency: {zs.size} estimates, fraction |z| < 3: {np.mean(np.abs(zs) < 3):.3f}")
    assert np.mean(np.abs(zs) < 3) >= 0.9
    assert np.exp(lp[ok]).min() < 1e-20
    near = ok & (0.5 * (edges[:-1] + edges[1:]) <= mu + 3 * sig)
    zr = (lp[near] - np.log(ref[near])) / el[near]
    print(f"near tail vs Edgeworth: {near.sum()} bins, fraction |z| < 3: {np.mean(np.abs(zr) < 3):.3f}")
    assert np.mean(np.abs(zr) < 3) >= 0.8


def test_power_law_bias_pearson_scan(fpt):
    phi_in, m, dN = math.sqrt(42.0), 0.001, 1e-4
    sig = math.sqrt(R.classical_var_quadratic(m, phi_in, math.sqrt(2.0)))
    target = R.classical_N(O.Model(m=m, phi_in=phi_in)) + 8 * sig
    insts, amps = [], []
    for p in (1, 2, 3, 4, 5):
        f = lambda lgA: R.classical_N(O.Model(m=m, phi_in=phi_in, bias=O.BIAS_POWER, A=math.exp(lgA), p=p),
                                      biased=True) - target
        hi = math.log(0.9 * 2.0 / phi_in ** (p + 1))
        lgA = optimize.brentq(f, hi - 40, hi, xtol=1e-12)
        amps.append(math.exp(lgA))
        insts.append(W.Instance(f"power_p{p}", m=m, phi_in=phi_in, bias=W.BIAS_POWER, A=math.exp(lgA), p=p, dN=dN,
                                n_traj=40_000, stream=p, edges=np.linspace(9.99, 10.05, 61)))
    print("[case] power-law bias scan p = 1..5", flush=True)
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    r = np.array([abs(res.pearson_r) for res in results])
    for p, A, rr, res in zip((1, 2, 3, 4, 5), amps, r, results):
        print(f"p = {p}: A_p = {A:.4e}, |r| = {rr:.4f}, ended {res.count[:res.n_bins + 2].sum()}")
    assert np.all(np.isfinite(r))
    assert r[2] > r[0] and r[1] > r[0]
    assert int(np.argmax(r)) + 1 in (3, 4)


def test_bump_potential_multi_bias(fpt):
    """The large-run configuration (bump potential, dN = 1e-4, 500 bins) at 7e6 runs: the
    combined lognormal estimates agree with each contributing amplitude, with the Edgeworth
    expansion of the bump potential's own cumulants near the peak, and reach below 1e-40 with
    errors under half a decade."""
    insts = W.c5_multi(n_total=7_000_000)
    print("[case] bump potential multi-bias, 7e6 runs", flush=True)
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    lp, el, nu = fpt.combine(results, 1)
    ok = nu > 0
    zs = []
    for r in results:
        s_lp, s_el, s_nu = fpt.combine([r], 1)
        both = ok & (s_nu > 0) & (nu > 1)
        zs.append((s_lp[both] - lp[both]) / np.sqrt(np.maximum(s_el[both] ** 2 - el[both] ** 2, 1e-30)))
    zs = np.concatenate(zs)
    good = ok & (el < 0.5 * math.log(10))
    reach = lp[good].min() / math.log(10)
    mdl = O.Model.from_instance(insts[0])
    mu, sig, gam, kap = R.edgeworth_for(mdl, n_grid=200001)
    e = results[0].edges
    c = 0.5 * (e[:-1] + e[1:])
    near = ok & (np.abs(c - mu) <= 2.5 * sig)
    ref = np.array([np.trapezoid(R.edgeworth_pdf(np.linspace(a, b, 33) - insts[0].dN, mu, sig, gam, kap),
                                 np.linspace(a, b, 33)) / (b - a) for a, b in zip(e[:-1], e[1:])])
    zr = (lp[near] - np.log(ref[near])) / el[near]
    print(f"consistency {zs.size} estimates, |z| < 3: {np.mean(np.abs(zs) < 3):.3f}; reach log10 P {reach:.1f}; "
          f"near peak vs Edgeworth ({near.sum()} bins, gamma {gam:.3f}): |z| < 3: {np.mean(np.abs(zr) < 3):.3f}")
    assert np.mean(np.abs(zs) < 3) >= 0.9
    assert reach < -40
    assert near.sum() >= 10 and np.mean(np.abs(zr) < 3) >= 0.8
