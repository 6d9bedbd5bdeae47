"""Statistical validation of the GPU estimates at full size against what the paper fixes.

Every comparison is judged by `helpers.check_z`: at most 1 % of the bins beyond 3 sigma (or, for
under 100 bins, no more than Gaussian errors give with probability 0.999) and a chi^2 p-value of
at least 0.001, with jackknife errors taken as Student-t with 15 degrees of freedom.

* Diffusion-dominated tail (the paper's m = 1, phi_in = phi_UV = sqrt 42 case of Sec. 3.1 and
  config C2's m = 1, phi_in = 6, wall at 8): P(N) = sum_n a_n exp(-Lambda_n N) (pole expansion,
  Sec. 1 and App. A) from the oracle's Sturm-Liouville solve, with the absorbing end moved out
  by beta S sqrt(dN) for the discrete monitoring; compared bin by bin within the estimated
  error in every bin the paper's own criteria trust.
* Drift-dominated case (m = 0.01, phi_in = 10), A = 1, 2, 4: the saddle-point density built from
  eight cumulants of N (the resummed form of App. B's cumulant expansion; App. B's Gaussian is
  off by factors of hundreds 12 standard deviations out at this skewness) on the simulation's
  lattice, against the naive estimates the paper's criteria trust and the lognormal estimates
  of Sec. 2.4 in every bin with at least 100 runs, down to P ~ 1e-99.
* Without a wall (the same potential): the branch-cut integral of App. A's infinite-phi_UV
  limit, bin by bin, for direct runs and for A = 0.3, with 1 % for the time step (reading R24).
* The three bias amplitudes of each case estimate the same P(N) where their samples overlap
  (Sec. 3: different A probe different regions of one distribution).
* Binary32 against binary64: the same runs through the oracle's binary64 mode differ from the
  binary32 histogram by a small fraction of the statistical error (stated for config C1).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import refmath as R
import workloads as W
from helpers import check_z, z_two_sided

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


@pytest.fixture(scope="module")
def c2_results(fpt):
    insts = W.c2()
    print("[case] C2 full statistics", flush=True)
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    return insts, results


def _bin_average(f, edges, n=64):
    out = np.empty(len(edges) - 1)
    for j in range(len(edges) - 1):
        x = np.linspace(edges[j], edges[j + 1], n + 1)
        y = f(x)
        out[j] = np.trapezoid(y, x) / (edges[j + 1] - edges[j])
    return out


def _trusted(res):
    """Bins whose naive estimate and error are reliable by the paper's own criteria: n_j > 400
    for the jackknife (Sec. 2.1) and n_j > <w>^2 exp(sigma^2_lnw) for the weight dispersion
    (Sec. 2.4; <w>^2 is the squared mean of the bin's weights relative to its typical weight,
    taken as 1 here, so the condition is n_j > exp(sigma^2_lnw))."""
    B = res.n_bins
    n = res.count[:B].astype(float)
    with np.errstate(over="ignore", invalid="ignore"):
        disp_ok = n > np.exp(np.nan_to_num(res.m2_lnw[:B], nan=np.inf))
    return (n > 400) & disp_ok & np.isfinite(res.log_p)


def _pole_reference(model, edges, dN, n_modes=6):
    S_end = model.m * model.phi_end / (2 * math.pi * math.sqrt(6))
    shifted = O.Model(m=model.m, phi_in=model.phi_in, phi_uv=model.phi_uv,
                      phi_end=model.phi_end - R.BGK_BETA * S_end * math.sqrt(dN))
    modes = R.sl_modes(shifted, n_modes, lam_max=4.0, n_scan=160)
    pdf = lambda N: np.sum(modes.amp[None, :] * np.exp(-modes.lam[None, :] * N[:, None]), axis=1)
    return _bin_average(pdf, edges), modes


def test_paper_diffusion_case_matches_pole_expansion(fpt):
    """Sec. 3.1 / Fig. 3: m = 1, phi_in = phi_UV = sqrt 42, 2e5 runs each for A = 0, 0.4, 0.8.
    The paper reaches P ~ 1e-3, 1e-6, 1e-12; here every trusted bin (N >= 10, where the six
    slowest poles have converged) agrees with the pole expansion within its jackknife error,
    and the reach with A = 0.8 is at least 1e-8 under the dispersion criterion.  The reach over
    bins with at least 100 runs (1.6e-3, 1.6e-6, 1.4e-14 in this run) matches the paper's; bins
    of n_j > 400 alone stop at 1.2e-10 with A = 0.8 (the reach depends on that count)."""
    insts = [W.paper_diffusion(A, stream=i) for i, A in enumerate((0.0, 0.4, 0.8))]
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    ref, modes = _pole_reference(O.Model.from_instance(insts[0]), insts[0].edges, insts[0].dN)
    assert abs(modes.lam[0] - 0.6528232) < 1e-4
    reach = []
    reach100 = []
    for inst, res in zip(insts, results):
        use = _trusted(res) & (res.edges[:-1] >= 10.0)
        z = (np.exp(res.log_p[use]) / ref[use] - 1) / res.rel_err_jk[use]
        reach.append(ref[use].min())
        n400 = (res.count[:res.n_bins] > 400) & np.isfinite(res.log_p)
        n100 = (res.count[:res.n_bins] >= 100) & np.isfinite(res.log_p)
        reach100.append(np.exp(res.log_p[n100]).min())
        print(f"{inst.name}: trusted bins {use.sum()}, reach P {ref[use].min():.2e} "
              f"(n_j > 400 only: {ref[n400].min():.2e}; n_j >= 100: {reach100[-1]:.2e})")
        check_z(z, 15, inst.name + " vs pole expansion")
    assert reach[0] > reach[1] > reach[2]
    assert reach[2] < 1e-8
    assert reach100[0] < 5e-3 and reach100[1] < 5e-6 and reach100[2] < 1e-12


def test_no_wall_tail_matches_branch_cut(fpt):
    """The C2 diffusion potential (m = 1, phi_in = 6) without a wall, where the characteristic
    function has a branch cut instead of poles (App. A, the infinite-phi_UV limit): trusted bins
    of width 0.5 from N = 10 out to the reach of 2e6 direct runs and of 1e7 runs with A = 0.3,
    against the branch-cut integral (end moved by beta S sqrt(dN)) at the bin centre, with 1 %
    added in quadrature to the jackknife error for the time step and the bin's curvature."""
    edges = np.arange(6.0, 60.001, 0.5)
    base = W.Instance("no_wall", m=1.0, phi_in=6.0, dN=1e-3, n_traj=2_000_000, k_max=200_000, edges=edges)
    insts = [base, W.Instance("no_wall_A0.3", m=1.0, phi_in=6.0, bias=W.BIAS_NOISE_SCALED, A=0.3, dN=1e-3,
                              n_traj=10_000_000, k_max=200_000, stream=1, edges=edges)]
    print("[case] no wall, A = 0 and 0.3", flush=True)
    results, _, _ = fpt.run_batch(insts, 0, block=512, wg_per_cu=2, chunk=1)
    S_end = base.m * base.phi_end / (2 * math.pi * math.sqrt(6))
    shifted = O.Model(m=base.m, phi_in=base.phi_in, phi_end=base.phi_end - R.BGK_BETA * S_end * math.sqrt(base.dN))
    centres = 0.5 * (edges[:-1] + edges[1:])
    ref = {}
    reach = []
    for inst, res in zip(insts, results):
        use = np.nonzero(_trusted(res) & (edges[:-1] >= 10.0))[0]
        use = use[::4]                                      # every fourth trusted bin (2 e-folds apart)
        z = []
        for j in use:
            if j not in ref:
                ref[j] = R.pdf_no_wall(float(centres[j]), shifted)
            d = math.exp(res.log_p[j]) / ref[j] - 1.0
            z.append(d / math.sqrt(res.rel_err_jk[j] ** 2 + 0.01 ** 2))
            print(f"{inst.name}: N = {centres[j]:.2f}, P {math.exp(res.log_p[j]):.4e} vs {ref[j]:.4e}, "
                  f"rel err {res.rel_err_jk[j]:.4f}")
        reach.append(min(ref[j] for j in use))
        assert len(use) >= 3
        check_z(z, 15, inst.name + " vs branch cut")
    assert reach[1] < reach[0] / 100


def test_c2_diffusion_tail_matches_pole_expansion(c2_results):
    """Config C2, diffusion-dominated, A = 1: trusted bins agree with the pole expansion; the
    reach is reported (the paper notes that with B = A S the weights spread in this regime,
    which limits how far a fixed bias goes, Sec. 3.1)."""
    insts, results = c2_results
    inst, res = insts[3], results[3]
    ref, _ = _pole_reference(O.Model.from_instance(inst), res.edges, inst.dN)
    use = _trusted(res) & (res.edges[:-1] >= 10.0)
    z = (np.exp(res.log_p[use]) / ref[use] - 1) / res.rel_err_jk[use]
    print(f"C2 diffusion A=1: trusted bins {use.sum()}, reach P {ref[use].min():.2e}")
    assert use.sum() >= 10
    check_z(z, 15, "C2 diffusion A=1 vs pole expansion")


def test_drift_case_matches_saddlepoint_reference(c2_results):
    """Config C2, drift-dominated (m = 0.01, phi_in = 10), A = 1, 2, 4 at 1e6 runs each: the naive
    estimates in the bins the paper's criteria trust (n_j > 400, n_j > exp(sigma^2_lnw); only
    A = 1 has such bins) and the lognormal estimates (Sec. 2.4, Cox interval) in every bin with
    at least 100 runs agree with the saddle-point reference built from eight cumulants of N on
    the lattice N = k dN, within their errors and the reference's truncation error.  The
    lognormal estimates reach P < 1e-30 with A = 2 and P < 1e-90 with A = 4."""
    insts, results = c2_results
    model = O.Model(m=0.01, phi_in=10.0, dN=1e-3)
    ref, trunc = R.saddlepoint_reference(model, insts[0].edges, order=8, n_grid=200001)
    ok_ref = np.isfinite(trunc)
    assert ok_ref.sum() == len(ref), "the truncation has converged over every bin of this workload"
    reach = []
    for inst, res in zip(insts[:3], results[:3]):
        B = res.n_bins
        n = res.count[:B]
        tn = _trusted(res)
        if tn.sum():
            z = (np.exp(res.log_p[tn] - ref[tn]) - 1) / np.sqrt(res.rel_err_jk[tn] ** 2 + trunc[tn] ** 2)
            check_z(z, 15, inst.name + " naive vs saddle point")
        use = (n >= 100) & np.isfinite(res.log_p_ln)
        with np.errstate(divide="ignore"):
            lo, hi = -np.log1p(-res.rel_err_ln_lo), np.log1p(res.rel_err_ln_hi)
        z = z_two_sided(res.log_p_ln - ref, np.sqrt(lo ** 2 + trunc ** 2), np.sqrt(hi ** 2 + trunc ** 2))
        check_z(z[use], None, inst.name + " lognormal vs saddle point")
        reach.append(float(np.exp(ref[use]).min()))
        print(f"{inst.name}: lognormal bins {use.sum()} reach P {reach[-1]:.2e}")
    assert reach[1] < 1e-30 and reach[2] < 1e-90


def test_bias_amplitudes_agree_where_samples_overlap(c2_results):
    """Bins trusted in two runs with different A estimate the same P(N)."""
    insts, results = c2_results
    for group in (results[:3], results[3:]):
        for a in range(3):
            for b in range(a + 1, 3):
                ra, rb = group[a], group[b]
                use = _trusted(ra) & _trusted(rb)
                if use.sum() == 0:
                    continue
                d = ra.log_p[use] - rb.log_p[use]
                err = np.sqrt(ra.rel_err_jk[use] ** 2 + rb.rel_err_jk[use] ** 2)
                # two jackknife errors of 15 degrees of freedom each: about 30 together
                check_z(d / err, 30, f"A pair {a},{b}")


def test_weights_average_to_one_with_censored_runs(c2_results):
    """E_S[w] = 1 over every launched run, censored and escaped ones included."""
    insts, results = c2_results
    for inst, res in zip(insts, results):
        mean_w = math.exp(res.lse_w_all) / inst.n_traj
        ess = math.exp(2 * res.lse_w_all - res.lse_w2_all)
        if ess > 1000:
            assert abs(mean_w - 1) < 6 / math.sqrt(ess), (inst.name, mean_w, ess)


def test_binary32_vs_binary64_on_c1(fpt):
    """Config C1: the binary32 histogram and the binary64 oracle's histogram of the same 1e4
    runs agree to a fraction of the statistical error (the error of every binary32 result
    against binary64 is stated by this comparison)."""
    inst = W.c1()
    res, _, _ = fpt.run(inst, 0, block=512, wg_per_cu=2, chunk=1)
    tr64 = O.simulate(O.Model.from_instance(inst), 0, inst.n_traj, mode=O.MODE_F64)
    h64 = O.histogram(tr64, inst.dN, inst.edges)
    c32 = res.count[:100].astype(float)
    c64 = h64.count[:100].astype(float)
    # per-bin count difference in units of the Poisson error of the bin
    err = np.sqrt(np.maximum(c64, 1.0))
    z = (c32 - c64) / err
    print("binary32 - binary64 per-bin |z| max", np.max(np.abs(z)), "rms", np.sqrt(np.mean(z ** 2)))
    assert np.sqrt(np.mean(z ** 2)) < 0.5
    assert abs(res.total_steps - int(tr64.k.sum())) / int(tr64.k.sum()) < 1e-4
