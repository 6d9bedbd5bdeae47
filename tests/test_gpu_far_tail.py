"""The fixed-bias far tail at P ~ 1e-30, at full size.

Config C2's drift-dominated case with the noise-scaled bias A = 2 (m = 0.01, phi_in = 10, no
wall, dN = 1e-3, 1e6 runs, 200 log-spaced bins): the amplitude that puts the most runs near
P ~ 1e-30 of the three the workload carries.

* Parity: all 1e6 runs against the oracle's runs of the same ids (2.5e10 steps on the host's
  cores): identical step counts, statuses, final fields and log-weights, bit for bit; every row
  of the histogram (counts per row and per jackknife subset, log-sums within 1e-12, moments,
  estimators) against the oracle's histogram of those runs.
* Reference: in the window of bins whose reference P lies between 1e-32 and 1e-28, the
  lognormal estimate (Sec. 2.4) with its Cox interval agrees with the saddle-point density of N
  built from eight of its cumulants (the resummed form of App. B's cumulant expansion) on the
  lattice N = k dN, bin by bin within 3 of its errors combined with the reference's truncation
  error; the reached P is stated.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import refmath as R
import workloads as W
from helpers import assert_dump_matches, assert_histogram_matches, check_z, to_model, z_two_sided

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


def test_drift_case_A2_far_tail_full_size(fpt):
    inst = W.c2()[1]
    assert inst.A == 2.0 and inst.n_traj == 1_000_000
    print(f"[case] C2 drift A = 2, {inst.n_traj} runs, every run dumped", flush=True)
    res, dump, _ = fpt.run(inst, 0, dump_n=inst.n_traj, block=512, wg_per_cu=2, chunk=1)
    print(f"[case] GPU done: {res.total_steps} steps; oracle on the host cores", flush=True)
    tr = O.simulate(to_model(inst), 0, inst.n_traj)
    print("[case] oracle done", flush=True)
    assert_dump_matches(dump, tr)
    h = O.histogram(tr, inst.dN, inst.edges)
    assert_histogram_matches(res, h)
    assert res.total_steps == int(tr.k.sum())

    ref, trunc = R.saddlepoint_reference(O.Model(m=0.01, phi_in=10.0, dN=inst.dN), inst.edges, order=8,
                                         n_grid=200001)
    B = res.n_bins
    n = res.count[:B]
    log10_ref = ref / math.log(10.0)
    window = (log10_ref >= -32.0) & (log10_ref <= -28.0)
    with np.errstate(divide="ignore"):
        lo, hi = -np.log1p(-res.rel_err_ln_lo), np.log1p(res.rel_err_ln_hi)
    z = z_two_sided(res.log_p_ln - ref, np.sqrt(lo ** 2 + trunc ** 2), np.sqrt(hi ** 2 + trunc ** 2))
    centres = 0.5 * (inst.edges[1:] + inst.edges[:-1])
    for j in np.nonzero(window)[0]:
        print(f"N {centres[j]:.4f}: runs {n[j]}, log10 P {res.log_p_ln[j] / math.log(10):.3f} "
              f"(+{math.log10(1 + res.rel_err_ln_hi[j]):.3f} / -{-math.log10(1 - res.rel_err_ln_lo[j]):.3f}), "
              f"reference {log10_ref[j]:.3f}, z {z[j]:.2f}, normality p {res.normal_p[j]:.3f}", flush=True)
    assert window.sum() >= 4
    assert np.all(n[window] >= 30), "every window bin holds runs"
    assert np.all(np.isfinite(trunc[window])) and np.all(np.abs(z[window]) < 3.0)
    check_z(z[window], None, "C2 drift A=2 window P in [1e-32, 1e-28]")
    reached = float(np.min(log10_ref[(n >= 30) & np.isfinite(res.log_p_ln)]))
    print(f"lognormal estimates in bins with >= 30 runs reach log10 P = {reached:.2f}", flush=True)
    assert reached < -30.0
