"""Learned proposals as the referee of the fixed-bias far tail on the bump potential (the large
run's configuration, dN = 1e-4, 500 bins, at a size a test can afford).

Importance sampling is unbiased for any proposal, and a proposal whose ln w spreads over a nat
or two in a bin gives a plain naive estimate there (no lognormal model) that its runs resolve.
Networks trained through windows at N = 17, 18 and 19 (the curriculum of the large run) are run
on noise streams of their own; the checks:

* each network's naive estimates agree with the combination of the others' bin by bin (the
  acceptance rule of the statistical tests, jackknife errors through Student's t);
* the learned combination agrees with direct sampling (A = 0) and A = 1 where their naive
  estimates are trusted;
* printed, not asserted: the fixed amplitudes' lognormal estimates minus the learned
  combination, in decades, beside the spread of their ln w.
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from helpers import check_z

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


def test_bump_potential_learned_proposals_agree_with_each_other_and_direct_sampling(fpt):
    L10 = math.log(10.0)
    fixed = W.c5_multi(amplitudes=(0.0, 1.0, 2.0, 3.0), n_total=40_000_000)
    print("[case] bump potential, A = 0..3, 1e7 runs each", flush=True)
    fixed_res, _, _ = fpt.run_batch(fixed, 0, block=512, wg_per_cu=2, chunk=1)

    base = fixed[0]
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    v[:4480] = np.random.default_rng(0).normal(0.0, 1e-2, 4480)
    v[4480] = 2.0
    p0 = W.MlpParams(W.bf16_round(v), in_mean=(8.0, 20.0, 20.0), in_inv_scale=(0.25, 0.1, 0.1),
                     out_scale=1.0, eval_every=16)
    inst0 = dataclasses.replace(base, name="C5_learned", bias=W.BIAS_MLP, A=0.0, mlp=p0, n_traj=1_000_000)
    theta = p0.values_f32()
    learned = []
    for si, centre in enumerate((17.0, 18.0, 19.0)):
        print(f"[case] training stage {centre:g}", flush=True)
        theta, _, rep = fpt.train_proposal(dataclasses.replace(inst0, target_N=centre), 1 + 100 * si, theta,
                                           window=(centre - 0.3, centre + 0.3), n_sample=100_000, rounds=3,
                                           steps=40, max_paths=8000, lr=3e-3, objective=1, temper=0.5)
        inst = dataclasses.replace(inst0, name=f"C5_learned_{centre:g}", target_N=centre,
                                   mlp=dataclasses.replace(p0, values=theta.copy()), stream=20 + si)
        res, _, _ = fpt.run(inst, 0, block=256, wg_per_cu=3, chunk=1)
        learned.append(res)
        print(f"  stage {centre:g}: window runs of the last round {rep[-1]['n_window']}", flush=True)

    edges = base.edges
    centres = 0.5 * (edges[1:] + edges[:-1])
    # leave-one-out among the learned proposals, naive estimates with their own trust rule
    z = []
    for i in range(len(learned)):
        lo, eo, no = fpt.combine([r for k, r in enumerate(learned) if k != i], 0)
        li, ei, ni = fpt.combine([learned[i]], 0)
        m = (ni > 0) & (no > 0)
        z += list((li[m] - lo[m]) / np.hypot(ei[m], eo[m]))
        print(f"  learned {i}: {m.sum()} bins shared with the others", flush=True)
    assert len(z) >= 30
    check_z(z, 15, "learned proposals, leave-one-out")

    ll, le, ln = fpt.combine(learned, 0)
    cov = centres[ln > 0]
    print(f"learned naive combination: {int((ln > 0).sum())} bins, N {cov.min():.2f} .. {cov.max():.2f}, "
          f"down to log10 P {ll[ln > 0].min() / L10:.1f}", flush=True)
    zd = []
    for A, r in zip((0, 1), fixed_res[:2]):
        fl, fe, fn = fpt.combine([r], 0)
        m = (fn > 0) & (ln > 0)
        zd += list((fl[m] - ll[m]) / np.hypot(fe[m], le[m]))
        print(f"  A = {A}: {m.sum()} trusted naive bins shared with the learned combination", flush=True)
    assert len(zd) >= 10
    check_z(zd, 15, "direct sampling and A = 1 against the learned proposals")

    B = len(centres)
    for A, r in zip((1, 2, 3), fixed_res[1:]):
        n = r.count[:B]
        m = (n >= 400) & (ln > 0) & np.isfinite(r.log_p_ln[:B])
        if not m.any():
            continue
        d = (r.log_p_ln[:B][m] - ll[m]) / L10
        s = np.sqrt(np.maximum(r.m2_lnw[:B][m] * n[m] / np.maximum(n[m] - 1, 1), 0.0))
        print(f"  A = {A}: lognormal minus learned over {m.sum()} bins (N {centres[m].min():.2f} .. "
              f"{centres[m].max():.2f}): median {np.median(d):+.2f} decades, spread of ln w {s.min():.1f} .. "
              f"{s.max():.1f} nats", flush=True)
