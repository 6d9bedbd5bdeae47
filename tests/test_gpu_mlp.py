"""The learned proposal (3 -> 64 -> 64 -> 1 tanh network, bfloat16 weights) on the GPU against
the oracle's binary64 evaluation of the same network with the same bfloat16 roundings.

The matrix cores accumulate in binary32 in their own order, so an activation can round to the
neighbouring bfloat16 now and then: the bias agrees to a small tolerance rather than bit for
bit, and runs of the learned sampler agree in step count for almost every run, with their
log-weights agreeing closely; their estimates agree statistically.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import to_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


@pytest.mark.parametrize("seed,scale", [(0, 1.0), (1, 3.0)])
def test_mlp_forward_matches_oracle(fpt, seed, scale):
    params = W.c4_params(seed, scale=scale, out_scale=1.5)
    rng = np.random.default_rng(10 + seed)
    n = 50_000
    phi = rng.uniform(1.4, 8.0, n).astype(np.float32)
    N = rng.uniform(0.0, 600.0, n).astype(np.float32)
    r_gpu = fpt.mlp_forward(params, 196.0, phi, N).astype(np.float64)
    model = O.Model(m=1.0, bias=O.BIAS_MLP, mlp=params, target_N=196.0)
    r_ref = O.mlp_r(model, phi, N)
    err = np.abs(r_gpu - r_ref)
    print(f"seed {seed}: r range [{r_ref.min():.3f}, {r_ref.max():.3f}], max |dr| {err.max():.2e}, "
          f"99.9% {np.quantile(err, 0.999):.2e}, median {np.median(err):.2e}, "
          f"bit-identical {np.mean(r_gpu.astype(np.float32) == r_ref.astype(np.float32)):.4f}")
    assert np.quantile(err, 0.999) < 5e-3 * params.out_scale
    assert err.max() < 3e-2 * params.out_scale
    assert np.median(err) < 2e-4 * params.out_scale


@pytest.mark.parametrize("every", [4, 1, 8, 16])
def test_mlp_sampler_matches_oracle(fpt, every):
    params = W.c4_params(3, out_scale=1.0, eval_every=every)
    inst = W.c4_instance(params, n_traj=600)
    res, dump, _ = fpt.run(inst, 0, block=256, wg_per_cu=1, chunk=1, dump_n=inst.n_traj)
    tr = O.simulate(to_model(inst), 0, inst.n_traj)
    k = dump.k[:inst.n_traj].astype(np.uint64)
    same = k == tr.k
    print(f"every {every}: identical step counts {same.mean():.4f}")
    assert same.mean() > 0.99
    # One activation flipping to the neighbouring bfloat16 moves r by ~ |w| 2^-8 ~ 1e-3 (the
    # forward test bounds it); that happens in ~1% of evaluations, each of which changes the
    # log-weight increment by ~ dr sqrt(dN) sigma / sigma ~ 1e-3 * 0.03.  Over the ~2e3
    # evaluations of a run, a few tens of flips accumulate to lw differences of ~1e-4.
    lw_rel = np.abs(dump.lw[same] - tr.lw[same]) / np.maximum(1.0, np.abs(tr.lw[same]))
    print(f"  lw rel diff max {lw_rel.max():.2e} median {np.median(lw_rel):.2e}")
    assert np.median(lw_rel) < 3e-4
    assert np.quantile(lw_rel, 0.99) < 3e-3
    assert int(res.count.sum()) == inst.n_traj


@pytest.mark.parametrize("every", [4, 1, 8, 16])
def test_constant_network_sampler_bit_exact(fpt, every):
    """A network whose only nonzero parameter is b3 gives r = out_scale b3 exactly on the matrix
    cores (zero weights times bounded activations add exact zeros), so the learned path must
    reproduce the oracle's noise-scaled bias of that value bit for bit."""
    from helpers import assert_dump_matches
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    v[4480] = 0.5
    params = W.MlpParams(v, out_scale=2.0, eval_every=every)
    base = W.c2(2000)[3]                  # A = 1
    inst = W.c4_instance(params, n_traj=2000, stream=base.stream)
    res, dump, _ = fpt.run(inst, 0, block=256, wg_per_cu=1, chunk=1, dump_n=inst.n_traj)
    tr = O.simulate(to_model(base), 0, base.n_traj)
    assert_dump_matches(dump, tr)


@pytest.mark.parametrize("every", [4, 16])
def test_bump_potential_constant_network_bit_exact(fpt, every):
    """The learned bias on the bump potential of the large run (the kernel variant that run
    uses): a constant network r = 2 reproduces the oracle's noise-scaled bias A = 2 bit for bit,
    and a random network matches the oracle's network-driven runs as closely as on the quadratic
    potential."""
    import dataclasses
    from helpers import assert_dump_matches
    base = dataclasses.replace(W.with_runs(W.c5(), 48), bias=W.BIAS_NOISE_SCALED, A=2.0, stream=3)
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    v[4480] = 0.5
    const = dataclasses.replace(base, bias=W.BIAS_MLP, A=0.0, target_N=20.0,
                                mlp=W.MlpParams(v, out_scale=4.0, eval_every=every))
    res, dump, _ = fpt.run(const, 0, block=256, wg_per_cu=2, chunk=1, dump_n=const.n_traj)
    assert_dump_matches(dump, O.simulate(to_model(base), 0, base.n_traj))
    rnd = dataclasses.replace(const, mlp=W.MlpParams.random(5, 1.0, in_mean=(8.0, 20.0, 20.0),
                                                            in_inv_scale=(0.25, 0.1, 0.1), out_scale=1.0,
                                                            eval_every=every))
    res, dump, _ = fpt.run(rnd, 0, block=256, wg_per_cu=2, chunk=1, dump_n=rnd.n_traj)
    tr = O.simulate(to_model(rnd), 0, rnd.n_traj)
    same = dump.k[:rnd.n_traj].astype(np.uint64) == tr.k
    print(f"bump, random network, every {every}: identical step counts {same.mean():.3f}")
    assert same.mean() > 0.99
    lw_rel = np.abs(dump.lw[same] - tr.lw[same]) / np.maximum(1.0, np.abs(tr.lw[same]))
    assert np.median(lw_rel) < 3e-4


def test_learned_bias_batches_match_single_runs(fpt):
    """Two learned-bias instances sharing a network in one batch (the general kernel) give each
    instance's runs exactly as a launch of that instance alone (the single-instance kernel), and
    a batch whose first instance has no runs takes the single-instance kernel for the other."""
    import dataclasses
    params = W.c4_params(3, out_scale=1.0)
    a = W.c4_instance(params, n_traj=700, stream=3)
    b = dataclasses.replace(W.c4_instance(params, n_traj=500, stream=4), target_N=150.0)
    _, dumps, _ = fpt.run_batch([a, b], 0, block=256, wg_per_cu=1, chunk=1, dump_n=700)
    for inst, d in zip((a, b), dumps):
        _, d1, _ = fpt.run(inst, 0, block=256, wg_per_cu=2, chunk=1, dump_n=700)
        n = inst.n_traj
        assert np.array_equal(d.k[:n], d1.k[:n]) and np.array_equal(d.lw[:n], d1.lw[:n])
        assert np.array_equal(d.status[:n], d1.status[:n])
    empty = dataclasses.replace(a, n_traj=0)
    res, dumps, _ = fpt.run_batch([empty, b], 0, block=256, wg_per_cu=2, chunk=1, dump_n=700)
    _, d1, _ = fpt.run(b, 0, block=256, wg_per_cu=2, chunk=1, dump_n=700)
    assert np.array_equal(dumps[1].k[:500], d1.k[:500]) and np.array_equal(dumps[1].lw[:500], d1.lw[:500])
    assert res[0].n_traj == 0 and int(res[0].count.sum()) == 0 and int(res[1].count.sum()) == 500
