"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Bar: identical step counts, statuses, final fields and log-weights for every
dumped run (the step count is decided in binary32 on both sides); identical
counts per row and per jackknife subset; binary64 log-sums within 1e-12
relative (only the summation order differs); log-weights within the
1e-5 relative tolerance a fortiori.
"""
import dataclasses
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import assert_dump_matches, assert_histogram_matches, to_model

pytestmark = pytest.mark.gpu

SEED = 0
CFG = dict(block=512, wg_per_cu=2, chunk=1)


@pytest.fixture(scope="module")
def fpt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_11234_amd as F
    return F


def _oracle(inst, n=None, stride=1):
    n = inst.n_traj if n is None else n
    tr = O.simulate(to_model(inst), SEED, n, t0=inst.t_first, stride=stride)
    return tr


def _print_case(label, **kw):
    print(f"[case] {label} {kw}", flush=True)


def test_c1_bit_exact_every_run(fpt):
    """Config C1 in full: 1e4 direct-sampling runs, every run compared."""
    inst = W.c1()
    _print_case("C1", n=inst.n_traj)
    res, dump, _ = fpt.run(inst, SEED, dump_n=inst.n_traj, dump_stride=1, **CFG)
    tr = _oracle(inst)
    assert_dump_matches(dump, tr)
    h = O.histogram(tr, inst.dN, inst.edges)
    assert_histogram_matches(res, h)
    assert np.all(dump.lw == 0.0)


def test_c2_batch_prefix_bit_exact(fpt):
    """All six C2 instances (drift- and diffusion-dominated, A = 1, 2, 4) in one batched launch,
    on the first ids of each; every run compared and the histograms of those runs."""
    sizes = [1536, 1536, 1536, 700, 300, 300]
    insts = [W.with_runs(i, n) for i, n in zip(W.c2(), sizes)]
    _print_case("C2 prefix batch", sizes=sizes)
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=max(sizes), dump_stride=1, **CFG)
    for inst, res, dump in zip(insts, results, dumps):
        tr = _oracle(inst)
        assert_dump_matches(dump, tr)
        h = O.histogram(tr, inst.dN, inst.edges)
        assert_histogram_matches(res, h)


def test_queue_order_does_not_change_results(fpt):
    """The shared queue hands out a batch's instances longest expected run first, and a
    caller's cost_hint overrides the estimate.  The six C2 instances handed out drift first
    (the reverse of the default, which puts the capped diffusion runs first) give the same
    runs and histograms as the oracle."""
    sizes = [1536, 1536, 1536, 700, 300, 300]
    insts = [dataclasses.replace(W.with_runs(i, n), cost_hint=float(len(sizes) - j))
             for j, (i, n) in enumerate(zip(W.c2(), sizes))]
    _print_case("C2 prefix batch, drift instances first", sizes=sizes)
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=max(sizes), dump_stride=1, **CFG)
    for inst, res, dump in zip(insts, results, dumps):
        tr = _oracle(inst)
        assert_dump_matches(dump, tr)
        assert_histogram_matches(res, O.histogram(tr, inst.dN, inst.edges))


@pytest.mark.parametrize("block,wg,chunk", [(64, 8, 1), (256, 4, 4), (1024, 1, 1), (512, 2, 16)])
def test_launch_shape_does_not_change_results(fpt, block, wg, chunk):
    """Counter-based noise: every run's path depends only on (seed, stream, t), so counts are
    identical for any workgroup size, grid and queue claim chunk; ragged n_traj."""
    inst = W.with_runs(W.c2()[3], 1237)
    _print_case("shape", block=block, wg=wg, chunk=chunk)
    res, dump, _ = fpt.run(inst, SEED, block=block, wg_per_cu=wg, chunk=chunk, dump_n=1237)
    tr = _oracle(inst)
    assert_dump_matches(dump, tr)
    assert_histogram_matches(res, O.histogram(tr, inst.dN, inst.edges))


def test_edge_cases(fpt):
    """Empty run, one run, a cap that censors every run mid-group, a start on the wall,
    escapes, the flat potential, the bump potential and the power-law bias."""
    base = W.c2()[3]
    cases = {
        "empty": W.with_runs(base, 0),
        "one": W.with_runs(base, 1),
        "all_censored": W.Instance("cens", m=1.0, phi_in=6.0, phi_uv=8.0, bias=W.BIAS_NOISE_SCALED, A=1.0,
                                   dN=1e-3, n_traj=333, k_max=7, edges=np.linspace(0, 0.1, 11)),
        "start_on_wall": W.Instance("wall", m=1.0, phi_in=math.sqrt(42), phi_uv=math.sqrt(42),
                                    bias=W.BIAS_NOISE_SCALED, A=0.4, dN=1e-3, n_traj=200,
                                    edges=np.geomspace(0.5, 60, 41)),
        "escape": W.Instance("esc", m=1.0, phi_in=3.0, bias=W.BIAS_NOISE_SCALED, A=4.0, dN=1e-3, n_traj=300,
                             phi_esc=4.0, edges=np.linspace(0, 5, 21)),
        "flat": W.Instance("flat", pot=W.POT_FLAT, V0=3 * (2 * math.pi) ** 2, phi_in=1.0, phi_end=0.0,
                           phi_uv=1.5, dN=1e-3, n_traj=500, edges=np.linspace(0, 8, 41)),
        "flat_levy_bias": W.Instance("levy", pot=W.POT_FLAT, V0=3 * (2 * math.pi) ** 2, phi_in=1.0, phi_end=0.0,
                                     phi_esc=5.0, bias=W.BIAS_NOISE_SCALED, A=-30.0, dN=1e-5, n_traj=500,
                                     edges=np.linspace(0.015, 0.06, 31)),
        "bump": W.with_runs(W.c5(), 64),
        "power": W.Instance("pow", m=0.01, phi_in=5.0, bias=W.BIAS_POWER, A=2e-5, p=3, dN=1e-3, n_traj=400,
                            edges=np.linspace(5.6, 6.0, 41)),
        # run ids across 2^32 (the counter's high word) and up to the last id 2^64 - 1
        "ids_across_2^32": dataclasses.replace(W.with_runs(W.c1(), 300), t_first=(1 << 32) - 150),
        "ids_at_the_top": dataclasses.replace(W.with_runs(W.c1(), 300), t_first=(1 << 64) - 1 - 300),
    }
    for name, inst in cases.items():
        _print_case("edge", name=name, n=inst.n_traj)
        res, dump, _ = fpt.run(inst, SEED, dump_n=max(1, inst.n_traj), block=256, wg_per_cu=2, chunk=1)
        tr = _oracle(inst)
        if inst.n_traj:
            assert_dump_matches(dump, tr)
        assert_histogram_matches(res, O.histogram(tr, inst.dN, inst.edges))
        if name == "all_censored":
            assert res.count[-2] == inst.n_traj and res.total_steps == 7 * inst.n_traj
        if name == "escape":
            assert res.count[-1] > 0


def test_id_range_shards_add_up(fpt):
    """One instance run as two id-range shards (as two launches, or two devices, would run it):
    counts and jackknife counts add exactly, the log-sum-exp sums combine, and each shard is
    the oracle's runs of its ids."""
    full = W.with_runs(W.c2()[0], 3000)
    a = dataclasses.replace(full, n_traj=1234)
    b = dataclasses.replace(full, n_traj=3000 - 1234, t_first=1234)
    rf, _, _ = fpt.run(full, SEED, **CFG)
    ra, da, _ = fpt.run(a, SEED, dump_n=a.n_traj, **CFG)
    rb, db, _ = fpt.run(b, SEED, dump_n=b.n_traj, **CFG)
    assert_dump_matches(db, _oracle(b))
    assert np.array_equal(ra.count + rb.count, rf.count)
    assert np.array_equal(ra.jk_count + rb.jk_count, rf.jk_count)
    assert ra.total_steps + rb.total_steps == rf.total_steps
    both = np.isfinite(ra.lse_w) & np.isfinite(rb.lse_w)
    assert both.any()
    assert np.allclose(np.logaddexp(ra.lse_w, rb.lse_w)[both], rf.lse_w[both], rtol=1e-12, atol=1e-12)


def test_largest_batch(fpt):
    """1024 instances (the batch limit) of 24 runs each, different streams and starting points,
    in one launch: every run accounted for, and sampled instances' runs match the oracle bit for
    bit."""
    insts = [dataclasses.replace(W.with_runs(W.c1(), 24), stream=i, phi_in=5.0 + 0.0005 * (i % 97),
                                 edges=np.linspace(5.6, 6.0, 11)) for i in range(1024)]
    _print_case("largest batch", n_inst=len(insts))
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=24, block=256, wg_per_cu=2, chunk=1)
    assert all(int(r.count.sum()) == 24 for r in results)
    for i in (0, 1, 511, 1023):
        assert_dump_matches(dumps[i], _oracle(insts[i]))


def test_single_entry_point_matches_batch(fpt):
    inst = W.with_runs(W.c2()[0], 2000)
    a = fpt.run_single_abi(inst, SEED)
    b, _, _ = fpt.run(inst, SEED, **CFG)
    assert np.array_equal(a.count, b.count)
    assert np.array_equal(a.jk_count, b.jk_count)
    assert a.total_steps == b.total_steps


def test_graph_replays_match_eager(fpt):
    """hipGraph capture of the launch sequence: several replays with eager work and
    synchronisations between them, each identical in counts to the eager run."""
    import torch
    inst = W.with_runs(W.c2()[0], 3000)
    eager, _, _ = fpt.run(inst, SEED, block=256, wg_per_cu=4, chunk=1)
    side = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(side):
            g, _, _ = fpt.run(inst, SEED, block=256, wg_per_cu=4, chunk=1, use_graph=True)
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.array_equal(g.count, eager.count), rep
        assert np.array_equal(g.jk_count, eager.jk_count), rep
        assert g.total_steps == eager.total_steps


def test_full_size_c2_sampled_runs(fpt):
    """C2 at its full size (6 x 1e6 runs) in the benchmark's launch: a sample of runs (every
    65536th id of each instance) is recomputed one by one by the oracle and must match bit for
    bit; the totals obey what holds at any size (every launched run lands in one row, the weight
    average is one within its error)."""
    insts = W.c2()
    stride = 65536
    n_dump = (insts[0].n_traj + stride - 1) // stride
    _print_case("C2 full", stride=stride)
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=n_dump, dump_stride=stride, **CFG)
    for inst, res, dump in zip(insts, results, dumps):
        assert int(res.count.sum()) == inst.n_traj
        tr = O.simulate(to_model(inst), SEED, n_dump, t0=0, stride=stride)
        assert_dump_matches(dump, tr)
        mean_w = math.exp(res.lse_w_all) / inst.n_traj
        ess = math.exp(2 * res.lse_w_all - res.lse_w2_all)
        if res.count[-2] == 0:
            assert abs(mean_w - 1) < 6 / math.sqrt(ess) + 1e-3, (inst.name, mean_w, ess)


def test_c5_top_of_range_bit_exact(fpt):
    """The bump-potential large run at its full size (1e9 runs over A = 0 .. 6, one instance of
    1.43e8 runs per amplitude): the last 4096 ids of the A = 0 and A = 6 instances, addressed
    by run id, in the benchmark's launch shape, every run against the oracle."""
    n_last = 4096
    insts = []
    for inst in (W.c5_multi()[0], W.c5_multi()[6]):
        insts.append(dataclasses.replace(inst, t_first=inst.n_traj - n_last, n_traj=n_last))
    _print_case("C5 top of range", t_first=insts[0].t_first, n=n_last)
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=n_last, dump_stride=1, **CFG)
    for inst, res, dump in zip(insts, results, dumps):
        tr = _oracle(inst)
        assert_dump_matches(dump, tr)
        assert_histogram_matches(res, O.histogram(tr, inst.dN, inst.edges))


def test_autotuned_launch_matches(fpt):
    """The autotuner only picks the launch shape: results equal the fixed-shape run."""
    inst = W.with_runs(W.c2()[1], 4000)
    a, _, _ = fpt.run(inst, SEED)
    b, _, _ = fpt.run(inst, SEED, **CFG)
    assert np.array_equal(a.count, b.count)
    assert np.array_equal(a.jk_count, b.jk_count)
    assert a.total_steps == b.total_steps


def test_mixed_none_and_noise_scaled_batch(fpt):
    """No bias and the noise-scaled bias share one launch (no bias = A 0): each instance's runs
    are bit-identical to the oracle's."""
    insts = [W.with_runs(W.c1(), 1500), W.with_runs(W.c2()[3], 300)]
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=1500, **CFG)
    for inst, res, dump in zip(insts, results, dumps):
        tr = _oracle(inst)
        assert_dump_matches(dump, tr)
        assert_histogram_matches(res, O.histogram(tr, inst.dN, inst.edges))


def test_c3_batch_prefix_bit_exact(fpt):
    """The 64-instance batch (config C3: phi_in, m, A, wall, dN drawn from splitmix64(0)) in one
    persistent launch over the shared longest-first queue: the first 96 runs of every instance
    are compared run by run with the oracle, and their histograms bin by bin."""
    insts = [W.with_runs(i, 96) for i in W.c3()]
    _print_case("C3 prefix batch", n=96)
    results, dumps, _ = fpt.run_batch(insts, SEED, dump_n=96, **CFG)
    for inst, res, dump in zip(insts, results, dumps):
        tr = _oracle(inst)
        assert_dump_matches(dump, tr)
        assert_histogram_matches(res, O.histogram(tr, inst.dN, inst.edges))


def test_c3_full_size_sampled_runs(fpt):
    """Config C3 at its full size (64 x 1e6 runs, lengths from ~1e3 steps to the cap) in one
    launch: sampled runs (every 262144th id) match the oracle bit for bit; every launched run
    is accounted for in exactly one row."""
    import torch
    insts = W.c3()
    stride = 1 << 18
    n_dump = (insts[0].n_traj + stride - 1) // stride
    _print_case("C3 full", stride=stride)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        results, dumps, tm = fpt.run_batch(insts, SEED, dump_n=n_dump, dump_stride=stride, timing=True, **CFG)
    steps = sum(r.total_steps for r in results)
    print(f"C3: {steps:.3e} steps in {tm[0]:.0f} ms -> {steps / tm[0] * 1e3:.3e} steps/s", flush=True)
    for inst, res, dump in zip(insts, results, dumps):
        assert int(res.count.sum()) == inst.n_traj
        tr = O.simulate(to_model(inst), SEED, n_dump, t0=0, stride=stride)
        assert_dump_matches(dump, tr)
