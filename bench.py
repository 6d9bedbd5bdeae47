"""Benchmark: the fixed-bias importance-sampling sweep (six instances, 1e6 runs each) on one GPU.

One step = one pass of the whole hot path over the batch: queue reset,
persistent Euler-Maruyama kernel with importance weights, first passage and
per-workgroup log-sum-exp histograms, merge and estimators, result copy-out.

Workload (configuration "C2"): quadratic V = m^2 phi^2/2, bias B = A sqrt(V/3)/(2 pi) with
A in {1, 2, 4}; drift-dominated m = 0.01, phi_in = 10, no wall; diffusion-dominated m = 1,
phi_in = 6, reflecting wall at 8; dN = 1e-3; 1e6 runs per instance; 200 log-spaced bins.

Prints one JSON line.  value = weighted trajectory-steps per second (sum over every run,
censored included, of its step count, divided by the wall time of the step).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz = 7.86e13
# lane-ops/s, i.e. the 157.3 TFLOP/s fp32 vector peak divided by 2 flops per FMA.  In the step
# kernel every VALU instruction kind it uses issues at that rate: its counters show 70.4 VALU
# instructions per wave-step in 171.4 SIMD-cycles, 29.5 of them fma, 32x32 integer multiplies,
# f64 adds and conversions; at two issue slots for those the wave-step would need 199.8 cycles.
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9
# MI355X binary32 vector peak (packed FMA on every lane), for the FLOP reading of the roofline
PEAK_FP32_FLOPS = 157.3e12
# Binary32 flops per trajectory-step: the algorithmic count of the step's arithmetic (about 35
# for half a Box-Muller pair with its log, sqrt and sincos, 13 for the step, 2 for the uniforms)
# and the count of the compiled kernel from its counters (SQ_INSTS_VALU_FLOPS_FP32 per
# trajectory-step), profiles/fpt_step_kernel_c2_sweep_valu_counters.md
FLOP_PER_STEP_ALGORITHMIC = 50.0
FLOP_PER_STEP_COUNTED = 61.7
# Algorithmic lane operations per trajectory-step of the quadratic, noise-scaled path: the VALU
# instructions of the compiled four-step pass of fpt_step_kernel<0,1,false>, loop control and
# retirement excluded (fma, three-input xor and 32x32->64 multiply one each):
#   Philox 40/4 (20 v_mad_u64_u32 and 20 v_bitop3_b32: ten rounds per 4 steps)
#   radius uniforms and the two Box-Muller pairs 119/4 (own log, sqrt and sincos)
#   the step 114/4 (reciprocal, drift/noise/bias, phi update, weight, wall, k, stopping tests)
OPS_PER_STEP = (40 + 119 + 114) / 4
# HBM bytes per launch of the step kernel on this workload: rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1
# (factors read off a plain 1 GiB copy, `--copy-calibration`), summaries under profiles/.
# Reset to None whenever the step kernel changes until the counters are taken again.
# Seed of the learned-vs-fixed evaluation runs: apart from every training seed (train_seed + 100 s
# + round) and every selection pilot seed (those + 2^30 + c), so the evaluated proposal does not
# depend on the evaluation's noise.
EVAL_SEED = 99991
TRAFFIC = (582272.875 * 1.99994 + 2624860.21875 * 1.0) * 1024


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n-traj", type=int, default=1_000_000)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    p.add_argument("--no-learned", action="store_true",
                   help="skip the learned-vs-fixed comparison in the main line (it adds about 40 s)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    # fixed launch shape (a sweep on MI355X put every shape from 64x16 to 1024x1 within 2%);
    # --autotune lets the library's measured autotuner pick it instead
    p.add_argument("--block", type=int, default=512)
    p.add_argument("--wg-per-cu", type=int, default=2)
    p.add_argument("--chunk", type=int, default=1)
    p.add_argument("--autotune", action="store_true")
    p.add_argument("--learned", action="store_true",
                   help="learned proposal vs the fixed-bias scan at equal error in the far-tail window")
    p.add_argument("--n-eval", type=int, default=10_000_000)
    p.add_argument("--n-sample", type=int, default=200_000)
    p.add_argument("--rounds", type=int, default=3)
    p.add_argument("--train-steps", type=int, default=40)
    p.add_argument("--max-paths", type=int, default=8000)
    p.add_argument("--lr", type=float, default=3e-3)
    p.add_argument("--target", type=float, default=196.0)
    p.add_argument("--eval-every", type=int, default=16,
                   help="steps the learned bias is held for (1, 4, 8 or 16); training records use the same groups")
    p.add_argument("--objective", type=int, default=1, help="0: log M2, 1: cross entropy")
    p.add_argument("--objective-compare", type=int, default=1,
                   help="also train with objective 0 (log M2) on the same seeds and budget and report it")
    p.add_argument("--fixed-budget-s", type=float, default=30.0,
                   help="GPU-seconds the best fixed bias runs for in the measured equal-error comparison (0: skip)")
    p.add_argument("--temper", type=float, default=0.5, help="w_0^temper in the path weights")
    p.add_argument("--train-seed", type=int, default=1)
    p.add_argument("--final-rounds", type=int, default=6, help="rounds of the final stage of the far-tail training (the C5 proposal uses --rounds)")
    p.add_argument("--select-pilot", type=int, default=200_000,
                   help="pilot runs scoring the final stage's candidate networks (0: keep the last)")
    p.add_argument("--eval-dn", type=str, default="",
                   help="comma-separated further step sizes at which the trained network is evaluated too "
                        "(the window estimate against the time step; --learned only)")
    p.add_argument("--stride", type=int, default=4,
                   help="record stride of the far-tail training sums (each kept record counts stride times)")
    p.add_argument("--curriculum", type=str, default="60,100,140",
                   help="comma-separated window centres trained in turn before the target")
    p.add_argument("--c5", action="store_true",
                   help="the large bump-potential run as one multi-bias batch, combined bin by bin")
    p.add_argument("--c5-total", type=int, default=1_000_000_000)
    p.add_argument("--c5-launches", type=int, default=7, help="launches the amplitudes are split over")
    p.add_argument("--c5-save", type=str, default="", help="write the per-amplitude result tables to this .npz")
    p.add_argument("--c5-analyse", type=str, default="",
                   help="only analyse result tables saved by --c5-save (CPU: the combination and the checks)")
    p.add_argument("--c5-learned", type=int, default=100_000_000,
                   help="runs of a learned proposal added to the combination (0: fixed amplitudes only)")
    p.add_argument("--c5-target", type=float, default=24.5, help="window centre N* of the learned proposal")
    p.add_argument("--c5-curriculum", type=str, default="17,18,19,20,21,22,23,24",
                   help="window centres the learned proposal is trained through before N*")
    p.add_argument("--c5-stage-runs", type=int, default=20_000_000,
                   help="runs of each curriculum stage's network from --c5-stage-from on (0: none)")
    p.add_argument("--c5-stage-from", type=float, default=18.0,
                   help="first curriculum centre whose network is run beside the final one")
    p.add_argument("--mlp-wg", type=int, default=3,
                   help="256-lane workgroups per CU of the learned-bias sampler (waves per SIMD)")
    p.add_argument("--mlp-sampler", action="store_true",
                   help="time the learned-bias sampler alone (untrained network, r ~ 1) on the diffusion case")
    p.add_argument("--c3", action="store_true",
                   help="the 64-instance batched sweep in one graph-replayed launch with the autotuned shape")
    p.add_argument("--no-c3", action="store_true",
                   help="skip the batched sweep in the main line (it adds about 40 s)")
    p.add_argument("--c3-steps", type=int, default=2, help="timed passes of the batched sweep in the main line")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only copy 1 GiB device-to-device 3 times (scale reference for HBM byte counters)")
    return p.parse_args()


def copy_calibration():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the step kernel."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 3}))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(insts, target_s, gpu_steps=None):
    """The oracle (binary32 mirror, all host threads) on a bounded sample of the same runs, and
    on one thread over the first runs of the same sample (a few seconds).  With gpu_steps (the
    GPU pass's trajectory-steps per instance) the rate is weighted by the GPU's step mix: the
    oracle's time for that pass is sum_i steps_i / rate_i, each instance at its own sampled rate."""
    import oracle as O
    to_model = O.Model.from_instance
    # per instance, double the prefix of ids until one run of the oracle takes at least a third
    # of the instance's share of target_s, and keep that run's measurement
    steps = 0
    elapsed = 0.0
    threads = 0
    share = target_s / len(insts)
    sample = []
    rates = []
    for inst in insts:
        n = 256
        while True:
            t0 = time.perf_counter()
            tr = O.simulate(to_model(inst), 0, n)
            dt = time.perf_counter() - t0
            if dt >= share / 3 or n >= inst.n_traj:
                break
            n = int(min(inst.n_traj, n * min(8.0, max(2.0, share / max(dt, 1e-3)))))
        elapsed += dt
        steps += int(tr.k.sum())
        threads = tr.threads
        rates.append(int(tr.k.sum()) / dt)
        sample.append(f"{inst.name}:{n}")
    # one thread: the first ids of the first drift-dominated instance (about 3 s)
    one = insts[0]
    n1, s1, e1 = 64, 0, 0.0
    while True:
        t0 = time.perf_counter()
        tr = O.simulate(to_model(one), 0, n1, threads=1)
        e1 = time.perf_counter() - t0
        s1 = int(tr.k.sum())
        if e1 >= 1.5 or n1 >= one.n_traj:
            break
        n1 = int(min(one.n_traj, n1 * min(8.0, max(2.0, 3.0 / max(e1, 1e-3)))))
    value = steps / elapsed
    weighting = "time share: each instance sampled for about the same time"
    if gpu_steps is not None and sum(gpu_steps) > 0:
        value = sum(gpu_steps) / sum(g / r for g, r in zip(gpu_steps, rates))
        weighting = "the GPU pass's step mix: sum of its steps over sum of steps_i / rate_i"
    return {"value": value, "unit": "traj-steps/s", "cores": threads, "kind": "oracle",
            "weighting": weighting, "rate_time_share": steps / elapsed,
            "rate_per_instance": {inst.name: r for inst, r in zip(insts, rates)},
            "cpu_model": cpu_model(), "single_core": s1 / e1,
            "single_core_sample": f"{one.name}: first {n1} ids, {s1} steps in {e1:.2f} s on one thread",
            "sample": "first ids of each instance: " + ", ".join(sample) + f"; {steps} steps in {elapsed:.1f} s"}


def window_stats(res, lo, hi):
    """Kish ESS and relative errors of the bins inside (lo, hi], with the jackknife relative
    errors (Sec. 2.1) beside the Kish ones as a cross-check."""
    import numpy as np
    e = res.edges
    j = [i for i in range(len(e) - 1) if e[i] >= lo - 1e-9 and e[i + 1] <= hi + 1e-9]
    lw, lw2 = res.lse_w[j], res.lse_w2[j]
    ess = np.exp(2 * lw - lw2)
    rel = np.sqrt(np.maximum(np.exp(lw2 - 2 * lw) - 1.0 / res.n_traj, 0.0))
    return {"bins": len(j), "ess": float(np.nansum(ess)), "median_rel_err": float(np.nanmedian(rel)),
            "median_rel_err_jk": float(np.nanmedian(res.rel_err_jk[j])),
            "log10_p": float(np.log10(np.nanmean(np.exp(res.log_p[j])))), "count": int(res.count[j].sum())}


def c5_run(args):
    """Bump potential V = m^2 phi^2/2 [1 + a exp(-(phi - phi0)^2/(2 w^2))], m = 0.05, a = 0.02,
    phi0 = 4, w = 0.1, phi_in = 8, wall at 12, dN = 1e-4, 500 bins: the runs split over noise-scaled
    amplitudes A = 0..6 (one noise stream each), run in persistent launches, plus a learned proposal
    aimed beyond their reach (args.c5_learned runs), all combined bin by bin (pyfpt_combine), the
    fixed amplitudes serving as the fallback wherever the learned proposal has no trusted
    estimate."""
    import numpy as np
    import torch
    import paper_2206_11234_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    insts = W.c5_multi(n_total=args.c5_total)
    F.run_batch([W.with_runs(i, 2000) for i in insts], 0, block=512, wg_per_cu=2, chunk=1)   # warm-up
    torch.cuda.synchronize()
    # the amplitudes in args.c5_launches consecutive groups, one persistent launch each (a launch
    # per group keeps each under a minute at 1e9 runs); the results do not depend on the grouping
    groups = [g for g in np.array_split(np.arange(len(insts)), max(1, args.c5_launches)) if len(g)]
    results, kern_ms = [], 0.0
    t0 = time.perf_counter()
    for g in groups:
        r, _, tm = F.run_batch([insts[i] for i in g], 0, block=512, wg_per_cu=2, chunk=1, timing=True)
        results += r
        kern_ms += tm[0]
        print(f"[c5] amplitudes {[insts[i].A for i in g]}: {tm[0] / 1e3:.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    steps = sum(r.total_steps for r in results)
    for inst_, r in zip(insts, results):
        r.amplitude = inst_.A
        r.label = f"A{inst_.A:g}"
    learned = None
    if args.c5_learned > 0:
        learned = c5_learned_run(args, insts[0], results)
        results.append(learned.pop("result"))
        results[-1].label = f"learned {args.c5_target:g}"
        for st, r in zip(learned["stages"], learned["stage_results"]):
            r.label = f"learned {st['centre']:g}"
        results += learned.pop("stage_results")
    # lognormal estimates gated bin by bin (the drift-dominated regime of Sec. 2.4), the naive
    # estimate where a bin fails its gate; with 500 bins and 1e8 runs per amplitude a whole-result
    # gate fails by chance
    if args.c5_save:
        np.savez_compressed(args.c5_save, **{f"counts_{i}": r.counts for i, r in enumerate(results)},
                            **{f"values_{i}": r.values for i, r in enumerate(results)},
                            edges=results[0].edges, amplitudes=np.array([i.A for i in insts]),
                            labels=np.array([r.label for r in results]))
    analysis = c5_analysis(results, n_fixed=len(insts))
    out = {"workload": "C5 bump potential, multi-bias A = 0..6" + (" + learned proposal" if learned else "") +
                       ", dN = 1e-4, 500 bins",
           "runs": sum(r.n_traj for r in results), "steps": steps, "wall_s": wall, "kernel_ms": kern_ms, "launches": len(groups),
           "traj_steps_per_s": steps / wall,
           "gate_passed": [bool(r.lognormal_accepted()) for r in results]}
    out.update(analysis)
    if learned is not None:
        out["learned"] = learned
    print(json.dumps(out), flush=True)


def c5_analysis(results, n_fixed):
    """The large run's results combined bin by bin, and the checks of what the combination rests on.

    - coverage and reach: estimator 3 (lognormal where a bin passes its gate, else the trusted
      naive estimate) and the same with the no-extrapolation rule (a lognormal bin also needs
      n_j >= exp(s_j^2/2)), over the fixed amplitudes alone and over every result;
    - the learned proposals against each other: each one's naive estimates (n_j > 400 and
      n_j > exp(s_j^2), no lognormal model) against the combination of the others, bin by bin,
      with the z of the jackknife errors mapped through Student's t (15 degrees of freedom);
    - the direct-sampling amplitudes' trusted naive estimates against the learned combination;
    - each fixed amplitude's lognormal estimate minus the learned naive combination, in decades."""
    import numpy as np
    from scipy import stats
    import paper_2206_11234_amd as F

    L10 = math.log(10.0)
    e = results[0].edges
    B = len(e) - 1
    centre = 0.5 * (e[1:] + e[:-1])

    def spans(mask):
        idx = np.nonzero(mask)[0]
        out = []
        for j in idx:
            if out and j <= out[-1][1] + 2:
                out[-1][1] = j
            else:
                out.append([j, j])
        return [[round(float(e[a]), 3), round(float(e[b + 1]), 3)] for a, b in out]

    def summary(res, est):
        lp, el, nu = F.combine(res, est)
        ok = nu > 0
        good = ok & (el < 0.5 * L10)
        deep = int(np.nonzero(good)[0].max()) if good.any() else -1
        return {"combined_bins": int(ok.sum()), "bins_within_half_decade": int(good.sum()),
                "reach_log10_p": float(lp[deep] / L10) if deep >= 0 else None,
                "reach_err_log10": float(el[deep] / L10) if deep >= 0 else None,
                "reach_N": float(centre[deep]) if deep >= 0 else None, "covered_N": spans(ok)}

    def zstats(z):
        z = np.asarray(z, np.float64)
        if z.size == 0:
            return None
        zn = stats.norm.ppf(np.clip(stats.t.cdf(z, 15), 1e-300, 1.0 - 1e-16))
        return {"comparisons": int(z.size), "beyond_3sigma": int(np.sum(np.abs(zn) > 3.0)),
                "rms_z": float(np.sqrt(np.mean(zn ** 2))),
                "chi2_p": float(stats.chi2.sf(float(np.sum(zn ** 2)), z.size))}

    NX = F.COMBINE_NO_EXTRAPOLATION
    out = {}
    out.update(summary(results, 3))
    out["no_extrapolation"] = summary(results, 3 + NX)
    out["fixed_only"] = summary(results[:n_fixed], 3)
    out["fixed_only_no_extrapolation"] = summary(results[:n_fixed], 3 + NX)
    lp, el, nu = F.combine(results, 3)
    below = np.nonzero((nu > 0) & (lp < -40 * L10))[0]
    out["p_1e-40_N"] = float(centre[below[0]]) if below.size else None
    learned = list(range(n_fixed, len(results)))
    if len(learned) >= 2:
        z = []
        for i in learned:
            lo, eo, no = F.combine([results[k] for k in learned if k != i], 0)
            li, ei, ni = F.combine([results[i]], 0)
            m = (ni > 0) & (no > 0)
            z += list((li[m] - lo[m]) / np.hypot(ei[m], eo[m]))
        out["learned_leave_one_out"] = zstats(z)
    if learned:
        ll, le, ln = F.combine([results[i] for i in learned], 0)
        out["learned_naive_covered_N"] = spans(ln > 0)
        direct, offsets = {}, {}
        for i in range(n_fixed):
            fl, fe, fn = F.combine([results[i]], 0)
            m = (fn > 0) & (ln > 0)
            st = zstats((fl[m] - ll[m]) / np.hypot(fe[m], le[m])) if m.any() else None
            if st is not None:
                direct[f"A{results[i].amplitude:g}"] = st
            n = results[i].count[:B]
            m = (n >= 400) & (ln > 0) & np.isfinite(results[i].log_p_ln[:B])
            if m.any():
                d = (results[i].log_p_ln[:B][m] - ll[m]) / L10
                offsets[f"A{results[i].amplitude:g}"] = {"bins": int(m.sum()), "median": float(np.median(d)),
                                                         "min": float(d.min()), "max": float(d.max()),
                                                         "N": [round(float(centre[m].min()), 2), round(float(centre[m].max()), 2)]}
        out["fixed_naive_vs_learned"] = direct
        out["fixed_lognormal_minus_learned_decades"] = offsets

    def val(c, j):
        lp_, el_, nu_ = c
        return [round(float(lp_[j] / L10), 3), round(float(el_[j] / L10), 3)] if nu_[j] > 0 else None

    # every 25th bin, combined: [log10 P, error in decades] or null where nothing contributes
    combos = {"all": F.combine(results, 3), "all_no_extrapolation": F.combine(results, 3 + NX),
              "fixed": F.combine(results[:n_fixed], 3), "fixed_no_extrapolation": F.combine(results[:n_fixed], 3 + NX)}
    out["selected_bins"] = [dict(bin=j, N=round(float(centre[j]), 3), **{k: val(c, j) for k, c in combos.items()})
                            for j in list(range(0, B, 25)) + [B - 1]]
    # each result's own estimates where it has at least 400 runs, at a few bins of the far tail
    rows = []
    for Nq in (18.85, 19.97, 21.16, 22.42, 23.49, 24.04):
        j = int(np.argmin(np.abs(centre - Nq)))
        for i, r in enumerate(results):
            n = int(r.count[j])
            if n < 400:
                continue
            s2 = float(r.m2_lnw[j]) * n / (n - 1)
            sd = math.sqrt(max(s2, 0.0))
            rows.append({"N": round(float(centre[j]), 3), "result": getattr(r, "label", str(i)), "runs": n,
                         "naive": round(float(r.log_p[j] / L10), 2), "lognormal": round(float(r.log_p_ln[j] / L10), 2),
                         "s_lnw": round(sd, 2), "n_ge_exp_s2_half": bool(n >= math.exp(min(s2 / 2, 700.0)))})
    out["per_result"] = rows
    return out


def c5_analyse_saved(path):
    """--c5-analyse: the analysis of result tables written by --c5-save (no GPU needed)."""
    import numpy as np
    import paper_2206_11234_amd as F
    from paper_2206_11234_amd import api

    z = np.load(path)
    edges = z["edges"]
    n_res = len([k for k in z.files if k.startswith("counts_")])
    lay = F.layout(len(edges) - 1, 16)
    res = [api.Result(edges=edges, n_sub=16, counts=z[f"counts_{i}"], values=z[f"values_{i}"], lay=lay)
           for i in range(n_res)]
    amps = list(z["amplitudes"])
    labels = list(z["labels"]) if "labels" in z.files else []
    for i, r in enumerate(res):
        r.amplitude = float(amps[i]) if i < len(amps) else float("nan")
        r.label = str(labels[i]) if i < len(labels) else (f"A{amps[i]:g}" if i < len(amps) else f"learned #{i - len(amps)}")
    print(json.dumps(c5_analysis(res, n_fixed=len(amps))), flush=True)


def c5_learned_run(args, base, fixed_results):
    """The learned proposal on the bump potential: a network started at r = 2 is trained through
    windows of half-width 0.3 in N centred at the curriculum points and then N* (cross entropy,
    tempered path weights), then run with args.c5_learned runs on its own noise stream.  Returns
    its result and, over the window bins around N*, its Kish ESS per 1e6 runs beside each fixed
    amplitude's."""
    import dataclasses
    import numpy as np
    import torch
    import paper_2206_11234_amd as F
    import workloads as W

    target = args.c5_target
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    v[:4480] = np.random.default_rng(0).normal(0.0, 1e-2, 4480)
    v[4480] = 2.0
    p0 = W.MlpParams(W.bf16_round(v), in_mean=(8.0, target, target), in_inv_scale=(0.25, 0.1, 0.1),
                     out_scale=1.0, eval_every=args.eval_every)
    inst0 = dataclasses.replace(base, name="C5_learned", bias=W.BIAS_MLP, A=0.0, mlp=p0, target_N=target,
                                stream=len(fixed_results), n_traj=args.c5_learned)
    theta = p0.values_f32()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rounds = []
    stage_thetas = []
    stages = [float(c) for c in args.c5_curriculum.split(",") if c] + [target]
    for si, centre in enumerate(stages):
        theta, _, rep = F.train_proposal(dataclasses.replace(inst0, target_N=centre), args.train_seed + 100 * si, theta,
                                         window=(centre - 0.3, centre + 0.3), n_sample=args.n_sample,
                                         rounds=args.rounds, steps=args.train_steps, max_paths=args.max_paths,
                                         lr=args.lr, objective=1, temper=args.temper,
                                         select=args.select_pilot if si == len(stages) - 1 else 0)
        for r in rep:
            r["centre"] = centre
            print(f"[c5] train round: {json.dumps(r)}", file=sys.stderr, flush=True)
        rounds += rep
        if si < len(stages) - 1:
            stage_thetas.append((centre, theta.copy()))
    train_s = time.perf_counter() - t0
    inst = dataclasses.replace(inst0, mlp=dataclasses.replace(p0, values=theta))
    res, _, tm = F.run(inst, 0, block=256, wg_per_cu=args.mlp_wg, chunk=1, timing=True)
    print(f"[c5] learned: {tm[0] / 1e3:.1f} s", file=sys.stderr, flush=True)
    # the curriculum's networks aimed between the fixed amplitudes' trusted reach and N*, each on
    # a noise stream of its own: their ln w spreads little in their windows, so those bins pass the
    # no-extrapolation rule of the combination
    stage_results, stage_info = [], []
    if args.c5_stage_runs > 0:
        for k, (centre, th) in enumerate([c for c in stage_thetas if c[0] >= args.c5_stage_from]):
            si = dataclasses.replace(inst0, name=f"C5_learned_{centre:g}", target_N=centre,
                                     mlp=dataclasses.replace(p0, values=th), n_traj=args.c5_stage_runs,
                                     stream=len(fixed_results) + 1 + k)
            r, _, tms = F.run(si, 0, block=256, wg_per_cu=args.mlp_wg, chunk=1, timing=True)
            stage_results.append(r)
            stage_info.append({"centre": centre, "runs": r.n_traj, "steps": r.total_steps, "kernel_ms": tms[0]})
            print(f"[c5] stage network {centre:g}: {tms[0] / 1e3:.1f} s", file=sys.stderr, flush=True)
    e = res.edges
    j = [i for i in range(len(e) - 1) if e[i] >= target - 0.3 and e[i + 1] <= target + 0.3]

    def ess_per_1e6(r):
        return float(np.nansum(np.exp(2 * r.lse_w[j] - r.lse_w2[j]))) / r.n_traj * 1e6

    return {"result": res, "stage_results": stage_results, "stages": stage_info,
            "runs": res.n_traj, "steps": res.total_steps, "kernel_ms": tm[0], "train_s": train_s,
            "window": [target - 0.3, target + 0.3], "window_bins": len(j),
            "window_runs": int(res.count[j].sum()), "ess_per_1e6_runs": ess_per_1e6(res),
            "fixed_ess_per_1e6_runs": {f"A{a.A:g}": ess_per_1e6(r) for a, r in zip(W.c5_multi(), fixed_results)},
            "train_rounds": rounds}


def learned_gain(args):
    """GPU-seconds to a 1% median relative error over the far-tail window, learned proposal vs
    the fixed noise-scaled bias scan, on the diffusion-dominated quadratic case (m = 1,
    phi_in = 6, wall at 8, dN = 1e-3).  The learned network starts at r = 1 (small random
    weights) and is trained with the tempered cross-entropy objective through a curriculum of
    windows, on runs of its own proposal (every args.stride-th record of each run kept, with
    weight args.stride), with args.final_rounds rounds at the target window;
    that stage's candidate networks are scored on pilots of args.select_pilot runs.  Both
    proposals are evaluated on EVAL_SEED, which no training round or pilot uses."""
    import dataclasses
    import numpy as np
    import torch
    import paper_2206_11234_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    lo, hi = args.target - 6.0, args.target + 6.0
    edges = np.linspace(0.0, 400.0, 201)
    base = dataclasses.replace(W.c2(args.n_eval)[3], edges=edges)
    eps = 0.01
    out = {"workload": f"far-tail window ({lo:g}, {hi:g}] of the diffusion case, P ~ 1e-30", "fixed": [],
           "n_eval": args.n_eval, "eval_every": args.eval_every}

    results = {}

    def evaluate(inst, label, **kw):
        F.run(dataclasses.replace(inst, n_traj=min(inst.n_traj, 20000)), EVAL_SEED, **kw)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _, tm = F.run(inst, EVAL_SEED, timing=True, **kw)
        results[label] = (res, tm[0])
        wall = time.perf_counter() - t0
        st = window_stats(res, lo, hi)
        st.update(label=label, kernel_ms=tm[0], wall_s=wall, steps=res.total_steps,
                  steps_per_s=res.total_steps / (tm[0] / 1e3))
        for key, rk in (("gpu_s_to_1pct", "median_rel_err"), ("gpu_s_to_1pct_jk", "median_rel_err_jk")):
            rel = st[rk]
            st[key] = (tm[0] / 1e3) * (rel / eps) ** 2 if np.isfinite(rel) and rel > 0 else None
        print(f"[learned] {label}: {json.dumps(st)}", file=sys.stderr, flush=True)
        return st

    for A in (0.6, 0.8, 1.0, 1.2, 1.4):
        out["fixed"].append(evaluate(dataclasses.replace(base, A=A), f"fixed A={A}", block=512, wg_per_cu=2, chunk=1))
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    v[:4480] = np.random.default_rng(0).normal(0.0, 1e-2, 4480)
    v[4480] = 1.0
    p0 = W.MlpParams(W.bf16_round(v), in_mean=(5.0, args.target, args.target), in_inv_scale=(0.4, 0.005, 0.01),
                     out_scale=1.0, eval_every=args.eval_every)
    inst0 = W.c4_instance(p0, n_traj=args.n_eval, target_N=args.target, stream=base.stream)
    inst0 = dataclasses.replace(inst0, edges=edges)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stages = [float(c) for c in args.curriculum.split(",") if c] + [args.target]
    theta = p0.values_f32()
    rep = []
    for si, centre in enumerate(stages):
        st_inst = dataclasses.replace(inst0, target_N=centre)
        theta, bf, r_stage = F.train_proposal(st_inst, args.train_seed + 100 * si, theta,
                                              window=(centre - 6.0, centre + 6.0), n_sample=args.n_sample,
                                              rounds=(args.final_rounds or args.rounds) if si == len(stages) - 1
                                              else args.rounds, steps=args.train_steps, max_paths=args.max_paths,
                                              lr=args.lr, objective=args.objective, temper=args.temper,
                                              stride=args.stride if args.objective == 1 else 1,
                                              select=args.select_pilot if si == len(stages) - 1 else 0)
        for r in r_stage:
            r["centre"] = centre
            print(f"[learned] train round: {json.dumps(r)}", file=sys.stderr, flush=True)
        rep += r_stage
    train_s = time.perf_counter() - t0
    p1 = W.MlpParams(theta, in_mean=p0.in_mean, in_inv_scale=p0.in_inv_scale, out_scale=1.0,
                     eval_every=args.eval_every)
    learned = evaluate(dataclasses.replace(inst0, mlp=p1), "learned", block=256, wg_per_cu=args.mlp_wg, chunk=1)
    # the same curriculum, seeds and budget with the second-moment objective (0: log M2, the
    # weight-variance criterion), whose path weights depend on theta, so every record is kept
    obj0 = None
    if args.objective_compare and args.objective != 0:
        t0 = time.perf_counter()
        theta0 = p0.values_f32()
        rep0 = []
        for si, centre in enumerate(stages):
            theta0, _, r_stage = F.train_proposal(dataclasses.replace(inst0, target_N=centre), args.train_seed + 100 * si,
                                                  theta0, window=(centre - 6.0, centre + 6.0), n_sample=args.n_sample,
                                                  rounds=(args.final_rounds or args.rounds) if si == len(stages) - 1
                                                  else args.rounds, steps=args.train_steps, max_paths=args.max_paths,
                                                  lr=args.lr, objective=0, temper=args.temper, stride=1,
                                                  select=args.select_pilot if si == len(stages) - 1 else 0)
            rep0 += r_stage
        train0_s = time.perf_counter() - t0
        p_obj0 = W.MlpParams(theta0, in_mean=p0.in_mean, in_inv_scale=p0.in_inv_scale, out_scale=1.0,
                             eval_every=args.eval_every)
        obj0 = evaluate(dataclasses.replace(inst0, mlp=p_obj0), "learned objective 0", block=256,
                        wg_per_cu=args.mlp_wg, chunk=1)
        obj0["train_s"] = train0_s
    # a fixed bias is a candidate only where its window estimate is trusted by the paper's
    # n_j > 400 criterion (Sec. 2.1); with fewer runs its error estimate is itself unreliable
    cands = [f for f in out["fixed"] if f["gpu_s_to_1pct"] and f["count"] > 400]
    best = min(cands, key=lambda f: f["gpu_s_to_1pct"]) if cands else None
    lg = learned["gpu_s_to_1pct"]
    # the same network at smaller time steps: the window estimate's dependence on dN
    out["learned_dn"] = []
    for dn in [float(x) for x in args.eval_dn.split(",") if x]:
        k_max = int(min(1 << 22, 64 * math.ceil(W.MU_SIGMA["C2_diff_T"][0] / dn)))
        st = evaluate(dataclasses.replace(inst0, mlp=p1, dN=dn, k_max=k_max), f"learned dN={dn:g}",
                      block=256, wg_per_cu=args.mlp_wg, chunk=1)
        st["dN"] = dn
        out["learned_dn"].append(st)
    lj = learned["gpu_s_to_1pct_jk"]
    # measured, not extrapolated: the best fixed bias runs on (id-range shards of n_eval runs)
    # for args.fixed_budget_s GPU-seconds; the error it reaches is the target eps, and each
    # learned proposal runs in shards of one run per lane until it reaches the same eps.  A shard
    # lasts as long as its longest run, so the learned side is latency-bound: it runs one wave per
    # SIMD (each run gets the SIMD to itself), and the gain is still a lower bound
    measured = None
    if best is not None and args.fixed_budget_s > 0:
        A_best = float(best["label"].split("=")[1])
        fx = run_until(F, dataclasses.replace(base, A=A_best), lo, hi, 0.0, args.n_eval, args.fixed_budget_s,
                       first=results[best["label"]], block=512, wg_per_cu=2, chunk=1)
        eps_m = fx["median_rel_err_jk"]
        measured = {"eps": eps_m, "fixed": dict(fx, label=best["label"])}
        for label, params in (("learned", p1),) + ((("learned objective 0", p_obj0),) if obj0 else ()):
            lanes = F.device_cus() * 256
            lm = run_until(F, dataclasses.replace(inst0, mlp=params), lo, hi, eps_m, lanes, 60.0,
                           block=256, wg_per_cu=1, chunk=1)
            lm["gain"] = fx["gpu_s"] / lm["gpu_s"] if lm["reached"] else None
            measured[label] = lm
            print(f"[learned] measured to eps {eps_m:.3f}: {label} {json.dumps(lm)}", file=sys.stderr, flush=True)
        print(f"[learned] measured fixed: {json.dumps(measured['fixed'])}", file=sys.stderr, flush=True)
    out.update(learned=learned, train_s=train_s, train_rounds=rep, best_fixed=best["label"] if best else None,
               objective_0=obj0, measured=measured,
               gain=(best["gpu_s_to_1pct"] / lg) if (best and lg) else None,
               gain_with_training=(best["gpu_s_to_1pct"] / (lg + train_s)) if (best and lg) else None,
               gain_jk=(best["gpu_s_to_1pct_jk"] / lj) if (best and lj and best["gpu_s_to_1pct_jk"]) else None)
    return out


def run_until(F, inst, lo, hi, eps, shard, budget_s, first=None, **kw):
    """Runs `inst` in id-range shards of `shard` runs (t_first = 0, shard, 2 shard, ...) until the
    median jackknife relative error over the window bins (lo, hi] of the merged shards is at most
    eps, or the kernel time reaches budget_s.  The shards' tables merge exactly (counts and
    jackknife counts add, log-sums combine by logaddexp; a run's subset is its id mod 16).
    `first`: an already computed result of the first shard (with its kernel ms).  Returns the
    kernel GPU-seconds, runs, and the error reached (jackknife and Kish)."""
    import dataclasses
    import numpy as np
    gpu_s, runs, i = 0.0, 0, 0
    acc = None
    while True:
        if first is not None and i == 0:
            res, ms = first
        else:
            res, _, tm = F.run(dataclasses.replace(inst, n_traj=shard, t_first=i * shard), EVAL_SEED, timing=True, **kw)
            ms = tm[0]
        gpu_s += ms / 1e3
        runs += shard
        i += 1
        e = res.edges
        j = np.array([b for b in range(len(e) - 1) if e[b] >= lo - 1e-9 and e[b + 1] <= hi + 1e-9])
        part = (res.jk_lse_w[:, j], res.jk_count[:, j].astype(np.float64), res.lse_w2[j])
        if acc is None:
            acc = [part[0].copy(), part[1].copy(), part[2].copy()]
        else:
            acc[0] = np.logaddexp(acc[0], part[0])
            acc[1] += part[1]
            acc[2] = np.logaddexp(acc[2], part[2])
        jk, jc, l2 = acc
        J = jk.shape[0]
        l = np.logaddexp.reduce(jk, axis=0)
        n_sub = np.array([runs // J + (1 if s < runs % J else 0) for s in range(J)], np.float64)
        with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
            ratio = np.exp(jk - l[None, :]) * (runs / n_sub[:, None])
            err_jk = np.std(ratio, axis=0, ddof=1) / np.sqrt(J)
            err_kish = np.sqrt(np.maximum(np.exp(l2 - 2 * l) - 1.0 / runs, 0.0))
        err_jk = np.where(jc.sum(axis=0) > 0, err_jk, np.inf)
        med_jk, med_kish = float(np.median(err_jk)), float(np.median(np.where(np.isfinite(err_jk), err_kish, np.inf)))
        if med_jk <= eps or gpu_s >= budget_s:
            return {"gpu_s": gpu_s, "runs": runs, "median_rel_err_jk": med_jk, "median_rel_err_kish": med_kish,
                    "reached": bool(med_jk <= eps)}


def learned_summary(full):
    """The learned-vs-fixed part of the headline metric, for the main bench line."""
    best = next((f for f in full["fixed"] if f["label"] == full["best_fixed"]), None)
    L = full["learned"]
    return {"workload": full["workload"], "eval_runs": full["n_eval"],
            "learned_gpu_s_to_1pct": L["gpu_s_to_1pct"], "learned_log10_p": L["log10_p"],
            "learned_median_rel_err": L["median_rel_err"], "learned_ess": L["ess"],
            "best_fixed": full["best_fixed"], "best_fixed_gpu_s_to_1pct": best["gpu_s_to_1pct"] if best else None,
            "train_s": full["train_s"], "gain": full["gain"], "gain_with_training": full["gain_with_training"],
            "gain_jackknife": full.get("gain_jk"),
            "note": "GPU-s to 1% median relative error over the window = kernel time x (error / 0.01)^2, "
                    "errors from the Kish ESS (gain_jackknife: the same with jackknife errors); "
                    "best fixed = lowest among the fixed amplitudes with > 400 window runs",
            "objective": "cross entropy (1), tempered",
            # the learned sampler on its evaluation runs: fpt_step_mlp1_kernel's rate, and its matrix-core
            # flop (34 MFMA 32x32x16 per 64 trajectories per evaluation) against the dense bf16 peak
            "sampler": {"kernel": "fpt_step_mlp1_kernel", "kernel_ms": L["kernel_ms"],
                        "traj_steps_per_s": L["steps_per_s"], "eval_every": full.get("eval_every"),
                        "mfma_frac_bf16_peak": (L["steps_per_s"] * 34 * 32 * 32 * 16 * 2 / 64 / full["eval_every"]
                                                / 2.5e15) if full.get("eval_every") else None},
            "objective_0": ({k: full["objective_0"][k] for k in ("ess", "median_rel_err", "median_rel_err_jk", "log10_p",
                                                                 "gpu_s_to_1pct", "train_s")}
                            if full.get("objective_0") else None),
            "measured": full.get("measured")}


def mlp_sampler_run(args):
    """The learned-bias step kernel alone: the diffusion-dominated quadratic case (m = 1,
    phi_in = 6, wall at 8, dN = 1e-3) under the untrained network (r ~ 1: small random weights,
    output bias 1), args.n_eval runs, network evaluated every args.eval_every steps."""
    import dataclasses
    import numpy as np
    import torch
    import paper_2206_11234_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    base = W.c2(args.n_eval)[3]
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    v[:4480] = np.random.default_rng(0).normal(0.0, 1e-2, 4480)
    v[4480] = 1.0
    p0 = W.MlpParams(W.bf16_round(v), in_mean=(5.0, args.target, args.target), in_inv_scale=(0.4, 0.005, 0.01),
                     out_scale=1.0, eval_every=args.eval_every)
    inst = dataclasses.replace(W.c4_instance(p0, n_traj=args.n_eval, target_N=args.target, stream=base.stream),
                               edges=np.linspace(0.0, 400.0, 201))
    F.run(dataclasses.replace(inst, n_traj=20000), 2, block=256, wg_per_cu=args.mlp_wg, chunk=1)   # warm-up
    kms, steps = [], 0
    for s in range(args.steps):
        res, _, tm = F.run(inst, 2, block=256, wg_per_cu=args.mlp_wg, chunk=1, timing=True)
        kms.append(tm[0])
        steps = res.total_steps
        print(f"[mlp] pass {s}: {tm[0]:.1f} ms", file=sys.stderr, flush=True)
    k = sum(kms) / len(kms) / 1e3
    flop = 34 * 32 * 32 * 16 * 2 / 64 / args.eval_every      # matrix-core flop per trajectory-step
    out = {"workload": f"learned-bias sampler, diffusion case, {args.n_eval} runs, network every {args.eval_every} steps",
           "kernel": "fpt_step_mlp1_kernel", "kernel_ms": k * 1e3, "steps": steps, "traj_steps_per_s": steps / k,
           "mfma_flop_per_step": flop, "mfma_pflops": steps / k * flop / 1e15,
           "mfma_frac_bf16_peak": steps / k * flop / 2.5e15}
    print(json.dumps(out), flush=True)


def c3_run(args, steps=None, warmup=None, quiet=False):
    """The batched sweep (64 instances of uneven length, 1e6 runs each) as one persistent launch,
    replayed from a HIP graph, launch shape and queue chunk from the library's autotuner.
    Returns the result line (printed unless quiet)."""
    import torch
    import paper_2206_11234_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    insts = W.c3(args.n_traj)
    side = torch.cuda.Stream()   # graph capture needs a non-null stream
    kw = dict(block=0, wg_per_cu=0, chunk=0)
    with torch.cuda.stream(side):
        # the first call runs the autotuner; one timed pass gives the kernel time (HIP events)
        _, _, tm = F.run_batch(insts, 0, timing=True, **kw)
        for _ in range(warmup):
            F.run_batch(insts, 0, use_graph=True, **kw)
        side.synchronize()
        steps_total = 0
        t_all = time.perf_counter()
        for s in range(steps):
            t0 = time.perf_counter()
            results, _, _ = F.run_batch(insts, 0, use_graph=True, **kw)
            side.synchronize()
            steps_total += sum(r.total_steps for r in results)
            print(f"[c3] pass {s} {(time.perf_counter() - t0) * 1e3:.1f} ms", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t_all
    steps_per_pass = steps_total / steps
    lens = [r.total_steps / i.n_traj for r, i in zip(results, insts)]
    out = {"metric": "weighted traj-steps/s", "value": steps_total / wall, "unit": "traj-steps/s",
           "steps": steps, "warmup": warmup, "ms_per_step": wall / steps * 1e3,
           "kernel_ms": tm[0], "kernel_rate": steps_per_pass / (tm[0] / 1e3),
           "issue_frac": OPS_PER_STEP * steps_per_pass / (tm[0] / 1e3) / PEAK_LANE_OPS,
           "config": {"workload": "C3 batched sweep: 64 instances from splitmix64(0), phi_in~U[3,12], "
                                  "m in {0.01,0.1,0.5,1}, A in {0..6}, wall on/off, dN in {1e-3,5e-4}, "
                                  "1e6 runs each, one graph-replayed launch, autotuned shape",
                      "instances": len(insts), "runs_per_instance": args.n_traj, "steps_per_pass": steps_per_pass,
                      "mean_len_min": min(lens), "mean_len_max": max(lens)}}
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the path runs on one GPU: --gpus must be 1 (sharding by run id is described, not launched)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.learned:
        print(json.dumps(learned_gain(args)), flush=True)
        return
    if args.c5_analyse:
        c5_analyse_saved(args.c5_analyse)
        return
    if args.c5:
        c5_run(args)
        return
    if args.c3:
        c3_run(args)
        return
    if args.mlp_sampler:
        mlp_sampler_run(args)
        return
    import numpy as np
    import torch
    import paper_2206_11234_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    insts = W.c2(args.n_traj)
    kw = dict(block=args.block, wg_per_cu=args.wg_per_cu, chunk=args.chunk)
    if args.autotune:
        kw = dict(block=0, wg_per_cu=0, chunk=0)
    for _ in range(args.warmup):
        F.run_batch(insts, 0, **kw)
    torch.cuda.synchronize()
    times, kern_ms, steps_total, ess_total, ess_target = [], [], 0, 0.0, 0.0
    # target window: the bin holding P ~ 1e-30 of the drift-dominated case (N* = 25.61, where the
    # A = 2 instance is the best fixed bias) and two bins on either side, over the three drift
    # instances
    N_STAR_DRIFT = 25.61

    def target_ess(r):
        j = int(np.searchsorted(r.edges, N_STAR_DRIFT)) - 1
        e = r.ess()[max(j - 2, 0):j + 3]
        return float(np.nansum(e))
    results = None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        results, _, tm = F.run_batch(insts, 0, timing=True, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        kern_ms.append(tm[0])
        steps_total += sum(r.total_steps for r in results)
        ess_total += float(sum(np.nansum(r.ess()) for r in results))
        ess_target += sum(target_ess(r) for inst, r in zip(insts, results) if inst.name.startswith("C2_drift"))
        print(f"[bench] step {s} {times[-1]*1e3:.1f} ms kernel {tm[0]:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    steps_per_pass = steps_total / args.steps
    value = steps_total / wall
    kmean = sum(kern_ms) / len(kern_ms) / 1e3
    achieved = OPS_PER_STEP * steps_per_pass / kmean
    kernel_steps_per_s = steps_per_pass / kmean
    out = {
        "metric": "weighted traj-steps/s",
        "value": value,
        "unit": "traj-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2 fixed-bias sweep: quadratic V, A in {1,2,4}, drift (m=0.01, phi_in=10) "
                               "and diffusion (m=1, phi_in=6, wall 8) cases, dN=1e-3, 6 x 1e6 runs, 200 bins",
                   "instances": len(insts), "runs_per_instance": args.n_traj,
                   "steps_per_pass": steps_per_pass},
        "ess_per_s": ess_total / wall,
        "ess_per_s_target": ess_target / wall,
        "ess_target_window": "drift case, the bin holding N* = 25.61 (P ~ 1e-30) and two bins on either side",
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": TRAFFIC, "traffic_unit": "bytes/launch",
                     "kernel": "fpt_step_kernel", "kernel_ms": kmean * 1e3,
                     "ops_per_step": OPS_PER_STEP,
                     "frac_reading": "VALU issue: compiled lane-ops per step over the lane-op issue peak",
                     "frac_flop": FLOP_PER_STEP_ALGORITHMIC * kernel_steps_per_s / PEAK_FP32_FLOPS,
                     "frac_flop_counted": FLOP_PER_STEP_COUNTED * kernel_steps_per_s / PEAK_FP32_FLOPS,
                     "flop_per_step": FLOP_PER_STEP_ALGORITHMIC, "flop_per_step_counted": FLOP_PER_STEP_COUNTED,
                     "flop_peak": PEAK_FP32_FLOPS / 1e12},
    }
    if not args.no_c3:
        c3 = c3_run(args, steps=args.c3_steps, warmup=1, quiet=True)
        out["c3_batched"] = {k: c3[k] for k in ("value", "unit", "steps", "ms_per_step", "kernel_ms", "kernel_rate",
                                                "issue_frac", "config")}
    if not args.no_learned:
        out["learned_vs_fixed"] = learned_summary(learned_gain(args))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts, args.cpu_seconds, [r.total_steps for r in results])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
