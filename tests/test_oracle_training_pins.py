"""Pins of the oracle's proposal-training quantities: the weight a fixed path would have under a
candidate bias (Sec. 2.2: ratio of the target and sample path densities), and the gradient of
log M2(theta).

- A constant candidate r = c on paths drawn with the constant bias r0 has the closed form
  ln w_c = (c/r0) ln w_0 + k dN (c^2 - c r0)/2 (eliminate sum xi between the two weights).
- The analytic gradient matches central finite differences of the loss in every parameter group.
- The replay reproduces the sampler's own runs (k, ln w, status) bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _fixed_model(A=1.0):
    return O.Model.from_instance(W.c2(64)[3]) if A == 1.0 else None


def _short_paths(model, lo, hi, n_want, seed=0, pool=4000):
    tr = O.simulate(model, seed, pool)
    ids = np.nonzero((tr.k >= lo) & (tr.k <= hi) & (tr.status == O.ST_ENDED))[0][:n_want]
    assert ids.size == n_want
    return ids.astype(np.uint64), tr


@pytest.mark.parametrize("E", [4, 16])
def test_replay_reproduces_sampler_runs(E):
    m = _fixed_model()
    ids, tr = _short_paths(m, 6000, 40000, 12)
    rec = O.records(m, 0, ids, E)
    assert np.array_equal(rec.k, tr.k[ids]) and np.array_equal(rec.status, tr.status[ids])
    assert np.array_equal(rec.lw, tr.lw[ids])
    n = np.diff(rec.off.astype(np.int64))
    assert np.array_equal(n, (rec.k.astype(np.int64) + E - 1) // E)
    # the last record of each path holds the remainder of its steps; all others hold E
    ln = rec.rec["pn"] & 31
    assert np.array_equal(rec.rec["pn"] >> 5, np.repeat(np.arange(len(ids)), n))
    last = rec.off[1:].astype(np.int64) - 1
    assert np.all(ln[last] == (rec.k - 1) % E + 1)
    mask = np.ones(len(ln), bool)
    mask[last] = False
    assert np.all(ln[mask] == E)
    assert np.all(rec.rec["k"][rec.off[:-1].astype(np.int64)] == 0)


@pytest.mark.parametrize("c", [0.0, 0.5, 1.0, 1.75])
def test_constant_candidate_closed_form(c):
    m = _fixed_model()                   # r0 = A = 1
    ids, _ = _short_paths(m, 6000, 200000, 10)
    rec = O.records(m, 0, ids, 4)
    v = np.zeros(4481)
    v[4480] = c
    net = W.MlpParams(np.zeros(4481, np.float32), out_scale=1.0)
    mm = O.Model.from_instance(W.c4_instance(net, n_traj=1, stream=m.stream))
    loss, grad, lwt = O.loss_grad(mm, v, rec, rec.lw, n_total=100.0)
    dN = float(np.float32(m.dN))
    want = c * rec.lw + rec.k * dN * (c * c - c) / 2
    # binary32 roundings of the per-step increments and of the group sums H, at most ~2^-24 of
    # |eta| ~ dN + sqrt(dN)|xi| per step, accumulated over k steps (a dropped term or a wrong
    # sign would move ln w by ~ k dN c^2/2 ~ 100)
    tol = rec.k * 2.0 ** -24 * (dN + np.sqrt(dN)) * (1 + c)
    assert np.all(np.abs(lwt - want) <= tol), np.max(np.abs(lwt - want) / tol)
    if c == 0.0:
        assert np.all(lwt == 0.0)
    x = rec.lw + lwt
    assert np.isclose(loss, np.log(np.sum(np.exp(x - x.max()))) + x.max() - np.log(100.0), rtol=0, atol=1e-12)


def test_gradient_matches_finite_differences():
    m = _fixed_model()
    ids, _ = _short_paths(m, 6000, 11000, 6)
    rec = O.records(m, 0, ids, 4)
    p = W.c4_params(7, scale=1.5, out_scale=0.8)
    mm = O.Model.from_instance(W.c4_instance(p, n_traj=1, stream=m.stream))
    theta = p.values_f32().astype(np.float64)
    loss, grad, _ = O.loss_grad(mm, theta, rec, rec.lw, n_total=1e4)
    rng = np.random.default_rng(3)
    groups = [(0, 192), (192, 256), (256, 4352), (4352, 4416), (4416, 4480), (4480, 4481)]
    idx = np.concatenate([rng.choice(np.arange(a, b), min(4, b - a), replace=False) for a, b in groups])
    h = 1e-5
    scale = np.max(np.abs(grad))
    assert scale > 1e-3
    for j in idx:
        tp = theta.copy(); tp[j] += h
        tm = theta.copy(); tm[j] -= h
        fd = (O.loss_grad(mm, tp, rec, rec.lw, 1e4)[0] - O.loss_grad(mm, tm, rec, rec.lw, 1e4)[0]) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 * scale + 1e-5 * abs(grad[j]), (j, fd, grad[j])


def test_cross_entropy_gradient_and_closed_form():
    """Objective 1 (cross entropy): the loss is sum_i c_i ln w_theta,i with c_i ~ w_0,i; for a
    constant candidate c its value follows from the closed form above, and its gradient matches
    central finite differences."""
    m = _fixed_model()
    ids, _ = _short_paths(m, 6000, 11000, 6)
    rec = O.records(m, 0, ids, 4)
    c = 0.7
    v = np.zeros(4481)
    v[4480] = c
    net = W.MlpParams(np.zeros(4481, np.float32), out_scale=1.0)
    mm = O.Model.from_instance(W.c4_instance(net, n_traj=1, stream=m.stream))
    loss, _, lwt = O.loss_grad(mm, v, rec, rec.lw, 1e4, objective=1)
    dN = float(np.float32(m.dN))
    ci = np.exp(rec.lw - rec.lw.max())
    ci /= ci.sum()
    want = np.sum(ci * (c * rec.lw + rec.k * dN * (c * c - c) / 2))
    # the binary32 rounding bound of the constant-candidate closed form, weighted by c_i
    tol = np.sum(ci * rec.k * 2.0 ** -24 * (dN + np.sqrt(dN)) * (1 + c))
    assert abs(loss - want) <= tol
    p = W.c4_params(5, scale=1.5, out_scale=0.8)
    mm = O.Model.from_instance(W.c4_instance(p, n_traj=1, stream=m.stream))
    theta = p.values_f32().astype(np.float64)
    loss, grad, _ = O.loss_grad(mm, theta, rec, rec.lw, 1e4, objective=1)
    scale = np.max(np.abs(grad))
    h = 1e-5
    for j in (5, 200, 300, 4000, 4360, 4420, 4480):
        tp = theta.copy(); tp[j] += h
        tm = theta.copy(); tm[j] -= h
        fd = (O.loss_grad(mm, tp, rec, rec.lw, 1e4, 1)[0] - O.loss_grad(mm, tm, rec, rec.lw, 1e4, 1)[0]) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 * scale + 1e-5 * abs(grad[j]), (j, fd, grad[j])


def test_record_stride_keeps_every_sth_group():
    """With stride s the records are exactly the groups g = 0, s, 2s, ... of the complete records
    (bit for bit); weighted by s, their sums estimate the complete sums."""
    m = _fixed_model()
    ids, _ = _short_paths(m, 6000, 40000, 8)
    full = O.records(m, 0, ids, 4)
    s4 = O.records(m, 0, ids, 4, stride=4)
    for i in range(len(ids)):
        f = full.rec[full.off[i]:full.off[i + 1]]
        g = s4.rec[s4.off[i]:s4.off[i + 1]]
        assert g.tobytes() == f[(f["k"] // 4) % 4 == 0].tobytes()
    # a constant candidate: the strided estimate of ln w_theta agrees with the complete sum
    net = W.MlpParams(np.zeros(4481, np.float32), out_scale=1.0)
    mm = O.Model.from_instance(W.c4_instance(net, n_traj=1, stream=m.stream))
    v = np.zeros(4481)
    v[4480] = 0.6
    _, _, lw_full = O.loss_grad(mm, v, full, full.lw, 1e4, objective=1)
    _, _, lw_s4 = O.loss_grad(mm, v, s4, s4.lw, 1e4, objective=1, rec_weight=4.0)
    # each group's term -c H + c^2 n dN/2 has spread ~ c sqrt(4 dN); the strided sum's error is
    # ~ sqrt(3 G) c sqrt(4 dN) for G groups
    G = np.diff(full.off.astype(np.int64))
    tol = 5 * np.sqrt(3 * G) * 0.6 * np.sqrt(4 * float(np.float32(m.dN)))
    assert np.all(np.abs(lw_s4 - lw_full) < tol)
