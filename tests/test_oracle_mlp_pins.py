"""Pins of the oracle's learned bias r_theta(phi, N, N*): its activation against tanh, and the
network against hand-built networks whose output is known in closed form (up to the
activation's bounded rounding difference): a constant network, and single paths through one hidden unit
of each layer chosen at asymmetric indices (a transposed weight matrix, a wrong parameter
offset or a mixed-up input would zero the path).  A constant network in the sampler must
reproduce the noise-scaled bias r = A of the same value bit for bit."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def bf16(x):
    """Round binary32 to bfloat16 (nearest, ties to even) on the bit pattern."""
    b = np.asarray(x, np.float32).reshape(-1).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def net(entries, **kw):
    v = np.zeros(W.MlpParams.N_PARAMS, np.float32)
    for off, val in entries:
        v[off] = val
    return W.MlpParams(v, **kw)


W1 = lambda u, i: 0 + 3 * u + i
B1 = lambda u: 192 + u
W2 = lambda o, i: 256 + 64 * o + i
B2 = lambda u: 4352 + u
W3 = lambda u: 4416 + u
B3 = 4480


def points(n=257, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(1.4, 8.0, n).astype(np.float32), rng.uniform(0.0, 600.0, n).astype(np.float32)


def bf16_ulp(y):
    """Spacing of bfloat16 numbers at |y| (8 significant bits)."""
    y = np.abs(np.asarray(y, np.float64))
    return np.exp2(np.floor(np.log2(np.maximum(y, 2.0 ** -120))) - 7)


def test_activation_is_tanh_to_a_third_of_a_bfloat16_ulp():
    """The sampler's activation against tanh itself: within 0.32 of a bfloat16 ulp of tanh x
    everywhere (a dense grid over the polynomial's range and the clamped tail, and random
    magnitudes from 2^-100 to 2^100), odd, saturating to +-1 once rounded to bfloat16, and once
    rounded never more than one bfloat16 ulp from the correctly rounded tanh, equal to it in at
    least 80 % of normally distributed pre-activations."""
    rng = np.random.default_rng(7)
    grid = np.linspace(-12.0, 12.0, 2_400_001).astype(np.float32)
    mags = np.exp2(rng.uniform(-100.0, 100.0, 400_000)).astype(np.float32)
    x = np.concatenate([grid, mags, -mags])
    x = x[x != 0]
    y = O.tanh_act(x).astype(np.float64)
    t = np.tanh(x.astype(np.float64))
    err = np.abs(y - t) / bf16_ulp(t)
    print(f"largest error {err.max():.3f} bfloat16 ulp at x = {x[np.argmax(err)]:.4f}")
    assert err.max() <= 0.32
    assert np.array_equal(O.tanh_act(-x), -O.tanh_act(x))
    big = np.concatenate([np.linspace(3.4, 50.0, 1000), [1e10, 3e38]]).astype(np.float32)
    assert np.all(bf16(O.tanh_act(big)) == 1.0) and np.all(bf16(O.tanh_act(-big)) == -1.0)
    z = rng.normal(0.0, 1.5, 1_000_000).astype(np.float32)
    a, b = bf16(O.tanh_act(z)), bf16(np.tanh(z.astype(np.float64)).astype(np.float32))
    steps = np.abs(a - b) / bf16_ulp(np.maximum(np.abs(a), np.abs(b)))
    print(f"rounded: equal {np.mean(a == b):.3f}, largest difference {steps.max():.2f} ulp")
    assert steps.max() <= 1.0 + 1e-12 and np.mean(a == b) >= 0.8


def test_constant_network():
    p = net([(B3, 0.5)], out_scale=2.0)
    phi, N = points()
    r = O.mlp_r(O.Model(bias=O.BIAS_MLP, mlp=p, target_N=196.0), phi, N)
    assert np.all(r == 1.0)


def test_single_path_through_phi():
    # unit 7 of layer 1 reads phi; unit 40 of layer 2 reads unit 7; the output reads unit 40
    p = net([(W1(7, 0), 1.0), (W2(40, 7), 0.5), (W3(40), 0.75)], in_mean=(5.0, 0.0, 0.0),
            in_inv_scale=(0.25, 1.0, 1.0), out_scale=1.5)
    phi, N = points()
    r = O.mlp_r(O.Model(bias=O.BIAS_MLP, mlp=p, target_N=0.0), phi, N)
    x = bf16((phi.astype(np.float64) - 5.0) * 0.25)
    h1 = bf16(np.tanh(x))
    h2 = bf16(np.tanh(0.5 * h1))
    want = 1.5 * 0.75 * h2
    # each rounded activation is the correctly rounded tanh or its neighbour (ulp <= 2^-8 below 1)
    assert np.max(np.abs(r - want)) <= 1.125 * (2.0 ** -8 + 0.5 * 2.0 ** -8) + 1e-15
    assert np.mean(np.abs(r - want) <= 1e-15) >= 0.5
    assert np.max(np.abs(want)) > 0.1
    # the transposed entry W2[7][40] carries nothing through unit 40
    q = net([(W1(7, 0), 1.0), (W2(7, 40), 0.5), (W3(40), 0.75)], in_mean=(5.0, 0.0, 0.0),
            in_inv_scale=(0.25, 1.0, 1.0), out_scale=1.5)
    assert np.all(O.mlp_r(O.Model(bias=O.BIAS_MLP, mlp=q, target_N=0.0), phi, N) == 0.0)


def test_single_paths_through_N_and_target_with_biases():
    # unit 3 reads N, unit 60 reads N* (with layer-1 bias); layer 2 unit 9 sums both with its bias
    p = net([(W1(3, 1), 1.0), (W1(60, 2), -2.0), (B1(60), 0.25), (W2(9, 3), 1.0), (W2(9, 60), 0.5),
             (B2(9), -0.125), (W3(9), 2.0), (B3, 0.0625)],
            in_mean=(0.0, 200.0, 100.0), in_inv_scale=(1.0, 0.005, 0.01), out_scale=1.0)
    phi, N = points(seed=1)
    for target in (0.0, 196.0, 400.0):
        r = O.mlp_r(O.Model(bias=O.BIAS_MLP, mlp=p, target_N=target), phi, N)
        xN = bf16((N.astype(np.float64) - 200.0) * np.float64(np.float32(0.005)))
        xT = bf16(np.array([(target - 100.0) * np.float64(np.float32(0.01))]))[0]
        h3 = bf16(np.tanh(xN))
        h60 = bf16(np.tanh(np.array([-2.0 * xT + 0.25])))[0]
        h9 = bf16(np.tanh(h3 + 0.5 * h60 - 0.125))
        want = 2.0 * h9 + 0.0625
        # one bfloat16 ulp (<= 2^-8) per activation on the path, through weights 1, 0.5 and 2
        assert np.max(np.abs(r - want)) <= 2.0 * (2.0 ** -8) * (1.0 + 1.0 + 0.5) + 1e-6, target
        assert np.mean(np.abs(r - want) <= 1e-6) >= 0.25, target


@pytest.mark.parametrize("every", [1, 4, 8, 16])
def test_constant_network_sampler_equals_noise_scaled_bias(every):
    base = W.c2(96)[3]                          # m = 1, phi_in = 6, wall at 8, A = 1
    m_fixed = O.Model.from_instance(base)
    p = net([(B3, 0.5)], out_scale=2.0, eval_every=every)
    m_net = O.Model.from_instance(W.c4_instance(p, n_traj=96, stream=base.stream))
    assert m_fixed.A == 1.0 and m_net.bias == O.BIAS_MLP
    a = O.simulate(m_fixed, 0, 96)
    b = O.simulate(m_net, 0, 96)
    assert np.array_equal(a.k, b.k) and np.array_equal(a.status, b.status)
    assert np.array_equal(a.lw, b.lw) and np.array_equal(a.phi, b.phi)
