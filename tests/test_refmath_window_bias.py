"""Pins of the zero-variance window bias of the oracle's reference math (the learned
proposal's ceiling).

For first passage in a window (lo, hi] the zero-variance proposal is the target process
conditioned on the event, whose extra drift is S^2 d/dphi ln h with h(phi, n) the probability
of ending in the window from phi at time n (App. A's pole expansion gives h).  On the flat well
(V = V0: D = 0, constant S, reflecting wall at L) everything is closed form:
psi_n = sin(k_n x)/k_n with k_n = (n + 1/2) pi / L, Lambda_n = S^2 k_n^2 / 2 and c_n = 2/L, and
the window probability is the difference of two values of the classical sine-series survival
function of Brownian motion between an absorbing and a reflecting end.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import refmath as R

L_WELL = 1.5
S2 = 1.0 / (12.0 * math.pi ** 2)          # V0 / (3 (2 pi)^2) with V0 = 1
S = math.sqrt(S2)
LO, HI = 300.0, 310.0


@pytest.fixture(scope="module")
def flat():
    m = O.Model(pot=O.POT_FLAT, V0=1.0, phi_in=1.0, phi_end=0.0, phi_uv=L_WELL)
    return R.window_bias(m, LO, HI, n_modes=6, lam_max=2.0)


def _closed(x, n, n_modes=6):
    k = (np.arange(n_modes) + 0.5) * math.pi / L_WELL
    lam = S2 * k ** 2 / 2.0
    t = (2.0 / L_WELL) * (np.exp(-lam * (LO - n)) - np.exp(-lam * (HI - n)))
    h = np.sum(t[:, None] * np.sin(np.outer(k, x)) / k[:, None], axis=0)
    dh = np.sum(t[:, None] * np.cos(np.outer(k, x)), axis=0)
    return h, S * dh / h


def test_flat_well_modes_and_weights(flat):
    k = (np.arange(6) + 0.5) * math.pi / L_WELL
    assert np.allclose(flat.lam, S2 * k ** 2 / 2.0, rtol=1e-9)
    assert np.allclose(flat.c, 2.0 / L_WELL, rtol=1e-8)


@pytest.mark.parametrize("n", [0.0, 200.0, 280.0])
def test_flat_well_bias_matches_closed_form(flat, n):
    x = np.linspace(0.05, L_WELL, 30)
    h_ref, r_ref = _closed(x, n)
    assert np.allclose(flat.h(x, n), h_ref, rtol=1e-8, atol=0)
    assert np.allclose(flat.r(x, n), r_ref, rtol=1e-7, atol=1e-12)
    # the bias vanishes at the reflecting wall; long before the window it pushes away from the
    # end everywhere (survive first), shortly before it pushes runs near the wall toward the end
    assert abs(flat.r(np.array([L_WELL]), n)[0]) < 1e-8
    if LO - n >= 100.0:
        assert np.all(flat.r(x[:-1], n) > 0)
    else:
        assert flat.r(x[:1], n)[0] > 0 and flat.r(x[-2:-1], n)[0] < 0


def test_window_probability_is_the_survival_difference(flat):
    """h from the mode sum against the sine series of the Brownian survival function, summed to
    400 terms independently (oracle.refmath.brownian_survival_wall)."""
    x, n = 1.0, 250.0
    surv = lambda T: R.brownian_survival_wall(np.array([T]), x, 0.0, L_WELL, S)[0]
    want = surv(LO - n) - surv(HI - n)
    assert flat.h(np.array([x]), n)[0] == pytest.approx(want, rel=1e-6)


def test_far_from_the_window_the_bias_is_quasi_stationary(flat):
    """Long before the window only the slowest mode is left: r* -> S k_0 cot(k_0 x)."""
    x = np.linspace(0.1, L_WELL - 0.1, 12)
    k0 = 0.5 * math.pi / L_WELL
    assert np.allclose(flat.r(x, LO - 2500.0), S * k0 / np.tan(k0 * x), rtol=1e-6)


def test_conditioned_density_of_the_flat_well(flat):
    """rho psi_0^2 with constant rho is sin^2(k_0 x), normalised."""
    x = np.linspace(0.0, L_WELL, 2001)
    k0 = 0.5 * math.pi / L_WELL
    want = np.sin(k0 * x) ** 2 / (L_WELL / 2.0)
    assert np.allclose(flat.conditioned_density(x), want, rtol=1e-6, atol=1e-9)
