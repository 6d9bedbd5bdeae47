"""Pins of the binary64 reference mathematics (oracle/refmath.py).

The quadrature of the paper's double integral and the Sturm-Liouville solver
are checked against closed forms that do not share their numerics: the
drift-dominated expansion of the same ODE, the paper's printed N_cl = 10,
Brownian first passage (the quantum well of Sec. 3), and the sine
eigen-series of an absorbing/reflecting interval.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import refmath as R
from conftest import read_golden


def _paper(name):
    for row in read_golden("paper_values.txt"):
        parts = row.split()
        if parts[0] == name:
            return float(parts[1])
    raise KeyError(name)


def test_classical_N_reproduces_paper_value():
    """Sec. 3: phi_in = sqrt(42) gives N_cl = 10 e-folds (phi_end = sqrt 2)."""
    m = O.Model(m=0.001, phi_in=math.sqrt(42.0), phi_end=math.sqrt(_paper("phi_end_sq")))
    assert abs(R.classical_N(m) - _paper("N_cl_phi_in_sqrt42")) < 1e-12


@pytest.mark.parametrize("mass,phi", [(0.01, 5.0), (0.01, 10.0), (0.001, math.sqrt(42.0))])
def test_mean_matches_drift_limit_expansion(mass, phi):
    """Small-v expansion of f_1'' - (v'/v^2) f_1' = -1/v (App. A with t -> 0) for
    v = v0 phi^2: f_1' = phi/2 + v0 phi^3/4 + O(v0^2), so
    <N> = (phi^2 - phi_end^2)/4 + v0 (phi^4 - phi_end^4)/16 + O(v0^2)."""
    m = O.Model(m=mass, phi_in=phi)
    v0 = mass ** 2 / (48 * math.pi ** 2)
    want = (phi ** 2 - 2.0) / 4 + v0 * (phi ** 4 - 4.0) / 16
    got = R.moments(m).mean
    assert abs(got - want) < 50 * v0 ** 2 * phi ** 6 + 1e-9


@pytest.mark.parametrize("mass,phi", [(0.01, 5.0), (0.01, 10.0)])
def test_variance_matches_classical_delta_N(mass, phi):
    """Drift-dominated variance m^2 (phi^6 - phi_end^6)/(1152 pi^2) (leading order)."""
    m = O.Model(m=mass, phi_in=phi)
    v = R.moments(m).var
    want = R.classical_var_quadratic(mass, phi, math.sqrt(2))
    v0 = mass ** 2 / (48 * math.pi ** 2)
    assert abs(v / want - 1) < 20 * v0 * phi ** 2


def test_moments_match_quantum_well_closed_forms():
    """Constant V with absorbing end a and reflecting wall b: E T = y (2L - y)/S^2,
    Var T = 2 (L^4 - (L-y)^4) / (3 S^4), y = x - a, L = b - a."""
    for V0, x, b in [(1.0, 1.0, 1.5), (118.4352528130723, 0.3, 2.0)]:
        m = O.Model(pot=O.POT_FLAT, V0=V0, phi_in=x, phi_end=0.0, phi_uv=b)
        S = math.sqrt(V0 / 3) / (2 * math.pi)
        mo = R.moments(m)
        assert abs(mo.mean / R.brownian_mean(x, 0.0, b, S) - 1) < 1e-9
        assert abs(mo.var / R.brownian_var(x, 0.0, b, S) - 1) < 1e-8


def test_moments_with_constant_bias_match_drifted_brownian():
    """Constant drift mu toward the end, no wall: E T = y/mu, Var T = y S^2/mu^3 (inverse
    Gaussian); the bias B = A S with A < 0 gives mu = |A| S on a flat potential."""
    S = 1.0
    V0 = 3 * (2 * math.pi) ** 2
    A = -2.0
    m = O.Model(pot=O.POT_FLAT, V0=V0, phi_in=1.0, phi_end=0.0, phi_esc=40.0,
                bias=O.BIAS_NOISE_SCALED, A=A)
    mo = R.moments(m, biased=True)
    mu = abs(A) * S
    assert abs(mo.mean - 1.0 / mu) < 1e-8
    assert abs(mo.var - 1.0 * S ** 2 / mu ** 3) < 1e-8


def test_sl_modes_match_sine_series():
    """Constant V: Lambda_n = (2n+1)^2 pi^2 S^2/(8 L^2),
    a_n = Lambda_n (4/((2n+1) pi)) sin((2n+1) pi y/(2L))."""
    m = O.Model(pot=O.POT_FLAT, V0=1.0, phi_in=1.0, phi_end=0.0, phi_uv=1.5)
    S = math.sqrt(1 / 3) / (2 * math.pi)
    modes = R.sl_modes(m, 3, lam_max=0.2)
    for n in range(3):
        lam = (2 * n + 1) ** 2 * math.pi ** 2 * S ** 2 / (8 * 1.5 ** 2)
        amp = lam * 4 / ((2 * n + 1) * math.pi) * math.sin((2 * n + 1) * math.pi / 3)
        assert abs(modes.lam[n] / lam - 1) < 1e-9
        assert abs(modes.amp[n] - amp) < 1e-9 * max(1, abs(amp))


def test_sl_modes_match_finite_difference_eigensolve():
    """Diffusion-dominated quadratic case (m = 1, phi_in = 6, wall at 8) and the paper's
    m = 1, phi_in = phi_UV = sqrt 42 case: the shooting eigenvalues agree with an independent
    finite-difference solve of the same Sturm-Liouville problem,
    (1/rho) (p psi')' = -Lambda psi with p = e^Psi, rho = (2/S^2) e^Psi, Psi' = 2D/S^2,
    symmetrised and solved as a tridiagonal eigenproblem."""
    from scipy.linalg import eigvalsh_tridiagonal
    for phi_in, phi_uv in [(6.0, 8.0), (math.sqrt(42.0), math.sqrt(42.0))]:
        m = O.Model(m=1.0, phi_in=phi_in, phi_uv=phi_uv)
        M = 20000
        x = np.linspace(m.phi_end, phi_uv, M + 1)
        h = x[1] - x[0]
        S2 = (m.m ** 2 * x ** 2 / 2) / 3 / (4 * math.pi ** 2)
        # Psi = int 2D/S^2 = int -4/(c^2 phi^3) = 2/(c^2 phi^2) + const, c^2 = m^2/(24 pi^2)
        c2 = m.m ** 2 / (24 * math.pi ** 2)
        Psi = 2.0 / (c2 * x ** 2)
        Psi -= Psi.max()
        xm = 0.5 * (x[1:] + x[:-1])
        Psim = 2.0 / (c2 * xm ** 2) - (2.0 / (c2 * x ** 2)).max()
        # unknowns psi_1..psi_M; volume weights rho_i h (half cell at the wall)
        vol = np.full(M + 1, h)
        vol[-1] = h / 2
        logw = np.log(2.0 / S2) + Psi + np.log(vol)
        i = np.arange(1, M + 1)
        pl = np.exp(Psim[i - 1])                       # p_{i-1/2}
        pr = np.zeros(M)
        pr[:-1] = np.exp(Psim[i[:-1]])                 # p_{i+1/2}, none past the wall
        diag = (pl + pr) / h / np.exp(logw[i])
        off = -np.exp(Psim[i[:-1]]) / h / np.exp(0.5 * (logw[i[:-1]] + logw[i[:-1] + 1]))
        ev = eigvalsh_tridiagonal(diag, off, select="i", select_range=(0, 2))
        modes = R.sl_modes(m, 3)
        assert np.all(np.abs(modes.lam / ev - 1) < 1e-5), (modes.lam, ev)


def test_lattice_gaussian_probs_normalise():
    edges = np.linspace(-1.0, 1.0, 201)
    p = R.lattice_gaussian_probs(0.0, 0.1, 1e-6, edges)
    assert abs(p.sum() - 1) < 1e-12
    from scipy import special
    q = np.diff(special.ndtr(edges / 0.1))
    assert np.max(np.abs(p - q)) < 1e-4
