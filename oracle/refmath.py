"""Binary64 reference mathematics that pins the simulation.

TEST INFRASTRUCTURE ONLY (part of the oracle; never imported by the product).

Contents, each citing the passage it follows:
  * ``drift_noise`` -- D = -V'/V, S = sqrt(V/3)/(2 pi) (Sec. 2.3,
    eq. eq_sr_diffusion with H^2 = V/3, Planck units), bias B = A f(phi)
    (eq. eq_importance_sampling_amplitude_general) with f = S, and the power
    law B = A_p phi^p (eq. eq_importance_sampling_amplitude_power_law).
  * ``moments`` -- mean first-passage time as the double integral of
    eq. eq:meanN:S:gen, and the variance from the same Green's function with
    the source of the moment recursion.  The recursion follows from the
    adjoint Fokker-Planck equation for the characteristic function
    (App. A, eq. eq_chracteristic_function_partial_diff_eqn with the
    boundary conditions eq_chracteristic_function_bc) and the moment formula
    <N^n> = i^-n d^n chi/dt^n at t = 0 (end of App. B): expanding chi in t
    gives L f_n = -n f_{n-1} with L = (S^2/2) d^2 + (D+B) d, f_n(phi_end) = 0,
    f_n'(phi_UV) = 0.  The variance g = f_2 - f_1^2 then obeys
    L g = -S^2 (f_1')^2 with the same boundary conditions (Ito product rule),
    which avoids the cancellation of f_2 - f_1^2 when sigma << mean.
  * ``sl_modes`` -- decay rates and amplitudes of the pole expansion
    P(N) = sum a_n exp(-Lambda_n N) (Sec. 1, eq. eq_pdf_expansion_in_exponentials;
    App. A, eq. eq_pdf_expansion_in_exponentials2), obtained as the
    Sturm-Liouville problem (S^2/2) psi'' + D psi' = -Lambda psi with
    psi(phi_end) = 0, psi'(phi_UV) = 0 by shooting.
  * ``brownian_*`` -- the quantum well (constant V, Sec. 3): Brownian first
    passage with an absorbing end and a reflecting wall.
  * ``classical_*`` -- the drift-dominated limit: N_cl = int dphi/|D|
    (Sec. 2.4) and the Gaussian of App. B with gamma = kappa = 0.
  * ``lattice_gaussian_probs`` -- that Gaussian mapped onto the lattice
    N = k dN of the simulation.
  * ``cumulants_to``, ``saddlepoint_logpdf``, ``saddlepoint_reference`` -- the
    cumulants of N to any order from the backward equation of the moment
    generating function, and Daniels' saddle-point density built from them
    (the resummed form of App. B's cumulant expansion, accurate far beyond
    the Edgeworth range), mapped onto the lattice with ``lattice_logprobs``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize, special

from . import BIAS_NONE, BIAS_NOISE_SCALED, BIAS_POWER, POT_FLAT, POT_QUADRATIC, POT_QUADRATIC_BUMP, Model


# --------------------------------------------------------------------------
# Drift, noise amplitude and bias in binary64 (Sec. 2.3).
# --------------------------------------------------------------------------
def potential(model: Model, phi):
    phi = np.asarray(phi, np.float64)
    if model.pot == POT_QUADRATIC:
        return 0.5 * model.m ** 2 * phi ** 2
    if model.pot == POT_QUADRATIC_BUMP:
        g = np.exp(-(phi - model.phi0) ** 2 / (2 * model.w ** 2))
        return 0.5 * model.m ** 2 * phi ** 2 * (1.0 + model.a * g)
    return np.full_like(phi, model.V0)


def dpotential(model: Model, phi):
    phi = np.asarray(phi, np.float64)
    if model.pot == POT_QUADRATIC:
        return model.m ** 2 * phi
    if model.pot == POT_QUADRATIC_BUMP:
        g = np.exp(-(phi - model.phi0) ** 2 / (2 * model.w ** 2))
        dg = -(phi - model.phi0) / model.w ** 2 * g
        return model.m ** 2 * phi * (1.0 + model.a * g) + 0.5 * model.m ** 2 * phi ** 2 * model.a * dg
    return np.zeros_like(phi)


def drift_noise(model: Model, phi, biased: bool = True):
    """(D, S, B) at phi: D = -V'/V (from 3H^2 = V), S = H/(2 pi) = sqrt(V/3)/(2 pi)."""
    V = potential(model, phi)
    D = -dpotential(model, phi) / V
    S = np.sqrt(V / 3.0) / (2.0 * np.pi)
    if not biased or model.bias == BIAS_NONE:
        B = np.zeros_like(S)
    elif model.bias == BIAS_NOISE_SCALED:
        B = model.A * S
    elif model.bias == BIAS_POWER:
        B = model.A * np.asarray(phi, np.float64) ** model.p
    else:
        raise ValueError("bias kind not supported by the reference math")
    return D, S, B


# --------------------------------------------------------------------------
# Moments of N from the Green's function of L (eq. eq:meanN:S:gen).
# --------------------------------------------------------------------------
def _cell_integrals(g, h):
    """E0 = int_0^h e^{g y} dy and E1 = int_0^h y e^{g y} dy, stable for any g h."""
    gh = g * h
    small = np.abs(gh) < 1e-3
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        e = np.exp(gh)
        E0 = np.where(small, h * (1 + gh / 2 + gh ** 2 / 6 + gh ** 3 / 24), np.expm1(gh) / g)
        E1 = np.where(small, h * h * (0.5 + gh / 3 + gh ** 2 / 8 + gh ** 3 / 30), (h * e - E0) / g)
    return e, E0, E1


def _green_derivative(x, psi_p, psi_p_mid, source):
    """J(x_i) = int_{x_i}^{x_M} source(y) exp(Psi(y) - Psi(x_i)) dy, backward over the grid.

    Per cell, dPsi = int Psi' (Simpson).  Where |dPsi| is small the source is taken linear
    in x and Psi linear in x (exact exponential integral); where |dPsi| is large (drift-
    dominated, the integrand lives within 1/|Psi'| of the cell's left end) the integral is
    taken in the variable Psi with source/Psi' linear in Psi, which is exact in the
    local-equilibrium limit J = source/|Psi'|."""
    h = np.diff(x)
    dpsi = h * (psi_p[:-1] + 4.0 * psi_p_mid + psi_p[1:]) / 6.0
    stiff = np.abs(dpsi) > 0.5
    s = source
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        # x-form: Psi(x_i + y) - Psi(x_i) = g y with g = dPsi/h
        g = dpsi / h
        e, E0x, E1x = _cell_integrals(g, h)
        cx = s[:-1] * E0x + (s[1:] - s[:-1]) * E1x / h
        # Psi-form: int_0^dPsi q(u) e^u du with q = source/Psi' linear in u
        q = s / psi_p
        E0p = np.expm1(dpsi)
        E1p = dpsi * np.exp(dpsi) - E0p
        cp = q[:-1] * E0p + (q[1:] - q[:-1]) * E1p / dpsi
        contrib = np.where(stiff, cp, cx)
        prop = np.exp(dpsi)
    J = np.zeros_like(x)
    for i in range(len(x) - 2, -1, -1):
        J[i] = J[i + 1] * prop[i] + contrib[i]
    return J


def _trapz_cum(x, y):
    out = np.zeros_like(x)
    out[1:] = np.cumsum(0.5 * (y[1:] + y[:-1]) * np.diff(x))
    return out


@dataclass
class Moments:
    mean: float
    var: float

    @property
    def std(self):
        return math.sqrt(self.var)


def _top(model: Model, biased: bool) -> float:
    if np.isfinite(model.phi_uv):
        return model.phi_uv
    top = model.esc()
    if biased and model.bias != BIAS_NONE:
        # beyond the zero of D + B the sample process runs away; the mean is
        # then finite only if that point is never reached in practice.
        xs = np.geomspace(model.phi_end, top, 200001) if model.phi_end > 0 else np.linspace(model.phi_end, top, 200001)
        D, S, B = drift_noise(model, xs)
        pos = np.nonzero(D + B > 0)[0]
        if pos.size:
            top = min(top, 0.9 * xs[pos[0]] + 0.1 * model.phi_in) if xs[pos[0]] > model.phi_in else top
    return top


def moments(model: Model, biased: bool = False, n_grid: int = 400001, phi=None) -> Moments:
    """Mean and variance of N for a start at phi (default phi_in).

    biased=False: the target process (drift D); biased=True: the sample process
    (drift D + B).  f_1' = J with source 2/S^2; g' = J with source 2 (f_1')^2.
    The result is Richardson-extrapolated over grids of n and n/2 cells."""
    phi = model.phi_in if phi is None else phi

    def solve(n):
        top = _top(model, biased)
        if model.pot != POT_FLAT and model.phi_end > 0:
            x = model.phi_end * np.exp(np.linspace(0.0, math.log(top / model.phi_end), n))
        else:
            x = np.linspace(model.phi_end, top, n)
        D, S, B = drift_noise(model, x, biased)
        psi_p = 2.0 * (D + B) / S ** 2
        xm = 0.5 * (x[1:] + x[:-1])
        Dm, Sm, Bm = drift_noise(model, xm, biased)
        psi_pm = 2.0 * (Dm + Bm) / Sm ** 2
        J1 = _green_derivative(x, psi_p, psi_pm, 2.0 / S ** 2)
        f1 = _trapz_cum(x, J1)
        Jg = _green_derivative(x, psi_p, psi_pm, 2.0 * J1 ** 2)
        gv = _trapz_cum(x, Jg)
        return np.interp(phi, x, f1), np.interp(phi, x, gv)

    m_a, v_a = solve(n_grid)
    m_b, v_b = solve((n_grid - 1) // 2 + 1)
    # cell rule is second order in h for smooth integrands
    mean = m_a + (m_a - m_b) / 3.0
    var = v_a + (v_a - v_b) / 3.0
    return Moments(float(mean), float(var))


# --------------------------------------------------------------------------
# Drift-dominated limit (Sec. 2.4 classical N; App. B Gaussian).
# --------------------------------------------------------------------------
def classical_N(model: Model, biased: bool = False, phi=None) -> float:
    """N_cl = int_{phi_end}^{phi} dphi' / |D + B| (noise set to zero)."""
    phi = model.phi_in if phi is None else phi
    f = lambda x: 1.0 / abs(float(sum(drift_noise(model, x, biased)[::2])))
    return integrate.quad(f, model.phi_end, phi, epsabs=0, epsrel=1e-13, limit=200)[0]


def classical_var_quadratic(m: float, phi_in: float, phi_end: float) -> float:
    """Drift-limit variance for V = m^2 phi^2/2: int S^2 (f_1')^2/|D| dphi with
    f_1' = phi/2, S^2 = m^2 phi^2/(24 pi^2): m^2 (phi_in^6 - phi_end^6)/(1152 pi^2)."""
    return m ** 2 * (phi_in ** 6 - phi_end ** 6) / (1152.0 * math.pi ** 2)


def noise_free_em(model: Model, biased: bool = False):
    """Euler-Maruyama with the noise set to zero, binary64: returns (k, tau) where k is
    the step count at first passage and tau the crossing time of the polygonal path."""
    phi = model.phi_in
    k = 0
    while True:
        D, S, B = drift_noise(model, phi, biased)
        nphi = phi + float(D + B) * model.dN
        k += 1
        if nphi <= model.phi_end:
            tau = (k - 1) * model.dN + model.dN * (phi - model.phi_end) / (phi - nphi)
            return k, tau
        phi = nphi


def lattice_gaussian_probs(mu: float, sigma: float, dN: float, edges, eps: float = 0.0):
    """P(e_j < k dN <= e_{j+1}) when k = ceil((N_c + eps)/dN) and N_c ~ Normal(mu, sigma):
    the Gaussian of App. B (gamma = kappa = 0) seen on the simulation's lattice; eps is
    the slowdown of the discrete drift (noise-free EM crossing time minus N_cl)."""
    edges = np.asarray(edges, np.float64)
    K = np.floor(edges / dN + 1e-9)
    # largest k with k dN <= e_j
    K = np.where((K + 1) * dN <= edges, K + 1, K)
    K = np.where(K * dN > edges, K - 1, K)
    z = (K * dN - eps - mu) / sigma
    cdf = special.ndtr(z)
    return np.diff(cdf)


# --------------------------------------------------------------------------
# Quantum well (constant V, Sec. 3): Brownian first passage.
# --------------------------------------------------------------------------
BGK_BETA = -special.zeta(0.5) / math.sqrt(2.0 * math.pi)   # 0.5826: Broadie-Glasserman-Kou


def brownian_mean(x: float, a: float, b: float, S: float) -> float:
    """E[T] for dx = S dW from x, absorbing at a < x, reflecting at b > x: solves
    (S^2/2) f'' = -1, f(a) = 0, f'(b) = 0."""
    return (x - a) * (2.0 * (b - a) - (x - a)) / S ** 2


def brownian_var(x: float, a: float, b: float, S: float) -> float:
    """Var T for the same process: (S^2/2) g'' = -S^2 f'^2, g(a) = 0, g'(b) = 0."""
    L = b - a
    y = x - a
    # f' = 2 (L - y)/S^2  ->  g'' = -2 f'^2 = -8 (L - y)^2 / S^4
    # g'(y) = 8/(3 S^4) (L - y)^3 ; g(y) = 2/(3 S^4) (L^4 - (L - y)^4)
    return 2.0 / (3.0 * S ** 4) * (L ** 4 - (L - y) ** 4)


def brownian_density_wall(T, x: float, a: float, b: float, S: float, n_terms: int = 400):
    """First-passage density with a reflecting wall: sum of the sine eigen-series
    P(T) = sum_n c_n (S^2 k_n^2 / 2) sin(k_n (x - a)) exp(-S^2 k_n^2 T/2),
    k_n = (2n+1) pi / (2L), c_n = 4/((2n+1) pi)."""
    T = np.asarray(T, np.float64)
    L = b - a
    n = np.arange(n_terms)
    kn = (2 * n + 1) * math.pi / (2 * L)
    cn = 4.0 / ((2 * n + 1) * math.pi)
    lam = 0.5 * S ** 2 * kn ** 2
    terms = cn[None, :] * lam[None, :] * np.sin(kn[None, :] * (x - a)) * np.exp(-lam[None, :] * T[..., None])
    return terms.sum(-1)


def brownian_survival_wall(T, x: float, a: float, b: float, S: float, n_terms: int = 400):
    T = np.asarray(T, np.float64)
    L = b - a
    n = np.arange(n_terms)
    kn = (2 * n + 1) * math.pi / (2 * L)
    cn = 4.0 / ((2 * n + 1) * math.pi)
    lam = 0.5 * S ** 2 * kn ** 2
    terms = cn[None, :] * np.sin(kn[None, :] * (x - a)) * np.exp(-lam[None, :] * T[..., None])
    return terms.sum(-1)


def levy_density(T, x: float, a: float, S: float):
    """No wall, no drift: (x - a)/(S sqrt(2 pi T^3)) exp(-(x - a)^2/(2 S^2 T))."""
    T = np.asarray(T, np.float64)
    y = x - a
    return y / (S * np.sqrt(2 * np.pi * T ** 3)) * np.exp(-y * y / (2 * S * S * T))


# --------------------------------------------------------------------------
# Pole expansion from the Sturm-Liouville problem (App. A).
# --------------------------------------------------------------------------
@dataclass
class Modes:
    lam: np.ndarray     # decay rates Lambda_n
    amp: np.ndarray     # a_n(phi_in)


def _scalar_drift_s2(model: Model):
    """Scalar (D, S^2) of the target process with math-module arithmetic (fast path for ODEs)."""
    four_pi2 = 4.0 * math.pi ** 2
    if model.pot == POT_QUADRATIC:
        m2 = model.m ** 2
        return lambda x: (-2.0 / x, 0.5 * m2 * x * x / (3.0 * four_pi2))
    if model.pot == POT_QUADRATIC_BUMP:
        m2, a, p0, w2 = model.m ** 2, model.a, model.phi0, model.w ** 2

        def f(x):
            g = math.exp(-(x - p0) ** 2 / (2 * w2))
            V = 0.5 * m2 * x * x * (1 + a * g)
            dV = m2 * x * (1 + a * g) - 0.5 * m2 * x * x * a * (x - p0) / w2 * g
            return -dV / V, V / (3.0 * four_pi2)
        return f
    s2 = model.V0 / (3.0 * four_pi2)
    return lambda x: (0.0, s2)


def _shoot(model: Model, lam: float, rtol=1e-12, dense=False):
    """psi(phi_end) = 0, psi'(phi_end) = 1 integrated up to phi_UV; carries Psi and the
    weighted integrals int rho psi and int rho psi^2 with rho = (2/S^2) e^Psi."""
    ds2 = _scalar_drift_s2(model)

    def rhs(x, y):
        psi, dpsi, Psi, i1, i2 = y
        D, S2 = ds2(x)
        rho = 2.0 / S2 * math.exp(Psi)
        return [dpsi, -2.0 / S2 * (D * dpsi + lam * psi), 2.0 * D / S2, rho * psi, rho * psi * psi]
    h0 = (model.phi_uv - model.phi_end) * 1e-4
    sol = integrate.solve_ivp(rhs, (model.phi_end, model.phi_uv), [0.0, 1.0, 0.0, 0.0, 0.0],
                              method="DOP853", rtol=rtol, atol=1e-300, dense_output=dense,
                              first_step=h0)
    return sol


def sl_modes(model: Model, n_modes: int = 3, lam_max: float | None = None, n_scan: int = 120) -> Modes:
    """First n_modes (Lambda_n, a_n) for a finite reflecting wall."""
    if not np.isfinite(model.phi_uv):
        raise ValueError("the pole expansion needs a finite reflecting wall")
    F = lambda lam: _shoot(model, lam, rtol=1e-10).y[1, -1]
    if lam_max is None:
        lam_max = 2.0
    grid = np.geomspace(lam_max * 1e-4, lam_max, n_scan)
    vals = np.array([F(l) for l in grid])
    roots = []
    for i in range(len(grid) - 1):
        if np.sign(vals[i]) != np.sign(vals[i + 1]):
            Fr = lambda lam: _shoot(model, lam).y[1, -1]
            roots.append(optimize.brentq(Fr, grid[i], grid[i + 1], xtol=1e-15, rtol=1e-14))
            if len(roots) == n_modes:
                break
    lams, amps = [], []
    for lam in roots:
        sol = _shoot(model, lam, dense=True)
        i1, i2 = sol.y[3, -1], sol.y[4, -1]
        c = i1 / i2
        psi_in = sol.sol(model.phi_in)[0]
        lams.append(lam)
        amps.append(lam * c * psi_in)
    return Modes(np.array(lams), np.array(amps))


def _prufer_shoot(model: Model, lam: float, rtol: float = 1e-12):
    """The Sturm-Liouville problem of `sl_modes` in Pruefer form, for drift-dominated cases where
    psi, psi' and rho span more than the binary64 range.  With psi = r sin(theta),
    psi' = r cos(theta), psi(phi_end) = 0, psi'(phi_end) = 1:
      theta' = cos^2 + (2/S^2)(D sin cos + Lambda sin^2),
      eta'   = (log r + Psi)' = sin cos - (2 Lambda/S^2) sin cos + (2D/S^2) sin^2,
      Psi'   = 2D/S^2,
      and the variation d theta/d Lambda along the path (its linearised equation).
    Returns the solution of (theta, eta, Psi, d theta/d Lambda) (a stiff system: LSODA, which
    switches to a stiff method where needed, with the implicit Runge-Kutta method as fallback)."""
    ds2 = _scalar_drift_s2(model)

    def rhs(x, y):
        th, _, _, thl = y
        D, S2 = ds2(x)
        sn, cs = math.sin(th), math.cos(th)
        g = 2.0 / S2
        a = -2.0 * sn * cs + g * (D * (cs * cs - sn * sn) + 2.0 * lam * sn * cs)
        return [cs * cs + g * (D * sn * cs + lam * sn * sn), sn * cs - g * lam * sn * cs + g * D * sn * sn,
                g * D, a * thl + g * sn * sn]

    def jac(x, y):
        th, _, _, thl = y
        D, S2 = ds2(x)
        sn, cs = math.sin(th), math.cos(th)
        g = 2.0 / S2
        c2 = cs * cs - sn * sn
        a = -2.0 * sn * cs + g * (D * c2 + 2.0 * lam * sn * cs)
        da = -2.0 * c2 + g * (-4.0 * D * sn * cs + 2.0 * lam * c2)
        return [[a, 0, 0, 0], [c2 - g * lam * c2 + 2.0 * g * D * sn * cs, 0, 0, 0], [0, 0, 0, 0],
                [da * thl + 2.0 * g * sn * cs, 0, 0, a]]

    sol = integrate.solve_ivp(rhs, (model.phi_end, model.phi_uv), [0.0, 0.0, 0.0, 0.0], method="LSODA",
                              rtol=rtol, atol=1e-14, dense_output=True)
    if sol.success and np.all(np.isfinite(sol.y[:, -1])):
        return sol
    return integrate.solve_ivp(rhs, (model.phi_end, model.phi_uv), [0.0, 0.0, 0.0, 0.0], method="Radau",
                               rtol=rtol, atol=1e-14, jac=jac, dense_output=True)


def sl_modes_prufer(model: Model, n_modes: int, lam_lo: float, lam_hi: float, n_scan: int = 40) -> Modes:
    """The first n_modes (Lambda_n, a_n) with Lambda_n in [lam_lo, lam_hi], from the Pruefer form.
    Mode n has theta(phi_UV) = pi/2 + n pi (psi'(phi_UV) = 0 with n interior zeros).  The
    amplitude uses the Sturm-Liouville identities int rho psi = p(phi_end) psi'(phi_end)/Lambda
    (integrate (p psi')' = -Lambda rho psi) and int rho psi^2 = p r^2 d theta/d Lambda at phi_UV
    (the Lambda-derivative of the same equation), p = e^Psi, so that
      a_n = Lambda c_n psi(phi_in) = sin(theta_in) exp(eta_in - Psi_in - 2 eta_UV + Psi_UV) / (d theta/d Lambda)_UV
    with every exponent formed before exponentiation."""
    if not np.isfinite(model.phi_uv):
        raise ValueError("the pole expansion needs a finite reflecting wall")
    grid = np.linspace(lam_lo, lam_hi, n_scan)
    th = np.array([_prufer_shoot(model, l, 1e-9).y[0, -1] for l in grid])
    lams, amps = [], []
    for n in range(64):
        tgt = math.pi / 2 + n * math.pi
        hit = np.nonzero((th[:-1] - tgt) * (th[1:] - tgt) <= 0)[0]
        if not hit.size:
            continue
        i = hit[0]
        # Newton's method on theta(phi_UV; Lambda) with the carried derivative d theta/d Lambda,
        # kept inside the bracket (bisection where a step would leave it)
        lo, hi = grid[i], grid[i + 1]
        lam = 0.5 * (lo + hi)
        for _ in range(60):
            sol = _prufer_shoot(model, lam)
            f = sol.y[0, -1] - tgt
            if f < 0:
                lo = lam
            else:
                hi = lam
            step = f / sol.y[3, -1]
            new = lam - step
            if not lo < new < hi:
                new = 0.5 * (lo + hi)
            if abs(new - lam) <= 1e-14 * max(1.0, abs(lam)):
                lam = new
                break
            lam = new
        sol = _prufer_shoot(model, lam)
        thb, etab, Psib, thlb = sol.y[:, -1]
        thi, etai, Psii, _ = sol.y[:, -1] if model.phi_in >= model.phi_uv else sol.sol(model.phi_in)
        lams.append(lam)
        amps.append(math.sin(thi) * math.exp(etai - Psii - 2.0 * etab + Psib) / thlb)
        if len(lams) == n_modes:
            break
    return Modes(np.array(lams), np.array(amps))


def cgf_walled(model: Model, s: float, order: int = 4, rtol: float = 1e-10, method: str = "Radau"):
    """K(s) = ln E[e^{sN}] of the first-passage time from phi_in and its first `order` derivatives
    in s, without truncation, for a reflecting wall at phi_UV (finite for s below the slowest decay
    rate Lambda_0).  y = d/dphi ln E[e^{sN}] obeys the Riccati form of the backward equation
    (App. A's equation for the characteristic function at t = -i s),
      (S^2/2)(y' + y^2) + D y = -s,  y(phi_UV) = 0,
    integrated from the wall down to phi_end (the direction in which it is stable), and
    K^(n)(s) = int_{phi_end}^{phi_in} d^n y / ds^n, the s-derivatives obeying the differentiated
    equations.  Returns [K, K', ..., K^(order)]."""
    if not np.isfinite(model.phi_uv):
        raise ValueError("cgf_walled needs a finite reflecting wall")
    ds2 = _scalar_drift_s2(model)
    n1 = order + 1
    binom = [[math.comb(n, k) for k in range(n + 1)] for n in range(n1)]

    def rhs(x, Y):
        D, S2 = ds2(x)
        g = 2.0 / S2
        y = Y[:n1]
        out = np.empty(2 * n1)
        for n in range(n1):
            sq = 0.0
            for k in range(n + 1):
                sq += binom[n][k] * y[k] * y[n - k]
            out[n] = -sq - g * D * y[n] - (g * s if n == 0 else (g if n == 1 else 0.0))
        out[n1:] = y
        return out

    def jac(x, Y):
        D, S2 = ds2(x)
        gD = 2.0 * D / S2
        J = np.zeros((2 * n1, 2 * n1))
        for n in range(n1):
            for k in range(n + 1):
                J[n, k] -= 2.0 * binom[n][k] * Y[n - k]
            J[n, n] -= gD
            J[n1 + n, n] = 1.0
        return J

    def blow_up(x, Y):              # beyond the slowest decay rate y diverges: stop before overflow
        return 1e100 - abs(Y[0]) if math.isfinite(Y[0]) else -1.0
    blow_up.terminal = True

    with np.errstate(over="ignore", invalid="ignore"):
        extra = {"jac": jac} if method in ("Radau", "BDF") else {}
        sol = integrate.solve_ivp(rhs, (model.phi_uv, model.phi_end), np.zeros(2 * n1), method=method,
                                  rtol=rtol, atol=1e-14, dense_output=True, events=blow_up, **extra)
    if not sol.success or sol.status == 1 or not np.all(np.isfinite(sol.y[:, -1])):
        raise ArithmeticError(f"cgf_walled: integration failed at s = {s}: {sol.message}")
    i_end = sol.y[n1:, -1]
    i_in = np.zeros(n1) if model.phi_in >= model.phi_uv else sol.sol(model.phi_in)[n1:]
    return [float(i_in[n] - i_end[n]) for n in range(n1)]


def saddlepoint_walled_reference(model: Model, edges, n_s: int = 120):
    """Bin-averaged log density of N on the simulation's lattice from Daniels' saddle-point density
    with the exact cumulant generating function of `cgf_walled` (no truncation of cumulants), with
    Daniels' second-order factor 1 + lambda_4/8 - 5 lambda_3^2/24 (lambda_k = K^(k)/K''^(k/2)), and
    the size of that factor squared as the reference's error:
    (log P_j, |log(1 + correction)|^2 at the bin centre).  The saddle points are tabulated over
    s up to just below the slowest decay rate (where K' -> infinity) and log p(x) is interpolated
    in x."""
    edges = np.asarray(edges, np.float64)
    _, tau = noise_free_em(model)
    eps = tau - classical_N(model)
    x_lo, x_hi = edges[0] - eps, edges[-1] - eps
    k0 = cgf_walled(model, 0.0, 2)
    # lower end of the s range: K'(s_lo) <= x_lo (bisected below when x_lo lies above the mean)
    if k0[1] > x_lo:
        s_lo = -1.0 / k0[2] * 0.5
        while cgf_walled(model, s_lo, 1)[1] > x_lo:
            s_lo *= 2.0
    else:
        s_lo = None
    # upper end: bracket K'(s) = x_hi, doubling toward the divergence (probed with the implicit
    # Runge-Kutta method, which stops quietly where y diverges)
    def probe(sv):
        try:
            v = cgf_walled(model, sv, 1, rtol=1e-7)[1]
        except ArithmeticError:
            return np.inf
        return v if np.isfinite(v) else np.inf

    s_a, s_b = 0.0, 1.0 / k0[2]
    while probe(s_b) < x_hi:
        s_a, s_b = s_b, 2.0 * s_b
    while s_b - s_a > 1e-5 * max(1.0, abs(s_b)):
        mid = 0.5 * (s_a + s_b)
        if probe(mid) < x_hi:
            s_a = mid
        else:
            s_b = mid
    s_hi = s_b if np.isfinite(probe(s_b)) else s_a
    if s_lo is None:
        a, b = 0.0, s_hi
        while b - a > 1e-5 * max(1.0, abs(b)):
            mid = 0.5 * (a + b)
            if probe(mid) <= x_lo:
                a = mid
            else:
                b = mid
        s_lo = a
    # grid: uniform in s below 0, denser toward s_hi above it
    u = np.linspace(0.0, 1.0, n_s)
    s0 = max(s_lo, 0.0)
    s_grid = s0 + (s_hi - s0) * (1.0 - (1.0 - u) ** 3)
    if s_lo < 0:
        s_grid = np.concatenate([np.linspace(s_lo, 0.0, n_s // 4, endpoint=False), s_grid])
    xs, lp, cr = [], [], []
    for sv in s_grid:
        try:
            K = cgf_walled(model, float(sv), 4, method="LSODA")
            if not (K[2] > 0):
                raise ArithmeticError
        except ArithmeticError:
            K = cgf_walled(model, float(sv), 4)
        if not (K[2] > 0):
            raise ArithmeticError(f"saddlepoint_walled_reference: K''({sv}) = {K[2]}")
        lam3 = K[3] / K[2] ** 1.5
        lam4 = K[4] / K[2] ** 2
        corr = math.log1p(lam4 / 8.0 - 5.0 * lam3 * lam3 / 24.0)
        xs.append(K[1])
        lp.append(K[0] - sv * K[1] - 0.5 * math.log(2.0 * math.pi * K[2]) + corr)
        cr.append(corr)
    xs, lp, cr = np.array(xs), np.array(lp), np.array(cr)
    order = np.argsort(xs)
    xs, lp, cr = xs[order], lp[order], cr[order]
    from scipy.interpolate import CubicSpline
    spl = CubicSpline(xs, lp)
    width = np.log(np.diff(edges))
    out = lattice_logprobs(lambda x: float(spl(x)), model.dN, edges, eps) - width
    centre = 0.5 * (edges[1:] + edges[:-1]) - eps
    return out, np.interp(centre, xs, cr) ** 2


# --------------------------------------------------------------------------
# The zero-variance proposal for a window of first-passage times.
#
# For the event N in (lo, hi], the proposal with zero weight variance is the target process
# conditioned on that event (a Doob h-transform): its drift is D + S^2 d/dphi ln h(phi, n) with
# h(phi, n) = P(N in (lo, hi] | field phi at time n).  From the pole expansion of the
# first-passage density from phi, p(s | phi) = sum_n Lambda_n c_n psi_n(phi) exp(-Lambda_n s)
# (App. A; psi_n(phi_end) = 0, psi_n'(phi_UV) = 0, c_n = <psi_n, 1>_rho / <psi_n, psi_n>_rho),
#   h(phi, n) = sum_n c_n psi_n(phi) [exp(-Lambda_n (lo - n)) - exp(-Lambda_n (hi - n))]
# for n <= lo, and the optimal bias in noise units is r*(phi, n) = S(phi) d/dphi ln h(phi, n).
# Far from the window only the slowest mode survives and r* tends to the quasi-stationary drift
# S psi_0'/psi_0, independent of n.  The truncated sum needs lo - n well above 1/Lambda_1.
# --------------------------------------------------------------------------
@dataclass
class WindowBias:
    lam: np.ndarray     # Lambda_n
    c: np.ndarray       # c_n
    sols: list          # dense shooting solutions (psi_n, psi_n') on [phi_end, phi_UV]
    lo: float
    hi: float
    s2: object          # phi -> S^2 of the target process

    def _terms(self, n):
        n = np.asarray(n, dtype=np.float64)
        return [ck * (np.exp(-lk * (self.lo - n)) - np.exp(-lk * (self.hi - n))) for lk, ck in zip(self.lam, self.c)]

    def h(self, phi, n):
        """Probability of ending in (lo, hi] from phi at time n (n <= lo)."""
        phi = np.asarray(phi, dtype=np.float64)
        return sum(t * sol.sol(phi)[0] for t, sol in zip(self._terms(n), self.sols))

    def r(self, phi, n):
        """The zero-variance bias in noise units, S d/dphi ln h."""
        phi = np.asarray(phi, dtype=np.float64)
        terms = self._terms(n)
        h = sum(t * sol.sol(phi)[0] for t, sol in zip(terms, self.sols))
        dh = sum(t * sol.sol(phi)[1] for t, sol in zip(terms, self.sols))
        S = np.sqrt(np.vectorize(lambda x: self.s2(x)[1])(phi))
        return S * dh / h

    def conditioned_density(self, phi):
        """Density of the field long before the window under the conditioned process:
        rho psi_0^2 (rho = (2/S^2) e^Psi, the weight that makes the generator self-adjoint),
        normalised by the trapezoid rule over the given ascending grid."""
        phi = np.asarray(phi, dtype=np.float64)
        y = self.sols[0].sol(phi)
        s2 = np.vectorize(lambda x: self.s2(x)[1])(phi)
        q = 2.0 / s2 * np.exp(y[2]) * y[0] ** 2
        return q / np.trapezoid(q, phi)


def window_bias(model: Model, lo: float, hi: float, n_modes: int = 6, lam_max: float | None = None,
                n_scan: int = 200) -> WindowBias:
    """The zero-variance bias r*(phi, n) for first passage in (lo, hi] (finite reflecting wall)."""
    if not np.isfinite(model.phi_uv):
        raise ValueError("the pole expansion needs a finite reflecting wall")
    modes = sl_modes(model, n_modes, lam_max=lam_max, n_scan=n_scan)
    sols, cs = [], []
    for lam in modes.lam:
        sol = _shoot(model, lam, dense=True)
        sols.append(sol)
        cs.append(sol.y[3, -1] / sol.y[4, -1])
    return WindowBias(modes.lam, np.array(cs), sols, float(lo), float(hi), _scalar_drift_s2(model))


# --------------------------------------------------------------------------
# Cumulants of N and the Edgeworth expansion (App. B).
#
# The cumulant generating function K(s, phi) = ln E[exp(s N)] of the first-passage time from
# phi satisfies L K + (S^2/2)(K')^2 + s = 0 with L = (S^2/2) d^2 + (D + B) d (the backward
# equation of E[exp(s N)] divided by it), K = 0 at phi_end and K' = 0 at phi_UV.  Order by order
# in s the cumulants solve the same linear problem with sources built from lower orders:
#   L k1 = -1,  L k2 = -S^2 k1'^2,  L k3 = -3 S^2 k1' k2',  L k4 = -S^2 (4 k1' k3' + 3 k2'^2).
# In the integrating-factor form used by `moments` (divide by S^2/2) the sources are
# 2/S^2, 2 k1'^2, 6 k1' k2' and 8 k1' k3' + 6 k2'^2.
# --------------------------------------------------------------------------
@dataclass
class Cumulants:
    k1: float
    k2: float
    k3: float
    k4: float

    @property
    def skewness(self):
        return self.k3 / self.k2 ** 1.5

    @property
    def excess_kurtosis(self):
        return self.k4 / self.k2 ** 2


def cumulants(model: Model, biased: bool = False, n_grid: int = 400001, phi=None) -> Cumulants:
    """The first four cumulants of N from phi (default phi_in), Richardson-extrapolated over grids
    of n and n/2 cells like `moments`."""
    phi = model.phi_in if phi is None else phi

    def solve(n):
        top = _top(model, biased)
        if model.pot != POT_FLAT and model.phi_end > 0:
            x = model.phi_end * np.exp(np.linspace(0.0, math.log(top / model.phi_end), n))
        else:
            x = np.linspace(model.phi_end, top, n)
        D, S, B = drift_noise(model, x, biased)
        psi_p = 2.0 * (D + B) / S ** 2
        xm = 0.5 * (x[1:] + x[:-1])
        Dm, Sm, Bm = drift_noise(model, xm, biased)
        psi_pm = 2.0 * (Dm + Bm) / Sm ** 2
        J1 = _green_derivative(x, psi_p, psi_pm, 2.0 / S ** 2)
        J2 = _green_derivative(x, psi_p, psi_pm, 2.0 * J1 ** 2)
        J3 = _green_derivative(x, psi_p, psi_pm, 6.0 * J1 * J2)
        J4 = _green_derivative(x, psi_p, psi_pm, 8.0 * J1 * J3 + 6.0 * J2 ** 2)
        return [float(np.interp(phi, x, _trapz_cum(x, J))) for J in (J1, J2, J3, J4)]

    a = solve(n_grid)
    b = solve((n_grid - 1) // 2 + 1)
    return Cumulants(*[ai + (ai - bi) / 3.0 for ai, bi in zip(a, b)])


def cumulants_to(model: Model, order: int = 8, biased: bool = False, n_grid: int = 400001, phi=None) -> list:
    """kappa_1 .. kappa_order of N from phi (default phi_in), by the same hierarchy as `cumulants`
    taken to any order.  With g = ln E[e^{sN}] the backward equation of the moment generating
    function (App. A, eq. eq_chracteristic_function_partial_diff_eqn at t = -i s) reads
    (S^2/2)(g'' + g'^2) + (D+B) g' = -s with g(phi_end) = 0, g'(phi_UV) = 0.  Matching powers of
    s in g = sum kappa_n s^n/n! gives L kappa_1 = -1 and, for n >= 2,
    L kappa_n = -(S^2/2) sum_{a=1}^{n-1} binom(n, a) kappa_a' kappa_{n-a}', the cumulants'
    derivatives being Green's-function integrals with these sources.  Richardson-extrapolated over
    grids of n and n/2 cells."""
    phi = model.phi_in if phi is None else phi

    def solve(n):
        top = _top(model, biased)
        if model.pot != POT_FLAT and model.phi_end > 0:
            x = model.phi_end * np.exp(np.linspace(0.0, math.log(top / model.phi_end), n))
        else:
            x = np.linspace(model.phi_end, top, n)
        D, S, B = drift_noise(model, x, biased)
        psi_p = 2.0 * (D + B) / S ** 2
        xm = 0.5 * (x[1:] + x[:-1])
        Dm, Sm, Bm = drift_noise(model, xm, biased)
        psi_pm = 2.0 * (Dm + Bm) / Sm ** 2
        J = [_green_derivative(x, psi_p, psi_pm, 2.0 / S ** 2)]
        for k in range(2, order + 1):
            src = sum(math.comb(k, a) * J[a - 1] * J[k - a - 1] for a in range(1, k))
            J.append(_green_derivative(x, psi_p, psi_pm, src))
        return [float(np.interp(phi, x, _trapz_cum(x, Jk))) for Jk in J]

    a = solve(n_grid)
    b = solve((n_grid - 1) // 2 + 1)
    return [ai + (ai - bi) / 3.0 for ai, bi in zip(a, b)]


def saddlepoint_root(x: float, K1, K2, s0: float = 0.0) -> float:
    """The saddle point: the root of K'(s) = x by Newton's method from s0 (K' is increasing, so
    the root is unique); nan where K'' is not positive along the way."""
    s = s0
    for _ in range(200):
        k2 = K2(s)
        if not (k2 > 0) or not math.isfinite(k2):
            return float("nan")
        ds = (K1(s) - x) / k2
        s -= ds
        if abs(ds) <= 1e-15 * max(1.0, abs(s)):
            break
    return s


def saddlepoint_logpdf_cgf(x: float, K, K1, K2, s0: float = 0.0) -> float:
    """Daniels' saddle-point density (Ann. Math. Stat. 25, 1954) from a cumulant generating
    function: log p(x) = K(s) - s x - log sqrt(2 pi K''(s)) at the root of K'(s) = x, found by
    Newton's method from s0 (K' is increasing, so the root is unique)."""
    s = s0
    for _ in range(200):
        k2 = K2(s)
        if not (k2 > 0) or not math.isfinite(k2):
            return float("nan")             # outside the range where the CGF is convex
        ds = (K1(s) - x) / k2
        s -= ds
        if abs(ds) <= 1e-15 * max(1.0, abs(s)):
            break
    return K(s) - s * x - 0.5 * math.log(2.0 * math.pi * K2(s))


def saddlepoint_logpdf(x: float, kappas) -> float:
    """The saddle-point density with the cumulant generating function truncated after the given
    cumulants, K(s) = sum_n kappa_n s^n / n!.  In the drift-dominated and interim regimes the
    standardised cumulants fall off with their order, so the truncation converges; its effect
    is the difference between successive orders (`saddlepoint_truncation`).  Near the mean this
    is the resummed form of the Edgeworth expansion of App. B built from the same cumulants."""
    kap = [float(k) for k in kappas]
    fact = [math.factorial(n) for n in range(len(kap) + 1)]
    K = lambda s: sum(kap[n] * s ** (n + 1) / fact[n + 1] for n in range(len(kap)))
    K1 = lambda s: sum(kap[n] * s ** n / fact[n] for n in range(len(kap)))
    K2 = lambda s: sum(kap[n] * s ** (n - 1) / fact[n - 1] for n in range(1, len(kap)))
    return saddlepoint_logpdf_cgf(x, K, K1, K2, (x - kap[0]) / kap[1])


def saddlepoint_term_ratio(x: float, kappas) -> float:
    """Ratio of the last two terms of the truncated cumulant series at the saddle point of x,
    kappa_n s / (n kappa_{n-1}) for n = len(kappas): small where the truncation has converged.
    Where it exceeds 0.35 the truncation error is not bounded by the change from the previous
    order (for the inverse Gaussian, whose series has a finite radius, it stops being so near
    half the radius)."""
    kap = [float(k) for k in kappas]
    fact = [math.factorial(n) for n in range(len(kap) + 1)]
    K1 = lambda s: sum(kap[n] * s ** n / fact[n] for n in range(len(kap)))
    K2 = lambda s: sum(kap[n] * s ** (n - 1) / fact[n - 1] for n in range(1, len(kap)))
    s = saddlepoint_root(x, K1, K2, (x - kap[0]) / kap[1])
    n = len(kap)
    return abs(kap[n - 1] * s / (n * kap[n - 2]))


def lattice_logprobs(logpdf, dN: float, edges, eps: float = 0.0, n_gauss: int = 24):
    """log P(e_j < k dN <= e_{j+1}) for k = ceil((N_c + eps)/dN) when N_c has the log-density
    `logpdf`: the bin holds the k with K_j < k <= K_{j+1}, K_j = max{k : k dN <= e_j}, i.e.
    N_c in (K_j dN - eps, K_{j+1} dN - eps], integrated by Gauss-Legendre in log space so that
    far-tail bins do not underflow (the lattice of `lattice_gaussian_probs` for any density).
    -inf for a bin that holds no lattice point."""
    edges = np.asarray(edges, np.float64)
    Kk = np.floor(edges / dN + 1e-9)
    Kk = np.where((Kk + 1) * dN <= edges, Kk + 1, Kk)
    Kk = np.where(Kk * dN > edges, Kk - 1, Kk)
    xg, wg = np.polynomial.legendre.leggauss(n_gauss)
    out = np.full(len(edges) - 1, -np.inf)
    for j, (a, b) in enumerate(zip(Kk[:-1] * dN - eps, Kk[1:] * dN - eps)):
        if b <= a:
            continue
        xs = 0.5 * (a + b) + 0.5 * (b - a) * xg
        lp = np.array([logpdf(float(x)) for x in xs])
        top = lp.max()
        out[j] = top + math.log(0.5 * (b - a) * float(np.sum(wg * np.exp(lp - top))))
    return out


def saddlepoint_reference(model: Model, edges, order: int = 8, n_grid: int = 400001):
    """Bin-averaged log density of N on the simulation's lattice (k = ceil((N_c + eps)/dN), eps
    the noise-free Euler-Maruyama lag) from the saddle-point density with `order` cumulants, and
    its truncation error, twice the change from the previous order:
    (log P_j, 2 |log P_j(order) - log P_j(order - 1)|).  The error is nan (no reference) in bins
    whose centre has a last-term ratio above 0.35 (`saddlepoint_term_ratio`)."""
    kap = cumulants_to(model, order, n_grid=n_grid)
    _, tau = noise_free_em(model)
    eps = tau - classical_N(model)
    edges = np.asarray(edges, np.float64)
    width = np.log(np.diff(edges))
    hi = lattice_logprobs(lambda x: saddlepoint_logpdf(x, kap), model.dN, edges, eps) - width
    lo = lattice_logprobs(lambda x: saddlepoint_logpdf(x, kap[:-1]), model.dN, edges, eps) - width
    centre = 0.5 * (edges[1:] + edges[:-1]) - eps
    q = np.array([saddlepoint_term_ratio(float(c), kap) for c in centre])
    with np.errstate(invalid="ignore"):
        err = 2.0 * np.abs(hi - lo)
    return hi, np.where(q <= 0.35, err, np.nan)


def hermite_he(n: int, x):
    """Probabilists' Hermite polynomials He_3, He_4, He_6 (He_3 = x^3 - 3x: the appendix prints
    x^2 - 1, which is not orthogonal to He_1 under the Gaussian weight)."""
    x = np.asarray(x, np.float64)
    if n == 3:
        return x ** 3 - 3 * x
    if n == 4:
        return x ** 4 - 6 * x ** 2 + 3
    if n == 6:
        return x ** 6 - 15 * x ** 4 + 45 * x ** 2 - 15
    raise ValueError(n)


def gaussian_pdf(N, mu: float, sigma: float):
    z = (np.asarray(N, np.float64) - mu) / sigma
    return np.exp(-0.5 * z * z) / (sigma * math.sqrt(2 * math.pi))


def edgeworth_pdf(N, mu: float, sigma: float, gamma: float, kappa: float):
    """App. B, eq. eq_edgeworth_expansion: the Gaussian times
    1 + gamma/6 He_3 + kappa/24 He_4 + gamma^2/72 He_6 of z = (N - mu)/sigma."""
    z = (np.asarray(N, np.float64) - mu) / sigma
    corr = 1 + gamma / 6 * hermite_he(3, z) + kappa / 24 * hermite_he(4, z) + gamma ** 2 / 72 * hermite_he(6, z)
    return gaussian_pdf(N, mu, sigma) * corr


def edgeworth_for(model: Model, n_grid: int = 400001):
    """(mu, sigma, gamma, kappa) of the target process of `model` from its cumulants."""
    c = cumulants(model, biased=False, n_grid=n_grid)
    return c.k1, math.sqrt(c.k2), c.skewness, c.excess_kurtosis


# --------------------------------------------------------------------------
# Characteristic function of N for quadratic inflation (App. A) with confluent hypergeometric
# functions, its poles and residues, and the branch-cut integral without a wall.
#   v(phi) = V/(24 pi^2) = v0 phi^2, v0 = m^2/(48 pi^2);  alpha(t) = sqrt(1 - 4 i t / v0);
#   f = v^((1+alpha)/4) 1F1((-1-alpha)/4; 1 - alpha/2; -1/v),
#   g = v^((1-alpha)/4) 1F1((-1+alpha)/4; 1 + alpha/2; -1/v);
#   A = f'(phi_UV)/g'(phi_UV), B = f(phi_end)/g(phi_end);
#   chi = B/(B - A) f/f_end - A/(B - A) g/g_end (eq. eq:characteristicFunction:generic).
# mpmath evaluates everything at `dps` digits.
# --------------------------------------------------------------------------
def _fg(alpha, v, deriv: bool, mp):
    """f and g (or their phi-derivatives times phi, using d/dphi = (2v/phi) d/dv) at v."""
    def one(s):
        a = (-1 - s * alpha) / 4
        b = 1 - s * alpha / 2
        z = -1 / v
        pref = v ** ((1 + s * alpha) / 4)
        F = mp.hyp1f1(a, b, z)
        if not deriv:
            return pref * F
        dF = (a / b) * mp.hyp1f1(a + 1, b + 1, z)          # d/dz 1F1(a;b;z)
        # d/dv [v^p F(-1/v)] = p v^(p-1) F + v^p F'(z) / v^2, times 2v (phi d/dphi)
        p = (1 + s * alpha) / 4
        return 2 * v * (p * v ** (p - 1) * F + pref * dF / v ** 2)
    return one(1), one(-1)


def char_function(t, model: Model, phi=None, dps: int = 50):
    """chi(t, phi) of the quadratic model with a reflecting wall (complex t allowed)."""
    import mpmath as mp
    mp.mp.dps = dps
    phi = model.phi_in if phi is None else phi
    v0 = mp.mpf(model.m) ** 2 / (48 * mp.pi ** 2)
    alpha = mp.sqrt(1 - 4j * mp.mpmathify(t) / v0)
    v = lambda x: v0 * mp.mpf(x) ** 2
    fe, ge = _fg(alpha, v(model.phi_end), False, mp)
    fu, gu = _fg(alpha, v(model.phi_uv), True, mp)
    f, g = _fg(alpha, v(phi), False, mp)
    A = fu / gu
    B = fe / ge
    return B / (B - A) * f / fe - A / (B - A) * g / ge


def _vfun(model: Model, mp):
    v0 = mp.mpf(model.m) ** 2 / (48 * mp.pi ** 2)
    return v0, (lambda x: v0 * mp.mpf(x) ** 2)


def pole_q(lam, model: Model, dps: int = 50) -> float:
    """A real function of Lambda whose zeros above v0/4 are the poles Lambda_n = i t_n of chi.
    There alpha is imaginary, f and g are complex conjugates, |A| = |B| = 1, and A = B exactly
    when g'(phi_UV) and g(phi_end) have the same phase modulo pi: this returns the sine of
    their phase difference."""
    import mpmath as mp
    mp.mp.dps = dps
    v0, v = _vfun(model, mp)
    alpha = mp.sqrt(mp.mpc(1 - 4 * mp.mpf(lam) / v0))
    _, ge = _fg(alpha, v(model.phi_end), False, mp)
    _, gu = _fg(alpha, v(model.phi_uv), True, mp)
    z = gu * mp.conj(ge)
    return float(mp.im(z) / abs(z))


def char_poles(model: Model, lam_brackets, dps: int = 50):
    """Poles Lambda_n inside the given brackets (roots of pole_q) with the residues
    a_n(phi_in) = lim (Lambda_n - i t) chi(t) (eq. eq_appendix_residual_numerical), taken on
    t = -i L as the mean of (Lambda_n - L) chi(-i L) at L = Lambda_n (1 -+ 1e-12)."""
    import mpmath as mp
    mp.mp.dps = dps
    out = []
    for lo, hi in lam_brackets:
        root = mp.findroot(lambda L: pole_q(L, model, dps), (mp.mpf(lo), mp.mpf(hi)), solver="illinois",
                           tol=mp.mpf(10) ** (-2 * dps // 3))
        eps = root * mp.mpf("1e-12")
        vals = [(root - L) * char_function(-1j * L, model, dps=dps) for L in (root - eps, root + eps)]
        out.append((float(root), float(mp.re(sum(vals) / 2))))
    return out


def char_function_no_wall(t, model: Model, phi=None, dps: int = 50, alpha=None):
    """chi(t, phi) of the quadratic model without a wall (eq.
    eq_appendix_characteristic_function_infinite_UV): only the g solution stays bounded as
    phi -> infinity, normalised to 1 at phi_end.  On the cut (t = -i y, y > v0/4) pass alpha
    explicitly to choose the side."""
    import mpmath as mp
    mp.mp.dps = dps
    phi = model.phi_in if phi is None else phi
    v0, v = _vfun(model, mp)
    if alpha is None:
        alpha = mp.sqrt(1 - 4j * mp.mpmathify(t) / v0)
    a = (-1 + alpha) / 4
    b = 1 + alpha / 2
    vp, ve = v(phi), v(model.phi_end)
    return (vp / ve) ** ((1 - alpha) / 4) * mp.hyp1f1(a, b, -1 / vp) / mp.hyp1f1(a, b, -1 / ve)


def pdf_no_wall(N: float, model: Model, phi=None, dps: int = 40) -> float:
    """P_phi(N) without a wall from the branch cut of chi (eq. eq_appendix_pdf_infinite_UV).

    chi has no poles here; its cut runs along t = -i y for y > v0/4, where alpha^2 = 1 - 4 y/v0
    is negative.  Inverting with the 1/(2 pi) of eq. eq:PDF:from:chi and wrapping the contour
    round the cut, across which chi jumps by 2 i Im chi, gives
        P(N) = -(1/pi) int_{v0/4}^inf Im chi(-i y) e^{-y N} dy,
    with chi taken on the side where alpha = +i sqrt(4 y/v0 - 1) (the limit from Re t < 0).
    The paper prints the prefactor as 2; the 1/pi follows from its own inversion formula and is
    pinned against simulated runs.  Evaluated with mpmath at `dps` digits; the integrand grows
    with y, so small N (below the bulk of the distribution) is not reachable this way."""
    import mpmath as mp
    mp.mp.dps = dps
    v0, _ = _vfun(model, mp)
    y0 = v0 / 4
    N = mp.mpf(N)

    def f(y):
        kappa = mp.sqrt(4 * y / v0 - 1)
        return mp.im(char_function_no_wall(None, model, phi, dps, alpha=mp.mpc(0, kappa))) * mp.exp(-y * N)

    # breakpoints: the edge of the cut on the scale 1/N, then decades of y
    pts = [y0] + [y0 + c / N for c in (1, 10, 100) if c / N < 1] + [mp.mpf(x) for x in (0.05, 0.5, 2, 6) if x > y0]
    pts = sorted(set(pts)) + [mp.inf]
    return float(-mp.quad(f, pts) / mp.pi)


def char_cumulants(model: Model, h: float = None, dps: int = 60, n_fit: int = 9):
    """The first four cumulants of N as the Taylor coefficients of ln chi(-i s) = ln E[exp(s N)]
    at s = 0, from a polynomial fit through points +-h, +-2h, ... (chi's formula has a removable
    singularity at s = 0 itself)."""
    import mpmath as mp
    mp.mp.dps = dps
    if h is None:
        h = 1e-4 / max(1.0, 10.0)
    pts = [mp.mpf(h) * k for k in range(-n_fit, n_fit + 1) if k != 0]
    vals = [mp.log(mp.re(char_function(-1j * x, model, dps=dps))) for x in pts]
    deg = 8
    A = mp.matrix([[x ** j for j in range(deg + 1)] for x in pts])
    b = mp.matrix(vals)
    c = mp.lu_solve(A.T * A, A.T * b)
    fac = [1, 1, 2, 6, 24]
    return Cumulants(*[float(c[n] * fac[n]) for n in (1, 2, 3, 4)])
