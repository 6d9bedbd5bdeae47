"""Seeded synthetic workloads: model parameters, trajectory counts, bin edges.

This module generates INPUTS only and holds none of the method's arithmetic;
both the product path and the oracle read their inputs from here.

The workloads are the parameter sets of the quadratic-inflation study
(V = m^2 phi^2 / 2 in Planck units, phi_end = sqrt 2 where the first slow-roll
parameter reaches one; Sec. 3) plus a Gaussian-bump variant, in five sizes:

  C1  direct sampling (bias 0), m = 0.01, phi_in = 5, no wall, dN = 1e-3,
      1e4 runs, 100 bins over mu +- 6 sigma;
  C2  fixed bias B = A sqrt(V/3)/(2 pi), A in {1, 2, 4}, dN = 1e-3, 1e6 runs each,
      200 log-spaced tail bins, in a drift-dominated case (m = 0.01,
      phi_in = 10, no wall) and a diffusion-dominated case (m = 1, phi_in = 6,
      reflecting wall at phi_UV = 8);
  C3  a batch of 64 instances drawn from splitmix64(0): phi_in ~ U[3, 12],
      m in {0.01, 0.1, 0.5, 1}, A in {0..6}, wall on (phi_UV = phi_in + 2) or
      off, dN in {1e-3, 5e-4}, 1e6 runs each;
  C4  the learned proposal on the diffusion-dominated case of C2;
  C5  1e9 runs, dN = 1e-4, V = m^2 phi^2/2 [1 + a exp(-(phi - phi0)^2/(2 w^2))]
      with m = 0.05, a = 0.02, phi0 = 4, w = 0.1, phi_in = 8, wall at 12,
      500 tail bins.

The paper measures on no dataset: its workloads are these model parameters.
mu and sigma below are the mean and standard deviation of N from the
stochastic-delta-N double integral (Sec. 2.3, eq. eq:meanN:S:gen and its
variance companion), evaluated once by the oracle's quadrature and frozen
here as inputs (a non-GPU test recomputes them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

POT_QUADRATIC, POT_QUADRATIC_BUMP, POT_FLAT = 0, 1, 2
BIAS_NONE, BIAS_NOISE_SCALED, BIAS_POWER, BIAS_MLP = 0, 1, 2, 3

PHI_END = math.sqrt(2.0)
K_MAX_CAP = 1 << 20


@dataclass
class Instance:
    """One (potential, boundary, bias, step, runs, bins) instance."""
    name: str
    pot: int = POT_QUADRATIC
    m: float = 1.0
    a: float = 0.0
    phi0: float = 0.0
    w: float = 1.0
    V0: float = 1.0
    bias: int = BIAS_NONE
    A: float = 0.0
    p: int = 1
    phi_in: float = 5.0
    phi_end: float = PHI_END
    phi_uv: float = math.inf
    phi_esc: float = 0.0     # 0 -> 100 phi_in when there is no wall
    dN: float = 1e-3
    n_traj: int = 10_000
    k_max: int = K_MAX_CAP
    stream: int = 0
    t_first: int = 0          # first run id: runs t_first .. t_first + n_traj - 1
    cost_hint: float = 0.0    # expected steps per run for the batch queue order (0: the library's estimate)
    edges: np.ndarray = field(default_factory=lambda: np.linspace(0.0, 1.0, 2))
    mlp: object = None        # MlpParams of the learned bias
    target_N: float = 0.0     # N* input of the learned bias

    def esc(self) -> float:
        if math.isfinite(self.phi_uv):
            return math.inf
        return self.phi_esc if self.phi_esc > 0 else 100.0 * self.phi_in


def k_max_rule(mean_target_N: float, dN: float) -> int:
    """Step cap: min(2^20, 64 ceil(<N>_T / dN))."""
    return int(min(K_MAX_CAP, 64 * math.ceil(mean_target_N / dN)))


def log_edges(lo: float, hi: float, n: int) -> np.ndarray:
    return np.geomspace(lo, hi, n + 1)


# Frozen quadrature values (mean, std of N under the target process; for the
# biased cases the sample process).  Recomputed by tests/test_workloads.py.
MU_SIGMA = {
    "C1": (5.750008188, 0.01171994848),
    "C2_drift_T": (24.50013188, 0.09378517290),
    "C2_drift_S_A1": (24.91508881, 0.09733255887),
    "C2_drift_S_A2": (25.34900611, 0.1011358309),
    "C2_drift_S_A4": (26.27994607, 0.1096266994),
    "C2_diff_T": (8.683042051, 2.263832420),
    "C5_T": (15.540996, 0.2406170),
}


def c1() -> Instance:
    mu, sig = MU_SIGMA["C1"]
    return Instance("C1", m=0.01, phi_in=5.0, dN=1e-3, n_traj=10_000,
                    k_max=k_max_rule(mu, 1e-3), edges=np.linspace(mu - 6 * sig, mu + 6 * sig, 101))


def c2(n_traj: int = 1_000_000):
    """The six fixed-bias instances, drift-dominated A = 1, 2, 4 then diffusion-dominated."""
    out = []
    mu_d, _ = MU_SIGMA["C2_drift_T"]
    lo = MU_SIGMA["C2_drift_T"][0] - 6 * MU_SIGMA["C2_drift_T"][1]
    hi = max(MU_SIGMA[f"C2_drift_S_A{A}"][0] + 6 * MU_SIGMA[f"C2_drift_S_A{A}"][1] for A in (1, 2, 4))
    e_drift = log_edges(lo, hi, 200)
    kd = k_max_rule(mu_d, 1e-3)
    for i, A in enumerate((1.0, 2.0, 4.0)):
        out.append(Instance(f"C2_drift_A{int(A)}", m=0.01, phi_in=10.0, bias=BIAS_NOISE_SCALED, A=A,
                            dN=1e-3, n_traj=n_traj, k_max=kd, stream=i, edges=e_drift))
    mu_f, _ = MU_SIGMA["C2_diff_T"]
    kf = k_max_rule(mu_f, 1e-3)
    e_diff = log_edges(0.5, kf * 1e-3, 200)
    for i, A in enumerate((1.0, 2.0, 4.0)):
        out.append(Instance(f"C2_diff_A{int(A)}", m=1.0, phi_in=6.0, phi_uv=8.0, bias=BIAS_NOISE_SCALED,
                            A=A, dN=1e-3, n_traj=n_traj, k_max=kf, stream=3 + i, edges=e_diff))
    return out


# ----------------------------------------------------------------------------
# splitmix64 (Steele, Lea, Flood 2014; the seeding generator of xoshiro):
# state += 0x9E3779B97F4A7C15; z = state; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
# z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31.
# ----------------------------------------------------------------------------
class SplitMix64:
    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53

    def choice(self, seq):
        return seq[self.next() % len(seq)]


def c3(n_traj: int = 1_000_000, n_inst: int = 64, seed: int = 0):
    """64 instances drawn from splitmix64(seed).  k_max uses the classical N_cl =
    (phi_in^2 - phi_end^2)/4 in place of <N>_T; bins are 200 log-spaced over
    [N_cl/4, k_max dN]."""
    rng = SplitMix64(seed)
    out = []
    for i in range(n_inst):
        phi_in = 3.0 + 9.0 * rng.uniform()
        m = rng.choice((0.01, 0.1, 0.5, 1.0))
        A = float(rng.choice((0, 1, 2, 3, 4, 5, 6)))
        wall = rng.choice((True, False))
        dN = rng.choice((1e-3, 5e-4))
        n_cl = (phi_in ** 2 - PHI_END ** 2) / 4.0
        kmax = k_max_rule(n_cl, dN)
        out.append(Instance(f"C3_{i:02d}", m=m, phi_in=phi_in, phi_uv=(phi_in + 2.0) if wall else math.inf,
                            bias=BIAS_NOISE_SCALED if A > 0 else BIAS_NONE, A=A, dN=dN, n_traj=n_traj,
                            k_max=kmax, stream=i, edges=log_edges(0.25 * n_cl, kmax * dN, 200)))
    return out


def c4_instance(params, n_traj: int = 1_000_000, target_N: float = 196.0, stream: int = 0) -> Instance:
    """The learned proposal on the diffusion-dominated case of C2 (m = 1, phi_in = 6, wall at 8),
    aimed at N* (P(N*) ~ 1e-30 near N* = 196 for this potential)."""
    base = c2(n_traj)[3]
    return replace(base, name="C4_mlp", bias=BIAS_MLP, A=0.0, mlp=params, target_N=target_N, stream=stream)


def c4_params(seed: int = 0, scale: float = 1.0, out_scale: float = 1.0, eval_every: int = 4) -> "MlpParams":
    """Network inputs normalised for the C4 case: phi in [sqrt 2, 8], N in [0, 600], N* ~ 200."""
    return MlpParams.random(seed, scale, in_mean=(5.0, 200.0, 200.0), in_inv_scale=(0.4, 0.005, 0.01),
                            out_scale=out_scale, eval_every=eval_every)


def c5(n_traj: int = 1_000_000_000) -> Instance:
    mu, sig = MU_SIGMA["C5_T"]
    kmax = k_max_rule(mu, 1e-4)
    return Instance("C5", pot=POT_QUADRATIC_BUMP, m=0.05, a=0.02, phi0=4.0, w=0.1, phi_in=8.0, phi_uv=12.0,
                    dN=1e-4, n_traj=n_traj, k_max=kmax, edges=log_edges(mu - 6 * sig, mu + 40 * sig, 500))


def c5_multi(amplitudes=(0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0), n_total: int = 1_000_000_000):
    """The large bump-potential run as a multi-bias batch: the runs split evenly over
    noise-scaled amplitudes (A = 0 is direct sampling), one noise stream per amplitude, the same
    500 bins."""
    base = c5(n_total // len(amplitudes))
    return [replace(base, name=f"C5_A{A:g}", bias=BIAS_NOISE_SCALED if A else BIAS_NONE, A=A, stream=i)
            for i, A in enumerate(amplitudes)]


def paper_diffusion(A: float, n_traj: int = 200_000, stream: int = 0) -> Instance:
    """The diffusion-dominated validation case of Sec. 3.1 (Fig. 3): m = 1,
    phi_in = phi_UV = sqrt 42, A in {0, 0.4, 0.8}, 2e5 runs each.  dN is not stated
    in the paper; 1e-3 is used."""
    phi = math.sqrt(42.0)
    return Instance(f"V2_A{A}", m=1.0, phi_in=phi, phi_uv=phi, bias=BIAS_NOISE_SCALED if A else BIAS_NONE,
                    A=A, dN=1e-3, n_traj=n_traj, k_max=K_MAX_CAP, stream=stream,
                    edges=np.linspace(0.0, 80.0, 161))


# ----------------------------------------------------------------------------
# Learned-proposal network parameters (inputs): 3 -> 64 -> 64 -> 1, tanh, bfloat16.
# ----------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    """Round binary32 values to the nearest bfloat16 (ties to even), kept as binary32."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


@dataclass
class MlpParams:
    """4481 parameters in the order W1[64][3], b1[64], W2[64][64], b2[64], w3[64], b3, every
    value a bfloat16 (stored here as binary32), plus the input normalisation and output scale."""
    values: np.ndarray
    in_mean: tuple = (0.0, 0.0, 0.0)
    in_inv_scale: tuple = (1.0, 1.0, 1.0)
    out_scale: float = 1.0
    eval_every: int = 4

    N_PARAMS = 4481

    def values_f32(self) -> np.ndarray:
        return bf16_round(self.values)

    def bf16_bits(self) -> np.ndarray:
        return (self.values_f32().view(np.uint32) >> 16).astype(np.uint16)

    @staticmethod
    def random(seed: int = 0, scale: float = 1.0, **kw) -> "MlpParams":
        """Glorot-uniform weights, zero biases except a small random b3 (seeded numpy)."""
        rng = np.random.default_rng(seed)
        v = np.zeros(4481, np.float32)
        lim1 = scale * np.sqrt(6.0 / (3 + 64))
        lim2 = scale * np.sqrt(6.0 / (64 + 64))
        lim3 = scale * np.sqrt(6.0 / (64 + 1))
        v[0:192] = rng.uniform(-lim1, lim1, 192)
        v[192:256] = rng.uniform(-0.1, 0.1, 64)
        v[256:4352] = rng.uniform(-lim2, lim2, 4096)
        v[4352:4416] = rng.uniform(-0.1, 0.1, 64)
        v[4416:4480] = rng.uniform(-lim3, lim3, 64)
        v[4480] = rng.uniform(-0.1, 0.1)
        return MlpParams(bf16_round(v), **kw)


def flat_well(L: float = 1.5, x: float = 1.0, V0: float = 1.0, dN: float = 1e-3, n_traj: int = 100_000,
              A: float = 0.0, wall: bool = True) -> Instance:
    """Quantum well (constant V, Sec. 3): Brownian motion from x, absorbing at 0,
    reflecting at L (or no wall)."""
    return Instance("flat", pot=POT_FLAT, V0=V0, phi_in=x, phi_end=0.0, phi_uv=L if wall else math.inf,
                    bias=BIAS_NOISE_SCALED if A != 0 else BIAS_NONE, A=A, dN=dN, n_traj=n_traj,
                    edges=np.linspace(0.0, 4000.0, 201))


def with_runs(inst: Instance, n_traj: int) -> Instance:
    return replace(inst, n_traj=n_traj)
