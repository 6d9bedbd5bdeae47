"""CPU oracle for the importance-sampled first-passage simulation.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py; never by the product package, which shares no
code with it.

Two parts:
  * ``simulate`` -- the per-trajectory Euler-Maruyama loop with the importance
    weight, in C (``fpt_oracle.c``), in a binary32 mirror mode (the step count
    is decided in the kernel's precision) and a binary64 reference mode;
  * ``histogram`` -- the per-bin estimators written out from their plain
    definitions in numpy, binary64: counts and weight sums per bin
    (Sec. 2.1 eq. eq_bin_pdf_reconstrcuted and Sec. 2.2
    eq. eq_bin_pdf_reconstrcuted_weighted_naive), jackknife subsets
    (Sec. 2.1), moments of ln w per bin (Sec. 2.4), and the Kish effective
    sample size of each bin.

``refmath`` holds the binary64 closed forms and quadratures that pin the
simulation (mean and variance of N, Sturm-Liouville tail, Brownian first
passage, lattice Gaussian).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "_liboracle.so")

POT_QUADRATIC, POT_QUADRATIC_BUMP, POT_FLAT = 0, 1, 2
BIAS_NONE, BIAS_NOISE_SCALED, BIAS_POWER, BIAS_MLP = 0, 1, 2, 3
ST_ENDED, ST_CENSORED, ST_ESCAPED = 1, 2, 3
MODE_F32, MODE_F64 = 0, 1
# the binary32 step of MODE_F32 with ln w summed in binary32 (Kahan-compensated, or plainly)
MODE_F32_KAHAN, MODE_F32_SUM = 2, 3


class _Params(ctypes.Structure):
    _fields_ = [
        ("pot_kind", ctypes.c_int),
        ("m", ctypes.c_double), ("a", ctypes.c_double), ("phi0", ctypes.c_double),
        ("w", ctypes.c_double), ("V0", ctypes.c_double),
        ("bias_kind", ctypes.c_int),
        ("A", ctypes.c_double),
        ("p", ctypes.c_int),
        ("phi_in", ctypes.c_double), ("phi_end", ctypes.c_double),
        ("phi_uv", ctypes.c_double), ("phi_esc", ctypes.c_double), ("dN", ctypes.c_double),
        ("k_max", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_uint32),
        ("mlp", ctypes.POINTER(ctypes.c_float)),
        ("in_mean", ctypes.c_float * 3), ("in_inv", ctypes.c_float * 3),
        ("out_scale", ctypes.c_float),
        ("target_N", ctypes.c_double),
        ("eval_every", ctypes.c_int),
    ]


_lib = None


def lib():
    """Load (building first if needed) the C oracle."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_uniform24.argtypes = [ctypes.c_uint32]
        L.oracle_uniform24.restype = ctypes.c_float
        L.oracle_log_f32.argtypes = [ctypes.c_float]
        L.oracle_log_f32.restype = ctypes.c_float
        L.oracle_exp_f32.argtypes = [ctypes.c_float]
        L.oracle_exp_f32.restype = ctypes.c_float
        L.oracle_log_f32_batch.argtypes = [f32p, f32p, ctypes.c_int64]
        L.oracle_exp_f32_batch.argtypes = [f32p, f32p, ctypes.c_int64]
        L.oracle_recip_f32_batch.argtypes = [f32p, f32p, ctypes.c_int64]
        L.oracle_sqrt_f32_batch.argtypes = [f32p, f32p, ctypes.c_int64]
        L.oracle_sincos2pi_f32_batch.argtypes = [f32p, f32p, f32p, ctypes.c_int64]
        L.oracle_normals_f32_batch.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                               ctypes.c_uint32, ctypes.c_uint32, f32p]
        L.oracle_normals_f64_batch.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                               ctypes.c_uint32, ctypes.c_uint32, f64p]
        L.oracle_drift_noise_bias_f32.argtypes = [ctypes.POINTER(_Params), ctypes.c_float, f32p]
        L.oracle_simulate.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_int, u64p, f64p, f64p, i32p,
                                      ctypes.c_int]
        L.oracle_simulate.restype = ctypes.c_int
        L.oracle_mlp_r_batch.argtypes = [ctypes.POINTER(_Params), f32p, f32p, f64p, ctypes.c_int64]
        L.oracle_tanh_act.argtypes = [f32p, f32p, ctypes.c_int64]
        vp = ctypes.c_void_p
        L.oracle_records.argtypes = [ctypes.POINTER(_Params), u64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, u64p,
                                     vp, u64p, f64p, i32p]
        L.oracle_records.restype = ctypes.c_int64
        L.oracle_loss_grad.argtypes = [ctypes.POINTER(_Params), f64p, vp, u64p, ctypes.c_int64, f64p,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double, f64p, f64p,
                                       f64p, f64p]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# --------------------------------------------------------------------------
# Model description (the paper's inputs: V, V', phi_in, phi_end, bias
# amplitude and shape, phi_UV, number of runs; Sec. 2.3 and Sec. 3).
# --------------------------------------------------------------------------
@dataclass
class Model:
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
    phi_end: float = float(np.sqrt(2.0))
    phi_uv: float = float("inf")
    phi_esc: float = 0.0          # 0 -> 100 phi_in without a wall (the paper's "infinite" wall)
    dN: float = 1e-3
    k_max: int = 1 << 20
    stream: int = 0
    mlp: object = None            # MlpParams for the learned bias
    target_N: float = 0.0

    @staticmethod
    def from_instance(inst) -> "Model":
        """The oracle's description of a workload instance (same field names)."""
        return Model(pot=inst.pot, m=inst.m, a=inst.a, phi0=inst.phi0, w=inst.w, V0=inst.V0,
                     bias=inst.bias, A=inst.A, p=inst.p, phi_in=inst.phi_in, phi_end=inst.phi_end,
                     phi_uv=inst.phi_uv, phi_esc=inst.phi_esc, dN=inst.dN, k_max=inst.k_max,
                     stream=inst.stream, mlp=getattr(inst, "mlp", None), target_N=getattr(inst, "target_N", 0.0))

    def esc(self) -> float:
        if np.isfinite(self.phi_uv):
            return float("inf")
        return self.phi_esc if self.phi_esc > 0 else 100.0 * self.phi_in

    def to_c(self, seed: int) -> _Params:
        P = _Params(self.pot, self.m, self.a, self.phi0, self.w, self.V0, self.bias, self.A,
                    self.p, self.phi_in, self.phi_end, self.phi_uv, self.esc(), self.dN,
                    int(self.k_max), int(seed), int(self.stream))
        if self.mlp is not None:
            m = self.mlp
            self._mlp_keep = np.ascontiguousarray(m.values_f32(), np.float32)
            P.mlp = self._mlp_keep.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            P.in_mean[:] = [float(v) for v in m.in_mean]
            P.in_inv[:] = [float(v) for v in m.in_inv_scale]
            P.out_scale = float(m.out_scale)
            P.target_N = float(self.target_N)
            P.eval_every = int(m.eval_every)
        return P


@dataclass
class Trajectories:
    t: np.ndarray       # uint64 trajectory ids
    k: np.ndarray       # uint64 step counts
    lw: np.ndarray      # float64 ln w
    phi: np.ndarray     # float64 final field value
    status: np.ndarray  # int32: 1 ended, 2 censored, 3 escaped
    threads: int = 1


def simulate(model: Model, seed: int, n: int, t0: int = 0, stride: int = 1,
             mode: int = MODE_F32, threads: int = 0) -> Trajectories:
    """Run trajectories t = t0 + i*stride, i < n, one by one."""
    L = lib()
    n = int(n)
    k = np.zeros(n, np.uint64)
    lw = np.zeros(n, np.float64)
    phi = np.zeros(n, np.float64)
    st = np.zeros(n, np.int32)
    P = model.to_c(seed)
    used = L.oracle_simulate(ctypes.byref(P), t0, stride, n, mode, _ptr(k, ctypes.c_uint64),
                             _ptr(lw, ctypes.c_double), _ptr(phi, ctypes.c_double),
                             _ptr(st, ctypes.c_int32), int(threads))
    t = (np.uint64(t0) + np.arange(n, dtype=np.uint64) * np.uint64(stride)).astype(np.uint64)
    return Trajectories(t, k, lw, phi, st, used)


def mlp_r(model: Model, phi, N) -> np.ndarray:
    """The learned bias r at the given (phi, N) points (binary64 with bfloat16 roundings)."""
    phi = np.ascontiguousarray(phi, np.float32)
    N = np.ascontiguousarray(N, np.float32)
    out = np.zeros(phi.size, np.float64)
    P = model.to_c(0)
    lib().oracle_mlp_r_batch(ctypes.byref(P), _ptr(phi, ctypes.c_float), _ptr(N, ctypes.c_float),
                             _ptr(out, ctypes.c_double), phi.size)
    return out


def tanh_act(x) -> np.ndarray:
    """The sampler's activation (binary32 in, binary32 out): tanh as a clamped polynomial,
    accurate to a third of a bfloat16 ulp (see the C source)."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros(x.size, np.float32)
    lib().oracle_tanh_act(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), x.size)
    return y.reshape(x.shape)


# --------------------------------------------------------------------------
# Training of the learned proposal: records of paths drawn from a proposal and
# the loss log M2(theta) with its gradient (see the C source for the derivation).
# --------------------------------------------------------------------------
RECORD_DTYPE = np.dtype([("phi", "<f4"), ("k", "<u4"), ("H", "<f4"), ("pn", "<u4")])


@dataclass
class Records:
    rec: np.ndarray        # RECORD_DTYPE, path i owns rec[off[i]:off[i+1]]
    off: np.ndarray        # uint64, n_paths + 1
    k: np.ndarray          # replayed step counts
    lw: np.ndarray         # replayed ln w under the sampling proposal
    status: np.ndarray


def records(model: Model, seed: int, t_ids, E: int, stride: int = 1) -> Records:
    """Replay the paths t_ids under the model's proposal (binary32 mirror) and cut each into
    records at multiples of E steps, keeping the groups g = 0, stride, 2 stride, ..."""
    L = lib()
    t = np.ascontiguousarray(t_ids, np.uint64)
    n = t.size
    P = model.to_c(seed)
    k = np.zeros(n, np.uint64)
    lw = np.zeros(n, np.float64)
    st = np.zeros(n, np.int32)
    off = np.zeros(n + 1, np.uint64)
    L.oracle_records(ctypes.byref(P), _ptr(t, ctypes.c_uint64), n, int(E), int(stride), _ptr(off, ctypes.c_uint64),
                     None, _ptr(k, ctypes.c_uint64), _ptr(lw, ctypes.c_double), _ptr(st, ctypes.c_int32))
    groups = (k + np.uint64(E - 1)) // np.uint64(E)
    off[1:] = np.cumsum((groups + np.uint64(stride - 1)) // np.uint64(stride))
    rec = np.zeros(int(off[-1]), RECORD_DTYPE)
    bad = L.oracle_records(ctypes.byref(P), _ptr(t, ctypes.c_uint64), n, int(E), int(stride), _ptr(off, ctypes.c_uint64),
                           ctypes.c_void_p(rec.ctypes.data), _ptr(k, ctypes.c_uint64), _ptr(lw, ctypes.c_double),
                           _ptr(st, ctypes.c_int32))
    assert bad == 0
    return Records(rec, off, k, lw, st)


def loss_grad(model: Model, theta, recs: Records, lw0, n_total: float, objective: int = 0, temper: float = 1.0,
              rec_weight: float = 1.0):
    """Objective 0: log M2(theta); objective 1: the cross entropy sum_i c_i ln w_theta,i with
    c_i proportional to w_0,i; temper = beta uses w_0^beta in the path weights.  Returns the
    loss, its gradient (4481) and ln w_theta per path.
    model supplies the input normalisation, out_scale, N* and dN."""
    L = lib()
    th = np.ascontiguousarray(theta, np.float64)
    assert th.size == 4481
    lw0 = np.ascontiguousarray(lw0, np.float64)
    n = recs.off.size - 1
    P = model.to_c(0)
    loss = np.zeros(1)
    grad = np.zeros(4481)
    lwt = np.zeros(n)
    scratch = np.zeros(max(n, 1) * 4481)
    L.oracle_loss_grad(ctypes.byref(P), _ptr(th, ctypes.c_double), ctypes.c_void_p(recs.rec.ctypes.data),
                       _ptr(recs.off, ctypes.c_uint64), n, _ptr(lw0, ctypes.c_double), float(n_total),
                       int(objective), float(temper), float(rec_weight), _ptr(loss, ctypes.c_double), _ptr(grad, ctypes.c_double), _ptr(lwt, ctypes.c_double),
                       _ptr(scratch, ctypes.c_double))
    return float(loss[0]), grad, lwt


def philox(ctr, key):
    L = lib()
    c = np.asarray(ctr, np.uint32).copy()
    kk = np.asarray(key, np.uint32).copy()
    o = np.zeros(4, np.uint32)
    L.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(kk, ctypes.c_uint32), _ptr(o, ctypes.c_uint32))
    return o


def normals_f32(seed: int, stream: int, t: int, j0: int, nj: int) -> np.ndarray:
    out = np.zeros(4 * nj, np.float32)
    lib().oracle_normals_f32_batch(seed, stream, t, j0, nj, _ptr(out, ctypes.c_float))
    return out


def normals_f64(seed: int, stream: int, t: int, j0: int, nj: int) -> np.ndarray:
    out = np.zeros(4 * nj, np.float64)
    lib().oracle_normals_f64_batch(seed, stream, t, j0, nj, _ptr(out, ctypes.c_double))
    return out


def log_f32(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().oracle_log_f32_batch(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), x.size)
    return y


def recip_f32(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().oracle_recip_f32_batch(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), x.size)
    return y


def sqrt_f32(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().oracle_sqrt_f32_batch(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), x.size)
    return y


def exp_f32(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().oracle_exp_f32_batch(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), x.size)
    return y


def sincos2pi_f32(u: np.ndarray):
    u = np.ascontiguousarray(u, np.float32)
    c = np.empty_like(u)
    s = np.empty_like(u)
    lib().oracle_sincos2pi_f32_batch(_ptr(u, ctypes.c_float), _ptr(c, ctypes.c_float),
                                     _ptr(s, ctypes.c_float), u.size)
    return c, s


def drift_noise_bias_f32(model: Model, phi: float):
    out = np.zeros(3, np.float32)
    P = model.to_c(0)
    lib().oracle_drift_noise_bias_f32(ctypes.byref(P), ctypes.c_float(phi), _ptr(out, ctypes.c_float))
    return out


# --------------------------------------------------------------------------
# Per-bin estimators from their plain definitions (binary64).
# --------------------------------------------------------------------------
def _lse(x: np.ndarray) -> float:
    """log(sum(exp(x))) with the maximum factored out; -inf for no terms."""
    if x.size == 0:
        return -np.inf
    mx = np.max(x)
    if not np.isfinite(mx):
        return float(mx)
    return float(mx + np.log(np.sum(np.exp(x - mx))))


@dataclass
class Histogram:
    edges: np.ndarray
    n_traj: int
    n_sub: int
    count: np.ndarray       # [B+4] rows: bins, underflow, overflow, censored, escaped
    lse_w: np.ndarray       # log sum w per row
    lse_w2: np.ndarray      # log sum w^2 per row
    jk_count: np.ndarray    # [n_sub, B+4]
    jk_lse_w: np.ndarray    # [n_sub, B+4]
    mean_lnw: np.ndarray    # per row (nan if empty)
    m2_lnw: np.ndarray      # central moments of ln w per row: (1/n) sum (x - mean)^j
    m3_lnw: np.ndarray
    m4_lnw: np.ndarray
    total_steps: int
    n_completed: int
    lse_w_all: float
    lse_w2_all: float
    lse_wk: float           # log sum w k
    lse_wk2: float          # log sum w k^2
    sum_k: float
    sum_k2: float
    n_per_sub: np.ndarray   # launched runs per jackknife subset
    s2_lnw: np.ndarray = None      # unbiased sample variance of ln w per row (nan if n < 2)
    normal_p: np.ndarray = None    # D'Agostino-Pearson p-value of ln w per row (nan if n < 8)
    pearson_r: float = float("nan")  # Pearson's r of log10 w with N over the ended runs (Sec. 3.4)

    # --- estimators ---
    def widths(self):
        return np.diff(self.edges)

    def lognormal(self):
        """Lognormal estimator of Sec. 2.4: <w_j> = exp(<ln w>_j + s_j^2/2) (eq.
        eq_lognormal_mean_maximum_likelihood), P_hat_j = n_j <w_j> / (n_total Delta_j) (eq.
        eq_lognormal_bin_pdf_reconstrcuted_weighted_maximum_likelihood), and the relative error
        factors |exp(-+u) - 1|, u = sqrt(s^2/n_j + s^4/(2 n_j - 2)) (eq.
        eq_log_normal_bin_pdf_reconstrcuted_error_maximum_likelihood).  s^2 is the unbiased sample
        variance.  Returns (log P_hat, rel_lo, rel_hi) per bin, nan where n_j < 2; rel_hi is +inf
        where u exceeds the binary64 range of exp (a wide ln w over few runs)."""
        B = len(self.edges) - 1
        n = self.count[:B].astype(np.float64)
        s2 = self.s2_lnw[:B]
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            lp = np.log(n) + self.mean_lnw[:B] + 0.5 * s2 - np.log(self.widths()) - np.log(self.n_traj)
            u = np.sqrt(s2 / n + s2 * s2 / (2 * n - 2))
            ok = n >= 2
            return np.where(ok, lp, np.nan), np.where(ok, -np.expm1(-u), np.nan), np.where(ok, np.expm1(u), np.nan)

    def log_p_naive(self):
        """log P_hat_j = log(sum_i w_i / (Delta_j n_total)), n_total = all launched runs."""
        B = len(self.edges) - 1
        return self.lse_w[:B] - np.log(self.widths()) - np.log(self.n_traj)

    def jackknife_rel_err(self):
        """Relative error of P_hat_j from the spread over subsets, rescaled by 1/sqrt(n_sub):
        sd_s(P_hat_j^(s)) / sqrt(n_sub) / P_hat_j, with each subset estimate taken relative to
        P_hat_j, P^(s)/P = exp(lse_s - lse) n_total/n_s (so far-tail values do not underflow)."""
        B = len(self.edges) - 1
        with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
            ratio = np.exp(self.jk_lse_w[:, :B] - self.lse_w[None, :B]) * (self.n_traj / self.n_per_sub[:, None])
            sd = np.std(ratio, axis=0, ddof=1)
            out = sd / np.sqrt(self.n_sub)
        out[~np.isfinite(self.lse_w[:B])] = np.nan
        return out

    def kish_rel_err2(self):
        """sum w^2 / (sum w)^2 - 1/n_total: the delta-method relative variance of P_hat_j."""
        B = len(self.edges) - 1
        with np.errstate(invalid="ignore"):
            return np.exp(self.lse_w2[:B] - 2 * self.lse_w[:B]) - 1.0 / self.n_traj

    def ess(self):
        B = len(self.edges) - 1
        with np.errstate(invalid="ignore"):
            return np.exp(2 * self.lse_w[:B] - self.lse_w2[:B])


COMBINE_NO_EXTRAPOLATION = 16


def combine(hists, estimator: int = 2):
    """Multi-bias reconstruction (Sec. 3.2, 3.3): per bin, the inverse-variance weighted mean of
    log P_hat over the histograms whose estimate is trusted there.  estimator 0: naive P_hat,
    error of log P = the jackknife relative error, trusted if n_j > 400 and n_j > exp(sigma^2);
    1: lognormal P_hat, error u = log(1 + rel_hi), trusted if n_j >= 8 and p >= 0.005; 2: the
    lognormal estimator for a histogram that passes the gate in every bin with a p-value, else
    the naive one; 3: bin by bin, the lognormal estimate where that bin passes the gate
    (n_j >= 8, p >= 0.005), else the naive one under its own rule -- the fallback of Sec. 2.4
    taken per bin.

    Adding COMBINE_NO_EXTRAPOLATION (16) also requires n_j >= exp(s_j^2 / 2) of a lognormal
    estimate: exp(<ln w> + s^2/2) draws its value from ln w near <ln w> + s^2, i.e. s standard
    deviations above the mean, which n draws reach only if s <= sqrt(2 ln n).

    Where several estimates contribute to a bin and scatter more than their errors allow
    (chi^2 = sum w_i (y_i - y_bar)^2 above n - 1), the error of the mean is scaled by
    sqrt(chi^2 / (n - 1)) (Birge's ratio).  Returns (log_p, err_log, n_used)."""
    kind = estimator & ~COMBINE_NO_EXTRAPOLATION
    if kind not in (0, 1, 2, 3):
        raise ValueError("estimator must be 0..3, optionally + COMBINE_NO_EXTRAPOLATION")
    strict = bool(estimator & COMBINE_NO_EXTRAPOLATION)
    B = len(hists[0].edges) - 1
    ys, ws = [], []
    for h in hists:
        est = kind
        pv = h.normal_p[:B]
        if est == 2:
            est = 1 if not np.any(np.isfinite(pv) & (pv < 0.005)) else 0
        n = h.count[:B].astype(np.float64)
        y0 = h.log_p_naive()
        e0 = h.jackknife_rel_err()
        with np.errstate(over="ignore", invalid="ignore"):
            ok0 = (n > 400) & (n > np.exp(h.m2_lnw[:B]))
        y1, _, hi = h.lognormal()
        e1 = np.log1p(hi)
        with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
            ok1 = (n >= 8) & np.isfinite(pv) & (pv >= 0.005)
            if strict:
                s2 = h.m2_lnw[:B] * n / (n - 1)
                ok1 &= n >= np.exp(0.5 * s2)
        if est == 0:
            y, e, ok = y0, e0, ok0
        elif est == 1:
            y, e, ok = y1, e1, ok1
        else:
            y, e, ok = np.where(ok1, y1, y0), np.where(ok1, e1, e0), ok1 | ok0
        with np.errstate(invalid="ignore"):
            ok &= np.isfinite(y) & np.isfinite(e) & (e > 0)
        ws.append(np.where(ok, 1.0 / np.where(ok, e, 1.0) ** 2, 0.0))
        ys.append(np.where(ok, y, 0.0))
    W = np.array(ws)
    Y = np.array(ys)
    used = np.sum(W > 0, axis=0).astype(np.int32)
    sw = W.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.sum(W * Y, axis=0) / sw
        chi2 = np.sum(W * (Y - mean[None, :]) ** 2, axis=0)
        birge = np.where(used > 1, np.sqrt(np.maximum(1.0, chi2 / np.maximum(used - 1, 1))), 1.0)
        return np.where(used > 0, mean, np.nan), np.where(used > 0, birge / np.sqrt(sw), np.nan), used


def bin_rows(k: np.ndarray, status: np.ndarray, dN: float, edges: np.ndarray) -> np.ndarray:
    """Row of each run: bin j with e_j < N <= e_{j+1} (N = k dN); B for N <= e_0;
    B+1 for N > e_B; B+2 censored; B+3 escaped."""
    B = len(edges) - 1
    N = k.astype(np.float64) * dN
    rows = np.searchsorted(edges, N, side="left") - 1   # e_j < N <= e_{j+1}  ->  j
    rows = np.where(N <= edges[0], B, rows)
    rows = np.where(N > edges[-1], B + 1, rows)
    rows = np.where(status == ST_CENSORED, B + 2, rows)
    rows = np.where(status == ST_ESCAPED, B + 3, rows)
    return rows.astype(np.int64)


def histogram(tr: Trajectories, dN: float, edges, n_sub: int = 16, n_traj: int | None = None) -> Histogram:
    edges = np.asarray(edges, np.float64)
    B = len(edges) - 1
    R = B + 4
    n_traj = len(tr.k) if n_traj is None else n_traj
    rows = bin_rows(tr.k, tr.status, dN, edges)
    sub = (tr.t % np.uint64(n_sub)).astype(np.int64)
    count = np.zeros(R, np.int64)
    lse_w = np.full(R, -np.inf)
    lse_w2 = np.full(R, -np.inf)
    jk_count = np.zeros((n_sub, R), np.int64)
    jk_lse_w = np.full((n_sub, R), -np.inf)
    mean = np.full(R, np.nan)
    s2 = np.full(R, np.nan)
    normal_p = np.full(R, np.nan)
    m2 = np.full(R, np.nan)
    m3 = np.full(R, np.nan)
    m4 = np.full(R, np.nan)
    order = np.argsort(rows, kind="stable")
    rs = rows[order]
    bounds = np.searchsorted(rs, np.arange(R + 1))
    for r in range(R):
        idx = order[bounds[r]:bounds[r + 1]]
        if idx.size == 0:
            continue
        x = tr.lw[idx]
        count[r] = idx.size
        lse_w[r] = _lse(x)
        lse_w2[r] = _lse(2.0 * x)
        mu = np.mean(x)
        d = x - mu
        mean[r] = mu
        m2[r] = np.mean(d ** 2)
        m3[r] = np.mean(d ** 3)
        m4[r] = np.mean(d ** 4)
        if idx.size >= 2:
            s2[r] = np.var(x, ddof=1)
        if idx.size >= 8:
            normal_p[r] = _normaltest_p(x)
        s = sub[idx]
        for q in range(n_sub):
            xs = x[s == q]
            jk_count[q, r] = xs.size
            jk_lse_w[q, r] = _lse(xs)
    kf = tr.k.astype(np.float64)
    with np.errstate(divide="ignore"):
        lnk = np.log(kf)
    n_per_sub = np.bincount(sub, minlength=n_sub).astype(np.float64)
    if n_traj != len(tr.k):
        # runs not simulated here (e.g. a sub-range) still count as launched
        n_per_sub = np.full(n_sub, n_traj / n_sub)
    return Histogram(edges, n_traj, n_sub, count, lse_w, lse_w2, jk_count, jk_lse_w,
                     mean, m2, m3, m4, int(tr.k.sum()), int(np.sum(tr.status == ST_ENDED)),
                     _lse(tr.lw), _lse(2 * tr.lw), _lse(tr.lw + lnk), _lse(tr.lw + 2 * lnk),
                     float(kf.sum()), float((kf * kf).sum()), n_per_sub, s2, normal_p,
                     _pearson(tr.lw[tr.status == ST_ENDED] / np.log(10.0), kf[tr.status == ST_ENDED] * dN))


def _pearson(x, y) -> float:
    """Pearson's correlation coefficient (library routine); nan with fewer than two points or
    no spread."""
    if x.size < 2 or np.ptp(x) == 0 or np.ptp(y) == 0:
        return float("nan")
    return float(np.corrcoef(x, y)[0, 1])


def _normaltest_p(x) -> float:
    """p-value of D'Agostino and Pearson's K^2 test (Sec. 2.4 uses it on ln w), as the library
    routine computes it; nan when the sample has no spread."""
    from scipy import stats
    x = np.asarray(x, np.float64)
    if np.ptp(x) == 0:
        return float("nan")
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        return float(stats.normaltest(x).pvalue)
