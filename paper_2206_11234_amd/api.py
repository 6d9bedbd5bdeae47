"""Python binding over the C ABI: argument marshalling only.

Every step of the path (stepping, binning, merging, estimators) runs in the
HIP kernels of libpyfpt.so.  PyTorch supplies device memory (results, dumps,
workspace) and the stream; numpy views of the returned buffers are built
after the stream has finished.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2206_11234_amd needs a HIP GPU (gfx950); no CPU path exists")
    return torch


def layout(n_bins: int, n_sub: int = 16) -> L.pyfpt_layout:
    lay = L.pyfpt_layout()
    L.check(L.load().pyfpt_result_layout(n_bins, n_sub, ctypes.byref(lay)))
    return lay


@dataclass
class Result:
    """Per-instance outputs (see the layout comment of include/pyfpt.h)."""
    edges: np.ndarray
    n_sub: int
    counts: np.ndarray          # uint64 flat buffer
    values: np.ndarray          # float64 flat buffer
    lay: L.pyfpt_layout = field(repr=False)

    def _c(self, off, n):
        return self.counts[off:off + n]

    def _v(self, off, n):
        return self.values[off:off + n]

    @property
    def n_bins(self):
        return len(self.edges) - 1

    @property
    def n_rows(self):
        return self.n_bins + 4

    @property
    def count(self):
        return self._c(self.lay.count, self.n_rows)

    @property
    def jk_count(self):
        return self._c(self.lay.jk_count, self.n_sub * self.n_rows).reshape(self.n_sub, self.n_rows)

    @property
    def n_traj(self):
        return int(self.counts[self.lay.n_traj])

    @property
    def total_steps(self):
        return int(self.counts[self.lay.total_steps])

    @property
    def lse_w(self):
        return self._v(self.lay.lse_w, self.n_rows)

    @property
    def lse_w2(self):
        return self._v(self.lay.lse_w2, self.n_rows)

    @property
    def jk_lse_w(self):
        return self._v(self.lay.jk_lse_w, self.n_sub * self.n_rows).reshape(self.n_sub, self.n_rows)

    @property
    def mean_lnw(self):
        return self._v(self.lay.mean_lnw, self.n_rows)

    @property
    def m2_lnw(self):
        return self._v(self.lay.m2_lnw, self.n_rows)

    @property
    def m3_lnw(self):
        return self._v(self.lay.m3_lnw, self.n_rows)

    @property
    def m4_lnw(self):
        return self._v(self.lay.m4_lnw, self.n_rows)

    @property
    def log_p(self):
        return self._v(self.lay.log_p, self.n_bins)

    @property
    def rel_err_jk(self):
        return self._v(self.lay.rel_err_jk, self.n_bins)

    @property
    def rel_err_kish(self):
        return self._v(self.lay.rel_err_kish, self.n_bins)

    @property
    def log_p_ln(self):
        return self._v(self.lay.log_p_ln, self.n_bins)

    @property
    def rel_err_ln_lo(self):
        return self._v(self.lay.rel_err_ln_lo, self.n_bins)

    @property
    def rel_err_ln_hi(self):
        return self._v(self.lay.rel_err_ln_hi, self.n_bins)

    @property
    def normal_p(self):
        return self._v(self.lay.normal_p, self.n_bins)

    def lognormal_accepted(self) -> bool:
        """The paper's gate (Sec. 2.4), as the library evaluates it: no bin with a normality
        p-value (n_j >= 8) below 0.5 %."""
        return bool(self.values[self.lay.lognormal_gate] == 1.0)

    @property
    def lse_w_all(self):
        return float(self.values[self.lay.lse_w_all])

    @property
    def lse_w2_all(self):
        return float(self.values[self.lay.lse_w2_all])

    @property
    def lse_wk(self):
        return float(self.values[self.lay.lse_wk])

    @property
    def lse_wk2(self):
        return float(self.values[self.lay.lse_wk2])

    @property
    def sum_k2(self):
        return float(self.values[self.lay.sum_k2])

    @property
    def pearson_r(self):
        return float(self.values[self.lay.pearson_r])

    def ess(self):
        """Kish's effective sample size per bin, as the library computes it."""
        return self._v(self.lay.ess, self.n_bins)


@dataclass
class Dump:
    k: np.ndarray
    lw: np.ndarray
    phi: np.ndarray
    status: np.ndarray
    stride: int


def _f(obj, name, default=0.0):
    return getattr(obj, name, default)


def mlp_struct(params, keep: list) -> L.pyfpt_mlp:
    """Device copy (bfloat16 bits) of a network's parameters and its constants."""
    torch = _torch()
    bits = params.bf16_bits().view(np.int16)
    t = torch.from_numpy(bits.copy()).to(torch.device("cuda", torch.cuda.current_device()))
    keep.append(t)
    m = L.pyfpt_mlp()
    m.params = ctypes.c_void_p(t.data_ptr())
    m.hidden = 64
    m.in_mean[:] = [float(v) for v in params.in_mean]
    m.in_inv_scale[:] = [float(v) for v in params.in_inv_scale]
    m.out_scale = float(params.out_scale)
    m.eval_every = int(params.eval_every)
    return m


def make_instance(inst, n_sub: int, keep: list) -> L.pyfpt_instance:
    edges = np.ascontiguousarray(np.asarray(inst.edges, dtype=np.float64))
    keep.append(edges)
    I = L.pyfpt_instance()
    I.pot = L.pyfpt_potential(int(_f(inst, "pot", 0)), float(_f(inst, "m", 1.0)), float(_f(inst, "a", 0.0)),
                              float(_f(inst, "phi0", 0.0)), float(_f(inst, "w", 1.0)), float(_f(inst, "V0", 1.0)))
    I.bias.kind = int(_f(inst, "bias", 0))
    I.bias.p = int(_f(inst, "p", 1))
    I.bias.A = float(_f(inst, "A", 0.0))
    I.bias.target_N = float(_f(inst, "target_N", 0.0))
    if I.bias.kind == L.BIAS_MLP:
        cache = keep[0] if keep and isinstance(keep[0], dict) else None
        key = id(inst.mlp)
        if cache is not None and key in cache:
            I.bias.mlp = cache[key]
        else:
            I.bias.mlp = mlp_struct(inst.mlp, keep)
            if cache is not None:
                cache[key] = I.bias.mlp
    I.phi_in = float(inst.phi_in)
    I.phi_end = float(inst.phi_end)
    I.phi_uv = float(_f(inst, "phi_uv", math.inf))
    I.phi_esc = float(_f(inst, "phi_esc", 0.0))
    I.dN = float(inst.dN)
    I.n_traj = int(inst.n_traj)
    I.t_first = int(_f(inst, "t_first", 0))
    I.k_max = int(_f(inst, "k_max", 0))
    I.stream = int(_f(inst, "stream", 0))
    I.cost_hint = float(_f(inst, "cost_hint", 0.0))
    I.bins = L.pyfpt_bins(len(edges) - 1, n_sub, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return I


def run_batch(instances, seed: int = 0, *, n_sub: int = 16, block: int = 0, chunk: int = 0, wg_per_cu: int = 0,
              use_graph: bool = False, dump_n: int = 0, dump_stride: int = 1, timing: bool = False,
              torch_workspace: bool = True, noalloc: bool = False):
    """Run a batch of instances in one persistent launch.  Returns (results, dumps, timing_ms).
    noalloc: through pyfpt_run_batch_noalloc (static scratch, no autotuning, no workspace)."""
    torch = _torch()
    lib = L.load()
    keep: list = [{}]          # [0]: device copies of networks shared by several instances
    n = len(instances)
    arr = (L.pyfpt_instance * n)(*[make_instance(i, n_sub, keep) for i in instances])
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream()
    lays, res_t, res = [], [], (L.pyfpt_result * n)()
    for i, inst in enumerate(instances):
        lay = layout(len(inst.edges) - 1, n_sub)
        c = torch.empty(int(lay.n_counts), dtype=torch.int64, device=dev)
        v = torch.empty(int(lay.n_values), dtype=torch.float64, device=dev)
        lays.append(lay)
        res_t.append((c, v))
        res[i] = L.pyfpt_result(c.data_ptr(), v.data_ptr(), 1)
    opt = L.pyfpt_options()
    opt.stream = ctypes.c_void_p(stream.cuda_stream)
    opt.block, opt.chunk, opt.wg_per_cu, opt.use_graph = block, chunk, wg_per_cu, int(use_graph)
    dump_t = None
    if dump_n:
        dump_t = (torch.zeros(n * dump_n, dtype=torch.int32, device=dev),
                  torch.zeros(n * dump_n, dtype=torch.float64, device=dev),
                  torch.zeros(n * dump_n, dtype=torch.float32, device=dev),
                  torch.zeros(n * dump_n, dtype=torch.int32, device=dev))
        opt.dump = L.pyfpt_dump(dump_n, dump_stride, dump_t[0].data_ptr(), dump_t[1].data_ptr(),
                                dump_t[2].data_ptr(), dump_t[3].data_ptr())
    ws_t = None
    if torch_workspace and not noalloc:
        nbytes = ctypes.c_size_t(0)
        L.check(lib.pyfpt_workspace_size(arr, n, ctypes.byref(opt), ctypes.byref(nbytes)))
        ws_t = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        opt.workspace = ctypes.c_void_p(ws_t.data_ptr())
        opt.workspace_bytes = int(nbytes.value)
    tm = (ctypes.c_float * 2)()
    if timing:
        opt.timing_ms = tm
    entry = lib.pyfpt_run_batch_noalloc if noalloc else lib.pyfpt_run_batch
    L.check(entry(arr, n, int(seed), res, ctypes.byref(opt)))
    stream.synchronize()
    results = []
    for i, inst in enumerate(instances):
        c, v = res_t[i]
        results.append(Result(np.asarray(inst.edges, np.float64), n_sub, c.cpu().numpy().view(np.uint64),
                              v.cpu().numpy(), lays[i]))
    dumps = None
    if dump_n:
        k, lw, phi, st = (t.cpu().numpy() for t in dump_t)
        dumps = [Dump(k[i * dump_n:(i + 1) * dump_n].view(np.uint32), lw[i * dump_n:(i + 1) * dump_n],
                      phi[i * dump_n:(i + 1) * dump_n], st[i * dump_n:(i + 1) * dump_n], dump_stride)
                 for i in range(n)]
    del ws_t
    return results, dumps, (list(tm) if timing else None)


def run(inst, seed: int = 0, **kw):
    """Single instance through pyfpt_run_batch (one persistent launch)."""
    results, dumps, tm = run_batch([inst], seed, **kw)
    return results[0], (dumps[0] if dumps else None), tm


def run_single_abi(inst, seed: int = 0, *, n_sub: int = 16, block: int = 512, chunk: int = 1, wg_per_cu: int = 2):
    """The same instance through the pyfpt_run entry point (host result buffers)."""
    _torch()
    lib = L.load()
    keep: list = []
    I = make_instance(inst, n_sub, keep)
    lay = layout(len(inst.edges) - 1, n_sub)
    counts = np.zeros(int(lay.n_counts), np.uint64)
    values = np.zeros(int(lay.n_values), np.float64)
    res = L.pyfpt_result(counts.ctypes.data, values.ctypes.data, 0)
    opt = L.pyfpt_options()
    opt.block, opt.chunk, opt.wg_per_cu = block, chunk, wg_per_cu
    opt.k_max = I.k_max
    opt.phi_esc = I.phi_esc
    opt.stream_id = I.stream
    opt.t_first = I.t_first
    L.check(lib.pyfpt_run(ctypes.byref(I.pot), I.phi_in, I.phi_end, I.phi_uv, I.dN, ctypes.byref(I.bias), I.n_traj,
                          int(seed), ctypes.byref(I.bins), ctypes.byref(res), ctypes.byref(opt)))
    return Result(np.asarray(inst.edges, np.float64), n_sub, counts, values, lay)


def mlp_forward(params, target_N: float, phi, N) -> np.ndarray:
    """r_theta at the given points through pyfpt_mlp_forward (matrix-core evaluation)."""
    torch = _torch()
    keep: list = []
    dev = torch.device("cuda", torch.cuda.current_device())
    m = mlp_struct(params, keep)
    p = torch.as_tensor(np.ascontiguousarray(phi, np.float32), device=dev)
    n_ = torch.as_tensor(np.ascontiguousarray(N, np.float32), device=dev)
    r = torch.empty_like(p)
    stream = torch.cuda.current_stream()
    L.check(L.load().pyfpt_mlp_forward(ctypes.byref(m), float(target_N), ctypes.c_void_p(p.data_ptr()),
                                       ctypes.c_void_p(n_.data_ptr()), ctypes.c_void_p(r.data_ptr()), p.numel(),
                                       ctypes.c_void_p(stream.cuda_stream)))
    stream.synchronize()
    return r.cpu().numpy()


def device_cus() -> int:
    n = ctypes.c_int32(0)
    L.check(L.load().pyfpt_device_cus(ctypes.byref(n)))
    return int(n.value)


COMBINE_NO_EXTRAPOLATION = 16     # PYFPT_COMBINE_NO_EXTRAPOLATION


def combine(results, estimator: int = 2):
    """Multi-bias reconstruction (pyfpt_combine): per-bin inverse-variance combination in
    log P of results sharing the same bins, errors scaled by Birge's ratio where contributors
    disagree; estimator + COMBINE_NO_EXTRAPOLATION adds the lognormal rule n_j >= exp(s^2/2).
    Returns (log_p, err_log, n_used)."""
    n = len(results)
    B = results[0].n_bins
    arr = (L.pyfpt_result * n)()
    keep = []
    for i, r in enumerate(results):
        c = np.ascontiguousarray(r.counts, np.uint64)
        v = np.ascontiguousarray(r.values, np.float64)
        keep += [c, v]
        arr[i] = L.pyfpt_result(c.ctypes.data, v.ctypes.data, 0)
    lp = np.zeros(B)
    el = np.zeros(B)
    nu = np.zeros(B, np.int32)
    L.check(L.load().pyfpt_combine(arr, n, B, results[0].n_sub, int(estimator), _ptr(lp), _ptr(el), _ptr(nu)))
    return lp, el, nu


# ---------------------------------------------------------------------------
# training of the learned proposal
# ---------------------------------------------------------------------------
RECORD_DTYPE = np.dtype([("phi", "<f4"), ("k", "<u4"), ("H", "<f4"), ("pn", "<u4")])


@dataclass
class Records:
    rec: np.ndarray         # RECORD_DTYPE; path i owns rec[off[i]:off[i+1]]
    off: np.ndarray         # uint64, n_paths + 1
    k: np.ndarray           # replayed step counts
    lw: np.ndarray          # replayed ln w
    status: np.ndarray


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def proposal_records(inst, seed: int, t_ids, k, group: int, stride: int = 1) -> Records:
    """Replay the runs t_ids (whose step counts k are known from a dump) under the instance's
    proposal and cut them into records, every stride-th group (pyfpt_proposal_records)."""
    _torch()
    keep: list = [{}]
    I = make_instance(inst, 16, keep)
    t = np.ascontiguousarray(t_ids, np.uint64)
    k = np.asarray(k, np.uint64)
    off = np.zeros(t.size + 1, np.uint64)
    groups = (k + np.uint64(group - 1)) // np.uint64(group)
    off[1:] = np.cumsum((groups + np.uint64(stride - 1)) // np.uint64(stride))
    rec = np.zeros(int(off[-1]), RECORD_DTYPE)
    k_out = np.zeros(t.size, np.uint32)
    lw_out = np.zeros(t.size, np.float64)
    st_out = np.zeros(t.size, np.int32)
    opt = L.pyfpt_options()
    opt.stream = ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    L.check(L.load().pyfpt_proposal_records(ctypes.byref(I), int(seed), _ptr(t), t.size, int(group), int(stride),
                                            _ptr(off),
                                            _ptr(rec), _ptr(k_out), _ptr(lw_out), _ptr(st_out), ctypes.byref(opt)))
    return Records(rec, off, k_out.astype(np.uint64), lw_out, st_out)


def proposal_loss_grad(params, target_N: float, dN: float, theta, recs: Records, lw0, n_total: float,
                       objective: int = 0, temper: float = 1.0, rec_weight: float = 1.0):
    """The objective (0: log M2, 1: cross entropy), its gradient (4481, binary64) and ln w_theta
    per path, from records."""
    _torch()
    keep: list = []
    m = mlp_struct(params, keep)
    th = np.ascontiguousarray(theta, np.float32)
    assert th.size == 4481
    lw0 = np.ascontiguousarray(lw0, np.float64)
    n = recs.off.size - 1
    loss = np.zeros(1)
    grad = np.zeros(4481)
    lwt = np.zeros(n)
    rec = np.ascontiguousarray(recs.rec)
    off = np.ascontiguousarray(recs.off, np.uint64)
    opt = L.pyfpt_options()
    opt.stream = ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    L.check(L.load().pyfpt_proposal_loss_grad(ctypes.byref(m), float(target_N), float(dN), _ptr(th), _ptr(rec),
                                              rec.size, _ptr(off), n, _ptr(lw0), float(n_total), int(objective),
                                              float(temper), float(rec_weight), _ptr(loss),
                                              _ptr(grad), _ptr(lwt), ctypes.byref(opt)))
    return float(loss[0]), grad, lwt


def train_proposal(inst, seed: int, theta, *, window, n_sample: int, rounds: int, steps: int, max_paths: int = 0,
                   lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, objective: int = 0,
                   temper: float = 1.0, stride: int = 1, select: int = 0):
    """Train the learned proposal of `inst` (pyfpt_train_proposal).  Returns (theta, bf16 bits,
    list of per-round report dicts).  select > 0: score the starting network and each round's
    end network on a pilot of that many runs and return the one with the largest window Kish
    ESS."""
    _torch()
    keep: list = [{}]
    I = make_instance(inst, 16, keep)
    th = np.ascontiguousarray(theta, np.float32).copy()
    bf = np.zeros(4481, np.uint16)
    cfg = L.pyfpt_train_config(float(window[0]), float(window[1]), int(n_sample), int(max_paths), int(rounds),
                               int(steps), int(inst.mlp.eval_every), float(lr), float(beta1), float(beta2), float(eps),
                               int(objective), float(temper), int(stride), int(select))
    rep = (L.pyfpt_train_report * rounds)()
    opt = L.pyfpt_options()
    opt.stream = ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    L.check(L.load().pyfpt_train_proposal(ctypes.byref(I), int(seed), ctypes.byref(cfg), _ptr(th), _ptr(bf),
                                          ctypes.cast(rep, ctypes.c_void_p), ctypes.byref(opt)))
    reports = [{f: getattr(r, f) for f, _ in L.pyfpt_train_report._fields_} for r in rep]
    return th, bf, reports
