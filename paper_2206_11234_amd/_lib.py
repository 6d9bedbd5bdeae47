"""ctypes declarations mirroring include/pyfpt.h (argument marshalling only).

Loading fails loudly when libpyfpt.so has not been built: there is no CPU
fallback anywhere in the package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpyfpt.so")

PYFPT_OK, PYFPT_EINVAL, PYFPT_ENOMEM, PYFPT_EDEVICE, PYFPT_EUNSUPPORTED = 0, -1, -2, -3, -4
NOALLOC_SCRATCH_BYTES = 64 << 20   # PYFPT_NOALLOC_SCRATCH_BYTES
POT_QUADRATIC, POT_QUADRATIC_BUMP, POT_FLAT = 0, 1, 2
BIAS_NONE, BIAS_NOISE_SCALED, BIAS_POWER, BIAS_MLP = 0, 1, 2, 3
ST_ENDED, ST_CENSORED, ST_ESCAPED = 1, 2, 3


class pyfpt_potential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_double), ("a", ctypes.c_double),
                ("phi0", ctypes.c_double), ("w", ctypes.c_double), ("V0", ctypes.c_double)]


class pyfpt_mlp(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("hidden", ctypes.c_int32),
                ("in_mean", ctypes.c_float * 3), ("in_inv_scale", ctypes.c_float * 3),
                ("out_scale", ctypes.c_float), ("eval_every", ctypes.c_int32)]


class pyfpt_bias(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_int32), ("A", ctypes.c_double),
                ("target_N", ctypes.c_double), ("mlp", pyfpt_mlp)]


class pyfpt_bins(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("n_sub", ctypes.c_int32),
                ("edges", ctypes.POINTER(ctypes.c_double))]


class pyfpt_instance(ctypes.Structure):
    _fields_ = [("pot", pyfpt_potential), ("bias", pyfpt_bias),
                ("phi_in", ctypes.c_double), ("phi_end", ctypes.c_double), ("phi_uv", ctypes.c_double),
                ("phi_esc", ctypes.c_double), ("dN", ctypes.c_double),
                ("n_traj", ctypes.c_uint64), ("t_first", ctypes.c_uint64), ("k_max", ctypes.c_uint64),
                ("stream", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("cost_hint", ctypes.c_double), ("bins", pyfpt_bins)]


class pyfpt_result(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("values", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class pyfpt_layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_counts", "n_values", "count", "jk_count", "n_traj", "total_steps",
        "lse_w", "lse_w2", "jk_lse_w", "mean_lnw", "m2_lnw", "m3_lnw", "m4_lnw",
        "log_p", "rel_err_jk", "rel_err_kish", "log_p_ln", "rel_err_ln_lo", "rel_err_ln_hi", "normal_p",
        "lse_w_all", "lse_w2_all", "lse_wk", "lse_wk2", "sum_k2", "pearson_r", "ess", "lognormal_gate")]


class pyfpt_dump(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("stride", ctypes.c_uint64), ("k", ctypes.c_void_p),
                ("lw", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class pyfpt_options(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("block", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("dump", pyfpt_dump), ("k_max", ctypes.c_uint64), ("phi_esc", ctypes.c_double),
                ("stream_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("t_first", ctypes.c_uint64),
                ("timing_ms", ctypes.POINTER(ctypes.c_float))]


class pyfpt_record(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_float), ("k", ctypes.c_uint32), ("H", ctypes.c_float), ("path_n", ctypes.c_uint32)]


class pyfpt_train_config(ctypes.Structure):
    _fields_ = [("window_lo", ctypes.c_double), ("window_hi", ctypes.c_double), ("n_sample", ctypes.c_uint64),
                ("max_paths", ctypes.c_int32), ("rounds", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("group", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("objective", ctypes.c_int32),
                ("temper", ctypes.c_float), ("stride", ctypes.c_int32), ("select", ctypes.c_int32)]


class pyfpt_train_report(ctypes.Structure):
    _fields_ = [("n_window", ctypes.c_int32), ("n_used", ctypes.c_int32), ("n_records", ctypes.c_uint64),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double), ("kish_window", ctypes.c_double),
                ("ms_sample", ctypes.c_float), ("ms_records", ctypes.c_float), ("ms_optimise", ctypes.c_float),
                ("selected", ctypes.c_int32), ("pilot_ess", ctypes.c_double)]


# every entry point declared in include/pyfpt.h
EXPORTS = ("pyfpt_result_layout", "pyfpt_bin_thresholds", "pyfpt_run", "pyfpt_run_batch", "pyfpt_run_batch_noalloc",
           "pyfpt_workspace_size",
           "pyfpt_mlp_forward", "pyfpt_combine", "pyfpt_proposal_records", "pyfpt_proposal_loss_grad", "pyfpt_train_proposal",
           "pyfpt_device_cus", "pyfpt_last_error")

_lib = None


class PyfptError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pyfpt error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_11234_amd.build` "
                          "(hipcc, gfx950); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.pyfpt_result_layout.argtypes = [ctypes.c_int32, ctypes.c_int32, P(pyfpt_layout)]
    L.pyfpt_bin_thresholds.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p]
    L.pyfpt_run.argtypes = [P(pyfpt_potential), ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            P(pyfpt_bias), ctypes.c_uint64, ctypes.c_uint64, P(pyfpt_bins), P(pyfpt_result),
                            P(pyfpt_options)]
    L.pyfpt_run_batch.argtypes = [P(pyfpt_instance), ctypes.c_int32, ctypes.c_uint64, P(pyfpt_result),
                                  P(pyfpt_options)]
    L.pyfpt_run_batch_noalloc.argtypes = [P(pyfpt_instance), ctypes.c_int32, ctypes.c_uint64, P(pyfpt_result),
                                          P(pyfpt_options)]
    L.pyfpt_workspace_size.argtypes = [P(pyfpt_instance), ctypes.c_int32, P(pyfpt_options), P(ctypes.c_size_t)]
    L.pyfpt_device_cus.argtypes = [P(ctypes.c_int32)]
    L.pyfpt_mlp_forward.argtypes = [P(pyfpt_mlp), ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    vp = ctypes.c_void_p
    L.pyfpt_combine.argtypes = [P(pyfpt_result), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                vp, vp, vp]
    L.pyfpt_proposal_records.argtypes = [P(pyfpt_instance), ctypes.c_uint64, vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, vp, vp, vp, vp, vp, P(pyfpt_options)]
    L.pyfpt_proposal_loss_grad.argtypes = [P(pyfpt_mlp), ctypes.c_double, ctypes.c_double, vp, vp, ctypes.c_uint64, vp,
                                           ctypes.c_int32, vp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, vp, vp, vp, P(pyfpt_options)]
    L.pyfpt_train_proposal.argtypes = [P(pyfpt_instance), ctypes.c_uint64, P(pyfpt_train_config), vp, vp, vp,
                                       P(pyfpt_options)]
    L.pyfpt_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_int if name != "pyfpt_last_error" else ctypes.c_char_p
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != PYFPT_OK:
        msg = load().pyfpt_last_error().decode(errors="replace")
        raise PyfptError(rc, msg)
