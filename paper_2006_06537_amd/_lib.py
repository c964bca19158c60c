"""ctypes binding of libfifagp.so (argument marshalling only).

Every operation runs in the HIP library; this module turns torch device tensors into
pointers, picks the current HIP stream and raises on non-zero status codes.  Loading
fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfifagp.so")

FP64, MIXED = 0, 1
FG_OK, FG_EINVAL, FG_ENOMEM, FG_ENOTSPD, FG_ETOL, FG_ENOTCONV, FG_EDEVICE = 0, -1, -2, -3, -4, -5, -6
KERNEL_SE, KERNEL_EXP, KERNEL_MATERN32, KERNEL_MATERN52 = 0, 1, 2, 3
STATUS_NAMES = {0: "FG_OK", -1: "FG_EINVAL", -2: "FG_ENOMEM", -3: "FG_ENOTSPD", -4: "FG_ETOL",
                -5: "FG_ENOTCONV", -6: "FG_EDEVICE"}

# names declared in include/fifa_gp.h, in declaration order
EXPORTS = ["hodlr_build", "hodlr_ranks", "hodlr_info", "hodlr_singular_values", "hodlr_entries",
           "hodlr_matvec", "hodlr_factor", "hodlr_factor_prec", "hodlr_solve_refined",
           "hodlr_solve_refined_noalloc",
           "hodlr_solve", "hodlr_logdet", "hodlr_logdet_parts", "hodlr_apply_w",
           "fg_normals", "gp_draw_f", "gp_draw_f_hetero", "gibbs_chain_create", "gibbs_step",
           "gibbs_step_batch", "gibbs_batch_tuning", "gibbs_chain_state", "gibbs_chain_create_grid", "gibbs_chain_create_collapsed",
           "gibbs_chain_inputs",
           "gibbs_predict_inputs", "gibbs_predict",
           "gibbs_predict_stats",
           "tp_chain_create", "tp_step", "tp_chain_state",
           "fg_footprint_bytes", "serve_create", "serve_submit", "serve_poll", "serve_drain",
           "serve_stats", "serve_destroy", "fg_timer_start", "fg_timer_stop", "fg_timer_start_mask", "fg_timer_result", "hodlr_status", "factor_status", "fg_last_error", "hodlr_destroy",
           "factor_destroy", "gibbs_chain_destroy", "tp_chain_destroy"]


class FgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lengthscale", C.c_double), ("nugget", C.c_double)]


class ChainCfg(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ell0", C.c_double), ("nugget", C.c_double),
                ("leaf", C.c_int32), ("tol", C.c_double), ("tau0", C.c_double),
                ("sigf2_0", C.c_double), ("a1", C.c_double), ("b1", C.c_double),
                ("a2", C.c_double), ("b2", C.c_double), ("grid_size", C.c_int32),
                ("grid_center", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("precision", C.c_int32)]


class ChainSnapshot(C.Structure):
    _fields_ = [("iteration", C.c_int64), ("tau", C.c_double), ("sigf2", C.c_double),
                ("ell", C.c_double), ("k", C.c_int32), ("last_proposal", C.c_int32),
                ("last_accept", C.c_int32), ("accepts", C.c_int32), ("logdet_sigma", C.c_double),
                ("yr", C.c_double), ("loglik", C.c_double), ("sse", C.c_double),
                ("q", C.c_double), ("logdet1", C.c_double), ("mh_log_ratio", C.c_double),
                ("status", C.c_int32), ("pcg_iters", C.c_int32), ("pcg_relres", C.c_double),
                ("precision_used", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TpCfg(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("ell0", C.c_double * 8),
                ("nugget", C.c_double), ("leaf", C.c_int32), ("tol", C.c_double),
                ("tau0", C.c_double), ("beta0", C.c_double), ("a1", C.c_double),
                ("b1", C.c_double), ("s_beta", C.c_double), ("grid_size", C.c_int32),
                ("grid_center", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("ncomp", C.c_int32)]


class TpSnapshot(C.Structure):
    _fields_ = [("iteration", C.c_int64), ("tau", C.c_double), ("beta", C.c_double),
                ("sse", C.c_double), ("beta_mean", C.c_double), ("beta_sd", C.c_double),
                ("k", C.c_int32 * 8), ("last_proposal", C.c_int32 * 8),
                ("last_accept", C.c_int32 * 8), ("accepts", C.c_int32 * 8),
                ("ell", C.c_double * 8), ("logdet", C.c_double * 8), ("q", C.c_double * 8),
                ("mh_log_ratio", C.c_double * 8), ("status", C.c_int32), ("ncomp", C.c_int32),
                ("betas", C.c_double * 4), ("beta_means", C.c_double * 4),
                ("beta_sds", C.c_double * 4)]

    def as_dict(self, d):
        out = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            if f in ("betas", "beta_means", "beta_sds"):
                out[f] = list(v)[:max(self.ncomp, 1)]
            else:
                out[f] = list(v)[:d] if hasattr(v, "__len__") else v
        return out


class ServeCfg(C.Structure):
    _fields_ = [("mem_budget", C.c_uint64), ("max_active", C.c_int32)]


class Job(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("n", C.c_int64), ("kind", C.c_int32),
                ("ell0", C.c_double), ("nugget", C.c_double), ("leaf", C.c_int32),
                ("tol", C.c_double), ("tau0", C.c_double), ("sigf2_0", C.c_double),
                ("iters", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("precision", C.c_int32), ("f_out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("snap", ChainSnapshot),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("bytes", C.c_uint64)]


class ServeStats(C.Structure):
    _fields_ = [("pending", C.c_int64), ("outstanding", C.c_int64), ("sweeps", C.c_int64),
                ("peak_bytes", C.c_uint64)]


_lib = None

P = C.c_void_p
DP = C.c_void_p  # device pointers travel as integers
I32, I64, U64, D = C.c_int32, C.c_int64, C.c_uint64, C.c_double


def lib():
    """Load libfifagp.so (raises FileNotFoundError if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is missing: build it with python -m paper_2006_06537_amd.build_lib")
    L = C.CDLL(LIB_PATH)
    sig = {
        "hodlr_build": ([DP, I64, Kernel, I32, D, P, C.POINTER(P)], I32),
        "hodlr_ranks": ([P, C.POINTER(I32), I32, C.POINTER(I32), P], I32),
        "hodlr_info": ([P, C.POINTER(I32), C.POINTER(I64)], I32),
        "hodlr_singular_values": ([P, C.POINTER(D), I32, P], I32),
        "hodlr_entries": ([P, DP, DP, I64, DP, P], I32),
        "hodlr_matvec": ([P, D, D, DP, DP, I32, I64, P], I32),
        "hodlr_factor": ([P, D, D, DP, P, C.POINTER(P)], I32),
        "hodlr_factor_prec": ([P, D, D, DP, I32, P, C.POINTER(P)], I32),
        "hodlr_solve_refined": ([P, P, D, D, DP, DP, I32, I64, D, I32, C.POINTER(I32),
                                 C.POINTER(D), P], I32),
        "hodlr_solve_refined_noalloc": ([P, P, D, D, DP, DP, I32, I64, D, I32, C.POINTER(I32),
                                 C.POINTER(D), P], I32),
        "hodlr_solve": ([P, DP, DP, I32, I64, P], I32),
        "hodlr_logdet": ([P, DP, P], I32),
        "hodlr_logdet_parts": ([P, DP, P], I32),
        "hodlr_apply_w": ([P, I32, I32, DP, DP, I32, I64, P], I32),
        "fg_normals": ([U64, U64, U64, U64, I64, DP, P], I32),
        "gp_draw_f": ([P, P, P, D, D, DP, U64, U64, U64, DP, DP, DP, P], I32),
        "gp_draw_f_hetero": ([P, P, P, DP, DP, U64, U64, U64, I32, DP, DP, P], I32),
        "tp_chain_create": ([C.POINTER(TpCfg), DP, DP, I64, P, C.POINTER(P)], I32),
        "tp_step": ([P, I32, P], I32),
        "tp_chain_state": ([P, C.POINTER(TpSnapshot), DP, P], I32),
        "tp_chain_destroy": ([P], None),
        "gibbs_chain_create": ([C.POINTER(ChainCfg), DP, DP, I64, P, C.POINTER(P)], I32),
        "gibbs_step": ([P, I32, P], I32),
        "gibbs_step_batch": ([C.POINTER(P), I32, I32, I32, I32, P], I32),
        "gibbs_batch_tuning": ([C.POINTER(P), I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(D)], I32),
        "gibbs_chain_state": ([P, C.POINTER(ChainSnapshot), DP, DP, DP, P], I32),
        "gibbs_chain_create_collapsed": ([C.POINTER(ChainCfg), DP, DP, I64, P, C.POINTER(P)], I32),
        "gibbs_chain_create_grid": ([C.POINTER(ChainCfg), DP, DP, I64, P, C.POINTER(P)], I32),
        "gibbs_chain_inputs": ([P, C.POINTER(I64), C.POINTER(I64), DP, DP, P], I32),
        "gibbs_predict_inputs": ([P, DP, I64, I32, P], I32),
        "gibbs_predict_stats": ([P, C.POINTER(I32), C.POINTER(I64)], I32),
        "gibbs_predict": ([P, DP, DP, DP, P], I32),
        "fg_footprint_bytes": ([C.POINTER(ChainCfg), P, I64, C.POINTER(U64)], I32),
        "serve_create": ([C.POINTER(ServeCfg), C.POINTER(P)], I32),
        "serve_submit": ([P, C.POINTER(Job), C.POINTER(U64)], I32),
        "serve_poll": ([P, C.POINTER(Result), I32, C.POINTER(I32)], I32),
        "serve_drain": ([P, D], I32),
        "serve_stats": ([P, C.POINTER(ServeStats)], I32),
        "serve_destroy": ([P], None),
        "fg_timer_start": ([I32], I32),
        "fg_timer_stop": ([C.POINTER(D), C.POINTER(I64), C.POINTER(D)], I32),
        "fg_timer_start_mask": ([C.c_uint32], I32),
        "fg_timer_result": ([I32, C.POINTER(D), C.POINTER(I64), C.POINTER(D)], I32),
        "hodlr_status": ([P, P], I32),
        "factor_status": ([P, P], I32),
        "fg_last_error": ([], C.c_char_p),
        "hodlr_destroy": ([P], None),
        "factor_destroy": ([P], None),
        "gibbs_chain_destroy": ([P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(code):
    if code != FG_OK:
        msg = lib().fg_last_error()
        raise FgError(code, msg.decode() if msg else "")
    return code
