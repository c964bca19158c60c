"""FIFA-GP hot path on MI355X: HODLR build / symmetric factor / solve / log-det,
Algorithm 1 draws and the Gibbs sweep of Moran & Wheeler (arXiv 2006.06537).

Thin Python face of libfifagp.so.  Tensors are torch FP64 tensors on the HIP
device; every call goes straight to the C ABI of include/fifa_gp.h on the current
stream.  Nothing here computes: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import (FP64, MIXED, KERNEL_EXP, KERNEL_SE, KERNEL_MATERN32, KERNEL_MATERN52, ChainCfg, ChainSnapshot, FgError, Job,
                   Kernel, Result, ServeCfg, ServeStats, TpCfg, TpSnapshot, check, lib)

__all__ = ["Hodlr", "Factor", "Chain", "TensorChain", "KernelTimer", "normals", "draw_f",
           "batch_tuning", "BATCH_EAGER", "BATCH_GRAPHS", "BATCH_GROUPED", "BATCH_AUTO",
           "draw_f_hetero", "step_batch", "solve_refined", "Server", "footprint_bytes", "FP64", "MIXED", "KERNEL_SE",
           "KERNEL_EXP", "KERNEL_MATERN32", "KERNEL_MATERN52", "FgError", "lib", "KID_LEAF", "KID_REDUCE", "KID_UPDATE", "KID_WHITEN",
           "KID_PREDICT"]

KID_LEAF, KID_REDUCE, KID_UPDATE, KID_WHITEN, KID_PREDICT = 1, 2, 3, 4, 5
KID_NAMES = {KID_LEAF: "k_leaf", KID_REDUCE: "k_reduce_panel", KID_UPDATE: "k_update_panel",
             KID_WHITEN: "k_whiten", KID_PREDICT: "k_predict_partial"}


class KernelTimer:
    """HIP-event timing of one library kernel over a region (fg_timer_start/stop).
    With `also` (more kernel ids) every listed kernel is timed in the same region
    (fg_timer_start_mask); stop() returns the first kernel's figures and result(kid)
    any listed kernel's."""

    def __init__(self, kernel_id, also=()):
        self.kid = kernel_id
        self.name = KID_NAMES[kernel_id]
        self.kids = [kernel_id] + [k for k in also if k != kernel_id]

    def start(self):
        if len(self.kids) == 1:
            check(lib().fg_timer_start(self.kid))
        else:
            check(lib().fg_timer_start_mask(sum(1 << k for k in self.kids)))

    def stop(self):
        ms, cnt, by = C.c_double(), C.c_int64(), C.c_double()
        check(lib().fg_timer_stop(C.byref(ms), C.byref(cnt), C.byref(by)))
        return self.result(self.kid)

    @staticmethod
    def result(kid):
        ms, cnt, by = C.c_double(), C.c_int64(), C.c_double()
        check(lib().fg_timer_result(kid, C.byref(ms), C.byref(cnt), C.byref(by)))
        return ms.value, cnt.value, by.value


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dev(t, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a float64 tensor on the HIP device")
    if not t.is_contiguous() and t.dim() == 1:
        raise ValueError("expected a contiguous tensor")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"expected {n} rows, got {t.shape[0]}")
    return C.c_void_p(t.data_ptr())


def _cols(t):
    """(nrhs, ld) of a vector or of a column-major block stored as a (nrhs, ld) tensor."""
    if t.dim() == 1:
        return 1, t.shape[0]
    if not t.is_contiguous():
        raise ValueError("multi-column blocks are (nrhs, n) contiguous tensors")
    return t.shape[0], t.shape[1]


class Hodlr:
    """Compressed K~_1 (hodlr_build)."""

    def __init__(self, x, lengthscale, nugget=1e-6, leaf=128, tol=1e-10, kind=KERNEL_SE):
        self.n = int(x.shape[0])
        h = C.c_void_p()
        check(lib().hodlr_build(_dev(x), self.n, Kernel(kind, lengthscale, nugget), leaf, tol,
                                _stream(), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def levels(self):
        L = C.c_int32()
        check(lib().hodlr_info(self._h, C.byref(L), None))
        return L.value

    def ranks(self):
        cnt = C.c_int32()
        nint = (1 << self.levels()) - 1
        buf = (C.c_int32 * max(nint, 1))()
        check(lib().hodlr_ranks(self._h, buf, max(nint, 1), C.byref(cnt), _stream()))
        return [buf[i] for i in range(cnt.value)]

    def singular_values(self, cap=60):
        nint = (1 << self.levels()) - 1
        buf = (C.c_double * max(nint * cap, 1))()
        check(lib().hodlr_singular_values(self._h, buf, cap, _stream()))
        return [[buf[h * cap + j] for j in range(cap)] for h in range(nint)]

    def entries(self, i, j):
        torch = _torch()
        out = torch.empty(i.shape[0], dtype=torch.float64, device=i.device)
        check(lib().hodlr_entries(self._h, C.c_void_p(i.data_ptr()), C.c_void_p(j.data_ptr()),
                                  int(i.shape[0]), _dev(out), _stream()))
        return out

    def matvec(self, v, alpha=1.0, beta=0.0):
        torch = _torch()
        y = torch.empty_like(v)
        nrhs, ld = _cols(v)
        check(lib().hodlr_matvec(self._h, alpha, beta, _dev(v), _dev(y), nrhs, ld, _stream()))
        return y

    def status(self):
        return lib().hodlr_status(self._h, _stream())

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and h.value and _lib._lib is not None:
                _lib._lib.hodlr_destroy(h)
        except Exception:  # interpreter shutdown
            pass
        self._h = None


class Factor:
    """W W' = alpha K~_1 + beta I + diag(d) (hodlr_factor)."""

    def __init__(self, H: Hodlr, alpha=1.0, beta=0.0, diag=None, precision=FP64):
        self.H = H  # keep the matrix alive
        f = C.c_void_p()
        check(lib().hodlr_factor_prec(H.handle, alpha, beta,
                                      _dev(diag) if diag is not None else None, precision,
                                      _stream(), C.byref(f)))
        self._f = f

    @property
    def handle(self):
        return self._f

    def logdet(self):
        torch = _torch()
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        check(lib().hodlr_logdet(self._f, _dev(out), _stream()))
        return out

    def logdet_parts(self):
        """(leaf part, node part) of the log-determinant, as a 2-element device tensor."""
        torch = _torch()
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        check(lib().hodlr_logdet_parts(self._f, _dev(out), _stream()))
        return out

    def solve(self, b):
        torch = _torch()
        x = torch.empty_like(b)
        nrhs, ld = _cols(b)
        check(lib().hodlr_solve(self._f, _dev(b), _dev(x), nrhs, ld, _stream()))
        return x

    def apply(self, v, transpose=False, inverse=False):
        torch = _torch()
        y = torch.empty_like(v)
        nrhs, ld = _cols(v)
        check(lib().hodlr_apply_w(self._f, int(transpose), int(inverse), _dev(v), _dev(y), nrhs,
                                  ld, _stream()))
        return y

    def status(self):
        return lib().factor_status(self._f, _stream())

    def __del__(self):
        f = getattr(self, "_f", None)
        try:
            if f is not None and f.value and _lib._lib is not None:
                _lib._lib.factor_destroy(f)
        except Exception:  # interpreter shutdown
            pass
        self._f = None


def solve_refined(A: Hodlr, F: Factor, alpha, beta, b, rtol=1e-10, maxit=50, noalloc=False,
                  out=None):
    """PCG on (alpha K~_1 + beta I) x = b preconditioned by F; returns (x, iters, relres).
    noalloc: hodlr_solve_refined_noalloc (the library's fixed scratch array, no
    allocation; pass `out` to avoid torch's allocation of x as well)."""
    torch = _torch()
    x = torch.empty_like(b) if out is None else out
    nrhs, ld = _cols(b)
    it, rr = C.c_int32(), C.c_double()
    fn = lib().hodlr_solve_refined_noalloc if noalloc else lib().hodlr_solve_refined
    check(fn(A.handle, F.handle, alpha, beta, _dev(b), _dev(x), nrhs, ld, rtol, maxit,
             C.byref(it), C.byref(rr), _stream()))
    return x, it.value, rr.value


def normals(n, seed, tag, iteration, stream_id):
    torch = _torch()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    check(lib().fg_normals(seed, tag, iteration, stream_id, n, _dev(out), _stream()))
    return out


def draw_f(K1: Hodlr, W1: Factor, WM: Factor, sigf2, tau, y, seed, iteration, stream_id):
    """Algorithm 1: returns (f, r, mu)."""
    torch = _torch()
    f = torch.empty_like(y)
    r = torch.empty_like(y)
    mu = torch.empty_like(y)
    check(lib().gp_draw_f(K1.handle, W1.handle, WM.handle, sigf2, tau, _dev(y), seed, iteration,
                          stream_id, _dev(f), _dev(r), _dev(mu), _stream()))
    return f, r, mu


def draw_f_hetero(K: Hodlr, WK: Factor, WP: Factor, D, y, seed, iteration, stream_id, factor=-1):
    """Algorithm 1.h: returns (f, R); WP must factor K~_1 + diag(1/D)."""
    torch = _torch()
    f = torch.empty_like(y)
    R = torch.empty_like(y)
    check(lib().gp_draw_f_hetero(K.handle, WK.handle, WP.handle, _dev(D), _dev(y), seed,
                                 iteration, stream_id, factor, _dev(f), _dev(R), _stream()))
    return f, R


class TensorChain:
    """Tensor-product surface chain (tp_chain_create / tp_step / tp_chain_state).
    x: (d, n) float64 device tensor in observation order; y: n.  ncomp > 1: a sum of
    that many tensor products; ell0 then holds d values (shared by the components) or
    ncomp * d (factor m = c d + h)."""

    def __init__(self, x, y, ell0, tau0=100.0, beta0=1.0, nugget=1e-6, leaf=128, tol=1e-10,
                 seed=0, stream_id=0, kind=KERNEL_SE, a1=1.0, b1=1.0, s_beta=10.0,
                 grid_size=100, grid_center=50, ncomp=1):
        torch = _torch()
        self.d, self.n = int(x.shape[0]), int(x.shape[1])
        self.ncomp = int(ncomp)
        self.nf = self.d * self.ncomp
        ell0 = [float(v) for v in ell0]
        if len(ell0) == self.d:
            ell0 = ell0 * self.ncomp
        if len(ell0) != self.nf or self.nf > 8:
            raise ValueError("one ell0 per dimension or per factor, at most 8 factors")
        x = x.contiguous()
        e = (C.c_double * 8)(*(ell0 + [0.0] * (8 - self.nf)))
        cfg = TpCfg(kind, self.d, e, nugget, leaf, tol, tau0, beta0, a1, b1, s_beta, grid_size,
                    grid_center, seed, stream_id, self.ncomp)
        c = C.c_void_p()
        check(lib().tp_chain_create(C.byref(cfg), _dev(x.reshape(-1)), _dev(y, self.n), self.n,
                                    _stream(), C.byref(c)))
        self._c = c
        self._torch = torch

    def step(self, iters=1):
        check(lib().tp_step(self._c, iters, _stream()))

    def state(self, with_factors=False):
        snap = TpSnapshot()
        F = None
        if with_factors:
            F = self._torch.empty((self.nf, self.n), dtype=self._torch.float64, device="cuda")
        check(lib().tp_chain_state(self._c, C.byref(snap), _dev(F.reshape(-1)) if F is not None
                                   else None, _stream()))
        out = snap.as_dict(self.nf)
        if F is not None:
            out["F"] = F
        return out

    def __del__(self):
        c = getattr(self, "_c", None)
        try:
            if c is not None and c.value and _lib._lib is not None:
                _lib._lib.tp_chain_destroy(c)
        except Exception:  # interpreter shutdown
            pass
        self._c = None


BATCH_EAGER, BATCH_GRAPHS, BATCH_GROUPED, BATCH_AUTO = 0, 1, 2, 3
BATCH_MODE_NAMES = {0: "eager", 1: "graphs", 2: "grouped", 3: "auto"}


def step_batch(chains, iters=1, nstreams=4, graphs=True, mode=None):
    """gibbs_step_batch over a list of Chain objects.  mode: BATCH_EAGER / _GRAPHS /
    _GROUPED / _AUTO (default: GRAPHS if graphs else EAGER)."""
    if mode is None:
        mode = BATCH_GRAPHS if graphs else BATCH_EAGER
    arr = (C.c_void_p * max(len(chains), 1))(*[c._c for c in chains])
    check(lib().gibbs_step_batch(arr, len(chains), iters, nstreams, int(mode), _stream()))


def batch_tuning(chains):
    """The autotuner's choice for this batch: (mode name or None while tuning, streams,
    ms per timed trial sweep)."""
    arr = (C.c_void_p * max(len(chains), 1))(*[c._c for c in chains])
    m, ns, ms = C.c_int32(), C.c_int32(), C.c_double()
    check(lib().gibbs_batch_tuning(arr, len(chains), C.byref(m), C.byref(ns), C.byref(ms)))
    return (BATCH_MODE_NAMES.get(m.value), ns.value, ms.value)


def footprint_bytes(x, ell0, leaf=128, tol=1e-10, nugget=1e-6, kind=KERNEL_SE, precision=FP64,
                    grid_size=100, grid_center=50):
    """fg_footprint_bytes for host inputs x (numpy, sorted): device bytes of a chain."""
    import numpy as np
    xh = np.ascontiguousarray(x, dtype=np.float64)
    cfg = ChainCfg(kind, ell0, nugget, leaf, tol, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, grid_size,
                   grid_center, 0, 0, precision)
    out = C.c_uint64()
    check(lib().fg_footprint_bytes(C.byref(cfg), C.c_void_p(xh.ctypes.data), xh.size,
                                   C.byref(out)))
    return out.value


class Server:
    """Serving loop (serve_create / serve_submit / serve_poll / serve_drain).  Jobs are
    host numpy arrays; the server copies them at submission."""

    def __init__(self, mem_budget, max_active=32):
        cfg = ServeCfg(int(mem_budget), max_active)
        s = C.c_void_p()
        check(lib().serve_create(C.byref(cfg), C.byref(s)))
        self._s = s
        self._keep = {}  # f buffers of jobs not yet polled

    def submit(self, x, y, ell0, iters, tau0=100.0, sigf2_0=1.0, nugget=1e-6, leaf=128,
               tol=1e-10, seed=0, stream_id=0, kind=KERNEL_SE, precision=FP64, want_f=True):
        import numpy as np
        xh = np.ascontiguousarray(x, dtype=np.float64)
        yh = np.ascontiguousarray(y, dtype=np.float64)
        f = np.empty_like(xh) if want_f else None
        job = Job(C.c_void_p(xh.ctypes.data), C.c_void_p(yh.ctypes.data), xh.size, kind, ell0,
                  nugget, leaf, tol, tau0, sigf2_0, iters, seed, stream_id, precision,
                  C.c_void_p(f.ctypes.data) if f is not None else None)
        jid = C.c_uint64()
        check(lib().serve_submit(self._s, C.byref(job), C.byref(jid)))
        self._keep[jid.value] = f
        return jid.value

    def poll(self, max_results=1024):
        buf = (Result * max_results)()
        got = C.c_int32()
        check(lib().serve_poll(self._s, buf, max_results, C.byref(got)))
        out = []
        for i in range(got.value):
            r = buf[i]
            d = {"id": r.id, "status": r.status, "t_submit": r.t_submit, "t_admit": r.t_admit,
                 "t_done": r.t_done, "bytes": r.bytes}
            d.update(r.snap.as_dict())
            d["f"] = self._keep.pop(r.id, None)
            out.append(d)
        return out

    def drain(self, timeout=600.0):
        check(lib().serve_drain(self._s, timeout))

    def stats(self):
        st = ServeStats()
        check(lib().serve_stats(self._s, C.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        s = getattr(self, "_s", None)
        try:
            if s is not None and s.value and _lib._lib is not None:
                _lib._lib.serve_destroy(s)
        except Exception:  # interpreter shutdown
            pass
        self._s = None

    def __del__(self):
        self.close()


class Chain:
    """One Gibbs chain (gibbs_chain_create / gibbs_step / gibbs_chain_state)."""

    def __init__(self, x, y, ell0, tau0, sigf2_0=1.0, nugget=1e-6, leaf=128, tol=1e-10,
                 seed=0, stream_id=0, kind=KERNEL_SE, priors=(1.0, 1.0, 1.0, 1.0),
                 grid_size=100, grid_center=50, precision=FP64, collapse=False, exact_rho=False):
        """collapse=True: repeated inputs are merged (gibbs_chain_create_collapsed) and the
        chain runs on the unique inputs (self.n of them; self.n_obs observations).
        exact_rho=True: the length-scale is drawn from its exact grid conditional
        (gibbs_chain_create_grid)."""
        if collapse and exact_rho:
            raise ValueError("collapse and exact_rho are separate chain kinds")
        m = int(x.shape[0])
        cfg = ChainCfg(kind, ell0, nugget, leaf, tol, tau0, sigf2_0, priors[0], priors[1],
                       priors[2], priors[3], grid_size, grid_center, seed, stream_id, precision)
        c = C.c_void_p()
        create = (lib().gibbs_chain_create_collapsed if collapse else
                  lib().gibbs_chain_create_grid if exact_rho else lib().gibbs_chain_create)
        check(create(C.byref(cfg), _dev(x, m), _dev(y, m), m, _stream(), C.byref(c)))
        self._c = c
        u, nobs = C.c_int64(), C.c_int64()
        check(lib().gibbs_chain_inputs(c, C.byref(u), C.byref(nobs), None, None, _stream()))
        self.n, self.n_obs = u.value, nobs.value

    def inputs(self):
        """(inputs, counts) of the chain on the device."""
        torch = _torch()
        xo = torch.empty(self.n, dtype=torch.float64, device="cuda")
        wo = torch.empty_like(xo)
        check(lib().gibbs_chain_inputs(self._c, None, None, _dev(xo), _dev(wo), _stream()))
        return xo, wo

    def step(self, iters=1):
        check(lib().gibbs_step(self._c, iters, _stream()))

    def state(self, with_vectors=False):
        torch = _torch()
        snap = ChainSnapshot()
        if with_vectors:
            f = torch.empty(self.n, dtype=torch.float64, device="cuda")
            r = torch.empty_like(f)
            mu = torch.empty_like(f)
            check(lib().gibbs_chain_state(self._c, C.byref(snap), _dev(f), _dev(r), _dev(mu),
                                          _stream()))
            d = snap.as_dict()
            d.update(f=f, r=r, mu=mu)
            return d
        check(lib().gibbs_chain_state(self._c, C.byref(snap), None, None, None, _stream()))
        return snap.as_dict()

    def predict_inputs(self, xstar, max_grid_points=4):
        """Set the new inputs of predict() (gibbs_predict_inputs); None clears them.  Z is
        kept for up to max_grid_points length-scale grid points (8 n m bytes each)."""
        if xstar is None:
            check(lib().gibbs_predict_inputs(self._c, None, 0, 1, _stream()))
            self.nstar = 0
            return
        m = int(xstar.shape[0])
        check(lib().gibbs_predict_inputs(self._c, _dev(xstar, m), m, int(max_grid_points),
                                         _stream()))
        self.nstar = m

    def predict_stats(self):
        """(grid points with Z cached, Z computations so far)."""
        k = C.c_int32()
        b = C.c_int64()
        check(lib().gibbs_predict_stats(self._c, C.byref(k), C.byref(b)))
        return k.value, b.value

    def predict(self):
        """One draw of f at the new inputs (gibbs_predict): (f*, mu*, s2*) on the device."""
        torch = _torch()
        m = getattr(self, "nstar", 0)
        fs = torch.empty(max(m, 1), dtype=torch.float64, device="cuda")
        mu = torch.empty_like(fs)
        s2 = torch.empty_like(fs)
        check(lib().gibbs_predict(self._c, _dev(fs), _dev(mu), _dev(s2), _stream()))
        return fs[:m], mu[:m], s2[:m]

    def __del__(self):
        c = getattr(self, "_c", None)
        try:
            if c is not None and c.value and _lib._lib is not None:
                _lib._lib.gibbs_chain_destroy(c)
        except Exception:  # interpreter shutdown
            pass
        self._c = None
