"""Thin ctypes binding of libse2ot.so (the C ABI in include/se2ot.h).

Argument marshalling only: every step of the transport path runs in the HIP
library.  Device arrays are passed as torch tensors on a ROCm device; streams
are torch streams (the current stream by default).  Importing this module
loads the library and raises if it is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libse2ot.so")

SE2_OK = 0
SE2_EINVAL = -1
SE2_ENOMEM = -2
SE2_EHIP = -3
SE2_ENUMERIC = -4
SE2_PENDING = 1
SE2_CONVERGED = 0
SE2_MAX_ITER = 1
SE2_BF16, SE2_F32, SE2_F64, SE2_F32_MFMA = 0, 1, 2, 3
SE2_REQ_OT, SE2_REQ_BARYCENTER = 0, 1

EXPORTED = [
    "se2_init", "se2_strerror", "se2_kernel_build", "se2_kernel_destroy", "se2_kernel_table", "se2_kernel_info",
    "se2_conv", "se2_conv_log", "se2_sinkhorn", "se2_barycenter", "se2_solve_queue_create",
    "se2_request_bytes", "se2_solve_queue_submit", "se2_solve_queue_poll", "se2_solve_queue_wait", "se2_solve_queue_times",
    "se2_solve_queue_stats", "se2_solve_queue_profile", "se2_solve_queue_kernel_time", "se2_solve_queue_destroy",
    "se2_solve_queue_release",
    "se2_lift_field", "se2_project", "se2_split_signed", "se2_jko_step", "se2_gradient_flow",
    "se2_split_signed_noalloc",
]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("ntheta", ctypes.c_int32),
                ("theta_axial", ctypes.c_int32)]


class Metric(ctypes.Structure):
    _fields_ = [("w1", ctypes.c_double), ("w2", ctypes.c_double), ("w3", ctypes.c_double),
                ("eps", ctypes.c_double), ("radius", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("tol_marg_l1", ctypes.c_double), ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("final_check", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("init_g", ctypes.c_void_p), ("eps_start", ctypes.c_double), ("eps_factor", ctypes.c_double),
                ("stage_iters", ctypes.c_int32), ("bulk", ctypes.c_int32), ("polish", ctypes.c_int32),
                ("switch_tol", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("marg_l1", ctypes.c_double),
                ("marg_l1_f64", ctypes.c_double), ("cost", ctypes.c_double), ("mass", ctypes.c_double),
                ("dual", ctypes.c_double), ("seconds", ctypes.c_double), ("terms_dense", ctypes.c_double),
                ("terms_sparse", ctypes.c_double), ("convs", ctypes.c_int32), ("scaling_iters", ctypes.c_int32),
                ("fallbacks", ctypes.c_int32), ("phase_switch_iter", ctypes.c_int32), ("terms_linear", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Flow(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("m", ctypes.c_double), ("ref", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("kernel", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("nu", ctypes.c_void_p), ("mus", ctypes.c_void_p),
                ("lambdas", ctypes.c_void_p), ("opts", Opts), ("f_out", ctypes.c_void_p),
                ("g_out", ctypes.c_void_p), ("bary_out", ctypes.c_void_p)]


class SE2Error(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {code} ({_strerror(code)})")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the library (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2402_15322_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_uint64
        sig = {
            "se2_init": ([], ctypes.c_int),
            "se2_strerror": ([ctypes.c_int], ctypes.c_char_p),
            "se2_kernel_build": ([ctypes.POINTER(Grid), ctypes.POINTER(Metric), ctypes.POINTER(vp)], ctypes.c_int),
            "se2_kernel_destroy": ([vp], ctypes.c_int),
            "se2_kernel_table": ([vp, vp, vp], ctypes.c_int),
            "se2_kernel_info": ([vp, ctypes.POINTER(Grid), ctypes.POINTER(Metric), ctypes.POINTER(i32)], ctypes.c_int),
            "se2_conv": ([vp, ctypes.c_int, vp, vp, i32, vp], ctypes.c_int),
            "se2_conv_log": ([vp, ctypes.c_int, vp, vp, i32, ctypes.POINTER(i32), vp], ctypes.c_int),
            "se2_lift_field": ([ctypes.POINTER(Grid), vp, vp, vp, i32, vp], ctypes.c_int),
            "se2_project": ([ctypes.POINTER(Grid), vp, vp, vp, vp, vp, i32, vp], ctypes.c_int),
            "se2_split_signed": ([vp, sz, vp, vp, vp], ctypes.c_int),
            "se2_split_signed_noalloc": ([vp, sz, vp, vp, vp], ctypes.c_int),
            "se2_jko_step": ([vp, vp, ctypes.POINTER(Flow), ctypes.POINTER(Opts), vp, vp, vp, ctypes.POINTER(Report),
                              vp], ctypes.c_int),
            "se2_gradient_flow": ([vp, vp, ctypes.POINTER(Flow), i32, ctypes.POINTER(Opts), vp, vp,
                                   ctypes.POINTER(Report), vp], ctypes.c_int),
            "se2_sinkhorn": ([vp, vp, vp, ctypes.POINTER(Opts), vp, vp, ctypes.POINTER(Report), vp], ctypes.c_int),
            "se2_barycenter": ([vp, i32, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(Report), vp],
                               ctypes.c_int),
            "se2_request_bytes": ([ctypes.POINTER(Request), ctypes.POINTER(sz)], ctypes.c_int),
            "se2_solve_queue_create": ([sz, i32, ctypes.POINTER(vp)], ctypes.c_int),
            "se2_solve_queue_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(u64)], ctypes.c_int),
            "se2_solve_queue_poll": ([vp, u64, ctypes.POINTER(Report)], ctypes.c_int),
            "se2_solve_queue_wait": ([vp, u64, ctypes.POINTER(Report)], ctypes.c_int),
            "se2_solve_queue_times": ([vp, u64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "se2_solve_queue_stats": ([vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
            "se2_solve_queue_release": ([vp, u64], ctypes.c_int),
            "se2_solve_queue_profile": ([vp, i32], ctypes.c_int),
            "se2_solve_queue_kernel_time": ([vp, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "se2_solve_queue_destroy": ([vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return load().se2_strerror(code).decode()
    except Exception:  # pragma: no cover - only while reporting another failure
        return "?"


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise SE2Error(rc, what)
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous and on the GPU")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def opts(tol: float = 1e-6, max_iter: int = 1000, check_every: int = 10, prec: int = SE2_F32,
         final_check: bool = True, prune: bool = True, init_g=None, eps_start: float = 0.0,
         eps_factor: float = 0.5, stage_iters: int = 0, bulk: Optional[int] = None,
         switch_tol: float = 1e-3) -> Opts:
    """se2_opts_t; eps_start > eps turns on eps-scaling (stage_iters iterations per coarser eps);
    bulk (an engine) turns on a bulk phase on that engine before `prec` (switch at switch_tol)."""
    return Opts(tol, max_iter, check_every, prec, int(final_check), int(prune), _ptr(init_g), float(eps_start),
                float(eps_factor), int(stage_iters), int(bulk) if bulk is not None else 0,
                1 if bulk is not None else 0, float(switch_tol))


def se2_init() -> None:
    _check(load().se2_init(), "se2_init")


class Kernel:
    """Owned handle of se2_kernel_build (destroyed with the object)."""

    def __init__(self, nx: int, ny: int, ntheta: int, axial: bool, w: Sequence[float], eps: float, radius: int):
        self.grid = Grid(nx, ny, ntheta, int(axial))
        self.metric = Metric(float(w[0]), float(w[1]), float(w[2]), float(eps), int(radius))
        h = ctypes.c_void_p()
        _check(load().se2_kernel_build(ctypes.byref(self.grid), ctypes.byref(self.metric), ctypes.byref(h)),
               "se2_kernel_build")
        self.handle = h.value
        self.shape = (ny, nx, ntheta)
        self.W = 2 * radius + 1

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.se2_kernel_destroy(h)
            self.handle = None

    def table(self):
        import numpy as np
        n = self.W * self.W * self.grid.ntheta ** 2
        lk = np.zeros(n)
        ct = np.zeros(n)
        _check(load().se2_kernel_table(self.handle, lk.ctypes.data, ct.ctypes.data), "se2_kernel_table")
        shp = (self.W, self.W, self.grid.ntheta, self.grid.ntheta)
        return lk.reshape(shp), ct.reshape(shp)

    def info(self):
        g, m, nz = Grid(), Metric(), ctypes.c_int32()
        _check(load().se2_kernel_info(self.handle, ctypes.byref(g), ctypes.byref(m), ctypes.byref(nz)),
               "se2_kernel_info")
        return {"nonzero_offsets_bf16": nz.value}


def se2_conv(k: Kernel, prec: int, x, out, stream=None) -> None:
    batch = x.numel() // (k.shape[0] * k.shape[1] * k.shape[2])
    _check(load().se2_conv(k.handle, prec, _ptr(x), _ptr(out), batch, _stream(stream)), "se2_conv")


def se2_conv_log(k: Kernel, prec: int, x, out, stream=None) -> int:
    """out = log(K * exp(x)); returns the groups recomputed in the log domain (matrix-core precisions)."""
    batch = x.numel() // (k.shape[0] * k.shape[1] * k.shape[2])
    fb = ctypes.c_int32(0)
    _check(load().se2_conv_log(k.handle, prec, _ptr(x), _ptr(out), batch, ctypes.byref(fb), _stream(stream)),
           "se2_conv_log")
    return fb.value


def _grid(nx: int, ny: int, nt: int, axial: bool) -> Grid:
    return Grid(int(nx), int(ny), int(nt), int(bool(axial)))


def se2_lift_field(nt: int, axial: bool, mag, angle, out, stream=None) -> None:
    """mag, angle: [..., ny, nx] float64 device tensors; out: [..., ny, nx, nt]."""
    ny, nx = mag.shape[-2], mag.shape[-1]
    batch = mag.numel() // (nx * ny)
    g = _grid(nx, ny, nt, axial)
    _check(load().se2_lift_field(ctypes.byref(g), _ptr(mag), _ptr(angle), _ptr(out), batch, _stream(stream)),
           "se2_lift_field")


def se2_project(axial: bool, u, mass, u_minus=None, argmax=None, angle=None, stream=None) -> None:
    """u (and u_minus): [..., ny, nx, nt] float64; mass, angle: [..., ny, nx] float64; argmax int32."""
    ny, nx, nt = u.shape[-3], u.shape[-2], u.shape[-1]
    batch = u.numel() // (nx * ny * nt)
    g = _grid(nx, ny, nt, axial)
    _check(load().se2_project(ctypes.byref(g), _ptr(u), _ptr(u_minus), _ptr(mass), _ptr(argmax), _ptr(angle), batch,
                              _stream(stream)), "se2_project")


def se2_split_signed(u, plus, minus, stream=None) -> None:
    _check(load().se2_split_signed(_ptr(u), u.numel(), _ptr(plus), _ptr(minus), _stream(stream)), "se2_split_signed")


def se2_split_signed_noalloc(u, plus, minus, stream=None) -> None:
    _check(load().se2_split_signed_noalloc(_ptr(u), u.numel(), _ptr(plus), _ptr(minus), _stream(stream)),
           "se2_split_signed_noalloc")


def se2_sinkhorn(k: Kernel, mu, nu, o: Opts, f_out=None, g_out=None, stream=None) -> dict:
    rep = Report()
    _check(load().se2_sinkhorn(k.handle, _ptr(mu), _ptr(nu), ctypes.byref(o), _ptr(f_out), _ptr(g_out),
                               ctypes.byref(rep), _stream(stream)), "se2_sinkhorn")
    return rep.as_dict()


def se2_jko_step(k: Kernel, mu, tau: float, m: float, ref: float, o: Opts, mu_next, f_out=None, g_out=None,
                 stream=None) -> dict:
    rep = Report()
    fl = Flow(float(tau), float(m), float(ref))
    _check(load().se2_jko_step(k.handle, _ptr(mu), ctypes.byref(fl), ctypes.byref(o), _ptr(mu_next), _ptr(f_out),
                               _ptr(g_out), ctypes.byref(rep), _stream(stream)), "se2_jko_step")
    return rep.as_dict()


def se2_gradient_flow(k: Kernel, mu0, tau: float, m: float, ref: float, nsteps: int, o: Opts, mu_out, traj=None,
                      stream=None) -> List[dict]:
    reps = (Report * int(nsteps))()
    fl = Flow(float(tau), float(m), float(ref))
    _check(load().se2_gradient_flow(k.handle, _ptr(mu0), ctypes.byref(fl), int(nsteps), ctypes.byref(o), _ptr(mu_out),
                                    _ptr(traj), reps, _stream(stream)), "se2_gradient_flow")
    return [r.as_dict() for r in reps]


def se2_barycenter(k: Kernel, mus: Sequence, lambdas: Sequence[float], o: Opts, bary_out, stream=None) -> dict:
    n = len(mus)
    ptrs = (ctypes.c_void_p * n)(*[_ptr(m) for m in mus])
    lam = (ctypes.c_double * n)(*[float(v) for v in lambdas])
    rep = Report()
    _check(load().se2_barycenter(k.handle, n, ptrs, lam, ctypes.byref(o), _ptr(bary_out), ctypes.byref(rep),
                                 _stream(stream)), "se2_barycenter")
    return rep.as_dict()


def ot_request_bytes(k: "Kernel", o: Opts) -> int:
    """Device bytes one OT request occupies in a SolveQueue."""
    r = Request(SE2_REQ_OT, 1, k.handle, None, None, None, None, o, None, None, None)
    b = ctypes.c_size_t()
    _check(load().se2_request_bytes(ctypes.byref(r), ctypes.byref(b)), "se2_request_bytes")
    return b.value


class SolveQueue:
    """se2_solve_queue_*: admission by HBM budget, continuous batching on a worker thread."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        h = ctypes.c_void_p()
        _check(load().se2_solve_queue_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)),
               "se2_solve_queue_create")
        self.handle = h.value
        self._keep = {}

    def submit_ot(self, k: Kernel, mu, nu, o: Opts, f_out=None, g_out=None) -> int:
        r = Request(SE2_REQ_OT, 1, k.handle, _ptr(mu), _ptr(nu), None, None, o, _ptr(f_out), _ptr(g_out), None)
        t = ctypes.c_uint64()
        _check(load().se2_solve_queue_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "submit")
        self._keep[t.value] = (k, mu, nu, f_out, g_out)
        return t.value

    def submit_barycenter(self, k: Kernel, mus: Sequence, lambdas: Sequence[float], o: Opts, bary_out) -> int:
        n = len(mus)
        ptrs = (ctypes.c_void_p * n)(*[_ptr(m) for m in mus])
        lam = (ctypes.c_double * n)(*[float(v) for v in lambdas])
        r = Request(SE2_REQ_BARYCENTER, n, k.handle, None, None, ctypes.cast(ptrs, ctypes.c_void_p),
                    ctypes.cast(lam, ctypes.c_void_p), o, None, None, _ptr(bary_out))
        t = ctypes.c_uint64()
        _check(load().se2_solve_queue_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "submit")
        self._keep[t.value] = (k, list(mus), bary_out)
        return t.value

    def poll(self, ticket: int) -> Optional[dict]:
        rep = Report()
        rc = load().se2_solve_queue_poll(self.handle, ticket, ctypes.byref(rep))
        if rc == SE2_PENDING:
            return None
        _check(rc, "poll")
        return rep.as_dict()

    def wait(self, ticket: int) -> dict:
        rep = Report()
        _check(load().se2_solve_queue_wait(self.handle, ticket, ctypes.byref(rep)), "wait")
        return rep.as_dict()

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        load().se2_solve_queue_times(self.handle, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def release(self, ticket: int) -> None:
        """Forget a finished ticket (its report and times); raises while it still runs."""
        rc = load().se2_solve_queue_release(self.handle, ticket)
        if rc == SE2_PENDING:
            raise SE2Error(rc, "release of a running ticket")
        _check(rc, "release")
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        out = (ctypes.c_int64 * 5)()
        _check(load().se2_solve_queue_stats(self.handle, out), "stats")
        return dict(zip(["admitted", "completed", "rejected", "peak_slots", "steps"], list(out)))

    def profile(self, enable: bool) -> None:
        _check(load().se2_solve_queue_profile(self.handle, int(enable)), "profile")

    def kernel_time(self) -> dict:
        out = (ctypes.c_double * 4)()
        _check(load().se2_solve_queue_kernel_time(self.handle, out), "kernel_time")
        return dict(zip(["seconds", "terms", "launches", "outputs"], list(out)))

    def close(self) -> None:
        if self.handle:
            load().se2_solve_queue_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            self.close()
