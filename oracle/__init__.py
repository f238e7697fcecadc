"""FP64 CPU oracle for entropic OT on SE(2) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never loads it and shares no code with it.

`se2_oracle.c` holds the arithmetic (FP64, log domain, OpenMP over output
pixels); this module builds it with gcc and wraps it with ctypes.  `dense.py`
holds an independent dense-matrix checker for tiny grids.

Paper references (arXiv 2402.15322): group law Section 2.3; rho_b Section 4.3;
group convolution Section 4.2; Sinkhorn Section 4.1; IBP barycenter Appendix A.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "se2_oracle.c")
_LIB = os.path.join(_HERE, "libse2oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str) -> ctypes.CDLL:
    """Load an oracle build from `path` with its ctypes signatures set.  `lib()` uses
    it for the normal build; the mutation tests load deliberately broken builds."""
    L = ctypes.CDLL(path)
    i, d = ctypes.c_int, ctypes.c_double
    L.oc_rho2.restype = d
    L.oc_rho2.argtypes = [d, d, d, d, d, d]
    L.oc_half_angle.restype = None
    L.oc_half_angle.argtypes = [d, d, d, _D]
    L.oc_kernel_table.restype = None
    L.oc_kernel_table.argtypes = [i, i, d, d, d, d, i, _D, _D]
    for fn in (L.oc_conv_log, L.oc_conv_linear):
        fn.restype = None
        fn.argtypes = [i, i, i, i, _D, _D, _D]
    L.oc_sinkhorn.restype = i
    L.oc_sinkhorn.argtypes = [i, i, i, i, _D, _D, _D, _D, i, d, _D, _D, _D, _D]
    L.oc_ibp.restype = i
    L.oc_ibp.argtypes = [i, i, i, i, _D, i, _D, _D, i, d, _D, _D, _D, _D, _D]
    L.oc_plan_stats.restype = None
    L.oc_plan_stats.argtypes = [i, i, i, i, _D, _D, _D, _D, _D, _D, _D, _D]
    L.oc_plan_l1.restype = d
    L.oc_plan_l1.argtypes = [i, i, i, i, _D, _D, _D, _D, _D]
    L.oc_num_threads.restype = i
    L.oc_num_threads.argtypes = []
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def num_threads() -> int:
    return int(lib().oc_num_threads())


def rho2(x: float, y: float, theta: float, w: Sequence[float]) -> float:
    """rho_b(g)^2 for g = (x, y, theta) (Section 4.3)."""
    return float(lib().oc_rho2(x, y, theta, *w))


def half_angle(x: float, y: float, theta: float) -> np.ndarray:
    b = np.zeros(3)
    lib().oc_half_angle(x, y, theta, _p(b))
    return b


def kernel_table(nt: int, axial: bool, w: Sequence[float], eps: float, R: int) -> Tuple[np.ndarray, np.ndarray]:
    """(logk, cost) over the window, shape [2R+1][2R+1][nt][nt], (dx,dy) = out - in."""
    W = 2 * R + 1
    logk = np.zeros((W, W, nt, nt))
    cost = np.zeros((W, W, nt, nt))
    lib().oc_kernel_table(nt, int(axial), w[0], w[1], w[2], eps, R, _p(logk), _p(cost))
    return logk, cost


def conv_log(logk: np.ndarray, login: np.ndarray) -> np.ndarray:
    """log of (K * exp(login)) on the grid [ny][nx][nt]."""
    ny, nx, nt = login.shape
    R = (logk.shape[0] - 1) // 2
    out = np.empty_like(login)
    lib().oc_conv_log(nx, ny, nt, R, _p(np.ascontiguousarray(logk)), _p(np.ascontiguousarray(login)), _p(out))
    return out


def conv_linear(logk: np.ndarray, x: np.ndarray) -> np.ndarray:
    ny, nx, nt = x.shape
    R = (logk.shape[0] - 1) // 2
    out = np.empty_like(x)
    lib().oc_conv_linear(nx, ny, nt, R, _p(np.ascontiguousarray(logk)), _p(np.ascontiguousarray(x)), _p(out))
    return out


def _window_at(logk: np.ndarray, arr: np.ndarray, iy: int, ix: int, ko: int):
    """Window terms of output (iy, ix, ko): (log K entries, input values) over the
    in-grid offsets d = out - in, all input orientations (Section 4.2, zero boundary)."""
    ny, nx, nt = arr.shape
    R = (logk.shape[0] - 1) // 2
    ks, vs = [], []
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            y, x = iy - dy, ix - dx
            if 0 <= y < ny and 0 <= x < nx:
                ks.append(logk[dy + R, dx + R, ko, :])
                vs.append(arr[y, x, :])
    return np.concatenate(ks), np.concatenate(vs)


def conv_log_points(logk: np.ndarray, login: np.ndarray, pts) -> np.ndarray:
    """log (K * exp(login)) at the given (iy, ix, ko) outputs only, one window sum each
    (the same definition as conv_log, evaluated point by point for large grids)."""
    out = np.empty(len(pts))
    for n, (iy, ix, ko) in enumerate(pts):
        k, v = _window_at(logk, login, iy, ix, ko)
        a = k + v
        m = np.max(a)
        out[n] = -np.inf if m == -np.inf else m + np.log(np.sum(np.exp(a - m)))
    return out


def conv_linear_points(logk: np.ndarray, x: np.ndarray, pts) -> np.ndarray:
    """(K * x) at the given (iy, ix, ko) outputs only, one window sum each."""
    out = np.empty(len(pts))
    for n, (iy, ix, ko) in enumerate(pts):
        k, v = _window_at(logk, x, iy, ix, ko)
        out[n] = np.sum(np.exp(k) * v)
    return out


def safe_log(m: np.ndarray) -> np.ndarray:
    with np.errstate(divide="ignore"):
        return np.log(m)


def sinkhorn(logk: np.ndarray, mu: np.ndarray, nu: np.ndarray, max_iter: int, tol: float,
             psi_init: Optional[np.ndarray] = None):
    """Log-domain Sinkhorn.  Returns (phi, psi, iters, err, err_hist) with phi = f/eps, psi = g/eps."""
    ny, nx, nt = mu.shape
    R = (logk.shape[0] - 1) // 2
    lmu, lnu = safe_log(mu), safe_log(nu)
    phi = np.empty_like(mu)
    psi = np.empty_like(mu)
    hist = np.zeros(max(max_iter, 1))
    err = ctypes.c_double(0.0)
    it = lib().oc_sinkhorn(nx, ny, nt, R, _p(np.ascontiguousarray(logk)), _p(lmu), _p(lnu),
                           _p(psi_init), max_iter, tol, _p(phi), _p(psi), _p(hist), ctypes.byref(err))
    if it < 0:
        raise MemoryError("oracle sinkhorn failed")
    return phi, psi, it, err.value, hist[:it]


def ibp(logk: np.ndarray, mus: Sequence[np.ndarray], lambdas: Sequence[float], max_iter: int, tol: float,
        lv_init: Optional[np.ndarray] = None, return_lv: bool = False):
    """Log-domain IBP barycenter.  Returns (bary, iters, err, err_hist), plus the log v_i of the
    returned iterate ([n][ny][nx][nt]) when return_lv; lv_init starts them (default 0)."""
    ny, nx, nt = mus[0].shape
    R = (logk.shape[0] - 1) // 2
    lm = np.ascontiguousarray(np.stack([safe_log(m) for m in mus]))
    lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
    logbar = np.zeros_like(mus[0])
    hist = np.zeros(max(max_iter, 1))
    err = ctypes.c_double(0.0)
    lv_out = np.zeros_like(lm)
    lv0 = None if lv_init is None else np.ascontiguousarray(lv_init, dtype=np.float64).reshape(lm.shape)
    it = lib().oc_ibp(nx, ny, nt, R, _p(np.ascontiguousarray(logk)), len(mus), _p(lm), _p(lam),
                      max_iter, tol, _p(logbar), _p(hist), ctypes.byref(err), _p(lv0), _p(lv_out))
    if it < 0:
        raise ValueError("oracle ibp failed")
    if return_lv:
        return np.exp(logbar), it, err.value, hist[:it], lv_out
    return np.exp(logbar), it, err.value, hist[:it]


# --------------------------------------------------------------------------
# Entropic JKO step for the porous-medium gradient flow (Section 5.4: the flow of
# F(nu) = 1/(m-1) int nu^m, eqs. (GF_JKO), (cost_GF); solved with the entropic scheme the
# paper cites, Peyre 2015: a = mu / K b, b = prox^KL_{tau F / eps}(K^T a) / K^T a)
# --------------------------------------------------------------------------

def porous_prox_log(s: np.ndarray, c: float, m: float) -> np.ndarray:
    """log q of the KL proximal step of the porous-medium energy at p = exp(s): the q > 0 with
    log q + c q^(m-1) = log p, the optimality condition of min_q c/m q^m + KL(q | p) (one
    scalar equation per element).  Solved by bisection in FP64 on [s - D, s],
    D = max(1, s + log(c)/(m - 1)), where the left end has a non-positive residual; -inf
    stays -inf."""
    s = np.asarray(s, dtype=np.float64)
    if c == 0.0:
        return s.copy()
    fin = np.isfinite(s)
    hi = np.where(fin, s, 0.0)
    lo = hi - np.maximum(1.0, hi + math.log(c) / (m - 1.0))
    target = np.where(fin, s, 0.0)
    for _ in range(200):          # the bracket (width < 2^11 here) shrinks to FP64 resolution
        mid = 0.5 * (lo + hi)
        with np.errstate(over="ignore"):
            pos = mid + c * np.exp((m - 1.0) * mid) - target > 0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    y = 0.5 * (lo + hi)
    return np.where(fin, y, s)


def porous_c(tau: float, eps: float, m: float, ref: float) -> float:
    """c of porous_prox_log for F(nu) = ref/(m-1) sum (nu/ref)^m (densities against a reference
    cell measure ref): c = (tau/eps) * m/(m-1) * ref^(1-m)."""
    return (tau / eps) * m / (m - 1.0) * ref ** (1.0 - m)


def jko_step(logk: np.ndarray, mu: np.ndarray, tau: float, m: float, eps: float, ref: float, max_iter: int,
             tol: float, psi_init: Optional[np.ndarray] = None):
    """One entropic JKO step from mu: the scaling iterations a = mu / K b and
    b = prox(K^T a) / K^T a in log form (phi = log a, psi = log b), psi_0 = psi_init (0 if None).
    Stops when the first-marginal L1 error sum mu |exp(phi_l - phi_{l+1}) - 1| <= tol or at
    max_iter.  Returns (phi_l, psi_l, nu_l, iters, err) with nu_l = b_l K^T a_l, the second
    marginal of the plan of iterate l (the next measure of the flow)."""
    c = porous_c(tau, eps, m, ref)
    lmu = safe_log(mu)
    psi = np.zeros_like(mu) if psi_init is None else np.array(psi_init, dtype=np.float64)
    phi = np.where(lmu == -np.inf, -np.inf, lmu - conv_log(logk, psi))
    err = math.inf
    nu = None
    for l in range(1, max_iter + 1):
        sv = conv_log(logk, phi)
        y = porous_prox_log(sv, c, m)
        psi = np.where(np.isfinite(sv), y - sv, -np.inf)
        nu = np.exp(y)
        phi_new = np.where(lmu == -np.inf, -np.inf, lmu - conv_log(logk, psi))
        with np.errstate(invalid="ignore"):
            err = float(np.sum(np.where(lmu == -np.inf, 0.0, mu * np.abs(np.expm1(phi - phi_new)))))
        if err <= tol or l == max_iter:
            return phi, psi, nu, l, err
        phi = phi_new
    return phi, psi, nu, max_iter, err


def gradient_flow(logk: np.ndarray, mu0: np.ndarray, tau: float, m: float, eps: float, ref: float, nsteps: int,
                  max_iter: int, tol: float):
    """nsteps JKO steps (the time marching of eq. (GF_JKO)): step t starts from the measure of
    step t-1 divided by its mass and from its log b.  Returns the list of the steps' measures
    (each scaled to mass one) and of (iters, err) per step."""
    mu, psi = mu0, None
    traj, info = [], []
    for _ in range(nsteps):
        _, psi, nu, it, err = jko_step(logk, mu, tau, m, eps, ref, max_iter, tol, psi)
        mu = nu / nu.sum()
        traj.append(mu)
        info.append((it, err))
    return traj, info


def porous_energy(nu: np.ndarray, m: float, ref: float) -> float:
    """F(nu) = ref/(m-1) sum (nu/ref)^m."""
    return float(ref / (m - 1.0) * np.sum((nu / ref) ** m))


# --------------------------------------------------------------------------
# Lift and projection around the transport path
# --------------------------------------------------------------------------

def lift_field(mag: np.ndarray, angle: np.ndarray, nt: int, axial: bool) -> np.ndarray:
    """Orientation-field lift, Section 5.3 eq. (lifting_vector_field): U(x, y, theta_k) = |v(x, y)|
    where the circular distance between the field's angle and theta_k is below half a step
    (pi/N for Theta = 2 pi), else 0.  Reading: the bin of theta_k is the half-open arc
    [theta_k - step/2, theta_k + step/2), so an angle exactly between two centres belongs to
    the upper one and every angle has exactly one bin.  mag, angle: [..., ny, nx]."""
    period = PI if axial else 2 * PI
    step = period / nt
    th = step * np.arange(nt)
    rel = np.mod(angle[..., None] - th + period / 2, period) - period / 2   # psi - theta_k in [-T/2, T/2)
    take = (rel >= -step / 2) & (rel < step / 2)
    return np.where(take, mag[..., None], 0.0)


def project(u: np.ndarray, u_minus: Optional[np.ndarray] = None):
    """Projection P(U) = integral over theta (Section 2.3, eq. (proj)) of an array of mass per cell:
    the sum over the orientation bins (minus that of u_minus: b_t = P(U+) - P(U-), Section 5.2
    eq. (final)), and the argmax bin of u (the first one on ties) of eq.
    (reconstruction_vector_field).  Returns (mass, argmax)."""
    mass = u.sum(axis=-1)
    if u_minus is not None:
        mass = mass - u_minus.sum(axis=-1)
    return mass, np.argmax(u, axis=-1)


def split_signed(u: np.ndarray):
    """Positive and negative parts of a signed score, each normalised to sum 1 (Section 5.2, step 2)."""
    plus = np.maximum(u, 0.0)
    minus = np.maximum(-u, 0.0)
    sp, sn = plus.sum(), minus.sum()
    return (plus / sp if sp > 0 else plus), (minus / sn if sn > 0 else minus)


# --------------------------------------------------------------------------
# eps-scaling: not in the paper.  The published warm-start scheme of Schmitzer,
# "Stabilized sparse scaling algorithms for entropy regularized transport problems"
# (SIAM J. Sci. Comput. 2019, Section 3.2): solve at a decreasing sequence of eps,
# each stage started from the previous stage's dual potentials in absolute units
# (g = eps log b kept, so log b is multiplied by eps_old / eps_new).
# --------------------------------------------------------------------------

def eps_schedule(eps: float, eps_start: float, factor: float):
    """eps_start * factor^s for every such value above eps, then eps (only eps when eps_start <= eps)."""
    if not eps_start > eps:
        return [eps]
    out = []
    e = eps_start
    while e > eps * (1.0 + 1e-12):
        out.append(e)
        e *= factor
    return out + [eps]


def sinkhorn_eps_scaling(kernel_at, eps: float, mu: np.ndarray, nu: np.ndarray, eps_start: float,
                         factor: float, stage_iters: int, max_iter: int, tol: float):
    """Sinkhorn with eps-scaling: stage_iters iterations at each coarser eps of the schedule, then
    at eps up to max_iter iterations in all (tol applies at eps only).  kernel_at(e) returns the
    log-kernel table at e.  Returns (phi, psi, iters, err, err_hist) as sinkhorn(), at eps."""
    sched = eps_schedule(eps, eps_start, factor)
    psi = None
    for s, e in enumerate(sched[:-1]):
        init = None if psi is None else psi * (sched[s - 1] / e)
        _, psi, _, _, _ = sinkhorn(kernel_at(e), mu, nu, stage_iters, -1.0, init)
    coarse = (len(sched) - 1) * stage_iters
    init = None if psi is None else psi * (sched[-2] / eps)
    phi, psi, it, err, hist = sinkhorn(kernel_at(eps), mu, nu, max_iter - coarse, tol, init)
    return phi, psi, it + coarse, err, hist


def ibp_eps_scaling(kernel_at, eps: float, mus: Sequence[np.ndarray], lambdas: Sequence[float], eps_start: float,
                    factor: float, stage_iters: int, max_iter: int, tol: float):
    """IBP with eps-scaling (the log v_i carried over as psi above).  Returns (bary, iters, err, err_hist)."""
    sched = eps_schedule(eps, eps_start, factor)
    lv = None
    for s, e in enumerate(sched[:-1]):
        init = None if lv is None else lv * (sched[s - 1] / e)
        _, _, _, _, lv = ibp(kernel_at(e), mus, lambdas, stage_iters, -1.0, init, return_lv=True)
    coarse = (len(sched) - 1) * stage_iters
    init = None if lv is None else lv * (sched[-2] / eps)
    bar, it, err, hist = ibp(kernel_at(eps), mus, lambdas, max_iter - coarse, tol, init)
    return bar, it + coarse, err, hist


def plan_stats(logk: np.ndarray, cost_tab: np.ndarray, phi: np.ndarray, psi: np.ndarray):
    """(cost, mass, marg1, marg2) of pi = exp(phi + logk + psi) (Section 4.1)."""
    ny, nx, nt = phi.shape
    R = (logk.shape[0] - 1) // 2
    m1 = np.empty_like(phi)
    m2 = np.empty_like(phi)
    c = ctypes.c_double(0.0)
    m = ctypes.c_double(0.0)
    lib().oc_plan_stats(nx, ny, nt, R, _p(np.ascontiguousarray(logk)), _p(np.ascontiguousarray(cost_tab)),
                        _p(np.ascontiguousarray(phi)), _p(np.ascontiguousarray(psi)),
                        ctypes.byref(c), ctypes.byref(m), _p(m1), _p(m2))
    return c.value, m.value, m1, m2


def plan_l1(logk, phi_a, psi_a, phi_b, psi_b) -> float:
    ny, nx, nt = phi_a.shape
    R = (logk.shape[0] - 1) // 2
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (logk, phi_a, psi_a, phi_b, psi_b)]
    return float(lib().oc_plan_l1(nx, ny, nt, R, *[_p(v) for v in a]))


def marginal_errors(logk, cost_tab, phi, psi, mu, nu):
    """(L1 error of marginal 1, of marginal 2, cost, mass) of the plan from (phi, psi)."""
    cost, mass, m1, m2 = plan_stats(logk, cost_tab, phi, psi)
    return float(np.abs(m1 - mu).sum()), float(np.abs(m2 - nu).sum()), cost, mass


PI = math.pi
