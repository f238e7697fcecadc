"""Checks that pin the FP64 oracle to facts the paper and the mathematics fix.

Each function raises AssertionError when the oracle disagrees.  They are
collected by `test_oracle_pins.py` and re-run by `test_oracle_mutants.py`
against deliberately broken copies of the oracle, to show that a plausible
mistake (dropped term, wrong sign, transposed operand) fails at least one pin.

Paper references (arXiv 2402.15322): group law Section 2.3; half-angle distance
Section 4.3 eqs. (rhob), (logcomp); group convolution and K = K^T Section 4.2;
Sinkhorn Section 4.1; equivariance Lemma (equivariance) and Corollary
(equivariance-sinkhorn); the SO(2) counterexample Lemma in Section 3;
barycenter algorithm Appendix A.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import linprog

import oracle
from oracle import dense

PI = math.pi


def _rand_measure(rng, shape, zero_frac=0.0):
    m = rng.uniform(0.1, 1.0, shape)
    if zero_frac > 0:
        m[rng.uniform(size=shape) < zero_frac] = 0.0
    return m / m.sum()


# --------------------------------------------------------------------------
# P1: closed-form values of rho_b at hand-checkable points, K(e) = 1,
#     rho_b(g^-1) = rho_b(g), and rho_b(., ., pi) = rho_b(., ., -pi)
# --------------------------------------------------------------------------

def pin_rho_closed_forms():
    # g = (1, 0, pi/2): b = (cos pi/4, -sin pi/4, pi/2)
    assert abs(oracle.rho2(1, 0, PI / 2, (1, 2, 1)) - (0.5 + 4 * 0.5 + PI ** 2 / 4)) < 1e-12
    # g = (0, 1, pi/2): b = (sin pi/4, cos pi/4, pi/2)
    assert abs(oracle.rho2(0, 1, PI / 2, (1, 2, 1)) - (0.5 + 4 * 0.5 + PI ** 2 / 4)) < 1e-12
    # g = (1, 1, 0): b = (1, 1, 0)
    assert abs(oracle.rho2(1, 1, 0.0, (1, 3, 1)) - 10.0) < 1e-12
    # g = (3, 4, pi) is represented with theta = -pi: b = (-4, 3, -pi)
    assert abs(oracle.rho2(3, 4, PI, (1, 2, 1)) - (16 + 4 * 9 + PI ** 2)) < 1e-12
    assert abs(oracle.rho2(3, 4, -PI, (1, 2, 1)) - (16 + 4 * 9 + PI ** 2)) < 1e-12
    # pure rotation: rho_b = w3 |theta|
    assert abs(oracle.rho2(0, 0, 0.7, (2, 5, 3)) - 9 * 0.49) < 1e-12
    # pure translation along the frame axes: rho_b = w1 |x|, w2 |y|
    assert abs(oracle.rho2(2.5, 0, 0.0, (3, 5, 7)) - 9 * 6.25) < 1e-12
    assert abs(oracle.rho2(0, -1.5, 0.0, (3, 5, 7)) - 25 * 2.25) < 1e-12
    # half-angle coordinates: half turn maps (x, y) to (y, -x)/...; theta = pi/3
    b = oracle.half_angle(2.0, 0.0, PI / 3)
    assert np.allclose(b, [2 * math.cos(PI / 6), -2 * math.sin(PI / 6), PI / 3], atol=1e-14)


def pin_rho_inverse_symmetry():
    rng = np.random.default_rng(11)
    for _ in range(200):
        x, y = rng.uniform(-5, 5, 2)
        th = rng.uniform(-PI, PI)
        w = rng.uniform(0.3, 4.0, 3)
        g = dense.se2_matrix(x, y, th)
        xi, yi, ti = dense.coords(np.linalg.inv(g))
        a = oracle.rho2(x, y, th, w)
        b = oracle.rho2(xi, yi, ti, w)
        assert abs(a - b) <= 1e-10 * max(1.0, a)


def pin_table_identity_and_symmetry():
    for nt, axial in ((8, False), (16, False), (8, True)):
        R = 3
        logk, cost = oracle.kernel_table(nt, axial, (1.0, 2.5, 1.3), 0.3, R)
        for k in range(nt):
            assert logk[R, R, k, k] == 0.0          # K(e) = 1
        # M = M^T  <=>  T[d, ko, ki] = T[-d, ki, ko]   (Section 4.2: K = K^T)
        flipped = logk[::-1, ::-1].transpose(0, 1, 3, 2)
        assert np.max(np.abs(logk - flipped)) <= 1e-12 * np.max(np.abs(logk))
        assert np.all(cost >= 0.0)
        assert np.allclose(logk, -cost / 0.3, rtol=1e-15, atol=0)


# --------------------------------------------------------------------------
# P2 / P3: the window convolution equals the explicit matrix built from
#          homogeneous SE(2) matrices; that matrix is symmetric
# --------------------------------------------------------------------------

def pin_conv_equals_dense_matrix():
    rng = np.random.default_rng(5)
    for (nx, ny, nt, axial, R, w, eps) in ((6, 5, 4, False, 2, (1.0, 2.0, 1.0), 0.7),
                                           (5, 5, 4, True, 2, (1.0, 3.0, 0.8), 0.9),
                                           (4, 6, 6, False, 1, (1.5, 1.0, 2.0), 2.0)):
        LM = dense.dense_logk(nx, ny, nt, axial, w, eps, R)
        logk, _ = oracle.kernel_table(nt, axial, w, eps, R)
        v = rng.uniform(0.0, 1.0, (ny, nx, nt))
        lin = oracle.conv_linear(logk, v)
        ref = (np.exp(LM) @ v.reshape(-1)).reshape(v.shape)
        assert np.max(np.abs(lin - ref)) <= 1e-13 * np.max(np.abs(ref))
        lv = rng.normal(0.0, 5.0, (ny, nx, nt))
        lv[0, 0, :2] = -np.inf
        got = oracle.conv_log(logk, lv)
        want = dense.conv_log(LM, lv)
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
        # symmetry of the operator
        finite = np.isfinite(LM)
        assert np.array_equal(finite, finite.T)
        assert np.max(np.abs(np.where(finite, LM - LM.T, 0.0))) <= 1e-12 * np.max(np.abs(LM[finite]))


def pin_pointwise_conv_equals_dense_matrix():
    """The point-by-point window sums (used to check large grids at sampled outputs)
    equal the explicit matrix product at every output of small grids, borders included."""
    rng = np.random.default_rng(6)
    for (nx, ny, nt, axial, R, w, eps) in ((7, 5, 4, False, 2, (1.0, 2.0, 1.0), 0.7),
                                           (5, 6, 4, True, 2, (1.0, 3.0, 0.8), 0.9)):
        LM = dense.dense_logk(nx, ny, nt, axial, w, eps, R)
        logk, _ = oracle.kernel_table(nt, axial, w, eps, R)
        pts = [(iy, ix, k) for iy in range(ny) for ix in range(nx) for k in range(nt)]
        v = rng.uniform(0.0, 1.0, (ny, nx, nt))
        ref = (np.exp(LM) @ v.reshape(-1)).reshape(-1)
        got = oracle.conv_linear_points(logk, v, pts)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
        lv = rng.normal(0.0, 5.0, (ny, nx, nt))
        lv[0, 0, :2] = -np.inf
        want = dense.conv_log(LM, lv).reshape(-1)
        got = oracle.conv_log_points(logk, lv, pts)
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


# --------------------------------------------------------------------------
# P4: one orientation -> separable anisotropic Gaussian (two 1-D passes)
# P5: one pixel -> circulant theta convolution (FFT)
# --------------------------------------------------------------------------

def pin_single_orientation_is_separable_gaussian():
    rng = np.random.default_rng(7)
    nx, ny, R, w, eps = 13, 9, 3, (1.2, 2.0, 5.0), 0.8
    logk, _ = oracle.kernel_table(1, False, w, eps, R)
    v = rng.uniform(0, 1, (ny, nx, 1))
    d = np.arange(-R, R + 1)
    gx = np.exp(-(w[0] * d) ** 2 / eps)
    gy = np.exp(-(w[1] * d) ** 2 / eps)
    tmp = np.stack([np.convolve(v[iy, :, 0], gx, mode="same") for iy in range(ny)])
    ref = np.stack([np.convolve(tmp[:, ix], gy, mode="same") for ix in range(nx)], axis=1)
    got = oracle.conv_linear(logk, v)[:, :, 0]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(ref)


def pin_single_pixel_is_circulant():
    rng = np.random.default_rng(8)
    for nt, axial in ((16, False), (12, False), (8, True)):
        w3, eps = 1.3, 0.6
        period = PI if axial else 2 * PI
        logk, _ = oracle.kernel_table(nt, axial, (1.0, 1.0, w3), eps, 0)
        phi = period * np.arange(nt) / nt
        d = np.mod(phi + PI, 2 * PI) - PI
        if axial:
            d = np.minimum(np.abs(d), np.abs(np.mod(phi + 2 * PI, 2 * PI) - PI))
        k = np.exp(-(w3 * d) ** 2 / eps)
        v = rng.uniform(0, 1, nt)
        ref = np.real(np.fft.ifft(np.fft.fft(k) * np.fft.fft(v)))
        got = oracle.conv_linear(logk, v.reshape(1, 1, nt)).reshape(-1)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(ref)


# --------------------------------------------------------------------------
# P6 / P11: exact grid symmetries (90-degree rotation with a quarter-turn
# shift of theta, mirror with theta -> -theta); equivariance of conv,
# Sinkhorn plans and barycenters, invariance and symmetry of the cost
# --------------------------------------------------------------------------

def rot90(a: np.ndarray, axial: bool = False) -> np.ndarray:
    """(ix, iy, k) -> (N-1-iy, ix, k + nt/4), nt/2 for axial grids (left translation by a quarter turn)."""
    ny, nx, nt = a.shape
    shift = nt // 2 if axial else nt // 4
    out = np.empty_like(a)
    for iy in range(ny):
        for ix in range(nx):
            out[ix, nx - 1 - iy] = np.roll(a[iy, ix], shift)
    return out


def mirror(a: np.ndarray) -> np.ndarray:
    """(ix, iy, k) -> (ix, N-1-iy, -k)."""
    out = a[::-1, :, :]
    idx = (-np.arange(a.shape[2])) % a.shape[2]
    return np.ascontiguousarray(out[:, :, idx])


def pin_conv_equivariance():
    rng = np.random.default_rng(9)
    for nt, axial in ((8, False), (8, True)):
        logk, _ = oracle.kernel_table(nt, axial, (1.0, 2.0, 1.0), 0.5, 2)
        v = rng.normal(0, 3, (7, 7, nt))
        c = oracle.conv_log(logk, v)
        assert np.max(np.abs(oracle.conv_log(logk, rot90(v, axial)) - rot90(c, axial))) < 1e-12
        assert np.max(np.abs(oracle.conv_log(logk, mirror(v)) - mirror(c))) < 1e-12


def pin_sinkhorn_equivariance_and_cost_symmetry():
    rng = np.random.default_rng(10)
    nt = 8
    logk, cost = oracle.kernel_table(nt, False, (1.0, 2.0, 1.0), 0.5, 2)
    mu = _rand_measure(rng, (6, 6, nt))
    nu = _rand_measure(rng, (6, 6, nt))
    phi, psi, it, err, _ = oracle.sinkhorn(logk, mu, nu, 60, -1.0)
    pr, sr, _, _, _ = oracle.sinkhorn(logk, rot90(mu), rot90(nu), 60, -1.0)
    assert np.max(np.abs(pr - rot90(phi))) < 1e-10 and np.max(np.abs(sr - rot90(psi))) < 1e-10
    pm, sm, _, _, _ = oracle.sinkhorn(logk, mirror(mu), mirror(nu), 60, -1.0)
    assert np.max(np.abs(pm - mirror(phi))) < 1e-10
    c0 = oracle.plan_stats(logk, cost, phi, psi)[0]
    c1 = oracle.plan_stats(logk, cost, pr, sr)[0]
    assert abs(c0 - c1) < 1e-12 * c0
    # symmetric in (mu, nu) at convergence: K = K^T makes the swapped plan the transpose
    phi, psi, it, err, _ = oracle.sinkhorn(logk, mu, nu, 3000, 1e-12)
    q, r, it2, err2, _ = oracle.sinkhorn(logk, nu, mu, 3000, 1e-12)
    assert err < 1e-12 and err2 < 1e-12
    ca = oracle.plan_stats(logk, cost, phi, psi)[0]
    cb = oracle.plan_stats(logk, cost, q, r)[0]
    assert ca > 0 and abs(ca - cb) < 1e-9 * ca


def pin_barycenter_equivariance():
    rng = np.random.default_rng(12)
    nt = 8
    logk, _ = oracle.kernel_table(nt, False, (1.0, 2.0, 1.0), 0.6, 2)
    mus = [_rand_measure(rng, (6, 6, nt)) for _ in range(3)]
    lam = [0.2, 0.5, 0.3]
    b, _, _, _ = oracle.ibp(logk, mus, lam, 40, -1.0)
    br, _, _, _ = oracle.ibp(logk, [rot90(m) for m in mus], lam, 40, -1.0)
    assert np.max(np.abs(br - rot90(b))) < 1e-12 * np.max(b) * 100


# --------------------------------------------------------------------------
# P7: marginals at convergence; the second marginal is exact after a b-update
# --------------------------------------------------------------------------

def pin_sinkhorn_marginals():
    rng = np.random.default_rng(13)
    nt = 8
    logk, cost = oracle.kernel_table(nt, False, (1.0, 2.0, 1.0), 0.8, 2)
    mu = _rand_measure(rng, (5, 6, nt))
    nu = _rand_measure(rng, (5, 6, nt))
    phi, psi, it, err, hist = oracle.sinkhorn(logk, mu, nu, 5000, 1e-11)
    assert err <= 1e-11 and it < 5000
    e1, e2, c, mass = oracle.marginal_errors(logk, cost, phi, psi, mu, nu)
    assert e1 <= 2e-11          # the reported error is the plan's first-marginal error
    assert abs(e1 - err) <= 1e-12
    assert e2 <= 1e-13          # exact after the b-update
    assert abs(mass - 1.0) <= 1e-11
    # an unconverged iterate: the reported error still equals the plan's
    phi, psi, it, err, hist = oracle.sinkhorn(logk, mu, nu, 3, -1.0)
    e1, e2, _, _ = oracle.marginal_errors(logk, cost, phi, psi, mu, nu)
    assert it == 3 and abs(e1 - err) <= 1e-12 * max(1.0, err) and e2 <= 1e-13


# --------------------------------------------------------------------------
# P8: the paper's SO(2) counterexample (Lemma in Section 3): two Diracs at
#     +-pi/4 against their half-turn; the optimal cost tends to (pi - 2 pi/4)^2,
#     not pi^2, as eps -> 0.  Needs zero-mass handling.
# --------------------------------------------------------------------------

def pin_so2_counterexample():
    nt = 16
    mu = np.zeros((1, 1, nt)); nu = np.zeros((1, 1, nt))
    mu[0, 0, 2] = mu[0, 0, 14] = 0.5       # +pi/4, -pi/4
    nu[0, 0, 10] = nu[0, 0, 6] = 0.5       # +pi/4 + pi, -pi/4 + pi
    for eps in (0.05, 0.02):
        logk, cost = oracle.kernel_table(nt, False, (1.0, 1.0, 1.0), eps, 0)
        phi, psi, it, err, _ = oracle.sinkhorn(logk, mu, nu, 200, 1e-13)
        c = oracle.plan_stats(logk, cost, phi, psi)[0]
        assert abs(c - (PI - 2 * PI / 4) ** 2) < 1e-8, c
        assert abs(c - PI ** 2) > 1.0


# --------------------------------------------------------------------------
# P9: barycenter closed forms (Appendix A with lambda = e_k, or identical inputs):
#     v stays 1 and bar = K*(mu_k / K*1) from the first iteration on
# --------------------------------------------------------------------------

def pin_barycenter_closed_form():
    rng = np.random.default_rng(14)
    nx, ny, nt, R, w, eps = 5, 4, 6, 2, (1.0, 2.0, 1.0), 0.7
    LM = dense.dense_logk(nx, ny, nt, False, w, eps, R)
    K = np.exp(LM)
    logk, _ = oracle.kernel_table(nt, False, w, eps, R)
    m0 = _rand_measure(rng, (ny, nx, nt))
    m1 = _rand_measure(rng, (ny, nx, nt))
    want0 = (K @ (m0.reshape(-1) / (K @ np.ones(m0.size)))).reshape(m0.shape)
    want1 = (K @ (m1.reshape(-1) / (K @ np.ones(m1.size)))).reshape(m1.shape)
    b, it, err, _ = oracle.ibp(logk, [m0, m1], [1.0, 0.0], 7, -1.0)
    assert np.max(np.abs(b - want0)) < 1e-13 * np.max(want0)
    b, it, err, _ = oracle.ibp(logk, [m0, m1], [0.0, 1.0], 3, -1.0)
    assert np.max(np.abs(b - want1)) < 1e-13 * np.max(want1)
    b, it, err, _ = oracle.ibp(logk, [m0, m0], [0.3, 0.7], 5, -1.0)
    assert np.max(np.abs(b - want0)) < 1e-12 * np.max(want0)
    assert err < 1e-12  # the w-side marginal is met at the fixed point


# --------------------------------------------------------------------------
# P10: brute force -- dense-matrix Sinkhorn / IBP, and an exact LP as eps -> 0
# --------------------------------------------------------------------------

def pin_dense_sinkhorn_and_ibp():
    rng = np.random.default_rng(15)
    nx, ny, nt, R, w, eps = 4, 5, 4, 2, (1.0, 2.0, 1.5), 0.4
    LM = dense.dense_logk(nx, ny, nt, False, w, eps, R)
    logk, cost = oracle.kernel_table(nt, False, w, eps, R)
    mu = _rand_measure(rng, (ny, nx, nt), zero_frac=0.1)
    nu = _rand_measure(rng, (ny, nx, nt))
    phi, psi, it, err, _ = oracle.sinkhorn(logk, mu, nu, 25, -1.0)
    dphi, dpsi = dense.sinkhorn(LM, mu, nu, 25)
    pa = dense.plan(LM, phi, psi)
    pb = dense.plan(LM, dphi, dpsi)
    assert np.sum(np.abs(pa - pb)) < 1e-12
    l1 = oracle.plan_l1(logk, phi, psi, dphi, dpsi)
    assert l1 < 1e-12
    # plan statistics of arbitrary potentials (mass not 1) against the dense plan's sums, the
    # cost from the dense matrix: rho^2 = -eps log K on the window
    p2, s2 = phi + rng.normal(0.0, 0.3, phi.shape), psi + rng.normal(0.0, 0.3, psi.shape)
    c_o, m_o, _, _ = oracle.plan_stats(logk, cost, p2, s2)
    pd = dense.plan(LM, p2, s2)
    fin = np.isfinite(LM)
    cd, md = float(np.sum(pd[fin] * (-eps * LM[fin]))), float(pd.sum())
    assert abs(md - 1.0) > 1e-3
    assert abs(c_o - cd) <= 1e-11 * cd and abs(m_o - md) <= 1e-12 * md
    mus = [_rand_measure(rng, (ny, nx, nt)) for _ in range(3)]
    lam = [0.5, 0.25, 0.25]
    b, _, _, _ = oracle.ibp(logk, mus, lam, 15, -1.0)
    bd = dense.ibp(LM, mus, lam, 15)
    assert np.max(np.abs(b - bd)) < 1e-12 * np.max(bd)


def pin_small_eps_matches_linear_program():
    rng = np.random.default_rng(16)
    nx, ny, nt, R, w = 3, 3, 4, 2, (1.0, 2.0, 1.0)
    mu = _rand_measure(rng, (ny, nx, nt))
    nu = _rand_measure(rng, (ny, nx, nt))
    _, cost_tab = oracle.kernel_table(nt, False, w, 1.0, R)
    LM = dense.dense_logk(nx, ny, nt, False, w, 1.0, R)     # = -rho^2 (eps = 1)
    C = -LM
    n = mu.size
    # exact LP over the full 3x3 grid (R = 2 covers every pair)
    A = np.zeros((2 * n, n * n))
    for i in range(n):
        A[i, i * n:(i + 1) * n] = 1.0
        A[n + i, i::n] = 1.0
    res = linprog(C.reshape(-1), A_eq=A, b_eq=np.concatenate([mu.reshape(-1), nu.reshape(-1)]),
                  bounds=(0, None), method="highs")
    assert res.status == 0
    for eps in (0.05, 0.02):
        logk, cost = oracle.kernel_table(nt, False, w, eps, R)
        phi, psi, it, err, _ = oracle.sinkhorn(logk, mu, nu, 20000, 1e-10)
        c = oracle.plan_stats(logk, cost, phi, psi)[0]
        # feasible plan => cost >= LP optimum; entropic gap <= eps * 2 log n
        assert c >= res.fun - 1e-8
        assert c - res.fun <= eps * 2 * math.log(n)


# --------------------------------------------------------------------------
# eps-scaling (not in the paper; Schmitzer 2019): off means plain Sinkhorn; the converged
# result is the unique minimiser at the final eps whatever the warm start; the carry-over
# keeps the dual potential g = eps log b, which the theory fixes as the quantity that
# converges as eps -> 0 (a converged stage at 2 eps is then a much better start at eps
# than log b carried over as it is, or a cold start)
# --------------------------------------------------------------------------

def pin_eps_scaling():
    rng = np.random.default_rng(17)
    nt, w, R = 8, (1.0, 2.0, 1.0), 2
    kat = lambda e: oracle.kernel_table(nt, False, w, e, R)[0]
    assert oracle.eps_schedule(0.1, 3.2, 0.5) == [3.2, 1.6, 0.8, 0.4, 0.2, 0.1]
    assert oracle.eps_schedule(0.1, 0.1, 0.5) == [0.1] and oracle.eps_schedule(0.1, 0.0, 0.5) == [0.1]
    mu = _rand_measure(rng, (6, 6, nt))
    nu = _rand_measure(rng, (6, 6, nt))
    eps = 0.3
    a = oracle.sinkhorn_eps_scaling(kat, eps, mu, nu, eps, 0.5, 5, 40, -1.0)
    b = oracle.sinkhorn(kat(eps), mu, nu, 40, -1.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2] == 40
    phi, psi, it, err, _ = oracle.sinkhorn_eps_scaling(kat, eps, mu, nu, 2.4, 0.5, 30, 5000, 1e-12)
    phi2, psi2, it2, err2, _ = oracle.sinkhorn(kat(eps), mu, nu, 5000, 1e-12)
    assert err <= 1e-12 and err2 <= 1e-12 and 90 < it < 5000
    assert oracle.plan_l1(kat(eps), phi, psi, phi2, psi2) < 1e-10
    # carry-over from a converged stage at 2 eps, one iteration at eps
    eps = 0.15
    _, psi_c, itc, errc, _ = oracle.sinkhorn(kat(2 * eps), mu, nu, 20000, 1e-13)
    assert errc <= 1e-13
    e_ok = oracle.sinkhorn_eps_scaling(kat, eps, mu, nu, 2 * eps, 0.5, itc, itc + 1, -1.0)[3]
    e_logb = oracle.sinkhorn(kat(eps), mu, nu, 1, -1.0, psi_c)[3]
    e_cold = oracle.sinkhorn(kat(eps), mu, nu, 1, -1.0)[3]
    assert e_ok < 0.5 * e_logb and e_ok < 0.5 * e_cold, (e_ok, e_logb, e_cold)
    # IBP: the converged barycenter does not depend on the warm start
    mus = [_rand_measure(rng, (5, 5, nt)) for _ in range(3)]
    lam = [0.3, 0.3, 0.4]
    eps = 0.4
    b1, it1, e1, _ = oracle.ibp_eps_scaling(kat, eps, mus, lam, 1.6, 0.5, 20, 5000, 1e-12)
    b2, it2, e2, _ = oracle.ibp(kat(eps), mus, lam, 5000, 1e-12)
    assert e1 <= 1e-12 and e2 <= 1e-12 and 40 < it1 < 5000
    assert np.max(np.abs(b1 - b2)) < 1e-10 * np.max(b2)
    # IBP carry-over: log v_i of a converged stage at 2 eps, rescaled by 2 (eps log v kept), starts
    # the stage at eps closer than the same log v_i unscaled or a cold start (measured: 0.48 and
    # 0.36 of their errors after one iteration)
    eps = 0.2
    _, itc, errc, _, lvc = oracle.ibp(kat(2 * eps), mus, lam, 20000, 1e-13, return_lv=True)
    assert errc <= 1e-13
    e_ok = oracle.ibp_eps_scaling(kat, eps, mus, lam, 2 * eps, 0.5, itc, itc + 1, -1.0)[2]
    e_raw = oracle.ibp(kat(eps), mus, lam, 1, -1.0, lvc)[2]
    e_cold = oracle.ibp(kat(eps), mus, lam, 1, -1.0)[2]
    assert e_ok < 0.6 * e_raw and e_ok < 0.5 * e_cold, (e_ok, e_raw, e_cold)


# --------------------------------------------------------------------------
# Lift and projection (Sections 2.3, 5.2, 5.3): projecting a lifted field returns its
# magnitude exactly and its angle to within half an orientation step; lifting commutes
# with the exact 90-degree grid symmetry; a split score recombines to the score
# --------------------------------------------------------------------------

def pin_lift_and_project():
    rng = np.random.default_rng(18)
    for nt, axial in ((8, False), (16, False), (32, True)):
        period = PI if axial else 2 * PI
        step = period / nt
        mag = rng.uniform(0.0, 1.0, (2, 9, 9))
        ang = rng.uniform(-3 * PI, 3 * PI, (2, 9, 9))
        U = oracle.lift_field(mag, ang, nt, axial)
        assert U.shape == (2, 9, 9, nt)
        assert np.all(np.count_nonzero(U, axis=-1) == (mag > 0))   # exactly one bin per pixel
        assert abs(U.sum() - mag.sum()) <= 1e-13
        m, k = oracle.project(U)
        assert np.array_equal(m, mag)
        d = np.abs(np.mod(k * step - ang + period / 2, period) - period / 2)
        assert np.all(d <= step / 2 + 1e-12)
        # away from the edges the bin is the nearest centre
        off = rng.uniform(-0.49, 0.49, 20) * step
        e = oracle.lift_field(np.ones(20), 3 * step + off, nt, axial)
        assert np.all(e[:, 3] == 1.0) and e.sum() == 20.0
        # the 90-degree rotation of the grid: pixels rotated and angles turned by a quarter turn
        f = rng.uniform(0.0, 1.0, (7, 7))
        a = rng.uniform(0.0, period, (7, 7))
        rot_f = np.empty_like(f)
        rot_a = np.empty_like(a)
        for iy in range(7):
            for ix in range(7):
                rot_f[ix, 6 - iy] = f[iy, ix]
                rot_a[ix, 6 - iy] = a[iy, ix] + PI / 2
        assert np.array_equal(oracle.lift_field(rot_f, rot_a, nt, axial),
                              rot90(oracle.lift_field(f, a, nt, axial), axial))
    # two measures, difference of projections
    u = rng.normal(0.0, 1.0, (5, 6, 8))
    plus, minus = oracle.split_signed(u)
    assert plus.min() >= 0 and minus.min() >= 0 and abs(plus.sum() - 1) < 1e-14 and abs(minus.sum() - 1) < 1e-14
    sp, sn = np.maximum(u, 0).sum(), np.maximum(-u, 0).sum()
    assert np.max(np.abs(sp * plus - sn * minus - u)) < 1e-14
    b, _ = oracle.project(plus, minus)
    assert np.max(np.abs(b - (plus.sum(-1) - minus.sum(-1)))) < 1e-15


# --------------------------------------------------------------------------
# JKO step of the porous-medium flow (Section 5.4; entropic scheme of Peyre 2015): the
# proximal step solves its scalar optimality condition and minimises its objective; tau = 0
# gives the entropic blur K^T (mu / K 1) after one iteration; the converged plan is a
# stationary point of the JKO objective on its constraint set {pi 1 = mu}; mass is kept;
# the step commutes with the 90-degree grid symmetry
# --------------------------------------------------------------------------

def pin_jko_step():
    rng = np.random.default_rng(19)
    for c in (1e-3, 1.0, 1e3):
        for m in (2.0, 5.0):
            sv = rng.uniform(-40.0, 40.0, 200)
            y = oracle.porous_prox_log(sv, c, m)
            assert np.all(np.abs(y + c * np.exp((m - 1) * y) - sv) <= 1e-11 * (1 + np.abs(sv)))
            p = np.exp(sv)
            obj = lambda q: c / m * q ** m + q * (np.log(q) - sv) - q
            q = np.exp(y)
            for f in (1 + 1e-5, 1 - 1e-5):
                assert np.all(obj(q) <= obj(q * f) + 1e-12 * np.abs(obj(q)))
    assert np.array_equal(oracle.porous_prox_log(sv, 0.0, 5.0), sv)
    # tau = 0: the entropic blur after one iteration
    nx, ny, nt, R, w, eps = 4, 3, 4, 2, (1.0, 2.0, 1.0), 0.7
    logk, cost = oracle.kernel_table(nt, False, w, eps, R)
    K = np.exp(dense.dense_logk(nx, ny, nt, False, w, eps, R))
    mu = _rand_measure(rng, (ny, nx, nt))
    phi, psi, nu, it, err = oracle.jko_step(logk, mu, 0.0, 5.0, eps, 1.0, 50, 1e-14)
    assert it == 1 and err == 0.0
    blur = K.T @ (mu.reshape(-1) / (K @ np.ones(mu.size)))
    assert np.max(np.abs(nu.reshape(-1) - blur)) <= 1e-14
    # converged step: mass, stationarity of J(pi) = <C, pi> + eps sum pi (log pi - 1) + tau F(pi^T 1)
    ref = 1.0 / mu.size
    # the flow moves probability measures: a step stopped after 3 iterations leaves its second
    # marginal off mass one, and the flow scales it back before the next step
    nu3 = oracle.jko_step(logk, mu, 0.05, 2.0, eps, ref, 3, -1.0)[2]
    assert abs(nu3.sum() - 1.0) > 1e-9
    traj, info = oracle.gradient_flow(logk, mu, 0.05, 2.0, eps, ref, 3, 3, -1.0)
    assert all(abs(t.sum() - 1.0) <= 1e-12 for t in traj) and [it for it, _ in info] == [3, 3, 3]
    for tau, m in ((1e-3, 5.0), (0.05, 2.0)):
        phi, psi, nu, it, err = oracle.jko_step(logk, mu, tau, m, eps, ref, 5000, 1e-13)
        assert err <= 1e-13 and abs(nu.sum() - 1.0) <= 1e-12
        LM = dense.dense_logk(nx, ny, nt, False, w, eps, R)          # -inf outside the window
        win = np.isfinite(LM)
        C = np.where(win, -eps * LM, 0.0)
        P = np.exp(phi.reshape(-1)[:, None] + LM + psi.reshape(-1)[None, :])
        assert np.max(np.abs(P.sum(axis=1) - mu.reshape(-1))) <= 1e-13
        assert np.max(np.abs(P.sum(axis=0) - nu.reshape(-1))) <= 1e-14
        F = lambda v: ref / (m - 1) * np.sum((v / ref) ** m)
        J = lambda Q: (np.sum(Q * C) + eps * np.sum(np.where(win, Q * (np.log(np.where(win, Q, 1.0)) - 1), 0.0))
                       + tau * F(Q.sum(axis=0)))
        h = rng.normal(0.0, 1.0, P.shape)
        h -= (P * h).sum(axis=1, keepdims=True) / P.sum(axis=1, keepdims=True)   # keeps pi 1 = mu
        t = 1e-4
        jp, j0, jm = J(P * (1 + t * h)), J(P), J(P * (1 - t * h))
        assert jp >= j0 and jm >= j0
        assert abs(jp - jm) <= 1e-6 * (jp + jm - 2 * j0) / t    # first variation vanishes
        # a wrong proximal constant breaks stationarity
        _, psi2, nu2, _, _ = oracle.jko_step(logk, mu, 2 * tau, m, eps, ref, 5000, 1e-13)
        P2 = np.exp(oracle.jko_step(logk, mu, 2 * tau, m, eps, ref, 5000, 1e-13)[0].reshape(-1)[:, None] + LM
                    + psi2.reshape(-1)[None, :])
        assert abs(J(P2 * (1 + t * h)) - J(P2 * (1 - t * h))) > 1e3 * abs(jp - jm)
    # the 90-degree grid symmetry
    logk, _ = oracle.kernel_table(8, False, (1.0, 2.0, 1.0), 0.5, 2)
    mu = _rand_measure(rng, (6, 6, 8))
    a = oracle.jko_step(logk, mu, 1e-4, 5.0, 0.5, 1.0 / mu.size, 40, -1.0)[2]
    b = oracle.jko_step(logk, rot90(mu), 1e-4, 5.0, 0.5, 1.0 / mu.size, 40, -1.0)[2]
    assert np.max(np.abs(b - rot90(a))) <= 1e-12 * np.max(a)


# --------------------------------------------------------------------------
# The plan-difference checker: sum |pi_a - pi_b| over the window (plan of Section 4.1,
# pi = exp(phi + log K + psi)) equals the same sum over the explicit dense plans of two
# different iterates; a shift of phi by c scales the plan by e^c, so the L1 difference is
# |1 - e^c| times the plan's mass; each of the four potentials enters
# --------------------------------------------------------------------------

def pin_plan_l1():
    rng = np.random.default_rng(20)
    nx, ny, nt, R, w, eps = 4, 5, 4, 2, (1.0, 2.0, 1.5), 0.4
    LM = dense.dense_logk(nx, ny, nt, False, w, eps, R)
    logk, _ = oracle.kernel_table(nt, False, w, eps, R)
    mu = _rand_measure(rng, (ny, nx, nt))
    nu = _rand_measure(rng, (ny, nx, nt))
    a = oracle.sinkhorn(logk, mu, nu, 3, -1.0)[:2]
    b = oracle.sinkhorn(logk, mu, nu, 25, -1.0)[:2]
    want = np.abs(dense.plan(LM, *a) - dense.plan(LM, *b)).sum()
    assert want >= 1e-3
    got = oracle.plan_l1(logk, a[0], a[1], b[0], b[1])
    assert abs(got - want) <= 1e-13 * want
    assert abs(oracle.plan_l1(logk, b[0], b[1], a[0], a[1]) - want) <= 1e-13 * want
    # each potential of the second pair enters: change only psi_b, then only phi_b
    for pair in ((a[0], b[1]), (b[0], a[1])):
        want2 = np.abs(dense.plan(LM, *a) - dense.plan(LM, *pair)).sum()
        assert want2 >= 1e-3
        assert abs(oracle.plan_l1(logk, a[0], a[1], *pair) - want2) <= 1e-13 * want2
    # closed form: phi + c scales the plan by e^c
    mass = dense.plan(LM, *b).sum()
    for c in (0.3, -1.2):
        got = oracle.plan_l1(logk, b[0], b[1], b[0] + c, b[1])
        assert abs(got - abs(1.0 - math.exp(c)) * mass) <= 1e-13 * mass
        got = oracle.plan_l1(logk, b[0], b[1], b[0], b[1] + c)
        assert abs(got - abs(1.0 - math.exp(c)) * mass) <= 1e-13 * mass
    assert oracle.plan_l1(logk, b[0], b[1], b[0], b[1]) == 0.0


# --------------------------------------------------------------------------
# The porous-medium energy F(nu) = ref/(m-1) sum (nu/ref)^m (Section 5.4, the energy of
# eq. (pde_ndiff) on densities against the cell measure ref): hand-evaluated values
# --------------------------------------------------------------------------

def pin_porous_energy():
    nu = np.array([0.5, 0.25, 0.25, 0.0])
    # m = 2, ref = 1/4: densities (2, 1, 1, 0); F = 1/4 * (4 + 1 + 1) = 1.5
    assert abs(oracle.porous_energy(nu, 2.0, 0.25) - 1.5) <= 1e-15
    # m = 5, ref = 1/4: (32 + 1 + 1) / 4 / 4 = 2.125
    assert abs(oracle.porous_energy(nu, 5.0, 0.25) - 2.125) <= 1e-15
    # m = 3, ref = 1/2: densities (1, 1/2, 1/2, 0); F = 1/2 / 2 * (1 + 1/8 + 1/8) = 0.3125
    assert abs(oracle.porous_energy(nu, 3.0, 0.5) - 0.3125) <= 1e-15
    # grid shape does not matter, only the values
    assert oracle.porous_energy(nu.reshape(2, 2), 5.0, 0.25) == oracle.porous_energy(nu, 5.0, 0.25)


ALL_PINS = [
    pin_rho_closed_forms,
    pin_rho_inverse_symmetry,
    pin_table_identity_and_symmetry,
    pin_conv_equals_dense_matrix,
    pin_pointwise_conv_equals_dense_matrix,
    pin_single_orientation_is_separable_gaussian,
    pin_single_pixel_is_circulant,
    pin_conv_equivariance,
    pin_sinkhorn_equivariance_and_cost_symmetry,
    pin_barycenter_equivariance,
    pin_sinkhorn_marginals,
    pin_so2_counterexample,
    pin_barycenter_closed_form,
    pin_dense_sinkhorn_and_ibp,
    pin_small_eps_matches_linear_program,
    pin_eps_scaling,
    pin_lift_and_project,
    pin_jko_step,
    pin_plan_l1,
    pin_porous_energy,
]
