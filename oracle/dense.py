"""Dense-matrix FP64 checker for tiny SE(2) grids -- TEST INFRASTRUCTURE ONLY.

An independent second route to the same quantities as `se2_oracle.c`:

  * group elements are 3x3 homogeneous matrices [[R_theta, x], [0, 1]], so the
    relative element h^{-1} g comes from a matrix inverse and product (the group
    law of Section 2.3) instead of the closed form used in C;
  * theta is read back from the product matrix with atan2;
  * the operator is built as an explicit matrix M[(x,ko),(y,ki)] = K(h^{-1} g)
    over the truncated window (Section 4.2), so a convolution is a matvec;
  * Sinkhorn (Section 4.1) and IBP (Appendix A) run on that matrix with
    scipy's logsumexp.

Meant for grids of at most a few hundred elements.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
from scipy.special import logsumexp


def se2_matrix(x: float, y: float, theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, x], [s, c, y], [0.0, 0.0, 1.0]])


def coords(m: np.ndarray):
    """(x, y, theta) of a homogeneous SE(2) matrix, theta in [-pi, pi)."""
    th = math.atan2(m[1, 0], m[0, 0])
    if th >= math.pi:
        th -= 2 * math.pi
    return m[0, 2], m[1, 2], th


def rho2_dense(x: float, y: float, th: float, w: Sequence[float]) -> float:
    """rho_b^2 (Section 4.3) from half-angle coordinates; th already in [-pi, pi]."""
    c, s = math.cos(th / 2), math.sin(th / 2)
    b1 = x * c + y * s
    b2 = -x * s + y * c
    return (w[0] * b1) ** 2 + (w[1] * b2) ** 2 + (w[2] * th) ** 2


def dense_logk(nx: int, ny: int, nt: int, axial: bool, w, eps: float, R: int) -> np.ndarray:
    """log M with M[(iy,ix,ko),(jy,jx,ki)] = exp(-rho^2(h^{-1}g)/eps) inside the window, -inf outside."""
    period = math.pi if axial else 2 * math.pi
    n = nx * ny * nt
    out = np.full((n, n), -np.inf)
    for iy in range(ny):
        for ix in range(nx):
            for ko in range(nt):
                g = se2_matrix(ix, iy, period * ko / nt)
                r = (iy * nx + ix) * nt + ko
                for jy in range(max(0, iy - R), min(ny, iy + R + 1)):
                    for jx in range(max(0, ix - R), min(nx, ix + R + 1)):
                        for ki in range(nt):
                            h = se2_matrix(jx, jy, period * ki / nt)
                            x, y, th = coords(np.linalg.inv(h) @ g)
                            d2 = rho2_dense(x, y, th, w)
                            if axial:
                                # the other lift of the output angle: g times a half turn
                                x2, y2, th2 = coords(np.linalg.inv(h) @ g @ se2_matrix(0, 0, math.pi))
                                d2 = min(d2, rho2_dense(x2, y2, th2, w))
                            out[r, (jy * nx + jx) * nt + ki] = -d2 / eps
    return out


def conv_log(LM: np.ndarray, login: np.ndarray) -> np.ndarray:
    flat = login.reshape(-1)
    return logsumexp(LM + flat[None, :], axis=1).reshape(login.shape)


def sinkhorn(LM: np.ndarray, mu: np.ndarray, nu: np.ndarray, iters: int):
    """`iters` Sinkhorn iterations on the explicit matrix; returns (phi, psi)."""
    lmu = np.log(mu.reshape(-1))
    lnu = np.log(nu.reshape(-1))
    psi = np.zeros_like(lmu)
    phi = None
    for _ in range(iters):
        phi = lmu - logsumexp(LM + psi[None, :], axis=1)
        psi = lnu - logsumexp(LM.T + phi[None, :], axis=1)
    return phi.reshape(mu.shape), psi.reshape(mu.shape)


def plan(LM: np.ndarray, phi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return np.exp(phi.reshape(-1)[:, None] + LM + psi.reshape(-1)[None, :])


def ibp(LM: np.ndarray, mus: Sequence[np.ndarray], lambdas: Sequence[float], iters: int) -> np.ndarray:
    """`iters` IBP iterations (Appendix A) in linear scaling variables on the explicit matrix."""
    K = np.exp(LM)
    n = len(mus)
    v = [np.ones(mus[0].size) for _ in range(n)]
    w = [np.ones(mus[0].size) for _ in range(n)]
    bar = None
    for _ in range(iters):
        bar = np.ones(mus[0].size)
        d = []
        for i in range(n):
            w[i] = mus[i].reshape(-1) / (K @ v[i])
            d.append(v[i] * (K @ w[i]))
            bar = bar * d[i] ** lambdas[i]
        for i in range(n):
            v[i] = v[i] * bar / d[i]
    return bar.reshape(mus[0].shape)
