"""The FP64 oracle against the stored fixtures of `tests/golden/`.

rho_b_halfangle.txt   hand-evaluated half-angle coordinates and rho_b^2 (Section 4.3,
                      eqs. (logcomp) and (rhob)), with rho_b(g^-1) = rho_b(g).
so2_counterexample.txt  the SO(2) counterexample of Section 3.2: entropic OT on one
                      pixel with 16 orientations tends to the cost (pi - 2a)^2 of the
                      better map, not the pi^2 of the right translation, as eps -> 0.
"""
from __future__ import annotations

import math
import os

import numpy as np

import oracle
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_NS = {"pi": math.pi, "cos": math.cos, "sin": math.sin, "__builtins__": {}}


def _expr(s: str) -> float:
    return float(eval(s, _NS))  # fixture arithmetic only: pi, cos, sin and numbers


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def test_rho_b_hand_values():
    n = 0
    for line in _rows("rho_b_halfangle.txt"):
        x, y, th, w1, w2, w3, b1, b2, b3, r2 = [_expr(t) for t in line.split()]
        w = (w1, w2, w3)
        b = oracle.half_angle(x, y, th)
        assert np.allclose(b, [b1, b2, b3], rtol=0, atol=1e-13), (line, b)
        got = oracle.rho2(x, y, th, w)
        assert abs(got - r2) <= 1e-12 * max(1.0, r2), (line, got, r2)
        # the inverse element, from the homogeneous matrix of Section 2.3
        xi, yi, ti = dense.coords(np.linalg.inv(dense.se2_matrix(x, y, th)))
        assert abs(oracle.rho2(xi, yi, ti, w) - r2) <= 1e-12 * max(1.0, r2), line
        n += 1
    assert n == 9


def test_so2_counterexample_fixture():
    kv = {}
    for line in _rows("so2_counterexample.txt"):
        k, v = [t.strip() for t in line.split("=", 1)]
        kv[k] = v
    nt = int(kv["ntheta"])
    assert int(kv["p"]) == 2
    a = _expr(kv["angle_a"])
    mu = np.zeros((1, 1, nt))
    nu = np.zeros((1, 1, nt))
    for k in map(int, kv["mu_bins"].split()):
        mu[0, 0, k] = 0.5
        assert abs(2 * math.pi * k / nt - a) < 1e-12 or abs(2 * math.pi * k / nt - (2 * math.pi - a)) < 1e-12
    for k in map(int, kv["nu_bins"].split()):
        nu[0, 0, k] = 0.5
    c_right = _expr(kv["cost_right_translation"])
    c_opt = _expr(kv["cost_optimal"])
    assert c_opt < c_right
    prev = None
    for eps in (0.2, 0.05, 0.02):
        # pure rotations with w3 = 1: rho_b = |theta|, the invariant metric of SO(2)
        logk, cost = oracle.kernel_table(nt, False, (1.0, 1.0, 1.0), eps, 0)
        phi, psi, it, err, _ = oracle.sinkhorn(logk, mu, nu, 500, 1e-13)
        assert err <= 1e-13
        c = oracle.plan_stats(logk, cost, phi, psi)[0]
        assert c >= c_opt - 1e-12            # a feasible plan never beats the optimum
        if prev is not None:
            assert c <= prev + 1e-12         # and approaches it as eps decreases
        prev = c
    assert abs(prev - c_opt) < 1e-8
    assert abs(prev - c_right) > 7.0
