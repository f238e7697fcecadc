"""JKO steps of the porous-medium gradient flow on the GPU (Section 5.4) against the oracle,
at equal iteration counts.

Bars (as for Sinkhorn): next measure and plan L1 <= 1e-5 and first-marginal L1 within 1e-6 of
the oracle's on the FP32-exp engine, 1e-9 on the FP64 engine; F(next measure) within 1e-6
relative.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host, torch_dev
from paper_2402_15322_amd import synth

pytestmark = pytest.mark.gpu

M = 5.0
W_FLOW = (1.0, math.sqrt(10.0), math.sqrt(2.0))   # the paper's metric for the flow


@pytest.fixture(scope="module")
def nat():
    torch_dev()
    from paper_2402_15322_amd import native
    native.se2_init()
    return native


def _gpu_step(nat, k, mu_d, tau, ref, o):
    torch = torch_dev()
    nxt = torch.empty_like(mu_d)
    f = torch.empty_like(mu_d)
    g = torch.empty_like(mu_d)
    rep = nat.se2_jko_step(k, mu_d, tau, M, ref, o, nxt, f, g)
    return rep, to_host(nxt), to_host(f), to_host(g)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_jko_step_matches_oracle(nat, prec):
    inst = synth.tiny_ot(4)
    g = inst.grid
    eps, R = 0.5, 4
    ref = 1.0 / inst.mu.size
    tau = 1e-3
    k = nat.Kernel(g.nx, g.ny, g.nt, False, W_FLOW, eps, R)
    p = nat.SE2_F32 if prec == "f32" else nat.SE2_F64
    rep, nu_g, f_g, g_g = _gpu_step(nat, k, to_dev(inst.mu), tau, ref,
                                   nat.opts(tol=-1, max_iter=40, check_every=10, prec=p))
    logk, cost = oracle.kernel_table(g.nt, False, W_FLOW, eps, R)
    phi_o, psi_o, nu_o, it_o, err_o = oracle.jko_step(logk, inst.mu, tau, M, eps, ref, 40, -1.0)
    assert rep["iters"] == it_o == 40
    tol = 1e-5 if prec == "f32" else 1e-9
    assert float(np.sum(np.abs(nu_g - nu_o))) <= tol
    assert oracle.plan_l1(logk, f_g / eps, g_g / eps, phi_o, psi_o) <= tol
    assert abs(rep["marg_l1"] - err_o) <= (1e-6 if prec == "f32" else 1e-10)
    e_o = oracle.porous_energy(nu_o, M, ref)
    assert abs(rep["dual"] - e_o) <= 1e-6 * e_o
    c_o = oracle.plan_stats(logk, cost, phi_o, psi_o)[0]
    assert abs(rep["cost"] - c_o) <= 1e-5 * c_o


def test_jko_step_lines64_pruned(nat):
    """A 64 x 64 x 16 stroke image with the paper's flow metric, 16 iterations, pruned engine."""
    inst = synth.lines64(6, paired=True)
    eps, R, tau = 0.5, 5, 1e-4
    ref = 1.0 / inst.mu.size
    k = nat.Kernel(64, 64, 16, False, W_FLOW, eps, R)
    rep, nu_g, f_g, g_g = _gpu_step(nat, k, to_dev(inst.mu), tau, ref, nat.opts(tol=-1, max_iter=16, check_every=4))
    logk, _ = oracle.kernel_table(16, False, W_FLOW, eps, R)
    phi_o, psi_o, nu_o, it_o, err_o = oracle.jko_step(logk, inst.mu, tau, M, eps, ref, 16, -1.0)
    assert rep["iters"] == it_o == 16
    assert float(np.sum(np.abs(nu_g - nu_o))) <= 1e-5
    assert abs(rep["marg_l1"] - err_o) <= 1e-6


def test_jko_tau_zero_is_the_entropic_blur(nat):
    inst = synth.tiny_ot(5)
    g = inst.grid
    k = nat.Kernel(g.nx, g.ny, g.nt, False, W_FLOW, 0.5, 4)
    # dense visits both times: the first a-update and the one after the (exact) b = 1 agree bitwise
    rep, nu_g, _, _ = _gpu_step(nat, k, to_dev(inst.mu), 0.0, 1.0,
                                nat.opts(tol=1e-12, max_iter=50, check_every=1, prune=False))
    assert rep["status"] == nat.SE2_CONVERGED and rep["iters"] == 1
    logk, _ = oracle.kernel_table(g.nt, False, W_FLOW, 0.5, 4)
    blur = oracle.conv_linear(logk, inst.mu / oracle.conv_linear(logk, np.ones_like(inst.mu)))
    assert float(np.max(np.abs(nu_g - blur) / blur)) <= 2e-6


def test_flow_of_three_warm_started_steps(nat):
    """Three steps, each warm-started from the previous step's log b: mass kept, F decreasing,
    every step equal to the oracle's."""
    inst = synth.tiny_ot(6)
    g = inst.grid
    eps, R, tau = 0.5, 4, 1e-3
    ref = 1.0 / inst.mu.size
    k = nat.Kernel(g.nx, g.ny, g.nt, False, W_FLOW, eps, R)
    logk, _ = oracle.kernel_table(g.nt, False, W_FLOW, eps, R)
    mu_g, mu_o = inst.mu, inst.mu
    init_g, psi_o = None, None
    energies = [oracle.porous_energy(inst.mu, M, ref)]
    for step in range(3):
        o = nat.opts(tol=-1, max_iter=60, check_every=20, init_g=init_g)
        rep, nu_g, f_g, g_g = _gpu_step(nat, k, to_dev(mu_g), tau, ref, o)
        _, psi_o, nu_o, _, _ = oracle.jko_step(logk, mu_o, tau, M, eps, ref, 60, -1.0, psi_o)
        assert float(np.sum(np.abs(nu_g - nu_o))) <= 1e-5, step
        assert abs(rep["mass"] - 1.0) <= 1e-3
        energies.append(rep["dual"])
        # the next step starts from the renormalised measure and this step's log b
        mu_g = nu_g / nu_g.sum()
        mu_o = nu_o / nu_o.sum()
        init_g = to_dev(g_g / eps)
    assert energies[1] < energies[0] and energies[2] < energies[1] and energies[3] < energies[2]


def test_jko_invalid_arguments(nat):
    inst = synth.tiny_ot(0)
    k = nat.Kernel(16, 16, 8, False, W_FLOW, 0.5, 4)
    mu = to_dev(inst.mu)
    for tau, m, ref, kw in ((-1.0, 5.0, 1.0, {}), (1.0, 1.0, 1.0, {}), (1.0, 5.0, 0.0, {}),
                            (1.0, 5.0, 1.0, dict(eps_start=2.0, eps_factor=0.5, stage_iters=5))):
        torch = torch_dev()
        with pytest.raises(nat.SE2Error) as e:
            nat.se2_jko_step(k, mu, tau, m, ref, nat.opts(tol=-1, max_iter=20, **kw), torch.empty_like(mu))
        assert e.value.code == nat.SE2_EINVAL


def test_gradient_flow_matches_oracle(nat):
    """se2_gradient_flow: four steps on the device (renormalised measures, carried log b)
    against the oracle's time marching, step by step."""
    torch = torch_dev()
    inst = synth.tiny_ot(7)
    g = inst.grid
    eps, R, tau, steps = 0.5, 4, 1e-3, 4
    ref = 1.0 / inst.mu.size
    k = nat.Kernel(g.nx, g.ny, g.nt, False, W_FLOW, eps, R)
    mu = to_dev(inst.mu)
    out = torch.empty_like(mu)
    traj = torch.empty((steps,) + g.shape, dtype=torch.float64, device="cuda")
    reps = nat.se2_gradient_flow(k, mu, tau, M, ref, steps, nat.opts(tol=-1, max_iter=50, check_every=25), out, traj)
    logk, _ = oracle.kernel_table(g.nt, False, W_FLOW, eps, R)
    traj_o, info_o = oracle.gradient_flow(logk, inst.mu, tau, M, eps, ref, steps, 50, -1.0)
    tg = to_host(traj)
    for t in range(steps):
        assert reps[t]["iters"] == info_o[t][0] == 50
        assert abs(reps[t]["marg_l1"] - info_o[t][1]) <= 1e-6
        assert float(np.sum(np.abs(tg[t] - traj_o[t]))) <= 1e-5, t
        assert abs(tg[t].sum() - 1.0) <= 1e-12
    assert np.array_equal(to_host(out), tg[-1])
    e = [oracle.porous_energy(x, M, ref) for x in [inst.mu] + list(tg)]
    assert all(e[i + 1] < e[i] for i in range(steps))
