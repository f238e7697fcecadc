"""eps-scaling on the GPU (an outer loop around Sinkhorn and IBP; Schmitzer 2019) against the
oracle's stage loop, at equal iteration counts in every stage.

Tolerances as for the plain solvers: plan or barycenter L1 <= 1e-5 and marginal L1 within 1e-6
of the oracle's for the FP32-exp engine, plan L1 <= 1e-9 for the FP64 engine.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host, torch_dev
from paper_2402_15322_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    torch_dev()
    from paper_2402_15322_amd import native
    native.se2_init()
    return native


def _kernel_at(inst):
    g = inst.grid
    return lambda e: oracle.kernel_table(g.nt, g.axial, inst.w, e, inst.radius)[0]


def _ot(nat, inst, o):
    torch = torch_dev()
    g = inst.grid
    k = nat.Kernel(g.nx, g.ny, g.nt, g.axial, inst.w, inst.eps, inst.radius)
    mu, nu = to_dev(inst.mu), to_dev(inst.nu)
    f = torch.empty_like(mu)
    gg = torch.empty_like(mu)
    rep = nat.se2_sinkhorn(k, mu, nu, o, f, gg)
    return rep, to_host(f) / inst.eps, to_host(gg) / inst.eps


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_ot_eps_scaling_matches_oracle(nat, prec):
    inst = synth.tiny_ot(2)  # eps = 0.5: stages 4, 2, 1, then 0.5
    p = nat.SE2_F32 if prec == "f32" else nat.SE2_F64
    o = nat.opts(tol=-1, max_iter=80, check_every=10, prec=p, eps_start=4.0, eps_factor=0.5, stage_iters=15)
    rep, phi_g, psi_g = _ot(nat, inst, o)
    phi_o, psi_o, it_o, err_o, _ = oracle.sinkhorn_eps_scaling(_kernel_at(inst), inst.eps, inst.mu, inst.nu,
                                                               4.0, 0.5, 15, 80, -1.0)
    assert rep["iters"] == it_o == 80 and rep["scaling_iters"] == 45
    logk, cost = oracle.kernel_table(inst.grid.nt, inst.grid.axial, inst.w, inst.eps, inst.radius)
    l1 = oracle.plan_l1(logk, phi_g, psi_g, phi_o, psi_o)
    assert l1 <= (1e-5 if prec == "f32" else 1e-9), l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6
    c_o = oracle.plan_stats(logk, cost, phi_o, psi_o)[0]
    assert abs(rep["cost"] - c_o) <= 1e-5 * c_o


def test_ot_eps_scaling_lines64_pruned(nat):
    """64 x 64 x 16 lines at eps = 0.1 with two coarser stages (0.4, 0.2) on the pruned engine."""
    inst = synth.lines64(5, paired=True)
    o = nat.opts(tol=-1, max_iter=28, check_every=4, eps_start=0.4, eps_factor=0.5, stage_iters=8)
    rep, phi_g, psi_g = _ot(nat, inst, o)
    phi_o, psi_o, it_o, err_o, _ = oracle.sinkhorn_eps_scaling(_kernel_at(inst), inst.eps, inst.mu, inst.nu,
                                                               0.4, 0.5, 8, 28, -1.0)
    assert rep["iters"] == it_o == 28 and rep["scaling_iters"] == 16
    logk, _ = oracle.kernel_table(16, False, inst.w, inst.eps, inst.radius)
    l1 = oracle.plan_l1(logk, phi_g, psi_g, phi_o, psi_o)
    assert l1 <= 1e-5, l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6, (rep["marg_l1"], err_o)


def test_barycenter_eps_scaling_matches_oracle(nat):
    torch = torch_dev()
    g = synth.Grid(16, 16, 8)
    mus = [synth.splat_segments(g, synth.draw_segments(synth.rng_for(79, s), g, 3, 3.0, 10.0), 1.0, 1e-6)
           for s in range(3)]
    lam = [0.2, 0.5, 0.3]
    w, eps, R = (1.0, 2.0, 1.0), 0.5, 4
    k = nat.Kernel(16, 16, 8, False, w, eps, R)
    out = torch.empty((16, 16, 8), dtype=torch.float64, device="cuda")
    o = nat.opts(tol=-1, max_iter=40, check_every=5, eps_start=2.0, eps_factor=0.5, stage_iters=10)
    rep = nat.se2_barycenter(k, [to_dev(m) for m in mus], lam, o, out)
    kat = lambda e: oracle.kernel_table(8, False, w, e, R)[0]
    bar_o, it_o, err_o, _ = oracle.ibp_eps_scaling(kat, eps, mus, lam, 2.0, 0.5, 10, 40, -1.0)
    assert rep["iters"] == it_o == 40 and rep["scaling_iters"] == 20
    l1 = float(np.sum(np.abs(to_host(out) - bar_o)))
    assert l1 <= 1e-5, l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6


def test_eps_scaling_off_changes_nothing(nat):
    """eps_start <= eps switches the scheme off: results bitwise equal to the plain solve."""
    inst = synth.tiny_ot(3)
    base = _ot(nat, inst, nat.opts(tol=-1, max_iter=50, check_every=10))
    for es in (0.0, inst.eps):
        r = _ot(nat, inst, nat.opts(tol=-1, max_iter=50, check_every=10, eps_start=es, eps_factor=0.5,
                                    stage_iters=5))
        assert r[0]["scaling_iters"] == 0
        assert np.array_equal(r[1], base[1]) and np.array_equal(r[2], base[2])


def test_eps_scaling_bad_schedules_rejected(nat):
    inst = synth.tiny_ot(0)
    for kw in (dict(eps_start=4.0, eps_factor=1.0, stage_iters=5),      # factor outside (0, 1)
               dict(eps_start=4.0, eps_factor=0.5, stage_iters=0),      # no iterations per stage
               dict(eps_start=4.0, eps_factor=0.5, stage_iters=20)):    # 3 x 20 coarse >= max_iter 60
        with pytest.raises(nat.SE2Error) as e:
            _ot(nat, inst, nat.opts(tol=-1, max_iter=60, **kw))
        assert e.value.code == nat.SE2_EINVAL


def test_eps_scaling_in_queue_alone_mixed_and_blocking(nat):
    """Scaled and plain requests together: each result is bitwise the same alone, in the mix,
    and from the blocking call."""
    torch = torch_dev()
    reqs = []
    for i, (n, nt, R, eps, w2) in enumerate(((16, 8, 4, 0.5, 2.0), (24, 16, 5, 0.2, 3.0))):
        g = synth.Grid(n, n, nt)
        r = synth.rng_for(9300 + i, 0)
        segs = synth.draw_segments(r, g, 3, 3.0, 8.0)
        mu = synth.splat_segments(g, segs, 1.0, 1e-6)
        nu = synth.splat_segments(g, synth.moved_segments(r, g, segs, 1.0, 0.1), 1.0, 1e-6)
        reqs.append((nat.Kernel(n, n, nt, False, (1.0, w2, 1.0), eps, R), to_dev(mu), to_dev(nu)))
    scaled = nat.opts(tol=-1, max_iter=45, check_every=5, eps_start=1.6, eps_factor=0.5, stage_iters=7)
    plain = nat.opts(tol=-1, max_iter=45, check_every=5)
    jobs = [(reqs[0], scaled), (reqs[1], scaled), (reqs[1], plain)]

    def run(slots):
        q = nat.SolveQueue(hbm_budget_bytes=256 << 20, max_slots=slots)
        outs, ts = [], []
        for (k, mu, nu), o in jobs:
            f, g = torch.empty_like(mu), torch.empty_like(mu)
            ts.append(q.submit_ot(k, mu, nu, o, f, g))
            outs.append((f, g))
        reps = [q.wait(t) for t in ts]
        q.close()
        return [(to_host(f), to_host(g)) for f, g in outs], reps

    alone, ra = run(1)
    mixed, rm = run(4)
    for j, ((k, mu, nu), o) in enumerate(jobs):
        assert ra[j]["iters"] == rm[j]["iters"] == 45
        assert np.array_equal(alone[j][0], mixed[j][0]) and np.array_equal(alone[j][1], mixed[j][1])
        f, g = torch.empty_like(mu), torch.empty_like(mu)
        rb = nat.se2_sinkhorn(k, mu, nu, o, f, g)
        assert rb["scaling_iters"] == ra[j]["scaling_iters"]
        assert np.array_equal(to_host(f), alone[j][0]) and np.array_equal(to_host(g), alone[j][1])
    assert ra[0]["scaling_iters"] == 14 and ra[1]["scaling_iters"] == 21 and ra[2]["scaling_iters"] == 0
