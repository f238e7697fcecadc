"""Serving queue: admission by budget, continuous batching, alone-vs-mixed identity."""
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


def _requests(nat):
    """Mixed sizes: two OT grids (8 and 16 orientations) and one barycenter."""
    torch = torch_dev()
    reqs = []
    for i, (n, nt, R, eps, w2) in enumerate(((16, 8, 4, 0.5, 2.0), (24, 16, 5, 0.2, 3.0), (16, 8, 4, 0.2, 3.0))):
        g = synth.Grid(n, n, nt)
        r = synth.rng_for(9000 + i, 0)
        segs = synth.draw_segments(r, g, 3, 3.0, 8.0)
        mu = synth.splat_segments(g, segs, 1.0, 1e-6)
        nu = synth.splat_segments(g, synth.moved_segments(r, g, segs, 1.0, 0.1), 1.0, 1e-6)
        k = nat.Kernel(n, n, nt, False, (1.0, w2, 1.0), eps, R)
        reqs.append(("ot", k, to_dev(mu), to_dev(nu), mu, nu))
    g = synth.Grid(16, 16, 8)
    ms = [synth.splat_segments(g, synth.draw_segments(synth.rng_for(9100, s), g, 3, 3.0, 8.0), 1.0, 1e-6)
          for s in range(3)]
    kb = nat.Kernel(16, 16, 8, False, (1.0, 2.0, 1.0), 0.5, 4)
    reqs.append(("bary", kb, [to_dev(m) for m in ms], [0.5, 0.3, 0.2], ms))
    return reqs


def _run(nat, reqs, max_slots, o):
    torch = torch_dev()
    q = nat.SolveQueue(hbm_budget_bytes=256 << 20, max_slots=max_slots)
    outs, tickets = [], []
    for r in reqs:
        if r[0] == "ot":
            f = torch.empty_like(r[2])
            g = torch.empty_like(r[2])
            tickets.append(q.submit_ot(r[1], r[2], r[3], o, f, g))
            outs.append((f, g))
        else:
            b = torch.empty_like(r[2][0])
            tickets.append(q.submit_barycenter(r[1], r[2], r[3], o, b))
            outs.append((b,))
    reps = [q.wait(t) for t in tickets]
    st = q.stats()
    q.close()
    return [tuple(to_host(x) for x in o_) for o_ in outs], reps, st


def test_alone_and_mixed_are_bitwise_identical(nat):
    reqs = _requests(nat)
    o = nat.opts(tol=1e-4, max_iter=150, check_every=5)
    alone, reps_a, st_a = _run(nat, reqs, 1, o)      # one solve at a time
    mixed, reps_m, st_m = _run(nat, reqs, 8, o)      # all resident together
    assert st_a["peak_slots"] == 1 and st_m["peak_slots"] == len(reqs)
    assert st_m["steps"] < st_a["steps"]
    for a, m, ra, rm in zip(alone, mixed, reps_a, reps_m):
        assert ra["iters"] == rm["iters"]
        for x, y in zip(a, m):
            assert np.array_equal(x, y)


def test_queue_matches_blocking_solver_and_oracle(nat):
    torch = torch_dev()
    reqs = _requests(nat)
    o = nat.opts(tol=-1, max_iter=40, check_every=10)
    res, reps, _ = _run(nat, reqs, 4, o)
    for r, out, rep in zip(reqs, res, reps):
        if r[0] != "ot":
            continue
        k = r[1]
        ny, nx, nt = k.shape
        f = torch.empty_like(r[2])
        g = torch.empty_like(r[2])
        rep_b = nat.se2_sinkhorn(k, r[2], r[3], o, f, g)
        assert np.array_equal(to_host(f), out[0]) and np.array_equal(to_host(g), out[1])
        assert rep_b["iters"] == rep["iters"] == 40
        eps = k.metric.eps
        logk, _ = oracle.kernel_table(nt, False, (k.metric.w1, k.metric.w2, k.metric.w3), eps, k.metric.radius)
        phi_o, psi_o, _, err_o, _ = oracle.sinkhorn(logk, r[4], r[5], 40, -1.0)
        assert oracle.plan_l1(logk, out[0] / eps, out[1] / eps, phi_o, psi_o) <= 1e-5
        assert abs(rep["marg_l1"] - err_o) <= 1e-6


def test_admission_respects_budget(nat):
    torch = torch_dev()
    g = synth.Grid(32, 32, 8)
    mu = synth.splat_segments(g, synth.draw_segments(synth.rng_for(9200, 0), g, 4, 5.0, 10.0), 1.0, 1e-6)
    k = nat.Kernel(32, 32, 8, False, (1.0, 2.0, 1.0), 0.2, 4)
    md = to_dev(mu)
    o = nat.opts(tol=-1, max_iter=20, check_every=5)
    # budget for roughly one solve at a time: everything still completes, never more than one resident
    need = nat.ot_request_bytes(k, o)
    q = nat.SolveQueue(hbm_budget_bytes=int(need * 1.5), max_slots=8)
    outs = [(torch.empty_like(md), torch.empty_like(md)) for _ in range(3)]
    ts = [q.submit_ot(k, md, md, o, f, gg) for f, gg in outs]
    reps = [q.wait(t) for t in ts]
    st = q.stats()
    assert st["peak_slots"] == 1 and st["completed"] == 3 and all(r["iters"] == 20 for r in reps)
    # a request larger than the whole budget is rejected at submit
    big = nat.Kernel(128, 128, 16, False, (1.0, 2.0, 1.0), 0.2, 4)
    bm = torch.full((128, 128, 16), 1.0 / (128 * 128 * 16), dtype=torch.float64, device="cuda")
    with pytest.raises(nat.SE2Error) as e:
        q.submit_ot(big, bm, bm, o)
    assert e.value.code == nat.SE2_ENOMEM
    q.close()


def test_kernel_time_accounts_every_convolution(nat):
    """Queue profiling: the algorithmic terms are exactly those of every convolution applied
    (one first a-update and two half-steps per iteration of each solve), the half-steps
    counted are those of the busiest lane, and the convolution time (the union of both
    lanes' launch intervals) is positive and within the wall time."""
    import time
    torch = torch_dev()
    n, nt, R = 24, 16, 5
    g = synth.Grid(n, n, nt)
    k = nat.Kernel(n, n, nt, False, (1.0, 3.0, 1.0), 0.2, R)
    reqs = []
    for i in range(4):
        r = synth.rng_for(9400 + i, 0)
        segs = synth.draw_segments(r, g, 3, 3.0, 8.0)
        reqs.append((to_dev(synth.splat_segments(g, segs, 1.0, 1e-6)),
                     to_dev(synth.splat_segments(g, synth.moved_segments(r, g, segs, 1.0, 0.1), 1.0, 1e-6))))
    it = 30
    o = nat.opts(tol=-1, max_iter=it, check_every=10)
    q = nat.SolveQueue(hbm_budget_bytes=256 << 20, max_slots=8)
    q.profile(True)
    t0 = time.perf_counter()
    ts = [q.submit_ot(k, mu, nu, o, torch.empty_like(mu), torch.empty_like(mu)) for mu, nu in reqs]
    reps = [q.wait(t) for t in ts]
    wall = time.perf_counter() - t0
    kt = q.kernel_time()
    q.close()
    per_conv = sum(max(0, n - abs(d)) for d in range(-R, R + 1)) ** 2 * nt * nt
    assert kt["terms"] == 4 * (2 * it + 1) * per_conv
    assert all(r["iters"] == it for r in reps)
    assert 2 * it <= kt["launches"] <= 2 * (it + 4)
    assert 0.0 < kt["seconds"] <= wall


@pytest.mark.parametrize("n,nt,R,iters", [(64, 16, 5, 300), (32, 32, 3, 120), (40, 8, 4, 120)])
def test_wide_and_narrow_rebuilds_are_bitwise_identical(nat, n, nt, R, iters):
    """The blocking solver rebuilds few uncertified tiles at 16 waves per item, the queue's
    lanes always at 8; the split of the window sums is the same for both widths, so the
    potentials agree bit for bit (pruned engine, the workload's shapes and more)."""
    torch = torch_dev()
    g = synth.Grid(n, n, nt)
    r = synth.rng_for(9200 + n, 0)
    segs = synth.draw_segments(r, g, 6, 4.0, 16.0)
    mu = synth.splat_segments(g, segs, 1.0, 1e-6)
    nu = synth.splat_segments(g, synth.moved_segments(r, g, segs, 2.0, 0.2), 1.0, 1e-6)
    k = nat.Kernel(n, n, nt, False, (1.0, 3.0, 1.0), 0.1, R)
    o = nat.opts(tol=-1, max_iter=iters, check_every=20)
    mud, nud = to_dev(mu), to_dev(nu)
    f, gb = torch.empty_like(mud), torch.empty_like(mud)
    rep_b = nat.se2_sinkhorn(k, mud, nud, o, f, gb)
    q = nat.SolveQueue(hbm_budget_bytes=256 << 20, max_slots=2)
    fq, gq = torch.empty_like(mud), torch.empty_like(mud)
    rep_q = q.wait(q.submit_ot(k, mud, nud, o, fq, gq))
    q.close()
    assert rep_b["iters"] == rep_q["iters"] == iters
    assert rep_b["terms_sparse"] > 0 and rep_b["terms_dense"] > 0
    assert np.array_equal(to_host(f), to_host(fq)) and np.array_equal(to_host(gb), to_host(gq))


def test_release_forgets_finished_tickets(nat):
    """A finished ticket can be released once; afterwards it is unknown.  Released tickets do
    not disturb the others' reports."""
    torch = torch_dev()
    g = synth.Grid(16, 16, 8)
    mu = synth.splat_segments(g, synth.draw_segments(synth.rng_for(9500, 0), g, 3, 3.0, 8.0), 1.0, 1e-6)
    k = nat.Kernel(16, 16, 8, False, (1.0, 2.0, 1.0), 0.5, 4)
    md = to_dev(mu)
    o = nat.opts(tol=-1, max_iter=20, check_every=10)
    q = nat.SolveQueue(hbm_budget_bytes=64 << 20, max_slots=4)
    ts = [q.submit_ot(k, md, md, o, torch.empty_like(md), torch.empty_like(md)) for _ in range(3)]
    reps = [q.wait(t) for t in ts]
    q.release(ts[0])
    with pytest.raises(nat.SE2Error) as e:
        q.release(ts[0])
    assert e.value.code == nat.SE2_EINVAL
    with pytest.raises(nat.SE2Error):
        q.wait(ts[0])
    assert q.wait(ts[1]) == reps[1] and q.times(ts[2])[2] > 0
    q.release(ts[1])
    q.release(ts[2])
    assert q.stats()["completed"] == 3
    q.close()


def test_converging_serving_requests_reach_tolerance(nat):
    """A burst of converging requests (theta-motion pairs of the converging serving trace on
    64x64x16 and 128x128x16, eps 0.1) through the queue: every one reaches marginal L1 1e-6
    with its FP64 check within 1.1e-6, and a sample equals the blocking call bit for bit."""
    torch = torch_dev()
    trace = synth.serving_trace(12, 1000.0, seed=3100, paired="theta", grids=synth.SERVE_GRIDS[1:])
    kernels = {}
    o = nat.opts(tol=1e-6, max_iter=3000, check_every=10, final_check=True)
    q = nat.SolveQueue(hbm_budget_bytes=1 << 30, max_slots=12)
    jobs = []
    for r in trace:
        x = r.inst
        key = (x.grid.nx, x.radius)
        if key not in kernels:
            kernels[key] = nat.Kernel(x.grid.nx, x.grid.ny, x.grid.nt, False, x.w, x.eps, x.radius)
        mu, nu = to_dev(x.mu), to_dev(x.nu)
        f, g = torch.empty_like(mu), torch.empty_like(mu)
        jobs.append((kernels[key], mu, nu, f, g, q.submit_ot(kernels[key], mu, nu, o, f, g)))
    reps = [q.wait(j[5]) for j in jobs]
    q.close()
    assert {x.inst.grid.nx for x in trace} == {64, 128}
    for rep in reps:
        assert rep["status"] == nat.SE2_CONVERGED and rep["marg_l1"] <= 1e-6, rep
        assert rep["marg_l1_f64"] <= 1.1e-6, rep
    for k, mu, nu, f, g, _ in (jobs[0], jobs[-1]):
        f2, g2 = torch.empty_like(mu), torch.empty_like(mu)
        nat.se2_sinkhorn(k, mu, nu, o, f2, g2)
        assert np.array_equal(to_host(f), to_host(f2)) and np.array_equal(to_host(g), to_host(g2))


def test_bulk_phase_switch_through_the_queue(nat):
    """A matrix-core bulk phase that ends on its fallback share (32 x 32 x 16 paired lines) and
    one that does not (theta motion), submitted together through the queue: the same switch
    iterations and the same bits as the blocking calls."""
    torch = torch_dev()
    insts = [synth.lines64(0, n=32), synth.lines64_theta(1, n=32)]
    o = nat.opts(tol=-1, max_iter=40, check_every=10, prec=nat.SE2_F32, bulk=nat.SE2_F32_MFMA, switch_tol=0.0)
    ks = [nat.Kernel(x.grid.nx, x.grid.ny, x.grid.nt, False, x.w, x.eps, x.radius) for x in insts]
    dev = [(to_dev(x.mu), to_dev(x.nu)) for x in insts]
    q = nat.SolveQueue(hbm_budget_bytes=256 << 20, max_slots=4)
    outs, tickets = [], []
    for k, (mu, nu) in zip(ks, dev):
        f, g = torch.empty_like(mu), torch.empty_like(mu)
        tickets.append(q.submit_ot(k, mu, nu, o, f, g))
        outs.append((f, g))
    reps = [q.wait(t) for t in tickets]
    q.close()
    assert reps[0]["phase_switch_iter"] in (10, 20, 30) and reps[1]["phase_switch_iter"] == -1
    for k, (mu, nu), (f, g), rq in zip(ks, dev, outs, reps):
        f2, g2 = torch.empty_like(mu), torch.empty_like(mu)
        rb = nat.se2_sinkhorn(k, mu, nu, o, f2, g2)
        assert rb["phase_switch_iter"] == rq["phase_switch_iter"] and rb["fallbacks"] == rq["fallbacks"]
        assert np.array_equal(to_host(f), to_host(f2)) and np.array_equal(to_host(g), to_host(g2))
