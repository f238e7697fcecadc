"""GPU parity at the grid shapes of the workloads (64x64x16, 128x128x16, 256x256x32).

Full grids are compared with the FP64 oracle on sampled outputs (window sums
evaluated point by point), on whole short runs where the oracle finishes in
seconds, and through properties that hold at any size: pruned against dense
evaluation, and the exact grid symmetry of Section 3.1 (a 90-degree rotation of
the grid with a quarter-turn shift of the orientation bins) for barycenters.

Tolerances follow tests/test_gpu_parity.py.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import pins
from gpu_util import to_dev, to_host, torch_dev
from paper_2402_15322_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [
    # n, nt, axial, w, eps, R, batch
    (64, 16, False, (1.0, 3.0, 1.0), 0.1, 5, 2),
    (128, 16, False, (1.0, 3.0, 1.0), 0.05, 7, 2),
    (256, 32, True, (1.0, 4.0, 1.0), 0.03, 10, 1),
]


@pytest.fixture(scope="module")
def nat():
    torch_dev()
    from paper_2402_15322_amd import native
    native.se2_init()
    return native


def _points(n, nt, rng, count=48):
    """Corners, edges and random interior outputs (iy, ix, ko)."""
    pts = [(0, 0, 0), (0, n - 1, nt - 1), (n - 1, 0, 1), (n - 1, n - 1, nt // 2), (n // 2, 0, 3), (0, n // 2, 5)]
    while len(pts) < count:
        pts.append((int(rng.integers(n)), int(rng.integers(n)), int(rng.integers(nt))))
    return pts


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[0]}x{s[1]}r{s[5]}")
def test_conv_full_size_sampled(nat, shape):
    torch = torch_dev()
    n, nt, axial, w, eps, R, batch = shape
    k = nat.Kernel(n, n, nt, axial, w, eps, R)
    logk, _ = oracle.kernel_table(nt, axial, w, eps, R)
    rng = np.random.default_rng(300 + n)
    pts = _points(n, nt, rng)
    nwin = (2 * R + 1) ** 2 * nt
    # linear: BF16 (MFMA), F32, F64 within the rigorous rounding bounds
    x = rng.uniform(0.0, 1.0, (batch, n, n, nt))
    for prec, u, dt in ((nat.SE2_BF16, 2.0 ** -8, torch.float32), (nat.SE2_F32, 2.0 ** -24, torch.float32),
                        (nat.SE2_F64, 2.0 ** -53, torch.float64)):
        xd = to_dev(x, dt)
        out = torch.empty_like(xd)
        nat.se2_conv(k, prec, xd, out)
        got = to_host(out).astype(np.float64)
        acc = 2.0 ** -24 if prec != nat.SE2_F64 else 2.0 ** -53
        gam = nwin * acc / (1 - nwin * acc)
        u_in = u if prec == nat.SE2_F64 else max(u, 2.0 ** -24)
        worst = 0.0
        for b in range(batch):
            ref = oracle.conv_linear_points(logk, x[b], pts)
            g = np.array([got[b, iy, ix, ko] for (iy, ix, ko) in pts])
            bound = (2 * u_in + u_in * u_in + gam) * ref + 1e-300
            worst = max(worst, float(np.max(np.abs(g - ref) / bound)))
        assert worst <= 1.0, (prec, worst)
    # log domain: F32 engine 2e-6, F64 1e-10 (natural-log units)
    lx = rng.normal(0.0, 300.0, (batch, n, n, nt))
    lx[:, :2, :3, 0] = -np.inf
    xd = to_dev(lx)
    for prec, tol in ((nat.SE2_F32, 2e-6), (nat.SE2_F64, 1e-10)):
        out = torch.empty_like(xd)
        nat.se2_conv_log(k, prec, xd, out)
        got = to_host(out)
        worst = 0.0
        for b in range(batch):
            ref = oracle.conv_log_points(logk, lx[b], pts)
            g = np.array([got[b, iy, ix, ko] for (iy, ix, ko) in pts])
            fin = np.isfinite(ref)
            assert np.array_equal(fin, np.isfinite(g))
            worst = max(worst, float(np.max(np.abs(g[fin] - ref[fin]))))
        assert worst <= tol, (prec, worst)


def _gpu_bary(nat, inst, iters, prune=True, tol=-1.0, check_every=None):
    torch = torch_dev()
    g = inst.grid
    k = nat.Kernel(g.nx, g.ny, g.nt, g.axial, inst.w, inst.eps, inst.radius)
    out = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    rep = nat.se2_barycenter(k, [to_dev(m) for m in inst.mus], inst.lambdas,
                             nat.opts(tol=tol, max_iter=iters, check_every=check_every or iters, prune=prune), out)
    return to_host(out), rep


def test_barycenter_curves128_matches_oracle(nat):
    """128x128x16 interpolation at t = 0.5 (two Bezier-stroke measures, no floor), 6 IBP
    iterations (certified pruning on): barycenter, error, mass and the transport cost
    sum_i lambda_i <pi_i, rho_b^2> of the returned iterate against the oracle."""
    inst = synth.curves128(0, t=0.5)
    g = inst.grid
    logk, cost = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
    bar_g, rep = _gpu_bary(nat, inst, 6)
    bar_o, it_o, err_o, _, lv = oracle.ibp(logk, inst.mus, inst.lambdas, 6, -1.0, return_lv=True)
    assert rep["iters"] == it_o == 6
    l1 = float(np.sum(np.abs(bar_g - bar_o)))
    assert l1 <= 1e-5, l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6
    assert abs(rep["mass"] - bar_o.sum()) <= 1e-6
    c_o = sum(lam * oracle.plan_stats(logk, cost, oracle.safe_log(m) - oracle.conv_log(logk, v), v)[0]
              for lam, m, v in zip(inst.lambdas, inst.mus, lv))
    assert abs(rep["cost"] - c_o) <= 1e-5 * c_o, (rep["cost"], c_o)


def test_barycenter_curves128_pruned_equals_dense(nat):
    """Certified pruning against dense evaluation over 40 IBP iterations at 128x128x16."""
    inst = synth.curves128(1, t=0.25)
    a, ra = _gpu_bary(nat, inst, 40, prune=True)
    b, rb = _gpu_bary(nat, inst, 40, prune=False)
    assert float(np.sum(np.abs(a - b))) <= 1e-6
    assert abs(ra["marg_l1"] - rb["marg_l1"]) <= 1e-7
    assert ra["terms_sparse"] > 0 and rb["terms_sparse"] == 0


def test_barycenter_fields_downsample_matches_oracle(nat):
    """The 256x256x32 axial field workload on its 64x64x8 downsample (same formula,
    eps, metric and 21x21 window), 4 measures, 4 IBP iterations against the oracle."""
    inst = synth.fields256(0, n=64, nt=8)
    g = inst.grid
    logk, _ = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
    bar_g, rep = _gpu_bary(nat, inst, 4)
    bar_o, it_o, err_o, _ = oracle.ibp(logk, inst.mus, inst.lambdas, 4, -1.0)
    assert rep["iters"] == it_o == 4
    l1 = float(np.sum(np.abs(bar_g - bar_o)))
    assert l1 <= 1e-5, l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6


def test_barycenter_fields256_symmetry(nat):
    """Full 256x256x32 axial barycenter of 4 fields: rotating every input by 90 degrees
    (grid rotation, orientation bins shifted by a quarter turn) rotates the barycenter;
    mass and positivity hold."""
    inst = synth.fields256(0)
    a, ra = _gpu_bary(nat, inst, 10)
    rot = synth.BaryInstance(inst.grid, inst.w, inst.eps, inst.radius,
                             [pins.rot90(m, axial=True) for m in inst.mus], inst.lambdas, inst.name + "/rot")
    b, rb = _gpu_bary(nat, rot, 10)
    assert np.all(a >= 0.0)
    assert abs(ra["mass"] - a.sum()) <= 1e-9
    l1 = float(np.sum(np.abs(pins.rot90(a, axial=True) - b)))
    assert l1 <= 1e-5 * a.sum(), l1
    assert abs(ra["marg_l1"] - rb["marg_l1"]) <= 1e-6


def test_bench_batch_matches_oracle(nat):
    """The benchmarked configuration: 32 paired 64x64x16 solves submitted together to the
    serving queue (three lanes, certified pruning), here for 20 iterations.  The first three
    solves (one per lane: requests go to the least-loaded lane in turn) are compared with
    the oracle at the same iteration count; solves of the batch are bitwise the blocking
    solve of the same pair."""
    torch = torch_dev()
    k = nat.Kernel(64, 64, 16, False, (1.0, 3.0, 1.0), 0.1, 5)
    insts = [synth.lines64(i, paired=True) for i in range(32)]
    mus = [to_dev(x.mu) for x in insts]
    nus = [to_dev(x.nu) for x in insts]
    fs = [torch.empty_like(m) for m in mus]
    gs = [torch.empty_like(m) for m in mus]
    it = 20
    o = nat.opts(tol=1e-6, max_iter=it, check_every=10)
    q = nat.SolveQueue(hbm_budget_bytes=nat.ot_request_bytes(k, o) * 32 + (64 << 20), max_slots=32)
    ts = [q.submit_ot(k, mus[i], nus[i], o, fs[i], gs[i]) for i in range(32)]
    reps = [q.wait(t) for t in ts]
    st = q.stats()
    q.close()
    assert st["peak_slots"] == 32 and all(r["iters"] == it for r in reps)
    logk, _ = oracle.kernel_table(16, False, (1.0, 3.0, 1.0), 0.1, 5)
    for i in (0, 1, 2):
        phi_o, psi_o, it_o, err_o, _ = oracle.sinkhorn(logk, insts[i].mu, insts[i].nu, it, -1.0)
        l1 = oracle.plan_l1(logk, to_host(fs[i]) / 0.1, to_host(gs[i]) / 0.1, phi_o, psi_o)
        assert l1 <= 1e-5, (i, l1)
        assert abs(reps[i]["marg_l1"] - err_o) <= 1e-6
    for i in (0, 17, 31):
        f, g = torch.empty_like(mus[i]), torch.empty_like(mus[i])
        nat.se2_sinkhorn(k, mus[i], nus[i], o, f, g)
        assert np.array_equal(to_host(f), to_host(fs[i])) and np.array_equal(to_host(g), to_host(gs[i]))
