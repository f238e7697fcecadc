"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances:
  * se2_conv BF16 -- the rigorous bound for products of two RNE-rounded bfloat16
    operands (unit roundoff u = 2^-8) summed in FP32 (gamma_n with 2^-24):
    |gpu - exact| <= (2u + u^2 + gamma_n) * (K * |x|) + n 2^-120 max|x|;
  * se2_conv F32 / F64 -- the same bound with u = 2^-24 / 2^-53;
  * log-domain paths -- absolute error of the natural log of K * exp(x):
    2e-6 for the FP32-exp engine (exponent arguments in FP64, FP32 exp2 and
    FP32 row sums), 1e-10 for the FP64 check path;
  * solvers at equal iteration counts -- plan L1 <= 1e-5, marginal L1 within
    1e-6 of the oracle's, relative transport cost within 1e-6 (the stated target
    is 1e-6 marginal L1 and 1e-3 relative cost).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from gpu_util import bf16_round, to_dev, to_host, torch_dev
from paper_2402_15322_amd import synth

pytestmark = pytest.mark.gpu

CONV_CASES = [
    # nx, ny, nt, axial, w, eps, R, batch
    (16, 16, 8, False, (1.0, 2.0, 1.0), 0.5, 4, 1),
    (13, 9, 16, False, (1.0, 3.0, 1.0), 0.8, 3, 2),
    (37, 21, 16, False, (1.0, 3.0, 1.0), 0.1, 5, 1),
    (20, 7, 32, True, (1.0, 4.0, 1.0), 0.3, 2, 2),
    (33, 40, 32, True, (1.0, 4.0, 1.0), 0.03, 10, 1),
    (9, 30, 8, False, (1.5, 1.0, 2.0), 2.0, 0, 1),
    # nt = 16 shapes of the FP32 matrix-core path: a single offset, a 15 x 15 window (dy
    # chunks of 8), a 25 x 25 window (chunks of 7, three zero rows), 8 rows per wave
    (16, 5, 16, False, (1.0, 2.0, 1.0), 1.0, 0, 3),
    (23, 50, 16, False, (1.0, 3.0, 1.0), 0.05, 7, 1),
    (30, 28, 16, False, (1.0, 3.0, 1.0), 0.5, 12, 1),
    (40, 70, 16, False, (1.0, 2.0, 1.0), 0.3, 2, 120),
    (12, 20, 32, False, (1.0, 2.0, 1.0), 1.0, 0, 2),   # nt = 32, a single offset (two passes)
    (20, 18, 32, True, (1.0, 4.0, 1.0), 0.4, 12, 1),   # nt = 32 at the largest window (25 x 25)
]


@pytest.fixture(scope="module")
def nat():
    torch_dev()
    from paper_2402_15322_amd import native
    native.se2_init()
    return native


def _kernel(nat, nx, ny, nt, axial, w, eps, R):
    return nat.Kernel(nx, ny, nt, axial, w, eps, R)


def test_kernel_table_matches_oracle(nat):
    for (nx, ny, nt, axial, w, eps, R, _) in CONV_CASES:
        k = _kernel(nat, nx, ny, nt, axial, w, eps, R)
        lk, ct = k.table()
        olk, oct_ = oracle.kernel_table(nt, axial, w, eps, R)
        # independent FP64 evaluations of the same closed form (different operation order)
        e_c = float(np.max(np.abs(ct - oct_) / np.maximum(1.0, np.abs(oct_))))
        e_l = float(np.max(np.abs(lk - olk) / np.maximum(1.0, np.abs(olk))))
        assert e_c <= 1e-13 and e_l <= 1e-13, (e_c, e_l)


@pytest.mark.parametrize("case", CONV_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{'a' if c[3] else ''}r{c[6]}")
def test_se2_conv_linear(nat, case):
    torch = torch_dev()
    nx, ny, nt, axial, w, eps, R, batch = case
    k = _kernel(nat, nx, ny, nt, axial, w, eps, R)
    logk, _ = oracle.kernel_table(nt, axial, w, eps, R)
    rng = np.random.default_rng(100 + nx)
    x = rng.uniform(0.0, 1.0, (batch, ny, nx, nt))
    x[:, 0, :, :] *= 1e-30  # a row of tiny values
    n = (2 * R + 1) ** 2 * nt
    ref = np.stack([oracle.conv_linear(logk, x[b]) for b in range(batch)])
    for prec, u, dt in ((nat.SE2_BF16, 2.0 ** -8, torch.float32), (nat.SE2_F32, 2.0 ** -24, torch.float32),
                        (nat.SE2_F64, 2.0 ** -53, torch.float64)):
        xin = x if prec != nat.SE2_BF16 else x  # the kernel rounds to bfloat16 itself
        xd = to_dev(xin.astype(np.float64), dt)
        out = torch.empty_like(xd)
        nat.se2_conv(k, prec, xd, out)
        got = to_host(out).astype(np.float64)
        acc = 2.0 ** -24 if prec != nat.SE2_F64 else 2.0 ** -53
        gam = n * acc / (1 - n * acc)
        # the FP32 input of BF16/F32 is itself a rounding of x
        u_in = u if prec == nat.SE2_F64 else max(u, 2.0 ** -24)
        bound = (2 * u_in + u_in * u_in + gam) * ref + n * 2.0 ** -120 * x.max()
        err = np.abs(got - ref)
        assert np.all(err <= bound), (prec, float(np.max(err / np.maximum(bound, 1e-300))))


def test_se2_conv_bf16_exact_operands(nat):
    """With inputs already bfloat16 the only error left is the FP32 accumulation:
    checks the MFMA operand/lane layout element by element."""
    torch = torch_dev()
    nx, ny, nt, R = 19, 18, 16, 3
    k = _kernel(nat, nx, ny, nt, False, (1.0, 2.0, 1.0), 1.5, R)
    logk, _ = oracle.kernel_table(nt, False, (1.0, 2.0, 1.0), 1.5, R)
    kb = bf16_round(np.exp(logk))
    rng = np.random.default_rng(7)
    x = bf16_round(rng.uniform(0, 1, (ny, nx, nt)))
    ref = oracle.conv_linear(np.log(np.maximum(kb, 1e-300)), x)
    out = torch.empty((ny, nx, nt), dtype=torch.float32, device="cuda")
    nat.se2_conv(k, nat.SE2_BF16, to_dev(x, torch.float32), out)
    got = to_host(out)
    n = (2 * R + 1) ** 2 * nt
    e = float(np.max(np.abs(got - ref) / ref))
    assert e <= n * 2.0 ** -24, e


@pytest.mark.parametrize("case", CONV_CASES[:5], ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}r{c[6]}")
def test_se2_conv_log(nat, case):
    torch = torch_dev()
    nx, ny, nt, axial, w, eps, R, batch = case
    k = _kernel(nat, nx, ny, nt, axial, w, eps, R)
    logk, _ = oracle.kernel_table(nt, axial, w, eps, R)
    rng = np.random.default_rng(200 + nx)
    # potentials with the spread seen in converged solves: hundreds per pixel
    x = rng.normal(0.0, 300.0, (batch, ny, nx, nt))
    x[:, :, :2, 0] = -np.inf  # zero mass
    ref = np.stack([oracle.conv_log(logk, x[b]) for b in range(batch)])
    xd = to_dev(x)
    for prec, tol in ((nat.SE2_F32, 2e-6), (nat.SE2_F64, 1e-10)):
        out = torch.empty_like(xd)
        nat.se2_conv_log(k, prec, xd, out)
        got = to_host(out)
        fin = np.isfinite(ref)
        assert np.array_equal(fin, np.isfinite(got))
        e = float(np.max(np.abs(got[fin] - ref[fin])))
        assert e <= tol, (prec, e)


def _ot_parity(nat, inst, iters, tol=-1.0):
    torch = torch_dev()
    g = inst.grid
    k = _kernel(nat, g.nx, g.ny, g.nt, g.axial, inst.w, inst.eps, inst.radius)
    logk, cost = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
    mu, nu = to_dev(inst.mu), to_dev(inst.nu)
    f = torch.empty_like(mu)
    gg = torch.empty_like(mu)
    rep = nat.se2_sinkhorn(k, mu, nu, nat.opts(tol=tol, max_iter=iters, check_every=1), f, gg)
    phi_g = to_host(f) / inst.eps
    psi_g = to_host(gg) / inst.eps
    phi_o, psi_o, it_o, err_o, _ = oracle.sinkhorn(logk, inst.mu, inst.nu, iters, tol)
    assert rep["iters"] == it_o
    l1 = oracle.plan_l1(logk, phi_g, psi_g, phi_o, psi_o)
    e1, e2, c_g, m_g = oracle.marginal_errors(logk, cost, phi_g, psi_g, inst.mu, inst.nu)
    c_o = oracle.plan_stats(logk, cost, phi_o, psi_o)[0]
    return rep, l1, e1, e2, err_o, c_g, c_o


def test_sinkhorn_tiny_200_iterations(nat):
    inst = synth.tiny_ot(0)
    rep, l1, e1, e2, err_o, c_g, c_o = _ot_parity(nat, inst, 200)
    assert l1 <= 1e-5, l1
    assert abs(e1 - err_o) <= 1e-6 and e2 <= 1e-6, (e1, err_o, e2)
    assert abs(rep["marg_l1"] - err_o) <= 1e-6
    assert abs(rep["marg_l1_f64"] - (e1 + e2)) <= 1e-9 * max(1.0, e1 + e2) + 1e-12
    assert abs(c_g - c_o) <= 1e-6 * c_o
    assert abs(rep["cost"] - c_o) <= 1e-5 * c_o


def test_sinkhorn_f64_engine(nat):
    """prec = F64 runs every convolution with FP64 exponentials and sums: the iterate
    then agrees with the FP64 oracle to rounding (plan L1 1e-9 after 200 iterations)."""
    torch = torch_dev()
    inst = synth.tiny_ot(1)
    g = inst.grid
    k = _kernel(nat, g.nx, g.ny, g.nt, g.axial, inst.w, inst.eps, inst.radius)
    logk, _ = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
    mu, nu = to_dev(inst.mu), to_dev(inst.nu)
    phi_o, psi_o, _, err_o, _ = oracle.sinkhorn(logk, inst.mu, inst.nu, 200, -1.0)
    l1 = {}
    for prec in (nat.SE2_F32, nat.SE2_F64):
        f = torch.empty_like(mu)
        gg = torch.empty_like(mu)
        rep = nat.se2_sinkhorn(k, mu, nu, nat.opts(tol=-1, max_iter=200, check_every=50, prec=prec), f, gg)
        l1[prec] = oracle.plan_l1(logk, to_host(f) / inst.eps, to_host(gg) / inst.eps, phi_o, psi_o)
        assert abs(rep["marg_l1"] - err_o) <= 1e-6
    assert l1[nat.SE2_F64] <= 1e-9, l1
    assert l1[nat.SE2_F32] <= 1e-5, l1


def test_sinkhorn_converges_to_tolerance(nat):
    """A smooth random pair at eps = 1 reaches 1e-6 in a few hundred iterations (478 in the oracle)."""
    rng = np.random.default_rng(31)
    g = synth.Grid(12, 10, 8)
    mu = rng.uniform(0.2, 1.0, g.shape)
    mu /= mu.sum()
    nu = rng.uniform(0.2, 1.0, g.shape)
    nu /= nu.sum()
    inst = synth.OTInstance(g, (1.0, 2.0, 1.0), 1.0, 3, mu, nu, "smooth12x10x8")
    rep, l1, e1, e2, err_o, c_g, c_o = _ot_parity(nat, inst, 3000, tol=1e-6)
    assert rep["status"] == nat.SE2_CONVERGED
    assert e1 + e2 <= 2e-6 and rep["marg_l1_f64"] <= 2e-6, (e1, e2, rep["marg_l1_f64"])
    assert abs(c_g - c_o) <= 1e-3 * c_o


@pytest.mark.parametrize("prune", [True, False])
def test_sinkhorn_lines64_matches_oracle(nat, prune):
    """The 64x64x16 workload at full size, 12 iterations, pruned and dense engines."""
    torch = torch_dev()
    inst = synth.lines64(3, paired=True)
    g = inst.grid
    k = _kernel(nat, g.nx, g.ny, g.nt, g.axial, inst.w, inst.eps, inst.radius)
    logk, cost = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
    mu, nu = to_dev(inst.mu), to_dev(inst.nu)
    f = torch.empty_like(mu)
    gg = torch.empty_like(mu)
    rep = nat.se2_sinkhorn(k, mu, nu, nat.opts(tol=-1, max_iter=12, check_every=4, prune=prune), f, gg)
    phi_o, psi_o, it_o, err_o, _ = oracle.sinkhorn(logk, inst.mu, inst.nu, 12, -1.0)
    phi_g, psi_g = to_host(f) / inst.eps, to_host(gg) / inst.eps
    l1 = oracle.plan_l1(logk, phi_g, psi_g, phi_o, psi_o)
    assert l1 <= 1e-5, l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6, (rep["marg_l1"], err_o)


def test_pruned_equals_dense_over_many_iterations(nat):
    """Certified pruning against the dense engine over 300 iterations at 64x64x16."""
    torch = torch_dev()
    inst = synth.lines64(4, paired=True)
    g = inst.grid
    k = _kernel(nat, g.nx, g.ny, g.nt, g.axial, inst.w, inst.eps, inst.radius)
    logk, cost = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
    mu, nu = to_dev(inst.mu), to_dev(inst.nu)
    out = {}
    for prune in (False, True):
        f = torch.empty_like(mu)
        gg = torch.empty_like(mu)
        rep = nat.se2_sinkhorn(k, mu, nu, nat.opts(tol=-1, max_iter=300, check_every=25, prune=prune), f, gg)
        out[prune] = (to_host(f) / inst.eps, to_host(gg) / inst.eps, rep)
    l1 = oracle.plan_l1(logk, out[True][0], out[True][1], out[False][0], out[False][1])
    assert l1 <= 1e-6, l1
    assert abs(out[True][2]["marg_l1"] - out[False][2]["marg_l1"]) <= 1e-7
    assert abs(out[True][2]["cost"] - out[False][2]["cost"]) <= 1e-6 * out[False][2]["cost"]


def test_barycenter_small(nat):
    torch = torch_dev()
    g = synth.Grid(16, 16, 8)
    mus = [synth.splat_segments(g, synth.draw_segments(synth.rng_for(77, s), g, 3, 3.0, 10.0), 1.0, 1e-6)
           for s in range(3)]
    lam = [0.2, 0.5, 0.3]
    w, eps, R = (1.0, 2.0, 1.0), 0.5, 4
    k = _kernel(nat, 16, 16, 8, False, w, eps, R)
    logk, _ = oracle.kernel_table(8, False, w, eps, R)
    out = torch.empty((16, 16, 8), dtype=torch.float64, device="cuda")
    rep = nat.se2_barycenter(k, [to_dev(m) for m in mus], lam, nat.opts(tol=-1, max_iter=60, check_every=1), out)
    bar_o, it_o, err_o, _ = oracle.ibp(logk, mus, lam, 60, -1.0)
    bar_g = to_host(out)
    assert rep["iters"] == it_o == 60
    l1 = float(np.sum(np.abs(bar_g - bar_o)))
    assert l1 <= 1e-5, l1
    assert abs(rep["marg_l1"] - err_o) <= 1e-6
    assert abs(rep["mass"] - bar_o.sum()) <= 1e-6


@pytest.mark.parametrize("shape", [(20, 13, 8, False), (21, 18, 16, False), (12, 10, 32, True)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{'a' if c[3] else ''}")
def test_barycenter_cost_matches_oracle(nat, shape):
    """Transport cost and barycenter mass of an IBP solve (Appendix A): the cost is
    sum_i lambda_i <pi_i, rho_b^2> with pi_i = diag(w_i) K diag(v_i) of the returned iterate,
    whose w_i comes from the w-update that measured its error (so pi_i has marginal mu_i),
    computed on the GPU from the measures' pointer tables; ragged tiles and all three
    orientation counts."""
    torch = torch_dev()
    nx, ny, nt, axial = shape
    g = synth.Grid(nx, ny, nt, axial)
    mus = [synth.splat_segments(g, synth.draw_segments(synth.rng_for(79, s), g, 3, 3.0, 9.0), 1.0, 1e-6)
           for s in range(3)]
    lam = [0.25, 0.45, 0.3]
    w, eps, R = (1.0, 2.0, 1.0), 0.4, 3
    k = _kernel(nat, nx, ny, nt, axial, w, eps, R)
    logk, cost = oracle.kernel_table(nt, axial, w, eps, R)
    out = torch.empty((ny, nx, nt), dtype=torch.float64, device="cuda")
    rep = nat.se2_barycenter(k, [to_dev(m) for m in mus], lam, nat.opts(tol=-1, max_iter=12, check_every=4), out)
    bar_o, it_o, _, _, lv = oracle.ibp(logk, mus, lam, 12, -1.0, return_lv=True)
    assert rep["iters"] == it_o == 12
    c_o = 0.0
    for i in range(3):
        lw = oracle.safe_log(mus[i]) - oracle.conv_log(logk, lv[i])
        c_i, m_i, _, _ = oracle.plan_stats(logk, cost, lw, lv[i])
        assert abs(m_i - mus[i].sum()) <= 1e-9 * mus[i].sum()   # the mu_i side of pi_i is exact
        c_o += lam[i] * c_i
    assert abs(rep["cost"] - c_o) <= 1e-5 * c_o, (rep["cost"], c_o)
    assert abs(rep["mass"] - bar_o.sum()) <= 1e-6


def test_plan_statistics_on_a_large_grid(nat):
    """Transport cost and plan mass on 256 x 256 x 16 (the plan statistics then take four
    orientations per lane): from the GPU's own potentials after 6 iterations, against the
    oracle's sums over the same plan."""
    torch = torch_dev()
    inst = synth.lines64(2, n=256)
    g = inst.grid
    k = _kernel(nat, g.nx, g.ny, g.nt, False, inst.w, inst.eps, inst.radius)
    logk, cost = oracle.kernel_table(g.nt, False, inst.w, inst.eps, inst.radius)
    mu, nu = to_dev(inst.mu), to_dev(inst.nu)
    f, gg = torch.empty_like(mu), torch.empty_like(mu)
    rep = nat.se2_sinkhorn(k, mu, nu, nat.opts(tol=-1, max_iter=6, check_every=3), f, gg)
    c_o, m_o, _, _ = oracle.plan_stats(logk, cost, to_host(f) / inst.eps, to_host(gg) / inst.eps)
    assert abs(rep["cost"] - c_o) <= 1e-6 * c_o, (rep["cost"], c_o)
    assert abs(rep["mass"] - m_o) <= 1e-6 * m_o, (rep["mass"], m_o)


def test_barycenter_cost_on_a_large_grid(nat):
    """The barycenter's plan statistics over the measures' pointer tables on 256 x 256 x 16
    (four orientations per lane there), 3 IBP iterations of two measures with a 3 x 3 window:
    cost and barycenter against the oracle."""
    torch = torch_dev()
    g = synth.Grid(256, 256, 16)
    mus = [synth.splat_segments(g, synth.draw_segments(synth.rng_for(80, s), g, 6, 20.0, 60.0), 2.0, 1e-6)
           for s in range(2)]
    lam = [0.4, 0.6]
    w, eps, R = (1.0, 2.0, 1.0), 0.5, 1
    k = _kernel(nat, 256, 256, 16, False, w, eps, R)
    logk, cost = oracle.kernel_table(16, False, w, eps, R)
    out = torch.empty((256, 256, 16), dtype=torch.float64, device="cuda")
    rep = nat.se2_barycenter(k, [to_dev(m) for m in mus], lam, nat.opts(tol=-1, max_iter=3, check_every=3), out)
    bar_o, it_o, _, _, lv = oracle.ibp(logk, mus, lam, 3, -1.0, return_lv=True)
    assert rep["iters"] == it_o == 3
    assert float(np.sum(np.abs(to_host(out) - bar_o))) <= 1e-5
    c_o = sum(l_ * oracle.plan_stats(logk, cost, oracle.safe_log(m) - oracle.conv_log(logk, v), v)[0]
              for l_, m, v in zip(lam, mus, lv))
    assert abs(rep["cost"] - c_o) <= 1e-5 * c_o, (rep["cost"], c_o)


def test_barycenter_weight_on_one_measure(nat):
    """lambda = e_1: the closed form bar = K*(mu_1 / K*1) (Appendix A with one active measure)."""
    torch = torch_dev()
    g = synth.Grid(12, 12, 16)
    mus = [synth.splat_segments(g, synth.draw_segments(synth.rng_for(78, s), g, 2, 3.0, 8.0), 1.0, 1e-6)
           for s in range(2)]
    w, eps, R = (1.0, 3.0, 1.0), 0.3, 3
    k = _kernel(nat, 12, 12, 16, False, w, eps, R)
    logk, _ = oracle.kernel_table(16, False, w, eps, R)
    want = oracle.conv_linear(logk, mus[0] / oracle.conv_linear(logk, np.ones_like(mus[0])))
    out = torch.empty((12, 12, 16), dtype=torch.float64, device="cuda")
    nat.se2_barycenter(k, [to_dev(m) for m in mus], [1.0, 0.0], nat.opts(tol=-1, max_iter=5), out)
    e = float(np.max(np.abs(to_host(out) - want) / want))
    assert e <= 2e-6, e


def test_invalid_inputs_rejected(nat):
    torch = torch_dev()
    k = _kernel(nat, 8, 8, 8, False, (1, 2, 1), 0.5, 2)
    good = np.full((8, 8, 8), 1.0 / 512)
    bad = good.copy()
    bad[0, 0, 0] = -1e-3
    bad[0, 0, 1] += 1e-3
    with pytest.raises(nat.SE2Error) as e:
        nat.se2_sinkhorn(k, to_dev(bad), to_dev(good), nat.opts())
    assert e.value.code == nat.SE2_EINVAL
    nanm = good.copy()
    nanm[1, 1, 1] = np.nan
    with pytest.raises(nat.SE2Error):
        nat.se2_sinkhorn(k, to_dev(nanm), to_dev(good), nat.opts())
    with pytest.raises(nat.SE2Error):
        nat.se2_barycenter(k, [to_dev(good), to_dev(good)], [0.7, 0.4], nat.opts(),
                           torch.empty((8, 8, 8), dtype=torch.float64, device="cuda"))


def test_conv_rejects_misaligned_float_input(nat):
    """The float paths stage their input with 16-byte loads: a misaligned input is refused on
    the host, before any launch."""
    torch = torch_dev()
    k = _kernel(nat, 8, 8, 16, False, (1, 2, 1), 0.5, 2)
    buf = torch.zeros(8 * 8 * 16 + 1, dtype=torch.float32, device="cuda")
    x = buf[1:].view(8, 8, 16)
    out = torch.empty((8, 8, 16), dtype=torch.float32, device="cuda")
    for prec in (nat.SE2_BF16, nat.SE2_F32):
        with pytest.raises(nat.SE2Error) as e:
            nat.se2_conv(k, prec, x, out)
        assert e.value.code == nat.SE2_EINVAL
    nat.se2_conv(k, nat.SE2_F32, buf[:8 * 8 * 16].view(8, 8, 16), out)   # aligned: accepted
    torch.cuda.synchronize()
