"""Lift and projection on the GPU (Sections 2.3, 5.2, 5.3) against the oracle.

Bars: the lift copies a magnitude or writes 0, so it is compared bit for bit (away from
bin edges, where the two sides' FP64 arithmetic may round an angle into different bins);
projected masses are sums of ntheta terms in a different order, within 1e-15 of the sum of
magnitudes; the argmax is an index and is compared exactly (both sides compare the same
FP64 values, lowest index on ties); the split is within 1e-15 relative.  The end-to-end
field pipeline (lift, barycenter, projection) follows the barycenter bar: L1 <= 1e-5.
"""
from __future__ import annotations

import math

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


CASES = [(8, False, (2, 33, 47)), (16, False, (1, 64, 64)), (32, True, (3, 17, 9)), (16, True, (1, 1, 1))]


@pytest.mark.parametrize("nt,axial,shape", CASES)
def test_lift_field_matches_oracle(nat, nt, axial, shape):
    torch = torch_dev()
    rng = np.random.default_rng(50 + nt)
    mag = rng.uniform(0.0, 1.0, shape)
    mag.flat[0] = 0.0
    ang = rng.uniform(-3 * math.pi, 3 * math.pi, shape)
    out = torch.empty(shape + (nt,), dtype=torch.float64, device="cuda")
    nat.se2_lift_field(nt, axial, to_dev(mag), to_dev(ang), out)
    got = to_host(out)
    want = oracle.lift_field(mag, ang, nt, axial)
    period = math.pi if axial else 2 * math.pi
    step = period / nt
    frac = np.mod(ang / step + 0.5, 1.0)
    clear = (frac > 1e-9) & (frac < 1 - 1e-9)          # not within rounding of a bin edge
    assert np.array_equal(got[clear], want[clear])
    assert np.all(np.count_nonzero(got, axis=-1) == (mag > 0))
    assert np.array_equal(got.sum(axis=-1), mag)


@pytest.mark.parametrize("nt,axial,shape", CASES)
def test_project_matches_oracle(nat, nt, axial, shape):
    torch = torch_dev()
    rng = np.random.default_rng(60 + nt)
    u = np.round(rng.uniform(0.0, 1.0, shape + (nt,)) * 4) / 4     # few levels: many ties in the argmax
    um = rng.uniform(0.0, 1.0, shape + (nt,))
    ud, umd = to_dev(u), to_dev(um)
    mass = torch.empty(shape, dtype=torch.float64, device="cuda")
    ang = torch.empty_like(mass)
    arg = torch.empty(shape, dtype=torch.int32, device="cuda")
    nat.se2_project(axial, ud, mass, argmax=arg, angle=ang)
    m_o, a_o = oracle.project(u)
    assert np.array_equal(to_host(mass), m_o)          # sums of quarters: exact in any order
    assert np.array_equal(to_host(arg), a_o)
    step = (math.pi if axial else 2 * math.pi) / nt
    assert np.array_equal(to_host(ang), a_o * step)
    nat.se2_project(axial, ud, mass, u_minus=umd)
    m_o, _ = oracle.project(u, um)
    bound = nt * 2.3e-16 * (u.sum(-1) + um.sum(-1))    # reordered FP64 sums of 2 nt terms
    assert np.all(np.abs(to_host(mass) - m_o) <= bound)


def test_split_signed_matches_oracle(nat):
    torch = torch_dev()
    rng = np.random.default_rng(70)
    for n in (100003, 7, 1):
        u = rng.normal(0.0, 1.0, n)
        if n == 1:
            u[0] = abs(u[0])                    # no negative part: it comes back as zeros
        p, m = torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda")
        nat.se2_split_signed(to_dev(u), p, m)
        po, mo = oracle.split_signed(u)
        assert np.max(np.abs(to_host(p) - po)) <= 1e-15 * max(po.max(), 1e-300)
        assert np.max(np.abs(to_host(m) - mo)) <= 1e-15 * max(mo.max(), 1e-300)


def test_field_pipeline_matches_oracle(nat):
    """Two smooth orientation fields on a 48 x 48 x 8 axial grid (the 256 x 256 x 32 field
    workload's formula, eps, metric and 21 x 21 window), lifted with the paper's one-bin lift,
    interpolated at t = 1/2 with 3 IBP iterations, projected back to magnitude and angle."""
    torch = torch_dev()
    n, nt = 48, 8
    w, eps, R = (1.0, 4.0, 1.0), 0.03, 10
    angs = [synth.orientation_field(synth.rng_for(4800 + s, 0), n) for s in range(2)]
    mag = np.full((n, n), 1.0 / (n * n))
    k = nat.Kernel(n, n, nt, True, w, eps, R)
    lifted = []
    for a in angs:
        out = torch.empty((n, n, nt), dtype=torch.float64, device="cuda")
        nat.se2_lift_field(nt, True, to_dev(mag), to_dev(a), out)
        lifted.append(out)
    bar = torch.empty((n, n, nt), dtype=torch.float64, device="cuda")
    rep = nat.se2_barycenter(k, lifted, [0.5, 0.5], nat.opts(tol=-1, max_iter=3, check_every=3), bar)
    mass = torch.empty((n, n), dtype=torch.float64, device="cuda")
    arg = torch.empty((n, n), dtype=torch.int32, device="cuda")
    nat.se2_project(True, bar, mass, argmax=arg)
    # oracle: the same three steps
    mus = [oracle.lift_field(mag, a, nt, True) for a in angs]
    for m, l in zip(mus, lifted):
        assert np.array_equal(to_host(l), m)
    logk, _ = oracle.kernel_table(nt, True, w, eps, R)
    bar_o, it_o, err_o, _ = oracle.ibp(logk, mus, [0.5, 0.5], 3, -1.0)
    assert rep["iters"] == it_o == 3
    bar_g = to_host(bar)
    assert float(np.sum(np.abs(bar_g - bar_o))) <= 1e-5
    m_o, a_o = oracle.project(bar_o)
    assert float(np.sum(np.abs(to_host(mass) - m_o))) <= 1e-5
    # the argmax is unique where the oracle's top two bins differ by more than the barycenter
    # bar; elsewhere (mass split between bins) the GPU's pick must be one of the top bins
    srt = np.sort(bar_o, axis=-1)
    clear = (srt[..., -1] - srt[..., -2]) > 1e-6 * srt[..., -1]
    assert clear.mean() > 0.3
    ga = to_host(arg)
    assert np.array_equal(ga[clear], a_o[clear])
    picked = np.take_along_axis(bar_o, ga[..., None].astype(np.int64), axis=-1)[..., 0]
    assert np.all(picked >= srt[..., -1] * (1 - 1e-5))
