"""se2_split_signed_noalloc (the entry point that allocates nothing) against se2_split_signed.

Both run the same kernels in the same order, so the outputs must agree bit for bit; two
calls in a row, the second on a smaller input, show that the library's scratch (which keeps
the last call's contents) leaves no trace in the next result.
"""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    torch_dev()
    from paper_2402_15322_amd import native
    native.se2_init()
    return native


def test_noalloc_split_equals_allocating_split(nat):
    torch = torch_dev()
    rng = np.random.default_rng(4242)
    for n in (3_000_017, 70_001):          # 184 then 5 partial blocks: the second call is smaller
        u = rng.normal(0.0, 1.0, n)
        ud = to_dev(u)
        p0 = torch.empty(n, dtype=torch.float64, device="cuda")
        m0 = torch.empty_like(p0)
        p1 = torch.full_like(p0, float("nan"))
        m1 = torch.full_like(p0, float("nan"))
        nat.se2_split_signed(ud, p0, m0)
        nat.se2_split_signed_noalloc(ud, p1, m1)
        a0, b0, a1, b1 = to_host(p0), to_host(m0), to_host(p1), to_host(m1)
        assert np.array_equal(a0.view(np.uint64), a1.view(np.uint64)), n
        assert np.array_equal(b0.view(np.uint64), b1.view(np.uint64)), n
        # and the parts are what the split means: normalised, disjoint supports
        assert abs(a1.sum() - 1.0) <= 1e-12 and abs(b1.sum() - 1.0) <= 1e-12
        assert not np.any((a1 > 0) & (b1 > 0))


def test_noalloc_split_at_its_maximum_and_empty(nat):
    """n = 4096 * 16384, the largest input the scratch serves (every one of its 4096 block
    partials used), bit for bit against the allocating split; then an empty input, which
    both entry points accept and which writes nothing."""
    torch = torch_dev()
    n = 4096 * 16384
    g = torch.Generator(device="cuda").manual_seed(77)
    ud = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    p0, m0 = torch.empty_like(ud), torch.empty_like(ud)
    p1, m1 = torch.full_like(ud, float("nan")), torch.full_like(ud, float("nan"))
    nat.se2_split_signed(ud, p0, m0)
    nat.se2_split_signed_noalloc(ud, p1, m1)
    assert torch.equal(p0.view(torch.int64), p1.view(torch.int64))
    assert torch.equal(m0.view(torch.int64), m1.view(torch.int64))
    assert abs(float(p1.sum()) - 1.0) <= 1e-9 and abs(float(m1.sum()) - 1.0) <= 1e-9
    del ud, p0, m0, p1, m1
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    nat.se2_split_signed(e, e, e)
    nat.se2_split_signed_noalloc(e, e, e)
    torch.cuda.synchronize()


def test_noalloc_split_rejects_oversized_input(nat):
    torch = torch_dev()
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    lib = nat.load()
    # n beyond 4096 * 16384 elements: refused on the host before any device work
    rc = lib.se2_split_signed_noalloc(x.data_ptr(), 4096 * 16384 + 1, x.data_ptr(), x.data_ptr(), None)
    assert rc == nat.SE2_EINVAL
    assert b"exceeds the maximum" in lib.se2_strerror(rc)
