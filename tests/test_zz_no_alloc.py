"""gxy_run_noalloc (runs in the library's static device scratch array)
against gxy_run, through the C ABI."""

import ctypes as C
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2609_20536_amd import hotrg as H
    c = H.Context(0)
    yield c
    c.close()


def _same(a, b):
    assert a.status == 0 and b.status == 0
    assert a.lnz_per_site == b.lnz_per_site, (a.lnz_per_site, b.lnz_per_site)
    for x, y in ((a.m_cos1, b.m_cos1), (a.m_cos2, b.m_cos2)):
        assert (math.isnan(x) and math.isnan(y)) or x == y, (x, y)
    assert [s["lnc"] for s in a.steps] == [s["lnc"] for s in b.steps]
    assert [s["side"] for s in a.steps] == [s["side"] for s in b.steps]


CASES = [
    # U(1) sectors with both impurity chains, then a smaller run
    (dict(beta=1.1, delta=0.6, nmax=5, dcut=20, nsteps=12, impurities=3),
     dict(beta=1.2, delta=0.7, nmax=3, dcut=12, nsteps=10, impurities=3)),
    # Z2 sectors, then one dense block (fields), smaller again
    (dict(beta=1.0, delta=0.5, nmax=4, dcut=16, nsteps=10, h1=0.05, impurities=2),
     dict(beta=1.0, delta=0.5, nmax=3, dcut=12, nsteps=8, h=0.05, impurities=1)),
]


@pytest.mark.parametrize("big,small", CASES)
def test_noalloc_matches_run_twice_in_a_row(ctx, big, small):
    a = ctx.run_noalloc(big)
    b = ctx.run_noalloc(small)          # second call, smaller input
    _same(a, ctx.run(big))
    _same(b, ctx.run(small))
    # and again after the context's own workspace was used
    _same(ctx.run_noalloc(small), b)


def test_noalloc_rejects_runs_beyond_the_scratch(ctx):
    from paper_2609_20536_amd import hotrg as H
    p = H.make_point(beta=1.2, delta=0.7, nmax=10, dcut=64, nsteps=40, impurities=3)
    r = H.Result()
    st = ctx.lib.gxy_run_noalloc(ctx.handle, C.byref(p), C.byref(r))
    assert st == 1
    msg = ctx.lib.gxy_last_error(ctx.handle).decode()
    assert "holds at most" in msg and str(256 << 20) in msg
    # the context still runs normally afterwards
    q = dict(beta=1.2, delta=0.7, nmax=3, dcut=12, nsteps=10, impurities=3)
    _same(ctx.run_noalloc(q), ctx.run(q))
