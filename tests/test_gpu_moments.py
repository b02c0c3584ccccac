"""Zero-field susceptibility from summed second-moment insertions on the GPU
(C ABI) against the CPU oracle.

A run with GXY_IMP_COS1_SQ / GXY_IMP_COS2_SQ carries, next to the pure and
one-insertion tensors, the tensor with two insertions averaged over ordered
pairs of sites: T2' = (T2 (x) T + T (x) T2 + 2 T1 (x) T1) / 4 with the pure
tensor's projector and norm; <m^2> = Tr T2 / Tr T and
chi = beta V (<m^2> - <m>^2) (Ch. 3, eq. susc by the fluctuation relation).
FP64 gates: ln Z/V 1e-12 (as every run), <m^2> and chi relative 1e-11, the
one-insertion values exactly zero at zero field.
"""

import math

import pytest

import oracle.hotrg as o
from paper_2609_20536_amd import workloads as W
from tests.test_gpu_parity import _compare

pytestmark = pytest.mark.gpu

SQ = W.IMP_COS1_SQ | W.IMP_COS2_SQ


@pytest.fixture(scope="module")
def ctx():
    from paper_2609_20536_amd import hotrg as H
    c = H.Context(0)
    yield c
    c.close()


def _moments_match(g, r, rel=1e-11):
    for a, b in ((g.msq_cos1, r.msq_cos1), (g.msq_cos2, r.msq_cos2),
                 (g.chi0, r.chi0), (g.chi0_n, r.chi0_n)):
        if math.isnan(b):
            assert math.isnan(a)
        else:
            assert a == pytest.approx(b, rel=rel), (a, b)


MOMENT_POINTS = [
    dict(beta=1.0, delta=0.5, nmax=3, dcut=12, nsteps=10, impurities=SQ),
    dict(beta=0.7, delta=0.8, nmax=4, dcut=13, nsteps=9, impurities=W.IMP_COS1_SQ),  # ragged
    dict(beta=1.1, delta=0.3, nmax=5, dcut=20, nsteps=12, impurities=SQ),
    dict(beta=1.2, delta=0.4, nmax=3, dcut=14, nsteps=10, impurities=SQ, q=3),
    dict(beta=0.9, delta=0.6, nmax=3, dcut=128, nsteps=2, impurities=SQ),   # 2x2, untruncated
    dict(beta=0.9, delta=0.6, nmax=1, dcut=128, nsteps=3, impurities=SQ),   # 4x2, untruncated
]


@pytest.mark.parametrize("pt", MOMENT_POINTS,
                         ids=lambda p: ",".join(f"{k}={v}" for k, v in p.items()))
def test_moment_runs_match_oracle(ctx, pt):
    g = ctx.run(pt)
    r = o.run_point(**pt)
    _compare(g, r, pt)
    _moments_match(g, r)
    assert g.chi0 > 0.0 and g.m_cos1 == 0.0


def test_beta_zero_half_per_site_exactly(ctx):
    g = ctx.run(dict(beta=0.0, delta=0.5, nmax=3, dcut=12, nsteps=11, impurities=SQ))
    V = 2.0 ** 11
    assert g.msq_cos1 * V == 0.5 and g.msq_cos2 * V == 0.5
    assert g.chi0 == 0.0 and g.chi0_n == 0.0


def test_moment_chains_do_not_change_the_rest(ctx):
    """Adding the second-moment chains changes neither ln Z/V nor the
    one-insertion values (the pure tensor's truncation drives them all)."""
    p = dict(beta=1.1, delta=0.3, nmax=5, dcut=20, nsteps=12)
    a = ctx.run(dict(p, impurities=3))
    b = ctx.run(dict(p, impurities=SQ))
    assert a.lnz_per_site == b.lnz_per_site
    assert a.m_cos1 == b.m_cos1 and a.m_cos2 == b.m_cos2
    assert math.isnan(a.chi0) and math.isnan(a.msq_cos1)


def test_moment_chains_need_zero_field(ctx):
    from paper_2609_20536_amd import hotrg as H
    with pytest.raises(H.GxyError) as e:
        ctx.run(dict(beta=1.0, delta=0.5, h=1e-3, nmax=3, dcut=12, nsteps=6, impurities=SQ))
    assert e.value.status == 5


def test_moment_batch_equals_single(ctx):
    pts = [dict(beta=b, delta=0.5, nmax=4, dcut=14, nsteps=10, impurities=SQ)
           for b in (0.8, 1.0, 1.2)]
    res = ctx.run_batch(pts, workers=3)
    for p, rb in zip(pts, res):
        rs = ctx.run(p)
        assert rb.chi0 == rs.chi0 and rb.chi0_n == rs.chi0_n and rb.lnz_per_site == rs.lnz_per_site


def test_bench_size_moment_run(ctx):
    """The bench workload (Dcut = 64, |n| <= 10, 40 steps) with both
    second-moment chains: finite, positive, deterministic."""
    p = W.precision_point(64).with_(impurities=SQ)
    a, b = ctx.run(p), ctx.run(p)
    assert a.status == 0 and a.chi0 > 0 and a.chi0_n > 0
    assert math.isfinite(a.chi0) and a.chi0 == b.chi0 and a.chi0_n == b.chi0_n
    assert a.m_cos1 == 0.0 and a.m_cos2 == 0.0
