"""Batched runs (worker contexts on their own streams) and the tile autotuner.

A batch must return, for every point, exactly (bit for bit) what a single
run of that point returns: the workers run the same deterministic kernels
on their own streams. The autotuner's tile choice must not change results
(every output element is accumulated over the same k-slices in order).
"""

import math

import pytest

from paper_2609_20536_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2609_20536_amd import hotrg as H
    c = H.Context(0)
    yield c
    c.close()


def _mixed_points():
    """Uneven Dcut, fields, chains and precisions in one batch."""
    base = W.Point(beta=1.1, delta=0.6, nmax=3, dcut=12, nsteps=14, impurities=3)
    return [
        base,
        base.with_(dcut=24, nmax=5, nsteps=10),
        base.with_(dcut=13, h=0.05, impurities=1, nsteps=8),
        base.with_(dcut=16, h1=0.07, impurities=2),
        base.with_(dcut=32, nmax=10, nsteps=8, impurities=0),
        base.with_(dcut=20, nmax=10, nsteps=6, prec=W.PREC_BF16X3, fp64_steps=2),
        base.with_(dcut=1, nsteps=5),
        base.with_(beta=0.7, dcut=12, nsteps=20, impurities=0),
        base.with_(dcut=14, nmax=4, nsteps=10, q=3),
        base.with_(dcut=12, h1=0.2, nsteps=8, q=4),
    ]


def _same(a, b):
    for f in ("lnz_per_site", "m_cos1", "m_cos2", "max_trunc_err", "min_cut_gap"):
        x, y = getattr(a, f), getattr(b, f)
        if not (x == y or (math.isnan(x) and math.isnan(y))):
            return False
    return a.status == b.status


@pytest.mark.parametrize("workers", [1, 3, 8])
def test_batch_equals_single_runs(ctx, workers):
    pts = _mixed_points()
    singles = [ctx.run(p) for p in pts]
    logs = [ctx.step_log(0) for _ in [0]]
    res = ctx.run_batch(pts, workers=workers)
    for i, (r, s) in enumerate(zip(res, singles)):
        assert _same(r, s), (i, r, s)
    assert [x["lnc"] for x in ctx.step_log(len(pts) - 1)] == [x["lnc"] for x in logs[0]]


def test_batch_reports_invalid_points_per_run(ctx):
    pts = _mixed_points()[:3]
    pts.insert(1, pts[0].with_(delta=2.0))
    res = ctx.run_batch(pts, workers=2)
    assert res[1].status == 1 and math.isnan(res[1].lnz_per_site)
    assert all(r.status == 0 for i, r in enumerate(res) if i != 1)


def test_autotune_picks_a_tile_and_keeps_results(ctx):
    pt = W.precision_point(dcut=24, impurities=0).with_(nsteps=8)
    before = ctx.run(pt)
    table = ctx.autotune(pt, [24, 32])
    for d, (tile, ms64, ms128, ms256) in table.items():
        assert tile in (64, 128, 256)
        assert ms64 > 0 and ms128 > 0 and ms256 > 0
        assert {64: ms64, 128: ms128, 256: ms256}[tile] == min(ms64, ms128, ms256)
    after = ctx.run(pt)
    assert after.lnz_per_site == before.lnz_per_site


@pytest.mark.parametrize("dma", ["0", "1"])
@pytest.mark.parametrize("chunk_mb", [8, 96])
def test_projection_chunks_do_not_change_results(ctx, chunk_mb, dma, monkeypatch):
    """Splitting the projection over the output index a (several chunks, each
    with its own planned launches) gives the same bits as one chunk: every
    element of X, Y and T' belongs to exactly one chunk and is reduced in the
    same order."""
    pts = [W.Point(beta=1.1, delta=0.6, nmax=5, dcut=24, nsteps=8, impurities=3),
           W.Point(beta=0.9, delta=0.4, nmax=4, dcut=20, nsteps=7, h1=0.05, impurities=3)]
    monkeypatch.setenv("GXY_GEMM_DMA", dma)
    whole = [ctx.run(p) for p in pts]
    monkeypatch.setenv("GXY_CHUNK_BYTES", str(chunk_mb << 20))
    for p, w in zip(pts, whole):
        r = ctx.run(p)
        assert _same(r, w), (p, r, w)


@pytest.mark.parametrize("prec,k,dma", [(W.PREC_FP64, 0, "0"), (W.PREC_FP64, 0, "1"),
                                        (W.PREC_FP32, 3, "0"), (W.PREC_BF16X3, 3, "0")])
def test_projection_tiles_give_the_same_bits(ctx, prec, k, dma, monkeypatch):
    """64 x 64, 128 x 128 and 256 x 128 projection tiles accumulate every
    output element over the same k-slices in the same order, in each
    arithmetic form and with either operand staging of the FP64 products."""
    monkeypatch.setenv("GXY_GEMM_DMA", dma)
    pts = [W.Point(beta=1.1, delta=0.6, nmax=6, dcut=32, nsteps=8, impurities=3, prec=prec,
                   fp64_steps=k),
           W.Point(beta=0.9, delta=0.4, nmax=5, dcut=24, nsteps=7, h1=0.05, impurities=3,
                   prec=prec, fp64_steps=k)]
    ref = None
    for tile in ("64", "128", "256"):
        monkeypatch.setenv("GXY_PROJ_TILE", tile)
        res = [ctx.run(p) for p in pts]
        if ref is None:
            ref = res
        for r, q in zip(res, ref):
            assert _same(r, q), (tile, r, q)
