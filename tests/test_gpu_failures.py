"""Failure reporting of a run (C ABI): non-finite values name the step at
which they appear, a caller workspace that is too small is refused before
any device work, and the context keeps working afterwards.

The NaN is planted from the host (GXY_INJECT_NAN_STEP = n puts one NaN into
the site tensor after step n's normalisation) only where no eigensolver sees
it: after the last step, or ahead of steps whose fused bond fits (no
truncation), so every kernel runs on its usual loop bounds and exits
normally.
"""

import ctypes as C
import math

import pytest

import oracle.hotrg as o

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2609_20536_amd import hotrg as H
    c = H.Context(0)
    yield c
    c.close()


def test_nan_after_the_last_step_fails_at_the_trace(ctx, monkeypatch):
    pt = dict(beta=1.0, delta=0.5, nmax=3, dcut=12, nsteps=6, impurities=3)
    monkeypatch.setenv("GXY_INJECT_NAN_STEP", "6")
    r = ctx.run(pt)
    assert r.status == 4 and r.fail_step == 6
    assert math.isnan(r.lnz_per_site)


def test_nan_ahead_of_untruncated_steps_names_the_first_bad_norm(ctx, monkeypatch):
    pt = dict(beta=0.9, delta=0.4, nmax=1, dcut=128, nsteps=3, impurities=3)
    monkeypatch.setenv("GXY_INJECT_NAN_STEP", "1")
    r = ctx.run(pt)
    assert r.status == 4 and r.fail_step == 2
    assert math.isnan(r.lnz_per_site) and math.isnan(r.m_cos1)


def test_context_runs_normally_after_a_failure(ctx, monkeypatch):
    pt = dict(beta=0.9, delta=0.4, nmax=1, dcut=128, nsteps=3, impurities=3)
    monkeypatch.setenv("GXY_INJECT_NAN_STEP", "1")
    assert ctx.run(pt).status == 4
    monkeypatch.delenv("GXY_INJECT_NAN_STEP")
    g = ctx.run(pt)
    assert g.status == 0 and g.fail_step == -1
    assert abs(g.lnz_per_site - o.run_point(**pt).lnz_per_site) <= 1e-13


def test_batch_reports_the_failed_runs(ctx, monkeypatch):
    pts = [dict(beta=b, delta=0.4, nmax=1, dcut=128, nsteps=3, impurities=0) for b in (0.7, 0.9)]
    monkeypatch.setenv("GXY_INJECT_NAN_STEP", "1")
    res = ctx.run_batch(pts, workers=2)
    assert all(r.status == 4 and r.fail_step == 2 for r in res)


def test_small_caller_workspace_is_refused(ctx):
    from paper_2609_20536_amd import hotrg as H
    import torch
    other = H.Context(0, torch_workspace=False)
    try:
        buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
        assert other.lib.gxy_set_workspace(other.handle, C.c_void_p(buf.data_ptr()),
                                           buf.numel()) == 0
        p = H.make_point(beta=1.0, delta=0.5, nmax=5, dcut=20, nsteps=8, impurities=3)
        r = H.Result()
        st = other.lib.gxy_run(other.handle, C.byref(p), C.byref(r))
        assert st == 2
        assert b"smaller than" in other.lib.gxy_last_error(other.handle)
        # with the caller's memory released the library allocates its own
        assert other.lib.gxy_set_workspace(other.handle, None, 0) == 0
        assert other.run(dict(beta=1.0, delta=0.5, nmax=3, dcut=12, nsteps=6)).status == 0
    finally:
        other.close()
