#!/usr/bin/env python3
"""HOTRG throughput on one MI355X, with roofline and CPU-oracle baseline.

One benchmark step is one full HOTRG run of the gXY workload at Dcut = 64:
beta = 1.2, Delta = 0.7, charges |n| <= 10 (D0 = 21), 40 coarse-graining
steps alternating y/x, both impurity chains (<cos theta>, <cos 2 theta>),
FP64 contractions, FP64 eigensolves. The input is resident on the device
(the initial tensor is built there from (beta, Delta)); the timed region
covers every step of the path.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line. value = coarse-graining steps per second (40 per run).
More legs ride on the same line (each skippable):
* "direct_lds": the workload with the FP64 projection products staged by
  direct global -> LDS loads (GXY_GEMM_DMA=1): steps/s, the D^7 product's
  launch time and MFMA fraction, |d ln Z/V| against the default staging;
* "precision": the same workload with the projection contractions in FP32
  and in split-BF16x3, with every step reduced and with the first 12 / 16
  steps in FP64: steps/s, |d ln Z/V| and |d C_v| against the FP64 GPU runs
  and against the stored oracle values, |d <cos 2 theta>| at h1 = 1.1e-3;
* "susceptibility": the workload with the second-moment chains (zero-field
  chi and chi_n from one run);
* "d96": the same model at Dcut = 96: 40-step FP64, FP32 and BF16x3 runs
  (steps/s, |d ln Z/V| against FP64) and FP64 against the stored oracle
  values (3 and 20 steps);
* "harmonic", "transition": the harmonic q = 3, 4 and the transition-
  temperature procedure;
* "surrogate": the surrogate's gain in locating the C_v peak at reduced
  size (the full-size refinement is `paper_2609_20536_amd.scan --refine`);
* "lgt": the configurational-temperature estimator of compact U(1) lattice
  gauge theory (the thesis's second workload, Ch. 4-5) on 16 configurations
  of 32^4: configurations/s, the gradient kernel's HBM roofline, the mean
  estimators and plaquette;
* "batched": a stratified 16-point subset of the 16 x 16 (beta, Delta) grid
  (4 points per Dcut in {24, 32, 48, 64}) by the zero-field route, three
  runs per point (beta -+ db for C_v, beta with the second-moment chains for
  chi, chi_n): points/s of the plain FP64 path (runs one after another) and,
  after the per-Dcut tile autotuner, of one batch on 16 worker streams (16
  hardware queues for the process) in FP64, FP32 and BF16x3 with schedules;
  max |d f| and relative d chi against FP64; the same for the Dcut = 64
  points alone.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
# hardware queues of this process (HIP reads it when it starts; an inherited
# smaller value is raised): the batched leg runs BATCH_WORKERS streams, and
# streams beyond the queue count share queues, which serialises their kernels
BATCH_WORKERS = 16
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < BATCH_WORKERS:
    os.environ["GPU_MAX_HW_QUEUES"] = str(BATCH_WORKERS)
sys.path.insert(0, ROOT)

METRIC = "HOTRG steps/s & MFMA util at D=64; batched (β,Δ) points/s at |δf|≤1e-9"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def workload_point(dcut: int):
    from paper_2609_20536_amd import workloads as W
    return W.precision_point(dcut=dcut, prec=W.PREC_FP64, impurities=W.IMP_COS1 | W.IMP_COS2)


def measured_traffic(name="ygemm_d64_chains_fp64_traffic.json"):
    """HBM bytes per launch of the D^7 GEMM from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if the sources it names (kernel, planner
    and the engine that issues the launches) are unchanged since the counters
    were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def stored_oracle(name):
    """ln Z/V (and the point) of a stored oracle run (tests/golden, written by
    the oracle's golden script), or None."""
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def precision_leg(ctx, pt, r64):
    """Reduced-precision contraction forms on the bench workload (Dcut = 64):
    steps/s, and the errors of ln Z/V and C_v (central differences at
    beta +- 1e-3) against the FP64 GPU runs and against the stored oracle
    values, for every step reduced (fp64_steps = 0) and with the first
    steps kept in FP64; <cos 2 theta> at h1 = 1.1e-3 (Dcut = 48) against its
    stored oracle value."""
    from paper_2609_20536_amd import workloads as W
    out = {}
    db = W.BETA_FD_STEP
    gold = [stored_oracle(n) for n in ("prec_d64_pure_m", "prec_d64_pure", "prec_d64_pure_p")]
    l_or = [g["lnz_per_site"] for g in gold] if all(gold) else None

    def lnz3(prec, k):
        base = pt.with_(impurities=0, prec=prec, fp64_steps=k)
        return [ctx.run(base.with_(beta=pt.beta + s)).lnz_per_site for s in (-db, 0.0, db)]

    def cv(l):
        return pt.beta ** 2 * (l[0] - 2.0 * l[1] + l[2]) / db ** 2
    l64 = lnz3(W.PREC_FP64, 0)
    out["cv_fp64"] = cv(l64)
    if l_or:
        out["fp64_vs_oracle"] = {"abs_dlnz_per_site": abs(l64[1] - l_or[1]),
                                 "abs_dcv": abs(cv(l64) - cv(l_or))}
    gm = stored_oracle("cv_b1.0_h1p")
    for name, prec, sched in (("fp32", W.PREC_FP32, (0, 12)), ("bf16x3", W.PREC_BF16X3, (0, 16))):
        rows = {}
        for k in sched:
            q = pt.with_(prec=prec, fp64_steps=k)
            ctx.run(q)
            t0 = time.perf_counter()
            r = ctx.run(q)
            el = time.perf_counter() - t0
            l = lnz3(prec, k)
            row = {"fp64_steps": k, "steps_per_s": q.nsteps / el,
                   "abs_dlnz_vs_fp64_gpu": abs(r.lnz_per_site - r64.lnz_per_site),
                   "abs_dcv_vs_fp64_gpu": abs(cv(l) - cv(l64))}
            if l_or:
                row["abs_dlnz_vs_oracle"] = abs(l[1] - l_or[1])
                row["abs_dcv_vs_oracle"] = abs(cv(l) - cv(l_or))
            if gm:
                g = ctx.run(W.Point(**{**gm["point"], "prec": prec, "fp64_steps": k}))
                row["abs_dm_cos2_h1_vs_oracle"] = abs(g.m_cos2 - gm["m_cos2"])
            rows[f"k{k}"] = row
        out[name] = rows
    return out


def d96_leg(ctx, note):
    """The precision workload at Dcut = 96 (beta = 1.2, Delta = 0.7, |n| <= 10):
    steps/s of 40-step FP64, FP32 and BF16x3 runs (first 16 steps FP64) and
    their |d ln Z/V| against FP64; the 3- and 20-step FP64 runs against the
    stored oracle values."""
    from paper_2609_20536_amd import workloads as W
    out = {}
    base = W.precision_point(96, impurities=0)
    for name, n in (("prec_d96_first3", 3), ("prec_d96_pure_n20", 20)):
        g = stored_oracle(name)
        if g:
            r = ctx.run(base.with_(nsteps=n))
            out[f"fp64_n{n}_abs_dlnz_vs_oracle"] = abs(r.lnz_per_site - g["lnz_per_site"])
    r64 = None
    for name, prec, k in (("fp64", W.PREC_FP64, 0), ("fp32", W.PREC_FP32, 16),
                          ("bf16x3", W.PREC_BF16X3, 16)):
        q = base.with_(prec=prec, fp64_steps=k)
        t0 = time.perf_counter()
        r = ctx.run(q)
        el = time.perf_counter() - t0
        row = {"fp64_steps": k, "steps_per_s": q.nsteps / el, "lnz_per_site": r.lnz_per_site}
        if r64 is None:
            r64 = r
        else:
            row["abs_dlnz_vs_fp64_gpu"] = abs(r.lnz_per_site - r64.lnz_per_site)
        out[name] = row
        note(f"bench: Dcut=96 {name} done in {el:.1f}s")
    return out


def surrogate_leg(ctx):
    """The surrogate's gain at reduced size: C_v peak location along beta at
    Delta = 0.6 and 0.9 from six HOTRG points spread uniformly against six
    placed around the surrogate's proposal (trained on a 21 x 6 grid of
    Dcut = 16 runs, |n| <= 5, 24 steps), against a 41-point reference scan.
    The full-size refinement (256-point grid, 512 proposals verified at
    Dcut = 64) is `python -m paper_2609_20536_amd.scan --refine`."""
    from paper_2609_20536_amd import surrogate as S
    t0 = time.perf_counter()
    out = S.gain_experiment(ctx, deltas=(0.6, 0.9), dcut=16, nmax=5, nsteps=24,
                            train_grid=(21, 6), workers=16)
    return {"seconds": time.perf_counter() - t0, "gain": out["gain"],
            "mean_err_uniform": out["mean_err_uniform"],
            "mean_err_guided": out["mean_err_guided"], "final_loss": out["final_loss"]}


def susceptibility_leg(ctx, pt):
    """The bench workload with both second-moment chains (zero-field chi and
    chi_n from one run): steps/s and the values."""
    from paper_2609_20536_amd import workloads as W
    p = pt.with_(impurities=W.IMP_COS1_SQ | W.IMP_COS2_SQ)
    ctx.run(p)
    t0 = time.perf_counter()
    r = ctx.run(p)
    el = time.perf_counter() - t0
    return {"steps_per_s": p.nsteps / el, "chi": r.chi0, "chi_n": r.chi0_n,
            "msq_cos1": r.msq_cos1, "lnz_per_site": r.lnz_per_site}


def harmonic_leg(ctx, pt):
    """The bench workload with the second coupling's harmonic q = 3 and 4
    (cos q phi, h1 and the second impurity on cos q theta): steps/s of one
    FP64 run each, with ln Z/V and <cos theta> for reference."""
    out = {}
    for q in (3, 4):
        p = pt.with_(q=q)
        ctx.run(p)
        t0 = time.perf_counter()
        r = ctx.run(p)
        el = time.perf_counter() - t0
        out[f"q{q}"] = {"steps_per_s": p.nsteps / el, "lnz_per_site": r.lnz_per_site,
                        "max_trunc_err": r.max_trunc_err}
    return out


def transition_leg(ctx):
    """The zero-field extrapolation of the transition temperature at
    Delta = 0.32 (field h1): susceptibility scans at four central fields
    and the C_v scan, Dcut = 24, |n| <= 10, 40 steps, in batches of 16."""
    from paper_2609_20536_amd import transition as T
    temps = [0.62 + 0.03 * i for i in range(13)]
    hbars = [0.001, 0.002, 0.004, 0.008]
    t0 = time.perf_counter()
    tr = T.transition_temperature(ctx, 0.32, temps, hbars, dcut=24, nmax=10, nsteps=40,
                                  workers=16)
    el = time.perf_counter() - t0
    runs = len(temps) * (2 * len(hbars) + 3)
    return {"delta": 0.32, "dcut": 24, "field": tr.field, "runs": runs, "seconds": el,
            "runs_per_s": runs / el, "hbars": hbars, "tpeaks": tr.tpeaks,
            "fit": {"a": tr.a, "b": tr.b, "c": tr.c, "rms": tr.rms}, "t_cv": tr.t_cv}


def batched_leg(ctx, note):
    """Points/s of (f, C_v, chi, chi_n) over a stratified grid subset by the
    zero-field route (three runs per point: beta -+ 1e-3, and beta with the
    second-moment chains), as one batch; plain FP64 one run after another
    against batched FP64 and batched reduced precision; also the Dcut = 64
    points alone."""
    from paper_2609_20536_amd import surrogate as S
    from paper_2609_20536_amd import workloads as W
    gp = W.grid_points()
    sub = []
    for d in W.GRID_DCUTS:
        sub += [g for g in gp if g.dcut == d][:4]
    tiles = ctx.autotune(W.Point(beta=1.0, delta=0.5, nmax=10, dcut=24, nsteps=10,
                                 impurities=0), list(W.GRID_DCUTS))
    note("bench: tile autotuner done")
    out = {"points": len(sub), "runs_per_point": 3,
           "route": "zero field: beta -+ 1e-3 for C_v, second-moment chains for chi, chi_n",
           "workers": BATCH_WORKERS,
           "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
           "plain": "the same runs one after another on one stream (FP64)",
           "tiles": {str(k): v[0] for k, v in tiles.items()}}
    for label, pts in (("stratified", sub), ("d64", [g for g in sub if g.dcut == 64])):
        res = {}
        row = {"points": len(pts)}
        for name, prec, k, workers in (("plain_fp64", W.PREC_FP64, 0, 1),
                                       ("fp64", W.PREC_FP64, 0, BATCH_WORKERS),
                                       ("fp32", W.PREC_FP32, 12, BATCH_WORKERS),
                                       ("bf16x3", W.PREC_BF16X3, 16, BATCH_WORKERS)):
            S.grid_observables_zero_field(ctx, pts[:1], workers=workers, prec=prec,
                                          fp64_steps=k)
            t0 = time.perf_counter()
            obs, _ = S.grid_observables_zero_field(ctx, pts, workers=workers, prec=prec,
                                                   fp64_steps=k)
            el = time.perf_counter() - t0
            res[name] = obs
            row[name + "_points_per_s"] = len(pts) / el
            note(f"bench: {label} {name} ({workers} worker(s)) done in {el:.1f}s")
        for name in ("fp32", "bf16x3"):
            row[f"speedup_{name}_batched_vs_plain_fp64"] = (row[name + "_points_per_s"] /
                                                            row["plain_fp64_points_per_s"])
            row[f"max_abs_df_{name}_vs_fp64"] = float(abs(res[name][:, 0] - res["fp64"][:, 0]).max())
            row[f"max_rel_dchi_{name}_vs_fp64"] = float(
                (abs(res[name][:, 2] - res["fp64"][:, 2]) / res["fp64"][:, 2]).max())
        out[label] = row
    return out


def direct_lds_leg(ctx, pt, r, steps, note):
    """The bench workload with the FP64 projection products staged by direct
    global -> LDS loads (GXY_GEMM_DMA=1): steps/s, the D^7 product's launch
    time and MFMA fraction, and ln Z/V against the default staging."""
    import torch

    os.environ["GXY_GEMM_DMA"] = "1"
    try:
        ctx.run(pt)
        os.environ["GXY_HOT_EVENTS"] = "1"
        ctx.hot_kernel_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rd = ctx.run(pt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        os.environ.pop("GXY_HOT_EVENTS", None)
        launches, ms, flops, _ = ctx.hot_kernel_stats(reset=True)
    finally:
        os.environ.pop("GXY_GEMM_DMA", None)
        os.environ.pop("GXY_HOT_EVENTS", None)
    avg = ms / max(launches, 1)
    tf = (flops / max(launches, 1)) / (avg * 1e-3) / 1e12 if ms > 0 else 0.0
    note("bench: direct-LDS leg done")
    return {"kernel": "ggemm_dma_kernel (FP64, operands by global_load_lds)",
            "steps_per_s": pt.nsteps * steps / el, "avg_launch_ms": avg, "achieved": tf,
            "frac": tf / PEAK_FP64_TFLOPS,
            "traffic": (measured_traffic("ygemm_dma_d64_chains_fp64_traffic.json")
                        if pt.dcut == 64 else None),
            "abs_dlnz_vs_default": abs(rd.lnz_per_site - r.lnz_per_site)}


def lgt_leg(ctx, note, reps: int = 10):
    """Configurational-temperature estimator of compact U(1) lattice gauge
    theory (Ch. 4-5) on the throughput batch, 16 configurations of 32^4
    (gauge-transformed Gaussian angles, plaquette near 0.58), full form
    (Tr h, |g|^2 and g^T h g): configurations/s; the gradient kernel's
    algorithmic HBM bytes per launch (every link's e^{i theta} read once and
    its g written once, 24 bytes per link) over its event-timed duration; and
    the whole call's rate on the 8 bytes per link of angles it must read."""
    import numpy as np
    import torch
    from paper_2609_20536_amd import workloads as W

    dims, nconf = W.LGT_BENCH_DIMS, W.LGT_BENCH_CONF
    th = torch.from_numpy(W.lgt_configs(nconf, dims)).to("cuda:0")
    ctx.lgt_estimator(th)
    os.environ["GXY_HOT_EVENTS"] = "1"
    try:
        ctx.hot_kernel_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = ctx.lgt_estimator(th)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        os.environ.pop("GXY_HOT_EVENTS", None)
    launches, ms, _, nbytes = ctx.hot_kernel_stats(reset=True)
    V = int(np.prod(dims))
    links = nconf * len(dims) * V
    avg = ms / max(launches, 1)
    gbs = (nbytes / max(launches, 1)) / (avg * 1e-3) / 1e9 if ms > 0 else 0.0
    note("bench: U(1) estimator leg done")
    return {
        "workload": (f"{nconf} configurations of {'x'.join(map(str, dims))} compact U(1), "
                     "full estimator (Tr h, |g|^2, g^T h g), FP64"),
        "configs_per_s": nconf * reps / el,
        "ms_per_call": 1000.0 * el / reps,
        "plaquette_mean": float(np.mean([r["plaquette"] for r in res])),
        "beta_diag_mean": float(np.mean([r["beta_diag"] for r in res])),
        "beta_full_mean": float(np.mean([r["beta_full"] for r in res])),
        "roofline": {"bound": "hbm", "kernel": "lgt_grad_kernel<4>", "achieved": gbs,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                     "traffic": measured_traffic("lgt_grad_32x4_traffic.json"),
                     "launches": int(launches), "avg_launch_ms": avg,
                     "algorithmic_bytes_per_launch": nbytes / max(launches, 1)},
        "end_to_end_angle_GBs": 8.0 * links / (el / reps) / 1e9,
    }


def cpu_baseline(pt, nimp: int, frac_cols: int = 8):
    """Time the CPU oracle on a bounded sample of the bench workload.

    Sample: the oracle runs the workload's first two coarse-graining steps
    (untimed: they bring both bond dimensions to Dcut), then its third step
    is timed: both environments, the per-sector eigensolves and the state
    selection in full, and the projection restricted to frac_cols of the
    Dcut output columns (the projection is linear in the number of output
    columns). One step costs env + eig + (1 + 2 nimp) projections; the
    metric's steps/s is the inverse.
    """
    import numpy as np
    import oracle.hotrg as o
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    D = pt.dcut
    t0 = time.perf_counter()
    r = o.run_point(beta=pt.beta, delta=pt.delta, h=pt.h, h1=pt.h1, nmax=pt.nmax, dcut=D,
                    nsteps=2, nquad=pt.nquad, impurities=0, keep_tensor=True)
    t_setup = time.perf_counter() - t0
    T = r.tensor
    lab_h, lab_v = r.labels_hv
    if T.shape != (D, D, D, D):   # pragma: no cover
        raise RuntimeError(f"sample tensor {T.shape}: both bonds should be at Dcut = {D}")
    # step 3 is a y-step (the run starts with one), on this tensor as it is
    sym = o.symmetry_of(pt.h, pt.h1)
    t0 = time.perf_counter()
    EL, ER = o.environments(T)
    t_env = time.perf_counter() - t0
    fused = o.fuse_labels(lab_h, lab_h, sym)
    t0 = time.perf_counter()
    secL = o.sector_eigh(EL, fused)
    secR = o.sector_eigh(ER, fused)
    sel = o.select_states(secL, secR, D, D * D)
    t_eig = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.project(sel.P[:, :frac_cols], T, T)
    t_proj = (time.perf_counter() - t0) * (D / frac_cols)
    per_step = t_env + t_eig + (1 + 2 * nimp) * t_proj
    return {
        "value": 1.0 / per_step,
        "unit": "HOTRG steps/s",
        "cores": int(cores),
        "cpu": cpu_model,
        "kind": "oracle",
        "sample": (f"step 3 of the bench workload (Dcut={D}, after the oracle's own first two "
                   f"steps, {t_setup:.1f}s untimed): environments {t_env:.2f}s + sector "
                   f"eigensolves and selection {t_eig:.2f}s + projection over "
                   f"{frac_cols}/{D} output columns scaled to {t_proj:.2f}s x {1 + 2 * nimp} "
                   f"placements (pure + 2 per impurity chain)"),
    }


def cpu_baseline_lgt():
    """The U(1) estimator's oracle on the host: the diagonal form on one
    32^4 configuration and the full form (explicit sparse Hessian) on one
    16^4 configuration, each as configurations/s at its size."""
    import oracle.lgt as ol
    from paper_2609_20536_amd import workloads as W
    th = W.lgt_configs(1, W.LGT_BENCH_DIMS)[0]
    t0 = time.perf_counter()
    ol.estimator(th, full=False)
    t_diag = time.perf_counter() - t0
    th16 = W.lgt_configs(1, (16, 16, 16, 16))[0]
    t0 = time.perf_counter()
    ol.estimator(th16, full=True)
    t_full = time.perf_counter() - t0
    return {"unit": "configurations/s", "kind": "oracle",
            "diag_32^4_configs_per_s": 1.0 / t_diag,
            "full_16^4_configs_per_s": 1.0 / t_full,
            "full_scaled_to_32^4_configs_per_s": 1.0 / (t_full * 16.0),
            "sample": "one 32^4 configuration (diagonal form) and one 16^4 configuration "
                      "(full form, scaled by volume to 32^4)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dcut", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-harmonic", action="store_true")
    ap.add_argument("--no-transition", action="store_true")
    ap.add_argument("--no-susceptibility", action="store_true")
    ap.add_argument("--no-d96", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-direct-lds", action="store_true")
    ap.add_argument("--no-lgt", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="one plain 1 GiB device copy first (known HBM bytes for counter scaling)")
    ap.add_argument("--phases", action="store_true", help="one extra untimed run with phase timers")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the HOTRG path here runs on a single MI355X "
              "(no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_20536_amd import hotrg as H

    pt = workload_point(args.dcut)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = H.Context(0)
    ctx.reserve([pt])
    os.environ.pop("GXY_TIMING", None)
    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    # projection tile for this Dcut, chosen by measurement (before any timing)
    tuned = ctx.autotune(pt.with_(nsteps=8, impurities=0), [pt.dcut])
    note(f"bench: tile autotuner: {tuned}")

    for i in range(args.warmup):
        t1 = time.perf_counter()
        ctx.run(pt)
        note(f"bench: warmup run {i + 1}/{args.warmup} done in {time.perf_counter() - t1:.1f}s")
    torch.cuda.synchronize()
    os.environ["GXY_HOT_EVENTS"] = "1"
    ctx.hot_kernel_stats(reset=True)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(ctx.run(pt))
        note(f"bench: timed run {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    os.environ.pop("GXY_HOT_EVENTS", None)
    launches, ms, flops, nbytes = ctx.hot_kernel_stats(reset=True)
    r = results[-1]
    if r.status != 0:
        raise SystemExit(f"run failed: status {r.status}")
    hot_avg_ms = ms / max(launches, 1)
    hot_tflops = (flops / max(launches, 1)) / (hot_avg_ms * 1e-3) / 1e12 if ms > 0 else 0.0
    phases = None
    if args.phases:
        os.environ["GXY_TIMING"] = "1"
        ctx.run(pt)
        note("bench: phase-timing run done")
        os.environ.pop("GXY_TIMING", None)
        phases = dict(zip(["init", "environment", "eigensolve", "selection", "projection",
                           "norm_permute"], [round(x, 2) for x in ctx.phase_times()]))
    steps_per_run = pt.nsteps
    value = steps_per_run * args.steps / elapsed
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "HOTRG steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"gxy-hotrg beta={pt.beta} Delta={pt.delta} nmax={pt.nmax} "
                         f"Dcut={pt.dcut} {pt.nsteps} steps, cos+cos2 impurity chains, "
                         f"FP64 contractions and eigensolves"),
            "coarse_graining_steps_per_run": steps_per_run,
            "lnz_per_site": r.lnz_per_site,
            "max_trunc_err": r.max_trunc_err,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "projection D^7 grouped GEMM (ggemm_contig_kernel, Y = X T, FP64)",
            "achieved": hot_tflops,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": hot_tflops / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic() if args.dcut == 64 else None,
            "launches": int(launches),
            "avg_launch_ms": hot_avg_ms,
            "flops_per_launch": flops / max(launches, 1),
            "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
        },
        "cpu_baseline": None,
    }
    if phases:
        line["phases_ms"] = phases
    if not args.no_direct_lds:
        line["direct_lds"] = direct_lds_leg(ctx, pt, r, args.steps, note)
    if not args.no_precision:
        line["precision"] = precision_leg(ctx, pt, r)
        note("bench: precision leg done")
    if not args.no_susceptibility:
        line["susceptibility"] = susceptibility_leg(ctx, pt)
        note("bench: susceptibility leg done")
    if not args.no_d96:
        line["d96"] = d96_leg(ctx, note)
    if not args.no_surrogate:
        line["surrogate"] = surrogate_leg(ctx)
        note("bench: surrogate leg done")
    if not args.no_harmonic:
        line["harmonic"] = harmonic_leg(ctx, pt)
        note("bench: harmonic-q leg done")
    if not args.no_transition:
        line["transition"] = transition_leg(ctx)
        note("bench: transition leg done")
    if not args.no_batched:
        line["batched"] = batched_leg(ctx, note)
    if not args.no_lgt:
        line["lgt"] = lgt_leg(ctx, note)
    if not args.no_cpu_baseline:
        note("bench: timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(pt, 2)
        if not args.no_lgt:
            line["cpu_baseline"]["lgt"] = cpu_baseline_lgt()
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
