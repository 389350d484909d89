"""Throughput and time to gap of the domain-decomposition hot path on one MI355X.

A step is one parallel DomDecIter half-iteration over every composite cell of
one partition (aggregation of the basic Y-marginals, cell inputs, the cell
Sinkhorn solves with the Newton Y-update and the PD stopping rule, re-split,
score pieces, GetWeights, update), alternating A and B.  The metric counts
grid points times inner Sinkhorn iterations: sum over the cells of
|X_J| * (Y-halves of that cell), divided by the wall time of the timed steps.
Every cell is solved in every step, whatever its Y-box size (variable-size
pools; boxes wider than the in-LDS layout are solved by gangs of workgroups);
`inner.overflow_cells` counts any cell that was not, and the headline `value`
is null if it is not 0.

Default run (the 1024 x 1024 workload, FP32 cells, FP64 reductions):
  1. the multiscale solve (Sec. 4.4: global Sinkhorn below 256^2, then DD
     layers with eps-scaling, eps = h^2 on the finest), timed from the host
     marginals: the time to each relative gap, certified by the polished
     bounds of dd_uot_score (FP32 and FP64);
  2. the headline: `--warmup` then `--steps` timed half-iterations continuing
     from the FP32 solve's final state, with the cell-solve launches timed
     by HIP events for the roofline;
  3. the FP32 error of one step against the FP64 step from the same state;
  4. the 256^2 workload at lambda 0.1, 1, 10 (eps from 64 h^2 to h^2), FP64
     and FP32, with the time to each gap and the FP32 error against FP64;
  5. the batched and differentiable forms (the latter from the grid
     problem's converged state, gradients at a converged state), and the CPU
     oracle timed on a sample of the headline state's cell solves (1 core
     and all cores).

Prints one JSON line on stdout, progress lines on stderr.  `--gpus` above 1
is refused: the solver runs on a single device.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2410_08859_amd import binding as B  # noqa: E402
from paper_2410_08859_amd.inputs import (WORKLOADS, batched_problems,  # noqa: E402
                                         displaced_points, displacement_theta,
                                         workload_marginals)

# MI355X: each of 256 CUs issues one wave64 VALU instruction per cycle (4
# SIMDs, each busy 4 cycles per instruction), 256 x 64 x 2.4e9 = 3.93e13
# lane-ops/s; the transcendental unit (v_exp_f32) runs at a quarter of that.
EXP_PEAK = 256 * 64 * 2.4e9 / 4.0
HBM_PEAK = 8.0e12

GW_NAMES = {B.GW_GREEDY: "greedy", B.GW_SAFE: "safe", B.GW_SWIFT: "swift",
            B.GW_STAGGERED: "staggered", B.GW_LINE: "line", B.GW_OPT: "opt"}
GW_IDS = {v: k for k, v in GW_NAMES.items()}
PROFILE = os.path.join(ROOT, "profiles", "k_cell_solve_grid1024_fp32_multiscale.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2410_08859_amd", "csrc", "cell_kernel.hip")
TARGETS = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)


def progress(msg):
    """One line on stderr per finished phase (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def profiled(args):
    """Counter figures that rocprofv3 measured for this workload, precision
    and final stage and this kernel source (HBM traffic per launch scaled by a
    copy probe, VALU issue fraction, VALU instructions per term: averages per
    launch over the profiled run's timed launches), or {} otherwise."""
    key = f"config: {args.workload} FP{args.precision} final {args.final32} max-inner " \
          f"{args.max_inner} err-ratio {args.err_ratio:g}"
    try:
        txt = open(PROFILE).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return {}
    if src not in txt or not re.search(r"^" + re.escape(key) + r"$", txt, re.M):
        return {}
    out = {}
    for name in ("traffic_bytes_per_launch", "valu_issue_frac", "valu_instr_per_term"):
        m = re.search(r"^" + name + r": ([0-9.eE+-]+)\s*$", txt, re.M)
        if m:
            out[name] = float(m.group(1))
    return out


def workload_config(name, precision, max_inner, err=2e-5, getweights=B.GW_LINE, cap=48, lam=None):
    w = WORKLOADS[name]
    n = w["n"]
    return B.dd_uot_default_config(
        n1=n, n2=n, h=1.0 / n, eps=w["eps_h2"] / n ** 2, lam=w["lam"] if lam is None else lam,
        cell=w["cell"],
        precision=precision, init=B.INIT_BLOCK, getweights=getweights, sinkhorn_err=err,
        sinkhorn_max_iter=max_inner, trunc=1e-15, lenience=0.0, box_margin=2, box_cap=cap)


def multiscale_solve(name, precision, final_max, polish, args, stream, lam=None, coarsest=16,
                     eps_start_h2=2.0):
    """The whole multiscale solve from the host marginals; returns the finest
    handle and the time to each target of the certified (polished) gap and
    of the DD-plan gap (tracked score against the certificate's dual).
    Layers from coarsest^2 up; every layer's eps starts at eps_start_h2 of
    its own h^2."""
    mu, nu = workload_marginals(name)
    cfg = workload_config(name, precision, args.max_inner, args.err, GW_IDS[args.getweights],
                          lam=lam)
    levels = int(round(np.log2(cfg.n1 / coarsest))) + 1
    extra = dict(eps_start_h2=float(eps_start_h2))
    ms = B.dd_uot_default_multiscale(levels=levels, final_max_halves=final_max, check_every=4,
                                     target_rel_gap=min(TARGETS), polish_iters=polish,
                                     final_err_ratio=args.err_ratio, final_err_min=1e-10, **extra)
    h, tr = B.dd_uot_solve_multiscale(cfg, ms, mu, nu, stream=stream)
    progress(f"multiscale {name} FP{precision} lambda {cfg.lambda_:g}: {tr[-1, 1] / 1e3:.1f} s, "
             f"certified gap {tr[-1, 4]:.3g}, DD-plan gap {tr[-1, 3]:.3g}")

    def reached(col):
        out = {}
        for t in TARGETS:
            hit = np.nonzero(tr[:, col] <= t)[0]
            out[f"{t:g}"] = None if hit.size == 0 else {"ms": float(tr[hit[0], 1]),
                                                        "half_iters": int(tr[hit[0], 0])}
        return out
    first = eps_start_h2 * (cfg.n1 / coarsest) ** 2
    sched = (f"{levels} layers from {coarsest}^2 (eps from {first:g} h^2 of the finest grid); "
             f"global Sinkhorn below 256^2 (tolerance {ms.global_tol:g} |mu|); eps "
             f"{eps_start_h2:g} h_l^2 -> h_l^2/2 per layer, then down to "
             f"{cfg.eps * cfg.n1 ** 2:g} h^2 on the finest")
    rec = {"workload": name, "precision": precision, "lambda": cfg.lambda_,
           "getweights": args.getweights,
           "certified_gap": reached(4), "dd_plan_gap": reached(3),
           "final": {"certified_gap": float(tr[-1, 4]), "dd_plan_gap": float(tr[-1, 3]),
                     "certificate_gap": float(tr[-1, 2]), "ms": float(tr[-1, 1]),
                     "half_iters": int(tr[-1, 0])},
           "not_reached": f"levels below the final certified gap {tr[-1, 4]:.3g} are not reached "
                          f"within the final stage's {final_max} half-iterations (null)",
           "schedule": f"{sched}; DD 4-16 half-iterations per stage; then at most {final_max} "
                       f"half-iterations with a certificate every 4 (polished by {polish} global "
                       f"Sinkhorn iterations); GetWeights {args.getweights} (lenience 0), Err "
                       f"{args.err:g} (final stage: min(Err, {args.err_ratio:g} x certified gap)), "
                       f"at most {args.max_inner} inner iterations per cell, cell problems on the "
                       f"support of nu_J, cells {cfg.cell}x{cfg.cell} on the finest layer, 4x4 below"}
    return h, rec


def timed_steps(h, steps, warmup):
    """Run warmup steps, then time `steps` half-iterations (wall clock between
    device synchronisations) and the cell-solve launches (HIP events)."""
    import torch
    B.dd_uot_iterate(h, warmup)
    torch.cuda.synchronize()
    B.dd_uot_set_timing(h, True)
    rec0 = len(B.dd_uot_history(h, 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.dd_uot_iterate(h, steps, stats=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms, kbytes = B.dd_uot_kernel_time(h)
    B.dd_uot_set_timing(h, False)
    hist = B.dd_uot_history(h, 0)[rec0:]
    return dict(dt=dt, launches=launches, kms=kms, kbytes=kbytes, hist=hist)


def box_stats(st):
    b = st["boxes"]
    side = np.maximum(b[:, 2], b[:, 3])
    return {"basic_box_side_p50": float(np.percentile(side, 50)),
            "basic_box_side_p90": float(np.percentile(side, 90)),
            "basic_box_side_max": int(side.max()),
            "stored_values_per_grid_point": float(st["values"].size / st["px"].size)}


def fp32_step_error(h64, name, args, stream, lam=None):
    """The FP32 error of one step: from the FP64 handle's state, one FP64 and
    one FP32 half-iteration; relative L1 differences of P_X, P_Y and the
    relative difference of the tracked score."""
    w = WORKLOADS[name]
    n = w["n"]
    nb = (n // w["cell"]) ** 2
    mu, nu = workload_marginals(name)
    st = B.dd_uot_get_state(h64, n, n, nb)
    c32 = workload_config(name, 32, args.max_inner, args.err, GW_IDS[args.getweights], lam=lam)
    h32 = B.dd_uot_init(c32, mu, nu, stream=stream)
    try:
        B.dd_uot_set_state(h32, st)
        B.dd_uot_iterate(h64, 1)
        B.dd_uot_iterate(h32, 1)
        (x64, y64), (x32, y32) = B.dd_uot_marginals(h64, 0, n, n), B.dd_uot_marginals(h32, 0, n, n)
        s64, s32 = B.dd_uot_score(h64, 0), B.dd_uot_score(h32, 0)
    finally:
        B.dd_uot_destroy(h32)
    rel = lambda a, b: float(np.abs(a - b).sum() / np.abs(b).sum())
    out = {"from": f"the FP64 state after {st['k']} half-iterations",
           "px_rel_l1": rel(x32, x64), "py_rel_l1": rel(y32, y64),
           "tracked_score_rel": abs(s32["tracked"] - s64["tracked"]) / abs(s64["tracked"])}
    progress(f"FP32 step error: P_X {out['px_rel_l1']:.2e}, P_Y {out['py_rel_l1']:.2e}, score "
             f"{out['tracked_score_rel']:.2e}")
    return out


def config2(args, stream):
    """The 256^2 workload (masses 1.0 / 0.8, cells 4x4, eps = h^2) at lambda
    in {0.1, 1, 10}: eps from 64 h^2 (the 64^2 layer at 4 of its h^2) down to
    h^2 through the 64^2, 128^2 and 256^2 layers, FP64 and FP32 solves with
    the time to each gap, and the FP32 error against FP64: the FP32 step from
    the FP64 solve's final state, and the two solves' final scores."""
    out = []
    for lam in (0.1, 1.0, 10.0):
        res = {"lambda": lam}
        h64, res["fp64"] = multiscale_solve("grid256", 64, args.final256, args.polish, args,
                                            stream, lam=lam, coarsest=64, eps_start_h2=4.0)
        try:
            s64 = B.dd_uot_score(h64, 0)
            h32, res["fp32"] = multiscale_solve("grid256", 32, args.final256, args.polish, args,
                                                stream, lam=lam, coarsest=64, eps_start_h2=4.0)
            try:
                s32 = B.dd_uot_score(h32, 0)
            finally:
                B.dd_uot_destroy(h32)
            res["fp32_vs_fp64"] = {
                "step": fp32_step_error(h64, "grid256", args, stream, lam=lam),
                "final_tracked_score_rel": abs(s32["tracked"] - s64["tracked"]) / abs(s64["tracked"]),
                "final_dual_rel": abs(s32["dual"] - s64["dual"]) / abs(s64["dual"])}
        finally:
            B.dd_uot_destroy(h64)
        out.append(res)
    return out


def plateau_study(stream, cap=10000):
    """The global GPU Sinkhorn (no decomposition) on the 256^2 marginals at
    eps = (8h)^2 from beta = 0, for lambda in {0.01, ..., 1000}: iterations
    and wall time until KL(P_X pi | e^{-alpha/lam} mu) / |mu| first reaches
    1e-2 ... 1e-6, and that error at 10, 30, 100, ... iterations (at most `cap`
    iterations per lambda).  Each call stops at the next target or milestone
    and the next continues from its beta: the uninterrupted iteration."""
    mu, nu = workload_marginals("grid256")
    n = mu.shape[0]
    mass = float(mu.sum())
    marks = [m for m in (10, 30, 100, 300, 1000, 3000, 10000) if m <= cap]
    out = []
    for lam in (0.01, 0.1, 1.0, 10.0, 100.0, 1000.0):
        cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=64.0 / n ** 2, lam=lam, cell=4,
                                      precision=64)
        beta = np.zeros((n, n))
        done, ms, pd = 0, 0.0, float("inf")
        first, at = {}, {}
        targets = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
        while done < cap:
            nxt = min([m for m in marks if m > done] + [cap])
            open_t = [t for t in targets if f"{t:g}" not in first]
            tol = open_t[0] * mass if open_t else 0.0
            t0 = time.perf_counter()
            r = B.dd_uot_global_sinkhorn(cfg, mu, nu, beta0=beta, max_iter=nxt - done, tol=tol,
                                         stream=stream)
            ms += 1e3 * (time.perf_counter() - t0)
            done += r["iters"]
            beta = r["beta"]
            pd = r["pd"] / mass
            for t in targets:
                if f"{t:g}" not in first and pd <= t:
                    first[f"{t:g}"] = {"iters": done, "ms": ms}
            if done in marks:
                at[str(done)] = pd
            if not open_t and done >= marks[-1]:
                break
        for t in targets:
            first.setdefault(f"{t:g}", None)
        out.append({"lambda": lam, "first_below": first, "error_at_iters": at, "iters": done,
                    "ms": ms})
        progress(f"plateau lambda {lam:g}: {done} iterations, error {pd:.2e}")
    return {"workload": "grid256", "eps": "(8h)^2", "beta0": 0.0, "runs": out}


def _oracle_cells(job):
    """Worker: the oracle's cell solves of `job["cells"]` on the exported
    state (the cells' basic boxes, the aggregated Y-marginal, the stored
    potential)."""
    from oracle import dd
    w = WORKLOADS[job["name"]]
    n = w["n"]
    mu, nu = workload_marginals(job["name"])
    p = dd.make_problem(mu, nu, w["eps_h2"] / n ** 2, w["lam"], 1.0 / n, w["cell"])
    boxes = job["boxes"]   # dict basic id -> (o1, o2, values)
    opt = dd.Options(err=job["err"], max_iter=job["max_inner"], trunc=1e-15, margin=2,
                     translate=True)
    warm = np.ones(p.nb1 * p.nb2, dtype=bool)
    t0 = time.perf_counter()
    pts = 0
    for cell in job["cells"]:
        r = dd.process_cell(p, cell, boxes, job["P"], opt, job["abar"], warm)
        pts += r["iters"] * r["xi"].size
    return pts, time.perf_counter() - t0


def cpu_baseline(state, name, args):
    """The oracle (plain FP64 NumPy, as it stands) timed on the GPU line's own
    state: the cell solves of the partition the next step solves, a sample of
    cells spread over the grid, on 1 core and on all cores of this process's
    CPU share (one process per core, cells split evenly)."""
    from concurrent.futures import ProcessPoolExecutor
    from oracle import dd
    w = WORKLOADS[name]
    n = w["n"]
    part = "A" if state["k"] % 2 == 0 else "B"
    mu, nu = workload_marginals(name)
    p = dd.make_problem(mu, nu, w["eps_h2"] / n ** 2, w["lam"], 1.0 / n, w["cell"])
    P = np.zeros((n, n))
    off = 0
    allboxes = []
    for o1, o2, l1, l2 in state["boxes"]:
        v = state["values"][off:off + l1 * l2].reshape(l1, l2)
        P[o1:o1 + l1, o2:o2 + l2] += v
        allboxes.append((int(o1), int(o2), v))
        off += l1 * l2
    cells = dd.composite_cells(p, part)
    stride = max(1, len(cells) // args.cpu_cells)
    sample = [cells[i] for i in range(0, len(cells), stride)][: args.cpu_cells]
    if not all(state["warm"]):
        raise RuntimeError("the CPU sample expects a warm-started state")

    def job(cs):
        bx = {b: allboxes[b] for c in cs for b in c["basic"]}
        return {"name": name, "cells": cs, "boxes": bx, "P": P, "abar": state["abar"],
                "err": args.err, "max_inner": args.max_inner}
    one = sample[: max(1, len(sample) // 8)]
    pts1, t1 = _oracle_cells(job(one))
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    chunks = [sample[i::cores] for i in range(cores)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(_oracle_cells, [job(c) for c in chunks if c]))
    tall = time.perf_counter() - t0
    ptsa = sum(r[0] for r in res)
    progress(f"CPU oracle: {pts1 / t1:.3g} (1 core), {ptsa / tall:.3g} ({cores} cores) grid-pts*iters/s")
    return {"value": ptsa / tall, "unit": "grid-pts*iters/s", "cores": cores, "kind": "oracle",
            "one_core": {"value": pts1 / t1, "cores": 1, "sample": f"{len(one)} cell solves"},
            "sample": f"{len(sample)} of {len(cells)} partition-{part} cell solves of the GPU line's "
                      f"state (the half-iteration after the timed ones), spread over the grid; FP64 "
                      f"dense NumPy per cell, Err {args.err:g}, at most {args.max_inner} inner "
                      f"iterations; wall time of the process pool including its start"}


def gang_times(ms):
    """The gang autotuner's times (ms, -1: the shape does not apply) by shape
    (G x workgroups per CU; one workgroup per wide cell first)."""
    names = ("one_workgroup", "2x2", "4x1", "4x2", "8x1", "8x2", "16x2")
    return {k: float(v) for k, v in zip(names, ms)}


def timed_iterate(h, steps, warmup):
    """(wall seconds, grid-pts*iters) of `steps` half-iterations after `warmup`."""
    import torch
    B.dd_uot_iterate(h, warmup, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = B.dd_uot_iterate(h, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, float(st["point_iters"])


def batched_form(steps, warmup):
    """The batched workload (64 problems, sides 64..512, lambda log-uniform in
    [0.1, 10], eps = h^2, FP32, cells 4x4): one handle whose launches cover
    every problem's cells, A+B pairs replayed from a hipGraph, threads per
    cell and the wide cells' launch autotuned; against the same problems
    stepped one handle at a time (eager, 256 threads per cell), and against
    the same batch in FP64 (same start and half-iterations): per-problem
    tracked scores and DD-plan gaps of both precisions."""
    probs = batched_problems(64)

    def configs(precision):
        return [B.dd_uot_default_config(n1=q["n"], n2=q["n"], h=1.0 / q["n"], eps=1.0 / q["n"] ** 2,
                                        lam=q["lam"], cell=4, precision=precision,
                                        sinkhorn_max_iter=100, box_cap=48, getweights=B.GW_LINE,
                                        lenience=0.0) for q in probs]

    def scores(h):
        sc = [B.dd_uot_score(h, p) for p in range(len(probs))]
        tracked = np.array([s["tracked"] for s in sc])
        dual = np.array([s["dual"] for s in sc])
        return tracked, (tracked - dual) / np.abs(dual)

    cfgs = configs(32)
    h = B.dd_uot_init_batch(cfgs, [q["mu"] for q in probs], [q["nu"] for q in probs])
    try:
        nt, _ = B.dd_uot_autotune(h)
        gG, gW, gms = B.dd_uot_autotune_gang(h)
        B.dd_uot_set_graph(h, True)
        dt, pts = timed_iterate(h, steps, warmup)
        tr32, gap32 = scores(h)
    finally:
        B.dd_uot_destroy(h)
    h = B.dd_uot_init_batch(configs(64), [q["mu"] for q in probs], [q["nu"] for q in probs])
    try:
        B.dd_uot_set_graph(h, True)
        dt64, pts64 = timed_iterate(h, steps, warmup)
        tr64, gap64 = scores(h)
    finally:
        B.dd_uot_destroy(h)
    dtr = np.abs(tr32 - tr64) / np.abs(tr64)
    dts, ptss = 0.0, 0.0
    for c, q in zip(cfgs, probs):
        hs = B.dd_uot_init(c, q["mu"], q["nu"])
        try:
            d, p = timed_iterate(hs, steps, warmup)
        finally:
            B.dd_uot_destroy(hs)
        dts += d
        ptss += p
    progress(f"batched form: {pts / dt:.3g} vs one by one {ptss / dts:.3g} grid-pts*iters/s; "
             f"FP64 batch {pts64 / dt64:.3g}; FP32 vs FP64 tracked score max {dtr.max():.2e}")
    return {"problems": len(probs), "grid_points": int(sum(q["n"] ** 2 for q in probs)),
            "steps": steps, "threads_per_cell": nt, "gangs": [gG, gW],
            "gang_tuned_ms": gang_times(gms),
            "value": pts / dt, "ms_per_step": 1e3 * dt / steps,
            "one_by_one": {"value": ptss / dts, "ms_per_step": 1e3 * dts / steps},
            "unit": "grid-pts*iters/s", "speedup": (pts / dt) / (ptss / dts),
            "fp64": {"value": pts64 / dt64, "ms_per_step": 1e3 * dt64 / steps,
                     "tracked_score_rel_diff": {"max": float(dtr.max()),
                                                "median": float(np.median(dtr))},
                     "dd_plan_gap_fp32": {"max": float(gap32.max()), "median": float(np.median(gap32))},
                     "dd_plan_gap_fp64": {"max": float(gap64.max()), "median": float(np.median(gap64))},
                     "note": "same start and half-iterations in both precisions"}}


def differentiable_form(args, stream, halves):
    """The differentiable workload (512^2, Y points displaced by the seeded
    8x8 cubic B-spline field of amplitude 2h, lambda 1, eps = h^2, cells 4x4):
    the FP64 multiscale solve of the grid problem, its state loaded into the
    displaced problem's handles (same grid indices, boxes and cells) in FP32
    and FP64, `halves` half-iterations there (the first greedy, since the
    loaded tracked scores belong to the grid cost), then the certificate
    (polished; its gap is reported: the gradients are those of that state)
    and the gradients d/dmu, d/dnu (dd_uot_backward) and d/dy'
    (dd_uot_backward_ypos); the FP32 gradients are compared with the FP64
    ones from the same start, relative to the FP64 gradient."""
    import torch
    name = "grid512"
    w = WORKLOADS[name]
    n = w["n"]
    nb = (n // w["cell"]) ** 2
    mu, nu = workload_marginals(name)
    y = displaced_points(n, n, 1.0 / n, displacement_theta(53, 1.0 / n))
    t0 = time.perf_counter()
    h0, ttg = multiscale_solve(name, 64, 32, args.polish, args, stream)
    try:
        st = B.dd_uot_get_state(h0, n, n, nb)
    finally:
        B.dd_uot_destroy(h0)
    out = {"grid_solve": {"precision": 64, "ms": 1e3 * (time.perf_counter() - t0),
                          "certified_gap": ttg["final"]["certified_gap"]}}
    grads = {}
    for prec in (32, 64):
        c = workload_config(name, prec, args.max_inner, args.err, GW_IDS[args.getweights])
        h = B.dd_uot_init_moved(c, mu, nu, y, stream=stream)
        try:
            B.dd_uot_set_state(h, st, force_greedy=True)
            B.dd_uot_set_polish(h, args.polish)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it = B.dd_uot_iterate(h, halves)
            torch.cuda.synchronize()
            tf = time.perf_counter() - t0
            t0 = time.perf_counter()
            s = B.dd_uot_score(h, 0)
            dmu, dnu = B.dd_uot_backward(h, 0, n, n)
            dy = B.dd_uot_backward_ypos(h, 0, n, n)
            tb = time.perf_counter() - t0
        finally:
            B.dd_uot_destroy(h)
        grads[prec] = (dmu, dnu, dy)
        out[f"fp{prec}"] = {"forward_ms": 1e3 * tf, "forward_value": it["point_iters"] / tf,
                            "backward_ms": 1e3 * tb, "certified_gap": s["rel_gap_polished"],
                            "certificate_gap": s["rel_pd_gap"],
                            "dd_plan_gap": (s["tracked"] - s["dual"]) / abs(s["dual"])}
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["grad_fp32_vs_fp64"] = {"dmu": rel(grads[32][0], grads[64][0]),
                                "dnu": rel(grads[32][1], grads[64][1]),
                                "dypos": rel(grads[32][2], grads[64][2])}
    out["half_iters"] = halves
    out["unit"] = "grid-pts*iters/s"
    f32 = out["fp32"]
    progress(f"differentiable form: grid solve {out['grid_solve']['ms']:.0f} ms, displaced FP32 "
             f"{f32['forward_ms']:.0f} ms (certified gap {f32['certified_gap']:.2g}; FP64 "
             f"{out['fp64']['certified_gap']:.2g}), backward "
             f"{f32['backward_ms']:.0f} ms; FP32 vs FP64 gradients "
             f"{out['grad_fp32_vs_fp64']['dmu']:.2g} / {out['grad_fp32_vs_fp64']['dnu']:.2g} / "
             f"{out['grad_fp32_vs_fp64']['dypos']:.2g}")
    return out


def copy_probe(mib):
    """One plain device copy of `mib` MiB (a reference dispatch of known HBM
    traffic for the profiler's FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def run(args):
    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
    stream = torch.cuda.current_stream(dev).cuda_stream
    w = WORKLOADS[args.workload]
    n = w["n"]
    nb = (n // w["cell"]) ** 2
    # 1. the solve in the headline precision; its final state is timed
    h, ttg_main = multiscale_solve(args.workload, args.precision, args.final32, args.polish, args,
                                   stream)
    try:
        gG, gW, gms = B.dd_uot_autotune_gang(h)
        gangs = {"G": gG, "wgs_per_cu": gW, "tuned_ms": gang_times(gms)}
        progress(f"gang autotune: G {gG}, {gW} workgroups per CU")
        r = timed_steps(h, args.steps, args.warmup)
        progress(f"timed {args.steps} steps: {1e3 * r['dt'] / args.steps:.1f} ms per step")
        B.dd_uot_set_polish(h, args.polish)
        score = B.dd_uot_score(h, 0)
        state = B.dd_uot_get_state(h, n, n, nb)
    finally:
        B.dd_uot_destroy(h)
    dt, launches, kms, kbytes, hist = r["dt"], r["launches"], r["kms"], r["kbytes"], r["hist"]
    point_iters = hist[:, 4].sum()
    terms = hist[:, 10].sum()
    avg_ms = kms / max(launches, 1)
    exp_rate = terms / launches / (avg_ms * 1e-3)
    hbm_rate = kbytes / launches / (avg_ms * 1e-3)
    prof = profiled(args)
    out = {
        "metric": "grid-pts·iters/s and time to PD-gap 1e-6, 1024² UOT, FP32 vs FP64 on 1 GPU",
        "value": point_iters / dt if hist[:, 7].sum() == 0 else None,
        "unit": "grid-pts·iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "cell": w["cell"], "lambda": w["lam"],
                   "eps": w["eps_h2"] / n ** 2, "precision": args.precision,
                   "start": f"multiscale solve ({ttg_main['final']['half_iters']} half-iterations, "
                            f"final certified gap {ttg_main['final']['certified_gap']:.3g})",
                   "getweights": args.getweights, "lenience": 0.0, "cell_err": args.err,
                   "max_inner": args.max_inner, "translate_step": True, "balance": False,
                   "box_margin": 2, "wide_cell_gangs": gangs},
        "roofline": {"bound": "alu", "achieved": exp_rate / 1e12, "peak": EXP_PEAK / 1e12,
                     "unit": "Texp/s", "frac": exp_rate / EXP_PEAK,
                     "traffic": prof.get("traffic_bytes_per_launch"), "traffic_unit": "bytes/launch",
                     "valu_issue_frac": prof.get("valu_issue_frac"),
                     "valu_instr_per_term": prof.get("valu_instr_per_term"),
                     "counters_from": os.path.relpath(PROFILE, ROOT) if prof else None,
                     "kernel": "k_cell_solve (all launch tiers of a step)",
                     "terms_per_launch": terms / launches, "avg_launch_ms": avg_ms,
                     "hbm_algorithmic_GBps": hbm_rate / 1e9, "hbm_frac": hbm_rate / HBM_PEAK},
        "inner": {"point_iters": float(point_iters),
                  "mean_inner_per_cell": float(hist[:, 8].sum() / max(hist[:, 3].sum(), 1)),
                  "unconverged_cells": float(hist[:, 6].sum()),
                  "overflow_cells": float(hist[:, 7].sum()),
                  "cells_solved": float(hist[:, 3].sum()),
                  "safe_steps": int((hist[:, 0] < 1).sum()),
                  "mean_theta": float(hist[:, 0].mean()),
                  "fp64_fallbacks": float(hist[:, 11].sum())},
        "state_after": {"certified_gap": score["rel_gap_polished"],
                        "dd_plan_gap": (score["tracked"] - score["dual"]) / abs(score["dual"]),
                        "certificate_gap": score["rel_pd_gap"], "tracked_score": score["tracked"],
                        "half_iters": score["half_iters"], "nnz": score["nnz"],
                        **box_stats(state)},
        "time_to_gap": [ttg_main],
    }
    # 2. the other precision: its own solve, and the FP32 error of one step
    if args.other_precision:
        prec = 64 if args.precision == 32 else 32
        h2, ttg2 = multiscale_solve(args.workload, prec, args.final64, args.polish, args, stream)
        try:
            out["time_to_gap"].append(ttg2)
            if prec == 64:
                out["fp32_step_error"] = fp32_step_error(h2, args.workload, args, stream)
        finally:
            B.dd_uot_destroy(h2)
    if args.config2:
        out["eps_scaling_256"] = config2(args, stream)
    if args.plateau:
        out["plateau"] = plateau_study(stream)
    if args.forms:
        out["batched_form"] = batched_form(args.steps, args.warmup)
        out["differentiable_form"] = differentiable_form(args, stream, args.moved_halves)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(state, args.workload, args)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid1024", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--max-inner", type=int, default=3000,
                    help="inner iterations per cell solve at most")
    ap.add_argument("--err", type=float, default=2e-5, help="cell tolerance Err (Sec. 4.4)")
    ap.add_argument("--getweights", default="line", choices=("swift", "staggered", "line", "opt"))
    ap.add_argument("--final32", type=int, default=64,
                    help="half-iterations of the final stage of the FP32 solve, at most")
    ap.add_argument("--final64", type=int, default=128,
                    help="half-iterations of the final stage of the FP64 solve, at most")
    ap.add_argument("--final256", type=int, default=96,
                    help="half-iterations of the final stage of the 256^2 eps-scaling solves")
    ap.add_argument("--moved-halves", type=int, default=8,
                    help="half-iterations of the displaced problem from the grid solution")
    ap.add_argument("--plateau", type=int, default=0,
                    help="1: also the global Sinkhorn plateau study (256^2, 6 lambdas)")
    ap.add_argument("--config2", type=int, default=1,
                    help="1: also the 256^2 eps-scaling solves at lambda 0.1, 1, 10")
    ap.add_argument("--err-ratio", type=float, default=0.001,
                    help="final stage: cell tolerance min(Err, ratio x certified gap)")
    ap.add_argument("--polish", type=int, default=10,
                    help="global Sinkhorn iterations polishing each certificate")
    ap.add_argument("--other-precision", type=int, default=1,
                    help="1: also the solve in the other precision and the FP32 step error")
    ap.add_argument("--forms", type=int, default=1,
                    help="1: also time the batched and the differentiable workloads")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-cells", type=int, default=64,
                    help="cell solves of the CPU oracle sample (all cores)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB of a plain device copy run once before the solver (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver "
              "runs on a single device)", file=sys.stderr)
        sys.exit(2)
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
