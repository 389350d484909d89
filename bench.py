"""Throughput of the domain-decomposition hot path on one MI355X.

A step is one parallel DomDecIter half-iteration over every composite cell of
one partition (aggregation of the basic Y-marginals, cell inputs, the cell
Sinkhorn solves with the Newton Y-update and the PD stopping rule, re-split,
score pieces, GetWeights, update), alternating A and B.  The metric counts
grid points times inner Sinkhorn iterations: sum over solved cells of
|X_J| * (Y-halves of that cell), divided by the wall time of the timed steps.

The headline steps start from the local block start (nu_i = nu on block i),
where every cell's Y-box fits the slot and every cell is solved; GetWeights
`line` (one launch over every cell of the partition per step).  With
--warm 1 the same steps are also timed on the finest layer after the
multiscale warm start (untimed).  Time to a relative primal-dual gap is
measured separately (--ttg): the whole multiscale solve, FP32 and FP64, from
the host marginals to each target.

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

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 9.83e13 FP32 lane-ops/s;
# v_exp_f32 runs at a quarter of that rate.
EXP_PEAK = 256 * 64 * 2.4e9 / 4.0
HBM_PEAK = 8.0e12


GW_NAMES = {B.GW_GREEDY: "greedy", B.GW_SAFE: "safe", B.GW_SWIFT: "swift",
            B.GW_STAGGERED: "staggered", B.GW_LINE: "line"}
PROFILE = os.path.join(ROOT, "profiles", "k_cell_solve_grid1024_fp32_block.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2410_08859_amd", "csrc", "cell_kernel.hip")
PROFILED = dict(workload="grid1024", precision=32, cap=48, start="block", steps=4, warmup=1,
                max_inner=100, getweights="line")


def profiled_traffic(args):
    """HBM bytes per cell launch that rocprofv3 measured (FETCH_SIZE and
    WRITE_SIZE scaled by a copy probe) for this bench configuration and this
    kernel source; None for any other configuration or a changed kernel."""
    if any(getattr(args, k) != v for k, v in PROFILED.items()):
        return None
    try:
        txt = open(PROFILE).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    return float(m.group(1)) if (m and src in txt) else None


def multiscale_params(levels, final_max, target, check_every=4):
    return B.dd_uot_default_multiscale(levels=levels, final_max_halves=final_max,
                                       check_every=check_every, target_rel_gap=target)


def time_to_gap(name, precision, max_inner, cap, final_max, targets, stream, err, getweights):
    """Wall time of the whole multiscale solve (host marginals in, certificate
    checks included) until each relative gap first reaches each target: the
    certificate's pd_gap/|dual| and the DD plan's (tracked - dual)/|dual|.
    Layers from 16 x 16 up; global Sinkhorn below 256 x 256."""
    mu, nu = workload_marginals(name)
    cfg = workload_config(name, precision, max_inner, cap, err)
    # strict GetWeights on every layer: with the paper's lenience the tracked
    # score drifts up by up to 0.5 % per step and the gap stalls far higher
    cfg.lenience = 0.0
    cfg.getweights = getweights
    levels = int(round(np.log2(cfg.n1 / 16))) + 1
    ms = multiscale_params(levels, final_max, min(targets))
    h, tr = B.dd_uot_solve_multiscale(cfg, ms, mu, nu, stream=stream)
    B.dd_uot_destroy(h)
    progress(f"time to gap {name} FP{precision}: {tr[-1, 1] / 1e3:.1f} s, final DD-plan gap "
             f"{tr[-1, 3]:.3g}")

    def reached(col):
        out = {}
        for t in targets:
            hit = np.nonzero(tr[:, col] <= t)[0]
            out[f"{t:g}"] = None if hit.size == 0 else {"ms": float(tr[hit[0], 1]),
                                                        "half_iters": int(tr[hit[0], 0])}
        return out
    return {"workload": name, "precision": precision, "getweights": GW_NAMES[getweights],
            "dd_plan_gap": reached(3),
            "certificate_gap": reached(2),
            "final": {"certificate_gap": float(tr[-1, 2]), "dd_plan_gap": float(tr[-1, 3]),
                      "ms": float(tr[-1, 1]), "half_iters": int(tr[-1, 0])},
            "schedule": f"{levels} layers from 16^2, global Sinkhorn below 256^2 (tolerance "
                        f"{ms.global_tol:g} |mu|), eps 2h^2 -> h^2/2 per layer (-> eps on the "
                        f"finest), DD 4-16 half-iterations per stage (to rel. gap 1e-3), coarser DD "
                        f"layers box cap {ms.coarse_box_cap} and lenience {ms.coarse_lenience:g}, "
                        f"then at most {final_max} half-iterations with a certificate every 4; "
                        f"GetWeights {GW_NAMES[getweights]} (lenience 0), box cap {cap}, cell Err {err:g}, "
                        f"at most {max_inner} inner iterations"}


def plateau_study(name, lams, targets, max_iter, stream):
    """Global UOT Sinkhorn (no decomposition) at eps = (8h)^2 from beta = 0:
    iterations and wall time until KL(P_X pi | e^{-alpha/lambda} mu) / |mu|
    first reaches each target, and that error at fixed iteration counts, for
    each lambda (the convergence-plateau study of Sec. 4.4).  The run is cut
    into calls that stop at the next target or the next milestone, each
    continuing from the previous beta (the same iteration run without a
    stop)."""
    mu, nu = workload_marginals(name)
    n = mu.shape[0]
    mass = float(mu.sum())
    miles = [m for m in (10, 30, 100, 300, 1000, 3000, 10000, 30000) if m < max_iter] + [max_iter]
    rows = []
    for lam in lams:
        cfg = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=64.0 / n ** 2, lam=lam, cell=4,
                                      precision=64)
        beta = np.zeros((n, n))
        done, ti, mi, kl = 0, 0, 0, None
        hits = {f"{t:g}": None for t in targets}
        trace = []
        t0 = time.perf_counter()
        while done < max_iter and ti < len(targets):
            tol = targets[ti] * mass
            r = B.dd_uot_global_sinkhorn(cfg, mu, nu, beta, max_iter=miles[mi] - done, tol=tol,
                                         stream=stream)
            done += r["iters"]
            beta = r["beta"]
            kl = r["pd"] / mass
            ms = 1e3 * (time.perf_counter() - t0)
            while ti < len(targets) and r["pd"] <= targets[ti] * mass:
                hits[f"{targets[ti]:g}"] = {"iters": done, "ms": ms}
                ti += 1
            if done >= miles[mi]:
                trace.append([done, kl])
                mi += 1
        rows.append({"lambda": lam, "to_tolerance": hits, "iters_run": done, "final_kl_rel": kl,
                     "kl_rel_at_iters": trace})
        progress(f"plateau study lambda={lam:g}: {done} iterations, KL/|mu| {kl:.3g}")
    return {"workload": name, "eps": "(8h)^2", "criterion": "KL(P_X pi | e^{-alpha/lambda} mu)/|mu|",
            "max_iter": max_iter, "rows": rows}


def progress(msg):
    """One line on stderr per finished phase (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_steps(h, steps, warmup):
    """Run warmup steps, then time `steps` half-iterations (wall clock between
    device synchronisations) and the cell-solve launches (HIP events)."""
    import torch
    B.dd_uot_iterate(h, warmup, stats=False)
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
    return dict(dt=dt, launches=launches, kms=kms, kbytes=kbytes, hist=hist,
                score=B.dd_uot_score(h, 0))


def workload_config(name, precision, max_inner, cap, err=2e-5, getweights=None):
    w = WORKLOADS[name]
    n = w["n"]
    return B.dd_uot_default_config(
        n1=n, n2=n, h=1.0 / n, eps=w["eps_h2"] / n ** 2, lam=w["lam"], cell=w["cell"],
        precision=precision, init=B.INIT_BLOCK,
        getweights=B.GW_LINE if getweights is None else getweights,
        sinkhorn_err=err, sinkhorn_max_iter=max_inner, trunc=1e-15, lenience=0.005,
        box_margin=2, box_cap=cap)


def cpu_baseline(name, max_inner, cap, budget_s=15.0):
    """The oracle timed on a bounded sample of the same workload: the cell
    solves of the first A cells of the first half-iteration, until the budget
    is spent.  Single-threaded numpy."""
    from oracle import dd
    w = WORKLOADS[name]
    n = w["n"]
    mu, nu = workload_marginals(name)
    p = dd.make_problem(mu, nu, w["eps_h2"] / n ** 2, w["lam"], 1.0 / n, w["cell"])
    st = dd.init_block(p)
    opt = dd.Options(err=2e-5, max_iter=max_inner, trunc=1e-15, lenience=0.005, margin=2, cap=cap,
                     translate=True)
    P = dd.aggregate(p, st.boxes)
    cells = dd.composite_cells(p, "A")
    t0 = time.perf_counter()
    pts = 0
    done = 0
    for c in cells:
        r = dd.process_cell(p, c, st.boxes, P, opt)
        pts += r["iters"] * r["xi"].size
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": pts / dt, "unit": "grid-pts*iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of {len(cells)} partition-A cell solves of the first half-iteration "
                      f"({n}x{n}, FP64 dense numpy, Err 2e-5, max {max_inner} inner iterations)"}


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
    [0.1, 10], eps = h^2, FP32, cells 4x4, box cap 48): one handle whose
    launches cover every problem's cells, A+B pairs replayed from a hipGraph,
    threads per cell autotuned; against the same problems stepped one handle
    at a time (eager, 256 threads per cell)."""
    probs = batched_problems(64)
    cfgs = [B.dd_uot_default_config(n1=q["n"], n2=q["n"], h=1.0 / q["n"], eps=1.0 / q["n"] ** 2,
                                    lam=q["lam"], cell=4, precision=32, sinkhorn_max_iter=100,
                                    box_cap=48, getweights=B.GW_STAGGERED) for q in probs]
    h = B.dd_uot_init_batch(cfgs, [q["mu"] for q in probs], [q["nu"] for q in probs])
    try:
        nt, _ = B.dd_uot_autotune(h)
        B.dd_uot_set_graph(h, True)
        dt, pts = timed_iterate(h, steps, warmup)
    finally:
        B.dd_uot_destroy(h)
    dts, ptss = 0.0, 0.0
    for c, q in zip(cfgs, probs):
        hs = B.dd_uot_init(c, q["mu"], q["nu"])
        try:
            d, p = timed_iterate(hs, steps, warmup)
        finally:
            B.dd_uot_destroy(hs)
        dts += d
        ptss += p
    progress(f"batched form: {pts / dt:.3g} vs one by one {ptss / dts:.3g} grid-pts*iters/s")
    return {"problems": len(probs), "grid_points": int(sum(q["n"] ** 2 for q in probs)),
            "steps": steps, "threads_per_cell": nt, "value": pts / dt, "ms_per_step": 1e3 * dt / steps,
            "one_by_one": {"value": ptss / dts, "ms_per_step": 1e3 * dts / steps},
            "unit": "grid-pts*iters/s", "speedup": (pts / dt) / (ptss / dts)}


def differentiable_form(halves):
    """The differentiable workload (512^2, Y points displaced by the seeded
    8x8 cubic B-spline field of amplitude 2h, lambda 1, eps = h^2, cells 4x4,
    box cap 32): forward half-iterations, then the certificate and the
    gradients d/dmu, d/dnu (dd_uot_backward) and d/dy' (dd_uot_backward_ypos),
    in FP32 and FP64; the gradient difference between the two is reported
    relative to the FP64 gradient."""
    import torch
    w = WORKLOADS["grid512"]
    n = w["n"]
    mu, nu = workload_marginals("grid512")
    y = displaced_points(n, n, 1.0 / n, displacement_theta(53, 1.0 / n))
    out, grads = {}, {}
    for prec in (32, 64):
        c = B.dd_uot_default_config(n1=n, n2=n, h=1.0 / n, eps=w["eps_h2"] / n ** 2, lam=w["lam"],
                                    cell=w["cell"], precision=prec, init=B.INIT_BLOCK,
                                    sinkhorn_max_iter=100, box_cap=32,
                                    getweights=B.GW_STAGGERED)
        h = B.dd_uot_init_moved(c, mu, nu, y)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = B.dd_uot_iterate(h, halves)
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
        out[f"fp{prec}"] = {"forward_ms": 1e3 * tf, "forward_value": st["point_iters"] / tf,
                            "backward_ms": 1e3 * tb, "certificate_gap": s["rel_pd_gap"],
                            "dd_plan_gap": (s["tracked"] - s["dual"]) / abs(s["dual"])}
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["grad_fp32_vs_fp64"] = {"dmu": rel(grads[32][0], grads[64][0]),
                                "dnu": rel(grads[32][1], grads[64][1]),
                                "dypos": rel(grads[32][2], grads[64][2])}
    out["half_iters"] = halves
    out["unit"] = "grid-pts*iters/s"
    progress(f"differentiable form: forward FP32 {out['fp32']['forward_ms']:.0f} ms, backward "
             f"{out['fp32']['backward_ms']:.0f} ms")
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
    mu, nu = workload_marginals(args.workload)
    gw = {v: k for k, v in GW_NAMES.items()}[args.getweights]
    cfg = workload_config(args.workload, args.precision, args.max_inner, args.cap, getweights=gw)
    stream = torch.cuda.current_stream(dev)
    if args.start == "multiscale":
        # untimed warm start: coarse layers and the eps stages of the finest
        h, _ = B.dd_uot_solve_multiscale(cfg, multiscale_params(args.levels, 0, 0.0), mu, nu,
                                         stream=stream.cuda_stream)
    else:
        h = B.dd_uot_init(cfg, mu, nu, stream=stream.cuda_stream)
    try:
        r = timed_steps(h, args.steps, args.warmup)
    finally:
        B.dd_uot_destroy(h)
    progress(f"timed {args.steps} steps: {1e3 * r['dt'] / args.steps:.2f} ms per step")
    dt, launches, kms, kbytes, hist, score = (r["dt"], r["launches"], r["kms"], r["kbytes"],
                                              r["hist"], r["score"])
    point_iters = hist[:, 4].sum()
    terms = hist[:, 10].sum()
    avg_ms = kms / max(launches, 1)
    exp_rate = terms / launches / (avg_ms * 1e-3)
    hbm_rate = kbytes / launches / (avg_ms * 1e-3)
    out = {
        "metric": "grid-pts\u00b7iters/s and time to PD-gap 1e-6, 1024\u00b2 UOT, FP32 vs FP64 on 1 GPU",
        "value": point_iters / dt,
        "unit": "grid-pts\u00b7iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": cfg.n1, "cell": cfg.cell, "lambda": cfg.lambda_,
                   "eps": cfg.eps, "precision": args.precision, "max_inner": args.max_inner,
                   "box_cap": cfg.box_cap, "start": args.start, "getweights": args.getweights,
                   "levels": args.levels if args.start == "multiscale" else 1},
        "roofline": {"bound": "alu", "achieved": exp_rate / 1e12, "peak": EXP_PEAK / 1e12,
                     "unit": "Texp/s", "frac": exp_rate / EXP_PEAK,
                     "traffic": profiled_traffic(args), "traffic_unit": "bytes/launch",
                     "kernel": "k_cell_solve", "avg_launch_ms": avg_ms,
                     "hbm_algorithmic_GBps": hbm_rate / 1e9, "hbm_frac": hbm_rate / HBM_PEAK},
        "inner": {"point_iters": float(point_iters), "mean_inner_per_cell":
                  float(hist[:, 8].sum() / max(hist[:, 3].sum(), 1)),
                  "unconverged_cells": float(hist[:, 6].sum()),
                  "overflow_cells": float(hist[:, 7].sum()),
                  "safe_steps": int((hist[:, 0] < 1).sum()),
                  "fp64_fallbacks": float(hist[:, 11].sum())},
        "state_after": {"certificate_gap": score["rel_pd_gap"],
                        "dd_plan_gap": (score["tracked"] - score["dual"]) / abs(score["dual"]),
                        "tracked_score": score["tracked"], "half_iters": score["half_iters"]},
    }
    if args.other_precision and args.start == "block":
        # the same workload and steps in the other cell precision (FP32 vs FP64)
        prec = 64 if args.precision == 32 else 32
        c2 = workload_config(args.workload, prec, args.max_inner, args.cap, getweights=gw)
        h = B.dd_uot_init(c2, mu, nu, stream=stream.cuda_stream)
        try:
            o = timed_steps(h, args.steps, args.warmup)
        finally:
            B.dd_uot_destroy(h)
        oh = o["hist"]
        out["other_precision"] = {
            "precision": prec, "value": float(oh[:, 4].sum() / o["dt"]),
            "ms_per_step": 1e3 * o["dt"] / args.steps,
            "avg_launch_ms": o["kms"] / max(o["launches"], 1),
            "mean_inner_per_cell": float(oh[:, 8].sum() / max(oh[:, 3].sum(), 1)),
            "unit": "grid-pts\u00b7iters/s"}
        progress(f"FP{prec} steps: {1e3 * o['dt'] / args.steps:.2f} ms per step")
    if args.warm and args.start != "multiscale":
        # the same steps after the multiscale warm start (the paper's pipeline)
        wcfg = workload_config(args.workload, args.precision, args.ms_max_inner, args.cap,
                               args.ms_err, gw)
        h, _ = B.dd_uot_solve_multiscale(wcfg, multiscale_params(args.levels, 0, 0.0), mu, nu,
                                         stream=stream.cuda_stream)
        try:
            w = timed_steps(h, args.steps, args.warmup)
        finally:
            B.dd_uot_destroy(h)
        wh = w["hist"]
        progress(f"warm-start steps: {1e3 * w['dt'] / args.steps:.2f} ms per step")
        out["warm_start_steps"] = {
            "value": float(wh[:, 4].sum() / w["dt"]), "ms_per_step": 1e3 * w["dt"] / args.steps,
            "mean_inner_per_cell": float(wh[:, 8].sum() / max(wh[:, 3].sum(), 1)),
            "overflow_cells": float(wh[:, 7].sum()), "unconverged_cells": float(wh[:, 6].sum()),
            "certificate_gap": w["score"]["rel_pd_gap"],
            "dd_plan_gap": (w["score"]["tracked"] - w["score"]["dual"]) / abs(w["score"]["dual"]),
            "start": f"multiscale, {args.levels} layers", "cell_err": args.ms_err,
            "max_inner": args.ms_max_inner}
    if args.ttg:
        targets = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)
        out["time_to_gap"] = [
            time_to_gap(name, prec, args.ms_max_inner, args.ttg_cap,
                        args.ttg_max32 if prec == 32 else args.ttg_max64, targets,
                        stream.cuda_stream, args.ms_err,
                        {v: k for k, v in GW_NAMES.items()}[args.ttg_getweights])
            for name in args.ttg_workloads.split(",") for prec in (32, 64)]
    if args.plateau:
        out["plateau_study"] = plateau_study("grid256", (0.01, 0.1, 1.0, 10.0, 100.0, 1000.0),
                                             (1e-2, 1e-3, 1e-4, 1e-5, 1e-6), args.plateau_max,
                                             stream.cuda_stream)
    if args.forms:
        out["batched_form"] = batched_form(args.steps, args.warmup)
        out["differentiable_form"] = differentiable_form(args.steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.max_inner, args.cap, args.cpu_budget)
        progress("CPU oracle sample timed")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid1024", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--max-inner", type=int, default=100)
    ap.add_argument("--getweights", default="line", choices=("swift", "staggered", "line"),
                    help="GetWeights of the timed steps")
    ap.add_argument("--cap", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--start", default="block", choices=("multiscale", "block"))
    ap.add_argument("--warm", type=int, default=0,
                    help="1: also time the steps after the multiscale warm start")
    ap.add_argument("--levels", type=int, default=7)
    ap.add_argument("--ttg", type=int, default=1, help="1: also measure time to gap (FP32, FP64)")
    ap.add_argument("--forms", type=int, default=1,
                    help="1: also time the batched and the differentiable workloads")
    ap.add_argument("--ms-err", type=float, default=2e-5,
                    help="cell tolerance Err of the multiscale runs")
    ap.add_argument("--ms-max-inner", type=int, default=1000)
    ap.add_argument("--ttg-workloads", default="grid256")
    ap.add_argument("--ttg-cap", type=int, default=80)
    ap.add_argument("--ttg-getweights", default="line", choices=("swift", "staggered", "line"),
                    help="GetWeights of the time-to-gap runs (line: the fastest decrement)")
    ap.add_argument("--ttg-max32", type=int, default=64)
    ap.add_argument("--ttg-max64", type=int, default=64)
    ap.add_argument("--other-precision", type=int, default=1,
                    help="1: also time the same steps in the other cell precision")
    ap.add_argument("--plateau", type=int, default=1,
                    help="1: also run the global-Sinkhorn convergence study over lambda")
    ap.add_argument("--plateau-max", type=int, default=10000,
                    help="iteration cap per lambda of the plateau study")
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
