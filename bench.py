"""Benchmark of the Leja phi-action hot path on one MI355X.

One step is one pass of the whole path over the 512^2 Allen-Cahn workload
(eps = 1e-3, u0 ~ U[-0.1, 0.1], h = 10x the explicit diffusive step, tol 1e-10):
  * an EXPRB2 step         -- power iteration + phi_1(hJ) h f(u)
  * an EPIRK4s3 step       -- power iteration + vertical phi_1 at 1/8, 1/9, 1 +
                              phi_3 + phi_4 on the stage remainders
  * a stand-alone phi_2(hJ) h f(u) (bound shared with the EPIRK4s3 step)
i.e. 7 delivered phi-actions per step, issued back to back and synchronised
once per step (deferred synchronisation: a rejected expansion is redone before
the step ends).  `value` is delivered phi-actions per
second with inputs resident in HBM.  The roofline object describes the fused
Leja iteration kernel, timed with HIP events on its launch stream over the
timed region; `cpu_baseline` times the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --form batch [--steps K] [--warmup W]
                        (the batching form: 256 uneven Allen-Cahn instances,
                         phi_1..phi_3 per instance in one graph-captured launch,
                         against the per-instance plain path)
       python bench.py --form sweep   (the other workloads: advection-diffusion 32^2,
                        Brusselator 1024^2 and Gray-Scott 1024^2 steps, an
                        advection-diffusion-reaction 512^2 step (Neumann),
                        Allen-Cahn 1024^2..8192^2)
       python bench.py --form stiffness   (the 512^2 step at 1..100x CFL; 10 Brusselator 1024^2 EXPRB3 steps)
       python bench.py --form adaptive   (variable step sizes, EPIRK4s3 on 512^2 Allen-Cahn)
       python bench.py --form user   (operators as callbacks: phi_1 on 512^2 Allen-Cahn, fused vs callbacks)
       python bench.py --form lekry  (EPIRK4s3 on 512^2 Allen-Cahn: all-Leja vs LeKry)
       python bench.py --form ceiling  (attainable HBM bandwidth: copy, read, Newton-step pattern)
       python bench.py --copy-calibration   (plain copy kernel for counter scaling)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TOL = 1e-10
CFL_MULT = 10.0
ACTIONS_PER_STEP = 7
METRIC = "\u03c6_l(hJ)v actions/sec + HBM GB/s (% peak), 512\u00b2 Allen\u2013Cahn, tol 1e-10"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "leja_kernel_allen_cahn_512_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_kernel_allen_cahn_256_instances_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per fused-kernel launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2211_08948_amd.rocprof_summary import kernel_source_hash
    if t.get("kernel_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def algorithmic_bytes(tm: dict, ncomp: int = 1) -> float:
    """Bytes the method must move through memory in the action kernel: per grid
    point and Newton iteration, read y_{m-1}, read the linearisation state,
    write y_m (24 B per component) and read+write every active accumulator
    (16 B per component); per power-iteration product, read x, read the state,
    write J x (24 B per component)."""
    return ncomp * (24.0 * tm["point_iters"] + 16.0 * tm["accum_point_iters"] + 24.0 * tm["power_point_iters"])


def copy_calibration():
    import torch
    n = 1 << 26  # 512 MiB of float64
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 10
    log(f"copy of {8 * n / 2**20:.0f} MiB: read {8 * n} B + write {8 * n} B per dispatch, "
        f"{2 * 8 * n / dt / 1e9:.0f} GB/s")


def cpu_baseline(prob, h):
    """The CPU oracle on one full step of the same workload (a bounded sample)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np

    from oracle.integrators import step as oracle_step
    from oracle.leja import Options, phi_action
    from oracle.operators import Operator
    op = Operator(prob)
    v = h * op.rhs(prob.state)
    t = time.perf_counter()
    steps = 0
    while steps < 50 and (steps == 0 or time.perf_counter() - t < 12.0):
        oracle_step(op, "EXPRB2", h, TOL)
        _, _, log4 = oracle_step(op, "EPIRK4S3", h, TOL)
        phi_action(op, v, 2, h, TOL, Options(bound=log4[0].bound))
        steps += 1
    dt = time.perf_counter() - t
    np.asarray(0)
    return {"value": round(ACTIONS_PER_STEP * steps / dt, 3), "unit": "phi-actions/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} full step(s) ({ACTIONS_PER_STEP * steps} actions) of the same 512^2 workload, "
                      f"FP64 NumPy oracle on 1 core, {dt:.1f} s; host nproc={os.cpu_count()}"}


def bench_batch(args):
    """The batching form on the 256-instance ensemble: one graph replay runs
    phi_1, phi_2, phi_3 of h_i f(u_i) for every instance (768 actions)."""
    import torch

    import paper_2211_08948_amd as lj
    from workloads import batch_instances
    probs = batch_instances()
    hs = [CFL_MULT * p.h_cfl for p in probs]
    ctx = lj.Context(0)
    ops = [lj.operator_from(p, "cuda:0") for p in probs]
    vs = []
    for J, h in zip(ops, hs):
        f = torch.empty_like(J.state)
        lj.lj_rhs(ctx, J, J.state, f)
        vs.append((h * f).contiguous())
    ws = [[torch.empty_like(v) for _ in range(3)] for v in vs]
    b = lj.Batch(ctx, ops, vs, hs, [1, 2, 3], [1.0, 1.0, 1.0], TOL, ws)
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        b.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    rc, sts = b.stats(stream)
    if rc != lj.LJ_OK or not all(st["converged"] for st in sts):
        raise SystemExit("batch: an instance did not converge")
    info = b.info()
    rejected = sum(1 for st in sts if st["rejections"] > 0)
    substepped = sum(1 for st in sts if max(st["substeps"]) > 1)
    # the same work through the plain path: one vertical call per instance
    # (each synchronises once), after a warm-up pass, timed by the same
    # events over the same number of passes
    plain_reps = max(1, min(args.steps, 5))

    def plain_pass():
        for i in range(len(probs)):
            rcp, _ = lj.lj_phi_vertical(ctx, ops[i], vs[i], [1, 2, 3], [1.0] * 3, hs[i], TOL, ws[i])
            if rcp != lj.LJ_OK:
                raise SystemExit("plain path: an instance did not converge")
    plain_pass()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(plain_reps):
        plain_pass()
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / plain_reps
    actions = 3 * len(probs)
    achieved = info["alg_bytes"] / (ms * 1e-3) / 1e9
    traffic = measured_traffic(BATCH_TRAFFIC_FILE)
    log(f"batch {ms:.3f} ms per launch (schedule {info['schedule']}: {info['block_size']} threads, team "
        f"{info['team']}), {info['alg_bytes'] / 1e9:.2f} GB algorithmic, {rejected} instances with a rejection, "
        f"{substepped} substepped inside the launch; plain path {plain_ms:.1f} ms per pass")
    out = {
        "metric": "\u03c6_l(hJ)v actions/sec, batching form: 256 uneven Allen\u2013Cahn instances, tol 1e-10",
        "value": round(actions / (ms * 1e-3), 1), "unit": "phi-actions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "256 Allen-Cahn instances, n in {128,192,256,384,512} uniform, eps log-uniform "
                               "[1e-4,1e-2] (seed 4), u0 seed 4000+i, h_i = 10x CFL_i, phi_1..phi_3 vertical, "
                               "tol 1e-10, one graph-captured launch",
                   "instances": len(probs), "total_points": int(info["total_values"]),
                   "schedule": {"block_size": info["block_size"], "team": info["team"]}},
        "speedup_vs_plain_vertical": round(plain_ms / ms, 2),
        "rejected_instances": rejected, "substepped_instances": substepped,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "dram_gbs": round(traffic / (ms * 1e-3) / 1e9, 1) if traffic else None,
                     "kernel": "lj_batch_kernel", "avg_launch_us": round(ms * 1e3, 1),
                     "algorithmic_bytes_per_launch": round(info["alg_bytes"])},
        "cpu_baseline": None,
    }
    b.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_sweep(args):
    """The other measured workloads, one JSON line each (not the headline
    metric): advection-diffusion 32^2 phi_1 (latency: us per action), the
    Brusselator 1024^2 (EXPRB43-u3 steps + a stand-alone phi_2), Gray-Scott
    1024^2 (EPIRK4s3 steps), advection-diffusion-reaction 512^2 with Neumann
    boundaries (EPIRK4s3 steps), and phi_1 on Allen-Cahn grids from 1024^2 to
    8192^2 (the HBM-bound regime)."""
    import statistics

    import torch

    import paper_2211_08948_amd as lj
    from workloads import adr_neumann, advdiff_bump, allen_cahn_noise, brusselator_perturbed, gray_scott_spots
    ctx = lj.Context(0)

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        lj.lj_timing_read(ctx, reset=True)
        lj.lj_timing_enable(ctx, True)
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        lj.lj_timing_enable(ctx, False)
        return statistics.median(ts), lj.lj_timing_read(ctx, reset=True), out

    def line(workload, metric, value, unit, ms, tm, ncomp, extra, bound="hbm", traffic_file=None):
        launches = max(tm["launches"], 1)
        avg_ms = tm["kernel_ms"] / launches
        bpl = algorithmic_bytes(tm, ncomp) / launches
        ach = bpl / (avg_ms * 1e-3) / 1e9
        traffic = measured_traffic(traffic_file) if traffic_file else None
        rec = {"metric": metric, "value": round(value, 2), "unit": unit, "n_gpus": 1, "ms_per_step": round(ms, 4),
               "dtype": "f64", "data": "synthetic", "config": {"workload": workload},
               "roofline": {"bound": bound, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_ms * 1e3, 2),
                            "algorithmic_bytes_per_launch": round(bpl), "traffic": traffic,
                            "dram_gbs": round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None}}
        rec.update(extra)
        print(json.dumps(rec), flush=True)

    def others(timed, line):
        # advection-diffusion 32^2, grid Peclet 1, phi_1 at 10x CFL
        prob, v0 = advdiff_bump()
        op = lj.operator_from(prob, "cuda:0")
        v = torch.as_tensor(v0, dtype=torch.float64, device="cuda:0")
        w = torch.empty_like(v)
        h = CFL_MULT * prob.h_cfl
        dt, tm, (rc, st) = timed(lambda: lj.lj_phi_action(ctx, op, v, w, 1, h, TOL), 50)
        line("advection-diffusion 32x32, nu 1, grid Peclet 1, bump + noise seed 1, phi_1 at 10x CFL, tol 1e-10",
             "\u00b5s per \u03c6_1 action", dt * 1e6, "us", dt * 1e3, tm, 1, {"m_star": st["m_star"][0]},
             bound="latency")

        # Brusselator 1024^2: EXPRB43-u3 steps + a stand-alone phi_2
        prob = brusselator_perturbed()
        op = lj.operator_from(prob, "cuda:0")
        h = CFL_MULT * prob.h_cfl
        u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
        f = torch.empty_like(u_out)
        lj.lj_rhs(ctx, op, op.state, f)
        v = (h * f).contiguous()
        w = torch.empty_like(v)

        def bstep():
            _, s3 = lj.lj_step(ctx, "EXPRB43_U3", op, h, TOL, u_out)
            lj.lj_phi_action(ctx, op, v, w, 2, h, TOL, lj.lj_default_options(bound=s3[0]["bound"]))
            return s3

        dt, tm, s3 = timed(bstep, 10)
        line("brusselator 1024x1024 periodic, D 2e-3, a 1, b 3, perturbation seed 3, h 10x CFL, tol 1e-10: "
             "one EXPRB43-u3 step + a phi_2 action (5 actions)", "\u03c6_l(hJ)v actions/sec", 5 / dt,
             "phi-actions/s", dt * 1e3, tm, 2, {"m_star": [s["m_star"][:2] for s in s3]})

        # Gray-Scott 1024^2 (Sec. 3 spots, a1 = a2 = 1e-3): one EPIRK4s3 step
        prob = gray_scott_spots(1024, a1=1e-3, a2=1e-3)
        op = lj.operator_from(prob, "cuda:0")
        h = CFL_MULT * prob.h_cfl
        u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
        err = torch.empty_like(u_out)
        dt, tm, s4 = timed(lambda: lj.lj_step(ctx, "EPIRK4S3", op, h, TOL, u_out, err)[1], 10)
        line("gray-scott 1024x1024 periodic, a1 = a2 = 1e-3, a 0.04, b 0.06, spot initial state, h 10x CFL, "
             "tol 1e-10: one EPIRK4s3 step (5 actions)", "\u03c6_l(hJ)v actions/sec", 5 / dt, "phi-actions/s",
             dt * 1e3, tm, 2, {"m_star": [s["m_star"][:3] for s in s4]})

        # advection-diffusion-reaction 512^2 (Sec. 3, Neumann boundaries, its initial
        # state; alpha 1e-2, beta -10, rate 100): one EPIRK4s3 step
        prob = adr_neumann(512, alpha=1e-2, beta=-10.0, rate=100.0)
        op = lj.operator_from(prob, "cuda:0")
        h = CFL_MULT * prob.h_cfl
        u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
        err = torch.empty_like(u_out)
        dt, tm, s5 = timed(lambda: lj.lj_step(ctx, "EPIRK4S3", op, h, TOL, u_out, err)[1], 20)
        line("advection-diffusion-reaction 512x512, homogeneous Neumann, alpha 1e-2, beta -10, rate 100, "
             "initial state 256(xy(1-x)(1-y))^2 + 0.3, h 10x CFL, tol 1e-10: one EPIRK4s3 step (5 actions)",
             "\u03c6_l(hJ)v actions/sec", 5 / dt, "phi-actions/s", dt * 1e3, tm, 1,
             {"m_star": [s["m_star"][:3] for s in s5]}, bound="latency")


    if not args.sweep_n:
        others(timed, line)
    # Allen-Cahn n^2, phi_1 of h f(u) at 10x CFL, bound given (Newton recurrence only);
    # 2000 is not a multiple of the 32-point tile (the narrower last tiles)
    for n in ((args.sweep_n,) if args.sweep_n else (1024, 2000, 2048, 4096, 8192)):
        prob = allen_cahn_noise(n, eps=1e-3, seed=2)
        op = lj.operator_from(prob, "cuda:0")
        h = CFL_MULT * prob.h_cfl
        f = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
        lj.lj_rhs(ctx, op, op.state, f)
        v = (h * f).contiguous()
        w = torch.empty_like(v)
        lam = lj.lj_spectral_bound(ctx, op, 20)
        o = lj.lj_default_options(bound=lam)
        dt, tm, (rc, st) = timed(lambda: lj.lj_phi_action(ctx, op, v, w, 1, h, TOL, o), 10 if n < 8192 else 4)
        # the register-tiled kernel (several 32 x 32 tiles per block) keeps 16
        # Newton steps per pass over HBM: its time goes to the steps' arithmetic
        # and workgroup synchronisation, not to memory traffic; with
        # LJ_NO_TILE=1 the streaming kernel runs and streams from HBM
        tiled = tm["tiled_launches"] > 0
        tf = None
        if n == 4096:
            tf = os.path.join(ROOT, "profiles", "action_regm_allen_cahn_4096_traffic.json" if tiled
                              else "action_stream_allen_cahn_4096_traffic.json")
        line(f"allen-cahn {n}x{n} periodic, eps 1e-3, u0~U[-0.1,0.1] seed 2, phi_1 at 10x CFL, bound given, "
             "tol 1e-10", "\u03c6_l(hJ)v actions/sec", 1 / dt, "phi-actions/s", dt * 1e3, tm, 1,
             {"m_star": st["m_star"][0], "kernel": "register-tiled" if tiled else "streaming"},
             bound="latency" if tiled else "hbm", traffic_file=tf)
    ctx.close()


def bench_stiffness(args):
    """The 512^2 Allen-Cahn step of the headline (EXPRB2 + EPIRK4s3 + phi_2) at
    h = 1, 3, 10, 30 and 100 times the explicit step, and the Brusselator
    1024^2 trajectory of 10 EXPRB43-u3 steps (u <- step(u)); one JSON line
    each (not the headline metric)."""
    import torch

    import paper_2211_08948_amd as lj
    from workloads import allen_cahn_noise, brusselator_perturbed
    ctx = lj.Context(0)
    prob = allen_cahn_noise(512, eps=1e-3, seed=2)
    op = lj.operator_from(prob, "cuda:0")
    u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    err = torch.empty_like(u_out)
    f = torch.empty_like(u_out)
    w2 = torch.empty_like(u_out)
    lj.lj_rhs(ctx, op, op.state, f)
    for mult in (1.0, 3.0, 10.0, 30.0, 100.0):
        h = mult * prob.h_cfl
        v = (h * f).contiguous()

        def one_step():
            _, s2 = lj.lj_step(ctx, "EXPRB2", op, h, TOL, u_out, None)
            _, s4 = lj.lj_step(ctx, "EPIRK4S3", op, h, TOL, u_out, err)
            _, s1 = lj.lj_phi_action(ctx, op, v, w2, 2, h, TOL, lj.lj_default_options(bound=s4[0]["bound"]))
            return s2, s4, s1

        for _ in range(3):
            one_step()
        torch.cuda.synchronize()
        lj.lj_timing_read(ctx, reset=True)
        lj.lj_timing_enable(ctx, True)
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            s2, s4, s1 = one_step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        lj.lj_timing_enable(ctx, False)
        tm = lj.lj_timing_read(ctx, reset=True)
        launches = max(tm["launches"], 1)
        avg_ms = tm["kernel_ms"] / launches
        bpl = algorithmic_bytes(tm) / launches
        ach = bpl / (avg_ms * 1e-3) / 1e9
        rec = {"metric": "\u03c6_l(hJ)v actions/sec, 512\u00b2 Allen\u2013Cahn step at h / h_CFL = %g" % mult,
               "value": round(ACTIONS_PER_STEP / dt, 1), "unit": "phi-actions/s", "n_gpus": 1,
               "ms_per_step": round(dt * 1e3, 4), "dtype": "f64", "data": "synthetic",
               "config": {"workload": "allen-cahn 512x512 periodic, eps 1e-3, u0~U[-0.1,0.1] seed 2, "
                                      "h=%gx CFL, tol 1e-10: EXPRB2 + EPIRK4s3 steps + phi_2 action" % mult},
               "m_star": {"EXPRB2": s2[0]["m_star"][0], "EPIRK4s3_vertical": s4[0]["m_star"][:3],
                          "phi_3": s4[1]["m_star"][0], "phi_4": s4[2]["m_star"][0], "phi_2": s1["m_star"][0]},
               "substeps": max(max(s2[0]["substeps"]), max(s4[0]["substeps"]), max(s1["substeps"])),
               "roofline": {"bound": "latency", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_ms * 1e3, 2),
                            "algorithmic_bytes_per_launch": round(bpl)}}
        print(json.dumps(rec), flush=True)

    # the Brusselator trajectory: 10 EXPRB43-u3 steps from the perturbed steady state
    prob = brusselator_perturbed()
    h = CFL_MULT * prob.h_cfl
    u = torch.as_tensor(prob.state, dtype=torch.float64, device="cuda:0").contiguous()
    ubuf = [u.clone(), torch.empty_like(u)]

    def trajectory():
        logs = []
        cur = 0
        for _ in range(10):
            J = lj.Operator(prob.kind, prob.nx, prob.ny, prob.ncomp, prob.dx, prob.dy,
                            tuple(float(c) for c in prob.coef), ubuf[cur])
            _, s3 = lj.lj_step(ctx, "EXPRB43_U3", J, h, TOL, ubuf[1 - cur])
            logs.append(s3)
            cur = 1 - cur
        return logs

    ubuf[0].copy_(u)
    trajectory()
    torch.cuda.synchronize()
    lj.lj_timing_read(ctx, reset=True)
    lj.lj_timing_enable(ctx, True)
    ubuf[0].copy_(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logs = trajectory()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lj.lj_timing_enable(ctx, False)
    tm = lj.lj_timing_read(ctx, reset=True)
    launches = max(tm["launches"], 1)
    avg_ms = tm["kernel_ms"] / launches
    bpl = algorithmic_bytes(tm, 2) / launches
    ach = bpl / (avg_ms * 1e-3) / 1e9
    rec = {"metric": "\u03c6_l(hJ)v actions/sec, Brusselator 1024\u00b2, 10 EXPRB3 steps",
           "value": round(4 * 10 / dt, 1), "unit": "phi-actions/s", "n_gpus": 1, "ms_per_step": round(dt * 100, 4),
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "brusselator 1024x1024 periodic, D 2e-3, a 1, b 3, perturbation seed 3, "
                                  "h 10x CFL, tol 1e-10: 10 EXPRB43-u3 steps u <- step(u) (4 actions each)"},
           "m_star": [[s["m_star"][:2] for s in step_log] for step_log in logs],
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_ms * 1e3, 2),
                        "algorithmic_bytes_per_launch": round(bpl)}}
    print(json.dumps(rec), flush=True)
    ctx.close()


def bench_adaptive(args):
    """Variable step sizes (Sec. 2.3) on the 512^2 Allen-Cahn workload: EPIRK4s3
    from u0 to T = 100 explicit diffusive steps, step tolerance 1e-6, phi
    actions to 1e-10; one JSON line (not the headline metric)."""
    import torch

    import paper_2211_08948_amd as lj
    from workloads import allen_cahn_noise
    prob = allen_cahn_noise(args.n, eps=1e-3, seed=2)
    ctx = lj.Context(0)
    op = lj.operator_from(prob, "cuda:0")
    out = torch.empty_like(op.state)
    T, dt0, tol = 100.0 * prob.h_cfl, CFL_MULT * prob.h_cfl, 1e-6
    lj.lj_integrate(ctx, "EPIRK4S3", op, 5 * prob.h_cfl, dt0, tol, TOL, out)  # warm-up
    torch.cuda.synchronize()
    lj.lj_timing_read(ctx, reset=True)
    lj.lj_timing_enable(ctx, True)
    t0 = time.perf_counter()
    rc, st, recs = lj.lj_integrate(ctx, "EPIRK4S3", op, T, dt0, tol, TOL, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lj.lj_timing_enable(ctx, False)
    tm = lj.lj_timing_read(ctx, reset=True)
    launches = max(tm["launches"], 1)
    avg_ms = tm["kernel_ms"] / launches
    bpl = algorithmic_bytes(tm) / launches
    ach = bpl / (avg_ms * 1e-3) / 1e9
    actions = 5 * (st["accepted"] + st["rejected"])  # phi_1 x3 (vertical), phi_3, phi_4 per attempt
    rec = {"metric": "time to solution, variable steps", "value": round(dt * 1e3, 3), "unit": "ms", "n_gpus": 1,
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"allen-cahn {args.n}x{args.n} periodic, eps 1e-3, u0~U[-0.1,0.1] seed 2, EPIRK4s3 "
                                  "from t = 0 to 100x the explicit diffusive step, step tol 1e-6 (relative "
                                  "embedded estimate), phi actions to 1e-10, first attempt 10x CFL"},
           "accepted": st["accepted"], "rejected": st["rejected"], "products": st["products"], "rc": rc,
           "actions_per_s": round(actions / dt, 1),
           "dt_over_cfl": [round(r["dt"] / prob.h_cfl, 3) for r in recs],
           # the tiled kernels keep the 512^2 working set on chip (latency-bound,
           # as the headline line); the streaming kernel streams from HBM
           "roofline": {"bound": "latency" if tm["tiled_launches"] > 0 else "hbm", "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_ms * 1e3, 2),
                        "algorithmic_bytes_per_launch": round(bpl)}}
    ctx.close()
    print(json.dumps(rec), flush=True)


def bench_user(args):
    """The user-operator path (lj_user_*) on 512^2 Allen-Cahn, phi_1 of h f(u)
    at 10x CFL with the bound given: the fused action kernel against the same
    operator through callbacks (the library's own lj_jv / lj_rhs called from
    Python), with analytic and with finite-difference products; one JSON line
    per variant (not the headline metric)."""
    import statistics

    import torch

    import paper_2211_08948_amd as lj
    from workloads import allen_cahn_noise
    prob = allen_cahn_noise(args.n, eps=1e-3, seed=2)
    ctx = lj.Context(0)
    J = lj.operator_from(prob, "cuda:0")
    h = CFL_MULT * prob.h_cfl
    f = torch.empty_like(J.state)
    lj.lj_rhs(ctx, J, J.state, f)
    v = (h * f).contiguous()
    w = torch.empty_like(v)
    lam = lj.lj_spectral_bound(ctx, J, 20)
    o = lj.lj_default_options(bound=lam)
    variants = [
        ("fused action kernel", lambda: lj.lj_phi_action(ctx, J, v, w, 1, h, TOL, o)),
        ("callbacks, analytic J v", lambda: lj.lj_user_phi_action(ctx, lj.family_user_operator(ctx, J), v, w, 1, h,
                                                                 TOL, o)),
        ("callbacks, finite-difference J v", lambda: lj.lj_user_phi_action(
            ctx, lj.family_user_operator(ctx, J, finite_difference=True), v, w, 1, h, TOL, o)),
    ]
    for name, fn in variants:
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(args.steps // 5, 5)):
            t0 = time.perf_counter()
            rc, st = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        dt = statistics.median(ts)
        m = st["m_star"][0]
        rec = {"metric": "\u03c6_1 action time", "value": round(dt * 1e6, 1), "unit": "us", "n_gpus": 1,
               "higher_is_better": False, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"allen-cahn {args.n}x{args.n} periodic, eps 1e-3, u0~U[-0.1,0.1] seed 2, "
                                      f"phi_1 at 10x CFL, bound given, tol 1e-10: {name}"},
               "m_star": m, "us_per_product": round(dt * 1e6 / max(m, 1), 2)}
        print(json.dumps(rec), flush=True)
    ctx.close()


def bench_lekry(args):
    """EPIRK4s3 on 512^2 Allen-Cahn at 10x CFL, bound given: all stages by
    Leja (fused action kernels) against LeKry (Leja internal stages, the third
    stage by Krylov); one JSON line each (not the headline metric)."""
    import statistics

    import torch

    import paper_2211_08948_amd as lj
    from workloads import allen_cahn_noise
    prob = allen_cahn_noise(args.n, eps=1e-3, seed=2)
    ctx = lj.Context(0)
    J = lj.operator_from(prob, "cuda:0")
    h = CFL_MULT * prob.h_cfl
    lam = lj.lj_spectral_bound(ctx, J, 20)
    o = lj.lj_default_options(bound=lam)
    u_out = torch.empty_like(J.state)
    err = torch.empty_like(u_out)
    for scheme in ("EPIRK4S3", "EPIRK4S3_LEKRY", "EPIRK4S3A", "EPIRK4S3A_LEKRY"):
        fn = lambda: lj.lj_step(ctx, scheme, J, h, TOL, u_out, err, o)
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(args.steps // 5, 5)):
            t0 = time.perf_counter()
            rc, sts = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        dt = statistics.median(ts)
        rec = {"metric": "step time", "value": round(dt * 1e3, 4), "unit": "ms", "n_gpus": 1,
               "higher_is_better": False, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"allen-cahn {args.n}x{args.n} periodic, eps 1e-3, u0~U[-0.1,0.1] seed 2, "
                                      f"one {scheme} step at 10x CFL, bound given, tol 1e-10"},
               "calls": [{"m_star": s["m_star"][:3], "substeps": s["substeps"][:3], "products": s["iters_total"]}
                         for s in sts]}
        print(json.dumps(rec), flush=True)
    ctx.close()


def bench_ceiling(args):
    """The attainable HBM bandwidth of the device: copy, read-only, and the
    Newton step's 3-read 2-write pattern over 1 GiB vectors, at launch shapes
    from 256 to 16384 blocks of 256 or 1024 threads, 1, 2 or 4 accesses in
    flight per thread and vector, ordinary or non-temporal loads and stores;
    the best of each pattern is the practical ceiling to read the roofline
    fractions against (one JSON line, every shape listed in it)."""
    import paper_2211_08948_amd as lj
    shapes = []
    for nt in (False, True):
        for threads in (256, 1024):
            for blocks in (256, 1024, 4096, 16384):
                for unroll in (1, 2, 4):
                    bw = lj.lj_measure_bandwidth_shape(1 << 30, blocks, threads, unroll, nt)
                    shapes.append({"blocks": blocks, "threads": threads, "unroll": unroll, "nontemporal": nt,
                                   **{k: round(v, 1) for k, v in bw.items()}})
                    log(json.dumps(shapes[-1]))
    best = {k: max(shapes, key=lambda r: r[k]) for k in ("copy", "read", "newton_step")}
    rec = {"metric": "attainable HBM bandwidth", "value": best["newton_step"]["newton_step"], "unit": "GB/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "streaming FP64 kernels over 1 GiB vectors, best of 5 per shape; value: the "
                                  "Newton-step pattern (3 reads + 2 writes) at its best shape"},
           "copy_gbs": best["copy"]["copy"], "read_gbs": best["read"]["read"],
           "newton_step_gbs": best["newton_step"]["newton_step"], "peak_gbs": HBM_PEAK_GBS,
           "fractions_of_peak": {k: round(best[k][k] / HBM_PEAK_GBS, 4) for k in best},
           "best_shapes": {k: {q: best[k][q] for q in ("blocks", "threads", "unroll", "nontemporal")} for k in best},
           "shapes": shapes}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512, help="grid points per axis (default: the 512^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--sweep-n", type=int, default=0,
                    help="--form sweep: run only the Allen-Cahn phi_1 line at this grid size (for profiling)")
    ap.add_argument("--form", choices=["plain", "batch", "sweep", "stiffness", "adaptive", "user", "lekry", "ceiling"],
                    default="plain")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the multi-GPU path is not "
              "implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.form == "batch":
        bench_batch(args)
        return
    if args.form == "sweep":
        bench_sweep(args)
        return
    if args.form == "stiffness":
        bench_stiffness(args)
        return
    if args.form == "adaptive":
        bench_adaptive(args)
        return
    if args.form == "user":
        bench_user(args)
        return
    if args.form == "lekry":
        bench_lekry(args)
        return
    if args.form == "ceiling":
        bench_ceiling(args)
        return

    import torch

    import paper_2211_08948_amd as lj
    from workloads import allen_cahn_noise

    prob = allen_cahn_noise(args.n, eps=1e-3, seed=2)
    h = CFL_MULT * prob.h_cfl
    ctx = lj.Context(0)
    op = lj.operator_from(prob, "cuda:0")
    u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    err = torch.empty_like(u_out)
    f = torch.empty_like(u_out)
    lj.lj_rhs(ctx, op, op.state, f)
    v = (h * f).contiguous()
    w2 = torch.empty_like(u_out)
    opt = lj.lj_default_options()

    # the three calls of a step are issued back to back and synchronised once
    # (deferred synchronisation): phi_2 reads the EPIRK4s3 step's bound on the
    # device; a rejected expansion would be redone at the end of the block
    opt2 = lj.lj_default_options(bound_device=lj.lj_bound_device(ctx))

    def one_step():
        with lj.Deferred(ctx) as d:
            d.step("EXPRB2", op, h, TOL, u_out, None, opt)
            d.step("EPIRK4S3", op, h, TOL, u_out, err, opt)
            d.phi_action(op, v, w2, 2, h, TOL, opt2)
        if d.rc != lj.LJ_OK:
            raise SystemExit("bench step: an expansion did not converge")
        return d.results[0][1], d.results[1][1]

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    lj.lj_timing_read(ctx, reset=True)
    lj.lj_timing_enable(ctx, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s2, s4 = one_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lj.lj_timing_enable(ctx, False)
    tm = lj.lj_timing_read(ctx, reset=True)
    dt = t1 - t0
    value = ACTIONS_PER_STEP * args.steps / dt
    launches = max(tm["launches"], 1)
    avg_ms = tm["kernel_ms"] / launches
    bytes_per_launch = algorithmic_bytes(tm) / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    log(f"step {dt / args.steps * 1e3:.3f} ms; action kernel: {tm['launches'] / args.steps:.1f} launches/step "
        f"({tm['tiled_launches']} of {tm['launches']} tiled), {avg_ms * 1e3:.1f} us avg, "
        f"{tm['iterations'] / launches:.1f} Newton + {tm['power_point_iters'] / launches / max(prob.n, 1):.1f} "
        f"power products per launch, {avg_ms * 1e3 * launches / max(tm['iterations'] + tm['power_point_iters'] / prob.n, 1):.2f} "
        f"us per product")
    log(f"m* EXPRB2 {s2[0]['m_star'][0]}, EPIRK4s3 vertical {s4[0]['m_star'][:3]}, phi_3 {s4[1]['m_star'][0]}, "
        f"phi_4 {s4[2]['m_star'][0]}")
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "phi-actions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"allen-cahn {args.n}x{args.n} periodic, eps 1e-3, u0~U[-0.1,0.1] seed 2, "
                               f"h={CFL_MULT:g}x CFL, tol 1e-10: EXPRB2 + EPIRK4s3 steps + phi_2 action",
                   "grid": [args.n, args.n], "actions_per_step": ACTIONS_PER_STEP},
        "roofline": {"bound": "latency", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "dram_gbs": round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                     "kernel": "lj_action (power iteration + divided differences + Newton recurrence)",
                     "avg_launch_us": round(avg_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": round(bytes_per_launch),
                     "note": "achieved = algorithmic bytes (24 + 16 K B per point and Newton step, 24 B per "
                             "power product) / kernel time against the HBM peak; the 512^2 working set stays "
                             "in registers, LDS and the caches, so the DRAM traffic the counters see (traffic, "
                             "dram_gbs) is far lower: the kernel is bound by the latency of its grid barriers "
                             "and per-step workgroup synchronisation, not by HBM"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, h)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
