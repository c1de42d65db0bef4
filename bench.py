#!/usr/bin/env python3
"""Benchmark of the batched Henry solve on one MI355X.

A step is one full pass of the hot path over one batch: random fields, the whole
implicit-Euler time horizon (Newton, multigrid-preconditioned BiCGStab, coarse
banded LU), mass balance and QoI, then the MLMC estimator over the batch.
Default workload: MLMC level 3 (256x128 cells, 384 steps, 512 samples, seed 1), FP64.
The metric is sample-timesteps/s = samples * time steps / wall time.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c1|c4|c5|qmc] [--model kl|paper]
  The default run (c2) adds an "extra" object with the rest of the metric: level 3 and level 4
  with the FP32 multigrid, and the MLMC hierarchy's wall time to RMSE (FP64 and FP32 multigrid).
  c4: MLMC wall time to RMSE for levels 0..4 in one ragged call; c5: discrete adjoint
  --model paper: the paper's own stochastic model (section 4; T = 6016 s) on the c1-c3 grids
  qmc: that model over 600 Halton points (section 5) at --level (default 3)
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from henry_inputs import WORKLOADS, draw_theta, level_grid  # noqa: E402

# HBM peak and the algorithmic bytes per unit of each kernel class (FP64 / FP32 multigrid)
from paper_2403_17018_amd.metrics import (BYTES_PER_UNIT as BYTES, HBM_PEAK_GBS, VC_BYTES_PER_UNIT,  # noqa: E402
                                          MetricsLog, batch_record)

METRICS = None   # MetricsLog of --metrics: one JSON line per measured batch
KERNEL_NAME = dict(gs="k_gs_colour", spmv="k_spmv_dot", assemble="k_assemble", restrict="k_residual_restrict",
                   prolong="k_gs_colour (fused prolongation)")


def host_cores():
    """Host threads the CPU baseline uses: the CPUs this process may run on, at most 16 (the
    host CPU share of one GPU on the benchmark machines), and what os.cpu_count() reports."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return min(16, avail), os.cpu_count() or 1


# oracle states stored along the level-3 horizon (tests/golden/make_golden.py span): the CPU
# baseline times short windows started from them so that every part of the horizon counts
WINDOW_SAMPLES = (68, 511)
WINDOW_STEPS = 4


def cpu_baseline(level, seed, nsamples_avail, steps_total, model="kl"):
    """The oracle (SuperLU Newton, one sample per process) on the host cores.

    Level 3 with the KL model: windows of WINDOW_STEPS steps started from the oracle's own
    states after steps 1, 96, 192 and 288 of two stored samples, plus the first step from the
    initial state; each window stands for the quarter of the horizon it starts, so a sample's
    full-horizon time is t_first + sum_q t_q / WINDOW_STEPS * (steps of quarter q).  The jobs
    are repeated cyclically over all `procs` processes so every core is loaded while they are
    timed.  Other workloads: level <= 1 runs the full horizon for `procs` samples; otherwise the
    first steps only (labelled as understating the rate)."""
    procs, ncpu = host_cores()
    nx, ny, _ = level_grid(level)
    gold = [os.path.join(ROOT, "tests", "golden", f"oracle_c2_s{s}.npz") for s in WINDOW_SAMPLES]
    windows = level == 3 and model == "kl" and seed == 1 and all(os.path.exists(f) for f in gold)
    code = f"""
import sys, time, json, numpy as np
sys.path.insert(0, {ROOT!r})
from henry_inputs import draw_theta
from oracle import henry as H
import multiprocessing as mp
pr = {"H.paper_problem()" if model == "paper" else "H.Problem()"}; g = H.Grid({nx}, {ny}, {steps_total})
mode = {"'windows'" if windows else ("'full'" if level <= 1 else "'first'")}
jobs = []
if mode == 'windows':
    for f in {gold!r}:
        z = np.load(f)
        jobs.append((z['theta'], None, 1))
        for k, n0 in enumerate(z['state_steps']):
            jobs.append((z['theta'], (int(n0), z['state_p'][k], z['state_c'][k]), {WINDOW_STEPS}))
else:
    th = draw_theta({seed}, {min(procs, nsamples_avail)}, level={level})
    n = {steps_total} if mode == 'full' else 10
    jobs = [(t, None, n) for t in th]
def one(j):
    th, start, n = j
    t0 = time.perf_counter()
    r = H.solve_sample(pr, g, th, nsteps=n, start=start)
    return time.perf_counter() - t0, r.newton_its
work = [jobs[i % len(jobs)] for i in range(max({procs}, len(jobs)))]
t0 = time.perf_counter()
with mp.get_context('fork').Pool({procs}) as p:
    out = p.map(one, work)
print(json.dumps(dict(mode=mode, njobs=len(jobs), wall=time.perf_counter() - t0, out=out)))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = json.loads(subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                                  check=True).stdout)
    out = r["out"]
    if r["mode"] == "windows":
        nj = r["njobs"]
        t = [sum(o[0] for o in out[i::nj]) / len(out[i::nj]) for i in range(nj)]   # mean over repeats
        per_sample = []
        starts = [1, 96, 192, 288, steps_total]
        for k in range(len(WINDOW_SAMPLES)):
            tk = t[5 * k:5 * k + 5]
            per_sample.append(tk[0] + sum(tk[1 + q] / WINDOW_STEPS * (starts[q + 1] - starts[q]) for q in range(4)))
        secs = sum(per_sample) / len(per_sample)
        value = procs * steps_total / secs
        sample = (f"{len(WINDOW_SAMPLES)} samples of the same workload on {nx}x{ny} cells: the first step and "
                  f"{WINDOW_STEPS}-step windows from the oracle's states after steps 1, 96, 192 and 288, each window "
                  f"standing for its quarter of the {steps_total}-step horizon ({len(out)} timed jobs, "
                  f"{r['wall']:.1f} s wall); full-horizon estimate {secs:.0f} s per sample per process, "
                  f"{procs} processes at once (os.cpu_count() = {ncpu})")
    elif r["mode"] == "full":
        ns = len(out)
        value = ns * steps_total / r["wall"]
        sample = f"{ns} samples x all {steps_total} steps on {nx}x{ny} cells, one sample per process"
    else:
        ns = len(out)
        value = ns * 10 / r["wall"]
        sample = (f"{ns} samples x first 10 of {steps_total} steps on {nx}x{ny} cells, one sample per process; the "
                  f"first steps are the costliest, so this understates the full-horizon rate")
    return {"value": value, "unit": "sample-timesteps/s", "cores": procs, "kind": "oracle", "sample": sample}


def solver_config(o):
    """The solver settings that ran, for the config label."""
    return {"coarse_grid": f"{o.coarse_nx}x{o.coarse_ny}",
            "coarse_solver": {1: "dense LU with partial pivoting",
                              2: "LU with partial pivoting in band storage (the dense elimination's pivots)"}.get(
                getattr(o, "coarse_solver", 0), "block-banded LU without pivoting"),
            "smoother": f"red-black 2x2-block Gauss-Seidel, {o.nu_pre} pre + {o.nu_post} post sweeps",
            "cycle": "V" if o.mg_cycle == 1 else "W",
            "krylov": f"right-preconditioned BiCGStab, forcing term {o.krylov_rtol:g}",
            "newton": f"tolerance {o.newton_tol:g}, first guess: extrapolation order {o.newton_extrapolate}, "
                      f"predictive stop {'on' if o.newton_predict > 0 else 'off'}, chord steps below "
                      f"{o.newton_jac_reuse:g}"}


def pmc_traffic(kernel, prec, workload, model, source="henry_kernels.hpp"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    this workload and model and the kernel source is unchanged."""
    f = os.path.join(ROOT, "profiles", f"pmc_{kernel}_fp{prec}.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("workload") != workload or d.get("model") != model:
        return None
    src = open(os.path.join(ROOT, "paper_2403_17018_amd", "csrc", source), "rb").read()
    if d.get("kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return d.get("hbm_bytes_per_launch")


def bench_mlmc(args):
    """Full MLMC hierarchy (levels 0..4, 4096/1024/256/64/16 samples, coupled fine/coarse
    pairs) in one ragged call, then the estimator: wall time to the reported RMSE."""
    import torch
    import paper_2403_17018_amd as P
    w = WORKLOADS["c4_mlmc_levels0to4"]
    prec = args.precision or 64
    graphs = 1 if args.graphs is None else args.graphs
    levels, m, seed = w["levels"], w["nsamples"], w["seed"]
    thetas = [torch.from_numpy(draw_theta(seed, k, level=l)).cuda() for l, k in zip(levels, m)]
    hx = P.Henry(0)
    opts = P.solver_opts(mg_precision=prec, use_graphs=graphs, step_graphs=args.step_graphs,
                         ragged_threads=args.ragged_threads)
    for _ in range(args.warmup):
        P.mlmc_run(hx, thetas, levels, opts=opts)
    torch.cuda.synchronize()
    n0 = hx.profile_read()["host_sync"]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        est = P.mlmc_run(hx, thetas, levels, opts=opts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    n1 = hx.profile_read()["host_sync"]
    if METRICS is not None:
        k = 0
        for l, lev in enumerate(levels):
            g = P.level_grid(lev)
            METRICS.write(batch_record(f"c4 level {lev}", g, est["results"][k], mg_precision=prec, call_seconds=dt))
            k += 1
            if l > 0:
                METRICS.write(batch_record(f"c4 level {lev} coarse partner", P.level_grid(levels[l - 1]),
                                           est["results"][k], mg_precision=prec, call_seconds=dt))
                k += 1
    # every batch's implicit-Euler steps: each level and each coarse partner
    nsteps_all = sum((48 << l) + ((48 << (l - 1)) if l > 0 else 0) for l in levels)
    work = sum(k * (48 << l) + (k * (48 << (l - 1)) if l > 0 else 0) for l, k in zip(levels, m))
    out = {
        "metric": "MLMC wall time to RMSE",
        "value": dt,
        "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 64 else "f64+f32mg", "data": "synthetic",
        "config": {"workload": "c4_mlmc_levels0to4: levels 0..4 (32x16..512x256 cells, 48..768 steps), "
                               "4096/1024/256/64/16 samples with coupled coarse partners (seed 3), one ragged call",
                   "mg_precision": prec, "hip_graphs": graphs, "step_graphs": args.step_graphs,
                   "parallelism": "one stream per grid on one GPU" if not args.ragged_threads
                   else "grids one after another from one host thread"},
        "host_syncs_per_batch_step": (n1[0] - n0[0]) / args.steps / nsteps_all,
        "host_sync_wait_ms": (n1[2] - n0[2]) / args.steps,
        "rmse": est["rmse"], "mlmc_mean_qoi": est["mean"], "var_of_estimator": est["var_of_estimator"],
        "V_l": est["V"], "sample_timesteps_per_s": work / dt, "failed_samples": est["nfailed"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_adjoint(args):
    """Discrete adjoint of the level-3 batch (256 samples, 384 steps, checkpoints every 32):
    forward with checkpoints, reverse sweep with segment recomputation and transposed solves."""
    import torch
    import paper_2403_17018_amd as P
    w = WORKLOADS["c5_adjoint_level3"]
    prec = args.precision or 64
    level, S, seed = w["level"], w["nsamples"], w["seed"]
    nx, ny, nsteps = level_grid(level)
    theta = torch.from_numpy(draw_theta(seed, S, level=level)).cuda()
    hx = P.Henry(0)
    g = P.grid(nx, ny, nsteps)
    opts = P.solver_opts(mg_precision=prec)
    for _ in range(args.warmup):
        hx.adjoint(theta, g, opts=opts, checkpoint_every=w["checkpoint_every"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, grad, st, nf = hx.adjoint(theta, g, opts=opts, checkpoint_every=w["checkpoint_every"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = {
        "metric": "adjoint sample-timesteps/s", "value": S * nsteps / dt, "unit": "sample-timesteps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 64 else "f64+f32mg", "data": "synthetic",
        "config": {"workload": f"c5_adjoint_level3: {nx}x{ny} cells, {nsteps} steps, {S} samples (seed {seed}), "
                               f"checkpoints every {w['checkpoint_every']} steps, gradient w.r.t. 13 parameters",
                   "mg_precision": prec, "parallelism": "samples batched on one GPU"},
        "failed_samples": nf, "mean_abs_grad": float(grad.abs().mean()), "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_qmc(args):
    """Quasi-Monte Carlo of the paper's own model (section 5: 600 Halton points): one batch
    at one level, then the single-level estimator (mean and variance of Q and of c at T)."""
    import torch
    import paper_2403_17018_amd as P
    from henry_inputs import qmc_theta
    level = 3 if args.level is None else args.level
    prec = args.precision or 64
    S = 600
    nx, ny, nsteps = level_grid(level)
    theta = torch.from_numpy(qmc_theta(S)).cuda()
    hx = P.Henry(0)
    opts = P.solver_opts(mg_precision=prec)
    prob = P.paper_problem()
    for _ in range(args.warmup):
        P.mlmc_run(hx, [theta], [level], prob=prob, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        est = P.mlmc_run(hx, [theta], [level], prob=prob, opts=opts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = {
        "metric": "sample-timesteps/s", "value": S * nsteps / dt, "unit": "sample-timesteps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 64 else "f64+f32mg", "data": "synthetic",
        "config": {"workload": f"qmc600: the paper's section-4 model, 600 Halton points (bases 2, 3, 5), level {level} "
                               f"({nx}x{ny} cells, {nsteps} steps, T = 6016 s), single-level estimator",
                   "mg_precision": prec, "parallelism": "samples batched on one GPU"},
        "qoi_mean": est["mean"], "qoi_var": est["V"][0],
        "c_mean_range": [float(est["mean_field"].min()), float(est["mean_field"].max())],
        "c_var_max": float(est["var_field"].max()), "failed_samples": est["nfailed"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_adaptive(args):
    """Adaptive MLMC (sections 3 and 5): pilot solves on levels 0..2 (32 samples each, with
    coarse partners), fitted rates, the level count and sample sizes for relative accuracy
    eps, then the production run in one ragged call.  Wall time of the whole driver to its
    RMSE, with the planned MLMC cost next to plain Monte Carlo's at the same level (Test B4).
    The paper's model (--model paper) has no decaying level differences on levels 1..3 (its
    80 s recharge period is aliased by the coarse steps), so its plan is refused there."""
    import torch
    import paper_2403_17018_amd as P
    prec = args.precision or 64
    eps = args.eps
    opts = P.solver_opts(mg_precision=prec)
    prob = P.paper_problem() if args.model == "paper" else P.problem()
    model = "the paper's section-4 model" if args.model == "paper" else "the KL model (T = 36000 s)"
    hx = P.Henry(0)

    def sampler(level, n, first):
        return torch.from_numpy(draw_theta(7, n, level=level, first_sample=first)).cuda()

    def run():
        return P.mlmc_adaptive(hx, sampler, eps=eps, prob=prob, opts=opts, pilot_levels=2, pilot_samples=32,
                               max_level=4)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        est = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    pl = est["plan"]
    out = {
        "metric": "MLMC wall time to RMSE (adaptive)", "value": dt, "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 64 else "f64+f32mg", "data": "synthetic",
        "config": {"workload": f"adaptive MLMC of {model}, relative accuracy {eps}, pilot levels "
                               f"0..2 x 32 samples (seed 7), at most level 4, production in one ragged call",
                   "mg_precision": prec, "parallelism": "samples batched on one GPU"},
        "levels": pl["L"], "m": pl["m"], "rmse": est["rmse"], "mlmc_mean_qoi": est["mean"],
        "rates": {k: pl[k] for k in ("alpha", "beta", "gamma")},
        "model_cost_s": pl["cost"], "plain_mc_cost_s": pl["mc_cost"], "production_wall_s": est["wall_s"],
        "failed_samples": est["nfailed"], "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def measure_batch(hx, theta, g, prob, opts, warmup, steps, workload, model):
    """Time `steps` whole-batch solves (plus the estimator over the batch) after `warmup`
    untimed ones; the dominant kernel class and its roofline from HIP events on the library's
    stream during the timed region."""
    import torch
    prec = opts.mg_precision
    S = theta.shape[0]

    def step():
        r = hx.solve(theta, g, prob, opts=opts, want_c=True)
        est = hx.mlmc_estimate([g], [r.qoi], [None], [r.c_T], [None])
        return r, est

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    hx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        r, est = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = hx.profile_read()
    hx.profile(False)
    dt = (t1 - t0) / steps
    if METRICS is not None:
        METRICS.write(batch_record(workload, g, r, seconds=dt, prof=prof, mg_precision=prec, timed_runs=steps,
                                   coarse=f"{opts.coarse_nx}x{opts.coarse_ny}", coarse_solver=opts.coarse_solver))
    st = r.stats.cpu()
    cls = max(BYTES[prec], key=lambda k: prof[k][2])      # dominant kernel class by summed time
    n, units, ms = prof[cls]
    per_launch_bytes = units / n * BYTES[prec][cls]
    achieved = per_launch_bytes / (ms / n * 1e-3) / 1e9
    return dict(value=S * g.nsteps / dt, ms_per_step=dt * 1e3,
                roofline={"bound": "hbm", "kernel": KERNEL_NAME[cls], "achieved": achieved, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                          "traffic": pmc_traffic(KERNEL_NAME[cls], prec, workload, model),
                          "avg_launch_us": ms / n * 1e3, "launches": n,
                          "algorithmic_bytes_per_launch": per_launch_bytes},
                kernel_classes_ms={k: round(v[2], 3) for k, v in prof.items()},
                newton_its_per_step=float(st[:, 0].mean()) / g.nsteps,
                krylov_its_per_newton=float(st[:, 1].sum() / st[:, 0].sum()),
                max_salt_defect=float(st[:, 3].max()), failed_samples=r.nfailed, mlmc_mean_qoi=est["mean"],
                _prof=prof)


VC_KERNEL_NAME = dict(gs="k_vc_gs", spmv="k_vc_spmv", assemble="k_vc_assemble")
VC_SAMPLES = 512
# one pre- and one post-smoothing sweep: the fastest of 1+1, 1+2, 2+1, 2+2 and 1+3 on this
# workload (the iteration counts barely change)
VC_OPTS = dict(krylov_maxit=1000, nu_pre=1, nu_post=1)


def bench_vc(hx, P, S=VC_SAMPLES, graphs=1, prec=64):
    """The paper's own discretisation (vertex-centred finite volumes, section 2.3) on level 1
    of its Table 2 (64 x 32 elements, 2145 vertices, 376 steps of 16 s) with its own model:
    one untimed short run, then the timed run (BiCGStab iterations replayed from a hipGraph
    when graphs = 1), then, since the library's HIP-event profiler times launches outside
    graphs only, a stream-launched repeat with the profiler on for the dominant kernel class
    and its roofline."""
    import torch
    g = P.vc_level_grid(1)
    th = torch.from_numpy(draw_theta(5, S)).cuda()
    o = P.solver_opts(use_graphs=graphs, mg_precision=prec, **VC_OPTS)
    hx.vc_solve(th, P.grid(g.nx, g.ny, 4), P.paper_problem(T=6016.0 * 4 / g.nsteps), o, want_c=False)
    torch.cuda.synchronize()
    hx.profile(True)      # resets the counters; event timing stays on only without graphs
    if graphs:
        hx.profile(False)
    t0 = time.perf_counter()
    r = hx.vc_solve(th, g, P.paper_problem(), o, want_c=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = hx.profile_read()
    if graphs:   # the graph replays were not timed: repeat stream-launched for the kernel timings
        torch.cuda.synchronize()
        hx.profile(True)
        t1 = time.perf_counter()
        hx.vc_solve(th, g, P.paper_problem(), P.solver_opts(use_graphs=0, mg_precision=prec, **VC_OPTS), want_c=False)
        torch.cuda.synchronize()
        dt_prof = time.perf_counter() - t1
        prof_k = hx.profile_read()
    else:
        dt_prof, prof_k = dt, prof
    hx.profile(False)
    st = r.stats.cpu()
    if METRICS is not None:
        METRICS.write(batch_record("f3_vc_level1_paper", g, r, seconds=dt))
    table = VC_BYTES_PER_UNIT[prec]
    cls = max(table, key=lambda k: prof_k[k][2])
    n, units, ms = prof_k[cls]
    per_launch = units / n * table[cls]
    achieved = per_launch / (ms / n * 1e-3) / 1e9
    return {
        "workload": "the paper's vertex-centred discretisation, level 1 of Table 2: 64x32 elements (2145 vertices), "
                    f"376 steps of 16 s, {S} samples (seed 5) of the section-4 model; BiCGStab preconditioned by a "
                    "vertex-grid multigrid V-cycle (1+1 four-colour Gauss-Seidel sweeps) with a pivoted LU on the "
                    "coarsest grid"
                    + ("; FP32 multigrid and Jacobian" if prec == 32 else "")
                    + ("; BiCGStab iterations replayed from a hipGraph" if graphs else ""),
        "unit": "sample-timesteps/s", "value": S * g.nsteps / dt, "ms_per_step": dt * 1e3,
        "roofline": {"bound": "hbm", "kernel": VC_KERNEL_NAME[cls], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": pmc_traffic(VC_KERNEL_NAME[cls], prec, "f3_vc_level1_paper", "paper", "henry_vc.hpp"),
                     "avg_launch_us": ms / n * 1e3, "launches": n, "algorithmic_bytes_per_launch": per_launch,
                     "timed_in": "a stream-launched repeat of the run" if graphs else "the timed run"},
        "kernel_classes_ms": {k: round(prof_k[k][2], 3) for k in table},
        "profiled_repeat_ms": dt_prof * 1e3 if graphs else None,
        "host_syncs": prof["host_sync"][0], "host_sync_ms": round(prof["host_sync"][2], 3),
        "newton_its_per_step": float(st[:, 0].mean()) / g.nsteps,
        "krylov_its_per_newton": float(st[:, 1].sum() / st[:, 0].sum()), "failed_samples": r.nfailed,
        "mean_qoi": float(r.qoi.mean())}


# Table 3 of the paper, eps = 0.05: L = 3 levels with m = 404, 49, 3 samples on levels 0, 1, 2
VC_MLMC_M = (404, 49, 3)


def bench_vc_mlmc(hx, P):
    """MLMC over the paper's own hierarchy (Table 2 levels 0..2, vertex-centred, the section-4
    model) with Table 3's sample allocation for relative accuracy 0.05: wall time of the whole
    estimate (each level and its coupled coarse partner, one after another, then the estimator),
    after a short untimed run on each grid."""
    import torch
    o = P.solver_opts(use_graphs=1, **VC_OPTS)
    ths = [torch.from_numpy(draw_theta(12 + l, m)).cuda() for l, m in enumerate(VC_MLMC_M)]
    for lev in range(len(VC_MLMC_M)):
        g = P.vc_level_grid(lev)
        hx.vc_solve(ths[lev], P.grid(g.nx, g.ny, 2), P.paper_problem(T=6016.0 * 2 / g.nsteps), o, want_c=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est = P.mlmc_run_vc(hx, ths, list(range(len(VC_MLMC_M))), P.paper_problem(), o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": "MLMC over Table 2's levels 0..2 of the paper's vertex-centred discretisation (16x8, 64x32 and "
                        "256x128 elements; 94, 376 and 1504 steps) with Table 3's allocation for eps = 0.05: "
                        f"{'/'.join(map(str, VC_MLMC_M))} samples (seeds 12..14) and coupled coarse partners, the "
                        "section-4 model, salt mass in x > 1 at T = 6016 s",
            "metric": "MLMC wall time", "unit": "s", "value": dt, "mlmc_mean_qoi": est["mean"], "rmse": est["rmse"],
            "V": est["V"], "failed_samples": est["nfailed"]}


def extra_lines(hx, P, args):
    """The rest of the metric at fixed small repeat counts (1 untimed + 1 timed run each, so the
    default run stays within minutes): level 3 with the FP32 multigrid, level 4 with the FP32
    multigrid (its workload), and the full MLMC hierarchy's wall time to RMSE with FP64 and
    FP32 multigrid."""
    import torch
    out = {}
    for key, name, prec in (("c2_fp32mg", "c2_fp64_level3", 32), ("c3_fp32mg_level4", "c3_mixed_level4", 32)):
        w = WORKLOADS[name]
        g = P.grid(*level_grid(w["level"]))
        th = torch.from_numpy(draw_theta(w["seed"], w["nsamples"], level=w["level"])).cuda()
        o = P.solver_opts(mg_precision=prec)
        m = measure_batch(hx, th, g, P.problem(), o, 1, 1, name, "kl")
        m.pop("_prof")
        out[key] = {"workload": f"{name}: {g.nx}x{g.ny} cells, {g.nsteps} steps, {w['nsamples']} samples "
                                f"(seed {w['seed']}), FP32 multigrid in FP64 BiCGStab/Newton",
                    "unit": "sample-timesteps/s", **m}
        del th
    # the workload as named: multigrid to a 32x16 coarse grid solved by the batched dense LU with
    # partial pivoting (four grids from 256x128); the factorisation's matrix-core roofline
    w = WORKLOADS["c2_fp64_level3"]
    g = P.grid(*level_grid(w["level"]))
    th = torch.from_numpy(draw_theta(w["seed"], w["nsamples"], level=w["level"])).cuda()
    o = P.solver_opts(coarse_nx=32, coarse_ny=16, coarse_solver=1)
    m = measure_batch(hx, th, g, P.problem(), o, 1, 1, "c2_fp64_level3", "kl")
    prof = m.pop("_prof")
    nf, uf, msf = prof["dense_factor"]
    n = 2 * 32 * 16
    flops = uf / nf * 2.0 * n ** 3 / 3.0                  # per launch: samples x 2n^3/3
    achieved = flops / (msf / nf * 1e-3) / 1e12
    out["c2_named_32x16_dense_lu"] = {
        "workload": f"c2_fp64_level3 with the 32x16 coarsest grid and the batched dense LU with partial pivoting "
                    f"(n = {n} unknowns per sample), FP64", "unit": "sample-timesteps/s", **m,
        "solver": solver_config(o),
        "dense_factor_roofline": {"bound": "mfma", "kernel": "k_dense_factor", "achieved": achieved,
                                  "peak": 78.6, "unit": "TFLOP/s", "frac": achieved / 78.6,
                                  "avg_launch_us": msf / nf * 1e3, "launches": nf,
                                  "flops_per_launch": flops}}
    # the same named configuration with the elimination in band storage: the dense LU's pivots
    # and factors, without its work on the zeros outside the band
    o = P.solver_opts(coarse_nx=32, coarse_ny=16, coarse_solver=2)
    m = measure_batch(hx, th, g, P.problem(), o, 1, 1, "c2_fp64_level3", "kl")
    prof = m.pop("_prof")
    out["c2_named_32x16_pivoted_band_lu"] = {
        "workload": f"c2_fp64_level3 with the 32x16 coarsest grid and Gaussian elimination with partial pivoting "
                    f"in band storage (n = {n}, 2 x 33 diagonals, pivots as the dense LU's), FP64",
        "unit": "sample-timesteps/s", **m, "solver": solver_config(o),
        "coarse_ms": {"factor": prof["band_factor"][2], "factor_launches": prof["band_factor"][0],
                      "solve": prof["band_solve"][2], "solve_launches": prof["band_solve"][0]}}
    del th
    w = WORKLOADS["c4_mlmc_levels0to4"]
    thetas = [torch.from_numpy(draw_theta(w["seed"], k, level=l)).cuda() for l, k in zip(w["levels"], w["nsamples"])]
    for prec in (64, 32):
        o = P.solver_opts(mg_precision=prec, use_graphs=1)
        P.mlmc_run(hx, thetas, w["levels"], opts=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est = P.mlmc_run(hx, thetas, w["levels"], opts=o)
        torch.cuda.synchronize()
        out[f"c4_mlmc_fp{prec}" if prec == 64 else "c4_mlmc_fp32mg"] = {
            "workload": "c4_mlmc_levels0to4: levels 0..4 (32x16..512x256 cells, 48..768 steps), "
                        "4096/1024/256/64/16 samples with coupled coarse partners (seed 3), one ragged call",
            "metric": "MLMC wall time to RMSE", "unit": "s", "value": time.perf_counter() - t0,
            "rmse": est["rmse"], "mlmc_mean_qoi": est["mean"], "failed_samples": est["nfailed"]}
    out["f3_vc_level1_paper"] = bench_vc(hx, P)
    out["f3_vc_level1_paper_fp32mg"] = bench_vc(hx, P, prec=32)
    out["f3_mlmc_table3_eps0.05"] = bench_vc_mlmc(hx, P)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "qmc", "adaptive", "f3"])
    ap.add_argument("--samples", type=int, default=None, help="f3: batch size (default 512)")
    ap.add_argument("--eps", type=float, default=0.002, help="relative accuracy of the adaptive workload")
    ap.add_argument("--level", type=int, default=None, help="level of the qmc workload (default 3)")
    ap.add_argument("--graphs", type=int, default=None, help="capture BiCGStab iterations in hipGraphs (c4 default 1)")
    ap.add_argument("--step-graphs", type=int, default=1,
                    help="c4: replay each settled step's first Newton iteration from a graph (the library default)")
    ap.add_argument("--ragged-threads", type=int, default=0, help="c4: 1 runs the grids one after another on one thread")
    ap.add_argument("--precision", type=int, default=None, help="multigrid precision (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra metric lines of the default run")
    ap.add_argument("--model", default="kl", choices=["kl", "paper"],
                    help="input model: KL fields (the workloads) or the paper's section-4 model")
    ap.add_argument("--metrics", default=None, metavar="FILE",
                    help="append one JSON line per measured batch (iteration histograms, kernel classes, "
                         "throughput, mass balance) to FILE")
    args = ap.parse_args()
    global METRICS
    if args.metrics:
        METRICS = MetricsLog(args.metrics)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(samples would shard across GPUs with one all-reduce of the MLMC sums)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        return bench_mlmc(args)
    if args.workload == "c5":
        return bench_adjoint(args)
    if args.workload == "qmc":
        return bench_qmc(args)
    if args.workload == "adaptive":
        return bench_adaptive(args)
    if args.workload == "f3":
        import paper_2403_17018_amd as P
        hx = P.Henry(0)
        m = bench_vc(hx, P, args.samples or VC_SAMPLES, 1 if args.graphs is None else args.graphs,
                     args.precision or 64)
        print(json.dumps({"metric": "sample-timesteps/s", "n_gpus": 1, "steps": 1, "warmup": 1,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f64+f32mg" if args.precision == 32 else "f64",
                          "data": "synthetic", "config": {"workload": m.pop("workload")}, **m}))
        return
    name = {"c1": "c1_fp64_level0", "c2": "c2_fp64_level3", "c3": "c3_mixed_level4"}[args.workload]
    w = WORKLOADS[name]
    prec = args.precision or w["mg_precision"]
    level, S, seed = w["level"], w["nsamples"], w["seed"]
    nx, ny, nsteps = level_grid(level)

    cpu = None if args.no_cpu_baseline else cpu_baseline(level, seed, S, nsteps, args.model)

    import torch
    import paper_2403_17018_amd as P

    theta = torch.from_numpy(draw_theta(seed, S, level=level)).cuda()
    hx = P.Henry(0)
    g = P.grid(nx, ny, nsteps)
    opts = P.solver_opts(mg_precision=prec)
    prob = P.paper_problem() if args.model == "paper" else P.problem()
    m = measure_batch(hx, theta, g, prob, opts, args.warmup, args.steps, name, args.model)
    m.pop("_prof")
    del theta
    out = {
        "metric": "sample-timesteps/s",
        "value": m["value"],
        "unit": "sample-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 64 else "f64+f32mg",
        "data": "synthetic",
        "config": {"workload": f"{name}: MLMC level {level}, {nx}x{ny} cells, {nsteps} implicit-Euler steps, "
                               f"{S} samples (seed {seed}), {'FP64' if prec == 64 else 'FP32'} multigrid"
                               + (", the paper's section-4 porosity/Kozeny-Carman/recharge model, T = 6016 s"
                                  if args.model == "paper" else ""),
                   "samples": S, "cells": nx * ny, "time_steps": nsteps, "mg_precision": prec,
                   "solver": solver_config(opts), "parallelism": "samples batched on one GPU"},
        "roofline": m["roofline"],
        **{k: m[k] for k in ("kernel_classes_ms", "newton_its_per_step", "krylov_its_per_newton", "max_salt_defect",
                             "failed_samples", "mlmc_mean_qoi")},
        "cpu_baseline": cpu,
    }
    if args.workload == "c2" and args.model == "kl" and args.precision is None and not args.no_extra:
        out["extra"] = extra_lines(hx, P, args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
