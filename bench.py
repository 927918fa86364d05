"""Benchmark of the LMM PF-SMC sampler's hot path on one MI355X.

A step is one observation step of Algorithm 1 (steps 2-6) for every particle
of the filter: shrink + predictor integration, first-stage weights, integer
systematic resampling, gather + proliferation + repropagation with the
local-error innovation, second-stage weights, weighted mean / covariance /
Cholesky.  The workload is the large Robertson configuration: N = 2^17
particles, 200 observation times log-spaced in [1e-3, 1e3], BDF2 with 20 fixed
steps per interval, served form = FP32 propagation with FP64 weights and
moments; the plain FP64 path is timed in the same run for comparison.

Prints one JSON line.  Inputs are synthetic (seeded), resident in HBM before
the timed region starts.  The timed region: a fresh filter, W untimed warm-up
steps on it, then K timed observation steps (the next ones of the schedule,
or the first K on a filter of their own when W + K exceed the schedule),
bracketed by device synchronisations; three untimed passes of the same form
come first, and four more follow for the spread.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1411_1702_amd import inputs  # noqa: E402

METRIC = "particle-steps/sec FP32 vs FP64 at stated error; p50/p99 assimilate latency"

# Algorithmic floating-point work of the integrator (Algorithm 1 steps 2 and
# 4), counted by the rule fma = 2, add/sub/mul = 1, reciprocals apart (they
# issue at quarter rate): per Newton iteration (f, J, the Newton matrix, the
# residual, its elimination and solve, the update and the test) and per
# integration step outside Newton (history, predictor, local-error term).
#   Robertson: 58 per iteration (+3 reciprocals), 33 per step;
#   chain:     304 per iteration with the bidiagonal solve (+32 reciprocals),
#              256 per step.
# Both passes are priced the same, so one particle-step costs
# 2 M (58 K + 33) (Robertson) with K the Newton iterations per step that the
# kernels count.  RNG, likelihood and moment arithmetic are not counted.
# Adams-Moulton steps add the derivative at the accepted value (Robertson 8,
# chain 64).  The filtered local-error estimate (one more solve with the
# Newton matrix per step, two at the first step of the interval; Robertson
# 13, chain 48 flop per solve) is the library's own reading and is reported
# as its own term, outside the count.
FLOPS = {
    # iter_exec: what the kernels execute per iteration (Robertson's solve
    # through the column sums of J: 45 FLOP and one reciprocal, where the
    # count of an iteration with the 3x3 LU is 58 and three)
    inputs.MODEL_ROBERTSON: {"iter": 58, "iter_exec": 45, "rcp_iter": 3, "sub": 33, "sub_am": 8, "solve": 13},
    inputs.MODEL_CHAIN: {"iter": 304, "iter_exec": 304, "rcp_iter": 32, "sub": 256, "sub_am": 64, "solve": 48},
}


def advdiff_flops(prob, update):
    """Algorithmic flops of one particle's pass on the advection-diffusion
    model: the 2D transforms (each 12 nt^2 (nt/2 + 1): a real-to-half-spectrum
    row pass of 4 flop per term and a complex column pass of 8, and the same
    back) -- one forward and one inverse per pass, plus one inverse per step
    for the local-error estimate in the repropagation -- and the per-mode
    recurrence (about 25 flop per mode and step in the predictor, 45 with the
    estimate).  RNG, likelihood and moments are not counted."""
    nt = int(prob.model_consts[0])
    modes = nt * (nt // 2 + 1)
    M = prob.substeps
    transforms = (2 + M) if update else 2
    return transforms * 12 * nt * nt * (nt // 2 + 1) + M * modes * (45 if update else 25)


def algorithmic_bytes(prob):
    """HBM bytes one FP32 update launch must move: kinetic models per
    particle the ancestor's state, parameters and predictor likelihood
    (4 d + 8 p + 8), the new state, parameters and weight (the same), the
    slot's drawn-ahead normals (4 (p + d)), the ancestor's integer-weight
    prefix that locates it (8) and the ancestor written out (4): Robertson
    124 bytes; advection-diffusion: the ancestor's field and the new field
    (4 d bytes each) plus the parameter and weight traffic and the ancestor
    read (its draw stays in the scatter pass)."""
    if prob.model == inputs.MODEL_ADVDIFF:
        return (8 * prob.d + 2 * 8 * prob.p + 3 * 8 + 4) * prob.n_particles
    d, p = prob.d, prob.p
    return (2 * (4 * d + 8 * p + 8) + 4 * (p + d) + 8 + 4) * prob.n_particles


# HBM bytes of one k_update launch (Robertson, N = 2^17, FP32 propagation)
# from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch),
# each scaled by what the counter reads for a plain 1 GiB device copy in the
# same run (FETCH_SIZE reads 524316 KiB for the copy's 1048576 KiB of reads:
# x2.0; WRITE_SIZE reads 1048576: x1.0).  Keyed by a hash of the kernel
# sources: once they change, the figure no longer applies and bench reports
# null until the counters are taken again.
TRAFFIC = {
    "5a36f625785c7981": {"fetch_kib": 5025.1, "write_kib": 6224.0, "fetch_scale": 2.0, "write_scale": 1.0},
}
KERNEL_SOURCES = ("pf_kernels.hip", "pf_device.hpp", "pf_types.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_1702_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def update_traffic_bytes(prob):
    """Counter-measured HBM bytes per k_update launch, or None when the
    counters were not taken on this workload and these kernel sources."""
    if (prob.model != inputs.MODEL_ROBERTSON or prob.n_particles != 1 << 17 or prob.lmm != 0
            or prob.order != 2 or prob.substeps != 20 or prob.resampling != 0):
        return None
    t = TRAFFIC.get(kernel_source_hash())
    if t is None:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


# MI355X vector ALU peak: 256 CU x 4 SIMD x 16 lanes x 2 flop (fma) x 2.4 GHz
PEAK_VALU_NONPACKED = 256 * 4 * 16 * 2 * 2.4e9 / 1e12      # 78.6 TFLOP/s (fp32 and fp64)
PEAK_FP32_PUBLISHED = 157.3                                   # TFLOP/s, packed fp32
PEAK_HBM_GBS = 8000.0                                         # GB/s, HBM3E


def progress(msg):
    """One line per finished phase on stderr (a long run shows it is alive)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def run_steps(pf, f, prob, steps):
    """Submit `steps` observation steps asynchronously and wait for them all."""
    tickets = []
    for j in range(steps):
        tickets.append(f.assimilate_async(prob.times[j], prob.y[j], prob.sigma[j]))
        if len(tickets) >= 48:      # keep within the per-filter ring of pending steps
            st = f.wait(tickets.pop(0))
            if st != pf.PF_OK:
                raise RuntimeError(f"step failed: {st}")
    for t in tickets:
        st = f.wait(t)
        if st != pf.PF_OK:
            raise RuntimeError(f"step failed: {st}")


def run_steps_from(pf, f, prob, first, steps):
    """Observation steps first .. first + steps - 1 of the schedule."""
    tickets = []
    for j in range(first, first + steps):
        tickets.append(f.assimilate_async(prob.times[j], prob.y[j], prob.sigma[j]))
        if len(tickets) >= 48:
            st = f.wait(tickets.pop(0))
            if st != pf.PF_OK:
                raise RuntimeError(f"step failed: {st}")
    for t in tickets:
        st = f.wait(t)
        if st != pf.PF_OK:
            raise RuntimeError(f"step failed: {st}")


def timed_pass(pf, ctx, prob, prec, steps, warmup):
    """One pass: a fresh filter, `warmup` untimed observation steps on it,
    then `steps` timed ones (the next steps of the schedule) bracketed by
    device synchronisations.  When the schedule is too short for both, the
    warm-up runs on a filter of its own and the timed steps start at the
    first observation.  Returns (ms per step, posterior of the timed filter,
    first timed observation)."""
    import torch
    same = warmup + steps <= prob.T
    if warmup and not same:
        fw = pf.Filter(ctx, pf.Config(prob, prec))
        run_steps(pf, fw, prob, warmup)
        fw.close()
    f = pf.Filter(ctx, pf.Config(prob, prec))
    first = warmup if same else 0
    if same and warmup:
        run_steps(pf, f, prob, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps_from(pf, f, prob, first, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    post = f.posterior()
    f.close()
    return 1e3 * (t1 - t0) / steps, post, first


def time_path(pf, ctx, prob, prec, steps, warmup):
    """The contract's timed region (a fresh filter, `warmup` untimed steps,
    then `steps` timed ones, no instrumentation), four more such passes for
    the spread, then the first steps once more with timing events between
    the kernel groups for the per-kernel durations."""
    import torch
    # three untimed passes first: on a GPU coming out of idle the first
    # passes of a run measure a few percent slow while its clocks settle
    for _ in range(3):
        timed_pass(pf, ctx, prob, prec, steps, warmup)
    ms0, post, first = timed_pass(pf, ctx, prob, prec, steps, warmup)
    t0, t1 = 0.0, ms0 * steps * 1e-3
    repeats = [ms0]
    for _ in range(4):
        repeats.append(timed_pass(pf, ctx, prob, prec, steps, warmup)[0])
    # instrumented pass over the same observation steps
    f = pf.Filter(ctx, pf.Config(prob, prec))
    if first:
        run_steps(pf, f, prob, first)
    s0 = f.stats()
    ctx.profile(True)
    run_steps_from(pf, f, prob, first, steps)
    times = {k: ctx.kernel_time(w) for k, w in
             (("step", pf.PF_TIME_STEP), ("predict", pf.PF_TIME_PREDICT),
              ("resample", pf.PF_TIME_RESAMPLE), ("update", pf.PF_TIME_UPDATE),
              ("moments", pf.PF_TIME_MOMENTS))}
    ctx.profile(False)
    s1 = f.stats()
    f.close()
    n = prob.n_particles
    iters_upd = s1["newton_update"] - s0["newton_update"]
    iters_pred = s1["newton_predict"] - s0["newton_predict"]
    extra_upd = 0.0
    if prob.model == inputs.MODEL_ADVDIFF:
        flop_upd = steps * n * advdiff_flops(prob, True)
        flop_pred = steps * n * advdiff_flops(prob, False)
        exec_upd, exec_pred = flop_upd, flop_pred
    else:
        # BDF with the SDIRK start-up is priced with the BDF model: its extra
        # per-stage right-hand sides are not counted (a lower bound)
        fl = FLOPS[prob.model]
        sub = fl["sub"] + (fl["sub_am"] if getattr(prob, "lmm", 0) == 1 else 0)
        flop_upd = iters_upd * fl["iter"] + steps * n * prob.substeps * sub
        flop_pred = iters_pred * fl["iter"] + steps * n * prob.substeps * sub
        exec_upd = iters_upd * fl["iter_exec"] + steps * n * prob.substeps * sub
        exec_pred = iters_pred * fl["iter_exec"] + steps * n * prob.substeps * sub
        extra_upd = steps * n * (prob.substeps + 1) * fl["solve"]
    wall = t1 - t0
    return {
        "wall_s": wall,
        "timed_observations": [first + 1, first + steps],
        "particle_steps_per_s": n * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "ms_per_step_5_passes": repeats,
        "ms_per_step_median_of_5": float(np.median(repeats)),
        "kernel_ms": {k: v[1] / max(v[0], 1) for k, v in times.items()},
        "launches": times["update"][0],
        "newton_per_substep": (iters_upd + iters_pred) / (2.0 * steps * n * prob.substeps),
        "flop_update_per_launch": flop_upd / steps,
        "flop_predict_per_launch": flop_pred / steps,
        "flop_update_executed_per_launch": exec_upd / steps,
        "flop_predict_executed_per_launch": exec_pred / steps,
        "flop_update_local_error_filter_per_launch": extra_upd / steps,
        "newton_fails": s1["newton_fails"] - s0["newton_fails"],
        "nonfinite": s1["nonfinite"] - s0["nonfinite"],
        "final_mean": post["mean"].tolist(),
        "final_ess": post["ess"],
    }


def lmm_label(prob):
    lmm = getattr(prob, "lmm", 0)
    return ("BDF", "AM", "BDF")[lmm] + str(prob.order) + ("+SDIRK" if lmm == 2 else "")


def latency(pf, ctx, prob, prec, count):
    """Wall time of synchronous pf_assimilate calls (call to result ready)."""
    f = pf.Filter(ctx, pf.Config(prob, prec))
    lat = []
    for j in range(count):
        t0 = time.perf_counter()
        st = f.assimilate(prob.times[j], prob.y[j], prob.sigma[j])
        lat.append(1e3 * (time.perf_counter() - t0))
        if st != pf.PF_OK:
            raise RuntimeError(f"step failed: {st}")
    f.close()
    return {"p50_ms": _percentile(lat, 50), "p99_ms": _percentile(lat, 99), "calls": count}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# the largest advection-diffusion grid (states) whose oracle step of one
# particle fits a bounded CPU sample (19 x 19 modes: ~4 s on one core)
ADVDIFF_CPU_MAX_STATES = 400


def cpu_baseline(prob, target_s):
    """The FP64 oracle on the host cores: the first S observation steps of the
    same workload, S chosen so the sample takes about target_s seconds.  The
    first two steps are also timed on one thread, for the speedup
    S_P = T_1 / T_P and efficiency E_P = S_P / P of the OpenMP run."""
    from oracle import oracle as O
    O.lib()
    threads = O.num_threads()
    if prob.model == inputs.MODEL_ADVDIFF:
        return cpu_baseline_particles(O, prob, target_s, threads)
    F = O.Filter(prob)
    t0 = time.perf_counter()
    F.step(prob.times[0], prob.y[0], prob.sigma[0])
    one = time.perf_counter() - t0
    S = 1
    t_two = None
    while S < prob.T and (time.perf_counter() - t0) + one < target_s:
        out = F.step(prob.times[S], prob.y[S], prob.sigma[S])
        if S == 1:
            t_two = time.perf_counter() - t0
        if out["status"]:
            break
        S += 1
    el = time.perf_counter() - t0
    res = {"value": prob.n_particles * S / el, "unit": "particle-steps/s", "cores": threads,
           "kind": "oracle", "cpu_model": _cpu_model(),
           "sample": f"first {S} of {prob.T} observation steps at N={prob.n_particles} "
                     f"(FP64 C oracle, OpenMP over particles, {el:.1f} s)"}
    if t_two is not None and threads > 1:
        O.set_threads(1)
        F1 = O.Filter(prob)
        a = time.perf_counter()
        F1.step(prob.times[0], prob.y[0], prob.sigma[0])
        F1.step(prob.times[1], prob.y[1], prob.sigma[1])
        t1 = time.perf_counter() - a
        O.set_threads(threads)
        sp = t1 / t_two
        res["single_thread_first_2_steps_s"] = t1
        res["threads_first_2_steps_s"] = t_two
        res["speedup_S_P"] = sp
        res["efficiency_E_P"] = sp / threads
    return res


def cpu_baseline_particles(O, prob, target_s, threads):
    """The oracle on the advection-diffusion workload: its dense LU makes one
    step of the full ensemble far longer than the budget, so the sample is
    the first observation step for a subset of the particles (its cost is
    linear in their number: the per-particle integrations dominate), sized
    from a pilot of one particle per thread.  A particle's step cannot be
    split, and its dense LU grows with the cube of the state count: at 361
    states it takes ~4 s on one core, at 1521 states ~75 times that, past
    any bounded sample, so larger grids report the leg as skipped."""
    if prob.d > ADVDIFF_CPU_MAX_STATES:
        return {"value": None, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
                "skipped": f"one particle's observation step of the FP64 oracle at {prob.d} states "
                           f"(dense LU, cubic in the state count) takes minutes on one core, past "
                           f"the {target_s:.0f} s sample; measured on grids of at most "
                           f"{ADVDIFF_CPU_MAX_STATES} states"}
    progress(f"cpu baseline: pilot of {threads} particles")
    t0 = time.perf_counter()
    O.Filter(prob.with_particles(threads)).step(prob.times[0], prob.y[0], prob.sigma[0])
    pilot = time.perf_counter() - t0
    n = max(threads, min(prob.n_particles, int(threads * max(1.0, 0.8 * target_s / max(pilot, 1e-3)))))
    t0 = time.perf_counter()
    O.Filter(prob.with_particles(n)).step(prob.times[0], prob.y[0], prob.sigma[0])
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"first observation step with N={n} of the workload's {prob.n_particles} particles "
                      f"(FP64 C oracle, OpenMP over particles, {el:.1f} s)"}


def precision_error(pf, ctx, prob, steps, reps=24):
    """FP32-propagation against FP64 at the stated error: `reps` seeds, each
    run in both precisions on the same data; after every step, the paired
    difference of each log-parameter's posterior mean, t = mean(d) /
    (sd(d)/sqrt(reps)) over the seeds.  Runs are compared only in
    distribution (a last-bit difference flips a resampling decision sooner
    or later and the paired runs decorrelate); |t| stays O(1) when the two
    precisions estimate the same posterior.  Paired runs share every random
    number and stay coupled for many steps, so sd(d) can be far below the
    Monte Carlo error of either run, and a tiny consistent offset then shows
    as a large t: the offset is also given in units of that Monte Carlo
    error (the spread over seeds of the FP64 run's posterior mean) and of
    the posterior standard deviation."""
    mu = {}
    for prec in (pf.PF_PREC_FP32_PROP, pf.PF_PREC_FP64):
        for r in range(reps):
            f = pf.Filter(ctx, pf.Config(prob, prec, seed=1000 + r))
            rows = []
            for j in range(steps):
                if f.assimilate(prob.times[j], prob.y[j], prob.sigma[j]) != pf.PF_OK:
                    rows.append(None)
                    continue
                post = f.posterior()
                rows.append((post["mean"], np.sqrt(np.maximum(np.diag(post["cov"]), 0.0))))
            f.close()
            mu[(prec, r)] = rows
    tt, eff, mce = [], [], []
    for j in range(steps):
        pairs = [(mu[(pf.PF_PREC_FP32_PROP, r)][j], mu[(pf.PF_PREC_FP64, r)][j]) for r in range(reps)]
        pairs = [(a, b) for a, b in pairs if a is not None and b is not None]
        if len(pairs) < 3:
            continue
        d = np.array([a[0] - b[0] for a, b in pairs])
        sd_post = np.mean([b[1] for _, b in pairs], axis=0)
        se = d.std(axis=0, ddof=1) / np.sqrt(len(pairs))
        mc = np.array([b[0] for _, b in pairs]).std(axis=0, ddof=1)
        tt.append(np.abs(d.mean(axis=0)) / np.maximum(se, 1e-300))
        eff.append(np.abs(d.mean(axis=0)) / np.maximum(sd_post, 1e-300))
        mce.append(np.abs(d.mean(axis=0)) / np.maximum(mc, 1e-300))
    tt, eff, mce = np.asarray(tt), np.asarray(eff), np.asarray(mce)
    if not tt.size:
        return None
    return {"seeds": reps, "steps": int(tt.shape[0]),
            "paired_t_median": float(np.median(tt)), "paired_t_p95": float(np.percentile(tt, 95)),
            "frac_abs_t_above_3": float(np.mean(tt > 3.0)),
            "mean_diff_in_mc_error_median": float(np.median(mce)),
            "mean_diff_in_mc_error_max": float(mce.max()),
            "mean_diff_in_posterior_sd_median": float(np.median(eff)),
            "mean_diff_in_posterior_sd_max": float(eff.max())}


def single_filter(pf, args, prob):
    """One filter, `steps` observation steps, FP32 served form and plain FP64."""
    steps = min(args.steps, prob.T)
    warm = min(args.warmup, prob.T)
    with pf.Context(0, 4 << 30) as ctx:
        r32 = time_path(pf, ctx, prob, pf.PF_PREC_FP32_PROP, steps, warm)
        progress(f"fp32 path timed: {r32['ms_per_step']:.4f} ms/step")
        r64 = None if args.no_fp64 else time_path(pf, ctx, prob, pf.PF_PREC_FP64, steps, warm)
        if r64:
            progress(f"fp64 path timed: {r64['ms_per_step']:.4f} ms/step")
        lat = latency(pf, ctx, prob, pf.PF_PREC_FP32_PROP, min(60, prob.T))
        progress("latency done")
        err = None if args.no_fp64 else precision_error(pf, ctx, prob, steps)
        if err:
            progress("precision comparison done")
    served = None
    if args.served_streams > 0 and prob.model == inputs.MODEL_ROBERTSON and prob.n_particles == 1 << 17:
        served = served_leg(pf, args.served_streams)
        progress(f"served leg done: p50 {served['latency_p50_ms']:.3f} ms, p99 {served['latency_p99_ms']:.3f} ms")
    upd_ms = r32["kernel_ms"]["update"]
    achieved = r32["flop_update_per_launch"] / (upd_ms * 1e-3) / 1e12
    traffic = update_traffic_bytes(prob)
    model = {inputs.MODEL_ROBERTSON: "robertson", inputs.MODEL_CHAIN: "chain16"}.get(prob.model)
    if prob.model == inputs.MODEL_ADVDIFF:
        nt = int(prob.model_consts[0])
        model = f"advdiff {nt}x{nt}"
    roofline = {
        "bound": "alu",
        "kernel": (f"k_ad_update + k_ad_part2 <{model}, fp32, {lmm_label(prob)}> (steps 3c-5: gather, "
                   "proliferate, repropagation mode by mode with the local-error innovation, weights, "
                   "tile moments and state sums)" if prob.model == inputs.MODEL_ADVDIFF else
                   f"k_update<{model}, fp32, {lmm_label(prob)}> (steps 3c-5: gather, proliferate, "
                   "repropagation with Newton and local-error innovation, weights, tile moments)"),
        "achieved": achieved, "peak": PEAK_FP32_PUBLISHED, "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_PUBLISHED,
        # the published FP32 peak counts packed (two-wide) FP32 instructions,
        # which this build does not emit; the one-wide VALU peak is 78.6
        "peak_nonpacked": PEAK_VALU_NONPACKED,
        "frac_of_nonpacked": achieved / PEAK_VALU_NONPACKED,
        # by the arithmetic the kernel executes (fewer operations per Newton
        # iteration than the count above for Robertson)
        "frac_executed": r32["flop_update_executed_per_launch"] / (upd_ms * 1e-3) / 1e12 / PEAK_FP32_PUBLISHED,
        "local_error_filter_flop_per_launch": r32["flop_update_local_error_filter_per_launch"],
        "traffic": traffic,
        "traffic_unit": "bytes per launch (HBM, counter-measured)",
        "algorithmic_bytes": algorithmic_bytes(prob),
        # the same launch against the HBM roofline: algorithmic bytes (and the
        # counter-measured ones) over the launch's duration, against 8 TB/s
        "hbm_gbs_algorithmic": algorithmic_bytes(prob) / (upd_ms * 1e-3) / 1e9,
        "hbm_frac_algorithmic": algorithmic_bytes(prob) / (upd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "hbm_frac_measured": (traffic / (upd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS) if traffic else None,
        "avg_launch_ms": upd_ms,
        "flop_per_launch": r32["flop_update_per_launch"],
    }
    # the predictor kernel alone: propagation and first-stage weights, no
    # random numbers and no local-error estimate
    pred_ms = r32["kernel_ms"]["predict"]
    pred_tf = r32["flop_predict_per_launch"] / (pred_ms * 1e-3) / 1e12
    propagation = {
        "kernel": (f"k_ad_predict<{model}, fp32, {lmm_label(prob)}>" if prob.model == inputs.MODEL_ADVDIFF else
                   f"k_predict<{model}, fp32, {lmm_label(prob)}> (steps 2-3a)"),
        "bound": "alu", "achieved": pred_tf, "peak": PEAK_FP32_PUBLISHED, "unit": "TFLOP/s",
        "frac": pred_tf / PEAK_FP32_PUBLISHED, "frac_of_nonpacked": pred_tf / PEAK_VALU_NONPACKED,
        "frac_executed": r32["flop_predict_executed_per_launch"] / (pred_ms * 1e-3) / 1e12 / PEAK_FP32_PUBLISHED,
        "avg_launch_ms": pred_ms,
        "flop_per_launch": r32["flop_predict_per_launch"],
    }
    out = {
        "metric": METRIC,
        "value": r32["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{model} N={prob.n_particles} T={prob.T} {lmm_label(prob)} "
                               f"M={prob.substeps} fp32-propagation, fp64 weights/moments"
                               + (", multinomial resampling" if prob.resampling else ""),
                   "resampling": "multinomial" if prob.resampling else "systematic",
                   "particles": prob.n_particles, "observations": prob.T, "lmm": ("BDF", "AM", "BDF_SDIRK")[prob.lmm], "order": prob.order,
                   "substeps": prob.substeps},
        "fp32": r32,
        "fp64": r64,
        "fp32_over_fp64": (r32["particle_steps_per_s"] / r64["particle_steps_per_s"]) if r64 else None,
        "fp32_error_vs_fp64": err,
        "lmm_substeps_per_s": r32["particle_steps_per_s"] * 2 * prob.substeps,
        "latency": lat,
        "served": served,
        "roofline": roofline,
        "roofline_propagation": propagation,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
        progress("cpu baseline done")
    return out


def batched(pf, args):
    """Many independent filters, one batched submission per observation round."""
    import torch
    probs = inputs.batched_mix(args.filters, seed=0)
    prec = pf.PF_PREC_FP32_PROP
    rounds = max(p.T for p in probs)
    total = sum(p.n_particles * p.T for p in probs)

    def run(ctx, timed):
        fs = [pf.Filter(ctx, pf.Config(p, prec)) for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending = []
        for r in range(rounds):
            idx = [i for i, p in enumerate(probs) if r < p.T]
            tk = ctx.assimilate_batch([fs[i] for i in idx], [probs[i].times[r] for i in idx],
                                      [probs[i].y[r] for i in idx], [probs[i].sigma[r] for i in idx])
            pending.append(list(zip(idx, tk)))
            if len(pending) >= 32:
                for i, t in pending.pop(0):
                    fs[i].wait(t)
        bad = 0
        for grp in pending:
            for i, t in grp:
                bad += fs[i].wait(t) != pf.PF_OK
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for f in fs:
            f.close()
        return wall, bad

    with pf.Context(0, 24 << 30) as ctx:
        run(ctx, False)                 # warm-up: captures nothing (shapes change every round)
        wall, bad = run(ctx, True)
    n_chain = sum(p.model == inputs.MODEL_CHAIN for p in probs)
    return {
        "metric": METRIC, "value": total / wall, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": rounds, "warmup": rounds, "ms_per_step": 1e3 * wall / rounds,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched {len(probs)} filters ({n_chain} chain16 BDF3 M=40 T=100, "
                               f"{len(probs) - n_chain} robertson BDF2 M=20 T=50), "
                               "N log-uniform in [512, 65536], one submission per round",
                   "particles_total": int(sum(p.n_particles for p in probs)),
                   "particle_steps": int(total)},
        "skipped_steps": int(bad),
    }


def serve_trace(pf, trace, pool, prec=None):
    """Replay a serving trace (stream arrivals and their observations) in real
    time through the continuous-batching server; the server's report plus the
    wall time, the replay's largest lag behind the trace, and throughput.
    FP32 propagation unless `prec` says otherwise."""
    prec = pf.PF_PREC_FP32_PROP if prec is None else prec
    cfgs = [pf.Config(r.problem, prec) for r in trace]
    events = []
    for k, r in enumerate(trace):
        events.append((r.arrival, 0, k, -1))
        for j, off in enumerate(r.obs_offsets):
            events.append((r.arrival + off, 1, k, j))
    events.sort()
    with pf.Context(0, pool) as ctx:
        srv = pf.Server(ctx, max_inflight=3)
        sids = [None] * len(trace)
        t0 = time.perf_counter()
        lag = 0.0
        for when, kind, k, j in events:
            now = time.perf_counter() - t0
            if when > now:
                time.sleep(when - now)
            else:
                lag = max(lag, now - when)
            if kind == 0:
                sids[k] = srv.open(cfgs[k])
            else:
                prob = trace[k].problem
                srv.submit(sids[k], prob.times[j], prob.y[j], prob.sigma[j])
                if j == prob.T - 1:
                    srv.close(sids[k])
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.destroy()
    st["wall_s"] = wall
    st["driver_max_lag_ms"] = 1e3 * lag
    st["particle_steps_per_s"] = st["particle_steps"] / st["busy_s"] if st["busy_s"] > 0 else None
    return st


def served_leg(pf, streams):
    """The serving workload at a reduced stream count (the same arrival rate,
    model mix and particle counts), for the default line: served p50/p99
    latency beside the throughput."""
    trace = inputs.serving_trace(n_streams=streams, rate=200.0, seed=0)
    st = serve_trace(pf, trace, 48 << 30)
    # the same trace served by the plain FP64 path
    s64 = serve_trace(pf, trace, 48 << 30, pf.PF_PREC_FP64)
    n_chain = sum(r.problem.model == inputs.MODEL_CHAIN for r in trace)
    return {"workload": f"serving {len(trace)} streams, Poisson arrivals 200/s, {n_chain} chain16 / "
                        f"{len(trace) - n_chain} robertson, N in {{4096, 16384, 65536}}, observation gaps "
                        "Exp(10 ms), fp32 propagation, uncapped pool",
            "latency_p50_ms": st["latency_p50_ms"], "latency_p99_ms": st["latency_p99_ms"],
            "latency_max_ms": st["latency_max_ms"], "particle_steps_per_s": st["particle_steps_per_s"],
            "steps_completed": st["steps_completed"], "steps_skipped": st["steps_skipped"],
            "mean_batch": st["mean_batch"], "ticks": st["ticks"], "wall_s": st["wall_s"],
            "driver_max_lag_ms": st["driver_max_lag_ms"],
            "fp64": {"latency_p50_ms": s64["latency_p50_ms"], "latency_p99_ms": s64["latency_p99_ms"],
                     "latency_max_ms": s64["latency_max_ms"], "mean_batch": s64["mean_batch"],
                     "driver_max_lag_ms": s64["driver_max_lag_ms"]}}


def serving(pf, args):
    """Poisson arrivals of filtering streams replayed in real time through the
    continuous-batching server; latency = submit -> result ready."""
    trace = inputs.serving_trace(n_streams=args.streams, rate=200.0, seed=0)
    runs = {}
    for label, pool in (("uncapped", 48 << 30), ("pool_256MiB", 256 << 20)):
        runs[label] = serve_trace(pf, trace, pool)
    # the same trace served by the plain FP64 path (uncapped pool)
    runs["fp64_uncapped"] = serve_trace(pf, trace, 48 << 30, pf.PF_PREC_FP64)
    main_run = runs["uncapped"]
    n_chain = sum(r.problem.model == inputs.MODEL_CHAIN for r in trace)
    return {
        "metric": METRIC, "value": main_run["particle_steps_per_s"], "unit": "particle-steps/s",
        "n_gpus": 1, "steps": int(main_run["ticks"]), "warmup": 0,
        "ms_per_step": 1e3 * main_run["busy_s"] / max(main_run["ticks"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving {len(trace)} streams, Poisson arrivals 200/s, "
                               f"{n_chain} chain16 / {len(trace) - n_chain} robertson, "
                               "N in {4096, 16384, 65536}, observation gaps Exp(10 ms), fp32 propagation"},
        "latency_p50_ms": main_run["latency_p50_ms"], "latency_p99_ms": main_run["latency_p99_ms"],
        "fp64_latency_p50_ms": runs["fp64_uncapped"]["latency_p50_ms"],
        "fp64_latency_p99_ms": runs["fp64_uncapped"]["latency_p99_ms"],
        "runs": runs,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--config", default="robertson",
                    choices=["robertson", "small", "chain", "advdiff", "advdiff40", "batched", "serving"])
    ap.add_argument("--filters", type=int, default=256)
    ap.add_argument("--streams", type=int, default=2000)
    ap.add_argument("--served-streams", type=int, default=200,
                    help="streams of the served leg of the default line (0: none)")
    ap.add_argument("--resampling", default="systematic", choices=["systematic", "multinomial"],
                    help="index draw of step 3(b) for the single-filter configurations")
    ap.add_argument("--lmm", default="bdf", choices=["bdf", "am", "bdf_sdirk"],
                    help="LMM family of the single-filter configurations (am: Adams-Moulton; "
                         "bdf_sdirk: BDF with the order-preserving SDIRK start-up)")
    ap.add_argument("--order", type=int, default=0,
                    help="BDF order or AM steps (0: the configuration's own)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters of a profiler pass)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); independent filters shard "
              "by whole filters across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1411_1702_amd import pf
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.init()
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.config == "batched":
        out = batched(pf, args)
    elif args.config == "serving":
        out = serving(pf, args)
    else:
        prob = {"robertson": inputs.config_robertson_large, "small": inputs.config_small,
                "chain": inputs.config_chain, "advdiff": lambda: inputs.config_advdiff(20),
                "advdiff40": lambda: inputs.config_advdiff(40)}[args.config]()
        if args.steps < 1:
            print("--steps must be >= 1", file=sys.stderr)
            sys.exit(2)
        prob.resampling = 1 if args.resampling == "multinomial" else 0
        prob.lmm = {"bdf": 0, "am": 1, "bdf_sdirk": 2}[args.lmm]
        if prob.model == inputs.MODEL_ADVDIFF and prob.lmm == 1:
            print("the advection-diffusion model runs BDF or BDF with the SDIRK start-up", file=sys.stderr)
            sys.exit(2)
        if args.order:
            prob.order = args.order
        out = single_filter(pf, args, prob)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
