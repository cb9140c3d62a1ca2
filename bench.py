"""Sliding-window cumulant update throughput on one MI355X.

Workload: the regime-change stream at n=60 columns, d=4, b=4, window t=20000
rows, p=1000 rows per update (Gaussian rows first, Gaussian-copula rows with
Student-t(6)/Exp(1) marginals after step 100).  One step = one cum_update:
the signed moment contraction of orders 1..4 with its compensated fold, the
FP64 moment->cumulant combine of every order and the norms / nu_k, all on the
GPU, with the stream's rows already resident in HBM.

Prints one JSON line: rows/s of the main path (--prec, default fp32) as
`value`, the per-path figures (fp64, fp32, split-bf16x3) with their sampled
error against the FP64 oracle, the dominant kernel's roofline, the oracle's
own throughput on the host cores (cpu_baseline), and further legs: the
200-step trajectory of the regime-change stream, the order-6 precision
sweep, the adjoint, 64 batched streams and the paper-scale nu_4 study.

The oracle runs only in the cpu_baseline leg: the GPU legs record sampled
stored elements (random pyramid offsets and the GPU's values there) and the
window they belong to, and that leg computes the oracle's values at those
elements and states each error.
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

N, D, B, T, P = 60, 4, 4, 20000, 1000
METRIC = "window updates/s + rows/s at n=60,d=4,b=4; split-BF16 vs FP64 GPU at stated err"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
EVENT_EVERY = 10  # timed region: one update launch in this many is bracketed by events
# Untimed steps after the warm-up, before the timed region: after the GPU has
# been idle (stream set-up, context creation) the shader clock rises over the
# first ~20 ms of back-to-back updates, and the update's duration falls by
# ~8 % meanwhile (kernel trace: fp32 46.0 -> 42.3 us over ~375 launches, fp64
# 86.0 -> 77.8 us over ~225); the timed region measures the settled clock.
SETTLE_STEPS = 500
TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


# HBM bytes per k_update launch at this workload from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE; mean over the sliding-update dispatches),
# each scaled by the ratio of known bytes to the same counter on a plain
# device copy.  Valid only for the kernel source they were taken on.
TRAFFIC = {"prec": "fp32",
           "kernels_sha256": "0ebc5875d8915f73b6e9cbf271e87bd43f334014309402b40ece0bba02a2f6c5",
           "fetch_bytes": 6139.53 * 1024 * 1.99988,   # FETCH_SIZE KiB x (256 MiB / 131080.1 KiB)
           "write_bytes": 6476.03 * 1024 * 1.00000}   # WRITE_SIZE KiB x (256 MiB / 262144.0 KiB)


def kernels_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1701_06446_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(prec: str):
    if TRAFFIC["kernels_sha256"] != kernels_sha256() or TRAFFIC["prec"] != prec:
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]


def copy_calibration(mib: int):
    """A plain elementwise pass (dst = -src) over mib MiB, three times: a
    reference for the FETCH_SIZE / WRITE_SIZE counters, each pass reading and
    writing mib MiB (an elementwise kernel, where a same-type copy could go to
    a DMA engine that the counters do not see)."""
    import torch

    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return {"bytes_each_way": mib << 20, "copies": 3}


def algorithmic_flops_per_update(p: int) -> float:
    """One FMA per stored pyramid element per signed row: 2 * (2p) * sum_k E_k."""
    import paper_1701_06446_amd as cum

    return 2.0 * (2 * p) * sum(cum.cum_num_elems(N, B, k) for k in range(1, D + 1))


# Deferred accuracy checks: (label, window rows, n, b, d, {k: (offsets,
# GPU values)}, tolerance), evaluated against the oracle in the cpu_baseline
# leg.
CHECKS = []


def record_check(label, ctx, window, n, b, d, rng, count=40, tol=None):
    """Samples `count` random stored elements of every order 2..d of ctx's
    cumulants (random pyramid offsets) and keeps them, with a host copy of
    the window, for the oracle comparison of the cpu_baseline leg."""
    import paper_1701_06446_amd as cum

    samples = {}
    for k in range(2, d + 1):
        ne = cum.cum_num_elems(n, b, k)
        offs = rng.integers(0, ne, size=count)
        samples[k] = (offs, cum.cum_get(ctx, k)[offs])
    CHECKS.append((label, np.asarray(window, dtype=np.float64), n, b, d, samples, tol))


def run_path(path, s, warmup, steps, check, host_leg=False):
    """path: a precision (sliding mode: the new and the leaving rows are both
    contracted) or '<precision>-fifo' (the batch-increment queue)."""
    import torch

    import paper_1701_06446_amd as cum

    prec, _, mode = path.partition("-")
    dt = np.float64 if prec == "fp64" else np.float32
    rows = np.ascontiguousarray(s.rows.astype(dt))
    dev = torch.from_numpy(rows).to("cuda")
    if mode == "fifo":
        ctx = cum.cum_init_fifo(N, D, B, dev[:T], P, prec=prec)
    else:
        ctx = cum.cum_init(N, D, B, dev[:T], prec=prec)
    w = 0

    def step():
        nonlocal w
        w += 1
        lo, hi = (w - 1) * P, w * P
        cum.cum_update(ctx, dev[T + lo:T + hi], None if mode == "fifo" else dev[lo:hi])

    for _ in range(warmup + SETTLE_STEPS):
        step()
    torch.cuda.synchronize()
    # timed region: HIP events on the context's stream bracket one update
    # kernel launch in EVENT_EVERY, the last of each group (each pair adds a gap)
    cum.cum_profile_enable(ctx, ["update"], every=EVENT_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    # every step's norms are formed inside the timed region: each update
    # launch forms the previous step's, cum_sync the last one
    cum.cum_sync(ctx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = cum.cum_profile_read(ctx)
    cum.cum_profile_enable(ctx, False)
    # the same number of steps without events (their overhead), then a few
    # with every kernel class bracketed (the smaller kernels' durations)
    t1 = time.perf_counter()
    for _ in range(steps):
        step()
    cum.cum_sync(ctx)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t1
    cum.cum_profile_enable(ctx, True)
    for _ in range(10):
        step()
    allk = cum.cum_profile_read(ctx)
    cum.cum_profile_enable(ctx, False)
    prof = {"update": prof["update"], "combine": allk["combine"], "norms": allk["norms"]}
    out = {
        "ms_per_step": elapsed / steps * 1e3,
        "updates_per_s": steps / elapsed,
        "rows_per_s": steps * P / elapsed,
        "ms_per_step_without_kernel_events": plain / steps * 1e3,
        "kernel_ms": {k: (v[1] / v[0] if v[0] else None) for k, v in prof.items()},
        "update_launches_timed_by_events": prof["update"][0],
        "launches_per_step": {"update": allk["update"][0] / 10, "combine": prof["combine"][0] / 10,
                              "norms": prof["norms"][0] / 10},
    }
    if host_leg:
        # the same updates from host (pageable numpy) rows: each call stages
        # both batches over PCIe and waits for the copies (never `value`)
        t3 = time.perf_counter()
        for _ in range(20):
            w += 1
            lo, hi = (w - 1) * P, w * P
            cum.cum_update(ctx, rows[T + lo:T + hi], None if mode == "fifo" else rows[lo:hi])
        torch.cuda.synchronize()
        out["host_input_rows_per_s"] = 20 * P / (time.perf_counter() - t3)
    # the recalculation the update replaces (Eq. (upcmplx), Sec. 2.4): the whole
    # current window contracted from scratch on the same context, with the
    # combine and norms; the paper's speed-up estimate is t / (2 t_up + B(d))
    win = dev[w * P: w * P + T]
    cum.cum_recompute(ctx, win)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(5):
        cum.cum_recompute(ctx, win)
    cum.cum_sync(ctx)  # the last recalculation's norms
    torch.cuda.synchronize()
    rec_ms = (time.perf_counter() - t2) / 5 * 1e3
    out["recompute_ms"] = rec_ms
    out["speedup_vs_recompute"] = rec_ms / out["ms_per_step_without_kernel_events"]
    out["speedup_theory"] = T / ((1 if mode == "fifo" else 2) * P + 15)  # B(4) = 15
    if check:
        record_check("paths." + path, ctx, rows[w * P: w * P + T], N, B, D, np.random.default_rng(7), tol=TOL[prec])
    if mode == "fifo":
        out["fifo_slots"] = T // P
    cum.cum_free(ctx)
    del dev
    torch.cuda.empty_cache()
    return out


def run_batched(steps, warmup, prec="fp32", autotune=True, reps=5):
    """64 uneven streams (n in 8..96, d in 3..4, t in 1000..20000, p = t/20)
    updated together by one captured graph; b per stream from the autotuner's
    cost model (deterministic)."""
    import torch

    import paper_1701_06446_amd as cum
    import streams
    from paper_1701_06446_amd import autotune as at

    ss = streams.batched_streams(m=64, steps=warmup + reps * steps)
    t0 = time.perf_counter()
    if autotune:
        for s in ss:
            s.b = at.choose_b(s.n, s.d, s.t, s.p, prec)
    tune_s = time.perf_counter() - t0
    dt = np.float64 if prec == "fp64" else np.float32
    rows = [np.ascontiguousarray(s.rows.astype(dt)) for s in ss]
    dev = [torch.from_numpy(r).to("cuda") for r in rows]
    ctxs = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec=prec) for s, d in zip(ss, dev)]
    bt = cum.cum_batch_create(ctxs)
    w = 0

    def step():
        nonlocal w
        w += 1
        cum.cum_batch_update(bt, [d[s.t + (w - 1) * s.p:s.t + w * s.p] for s, d in zip(ss, dev)],
                             [d[(w - 1) * s.p:w * s.p] for s, d in zip(ss, dev)])

    for _ in range(warmup):
        step()
    cum.cum_batch_sync(bt)
    # `reps` timed blocks of `steps` steps: the median block is reported, the
    # spread is (max - min) / median over the blocks
    runs = []
    for _ in range(reps):
        t1 = time.perf_counter()
        for _ in range(steps):
            step()
        cum.cum_batch_sync(bt)
        runs.append(time.perf_counter() - t1)
    el = float(np.median(runs))
    rows_per_step = sum(s.p for s in ss)
    flops = sum(2.0 * 2 * s.p * sum(cum.cum_num_elems(s.n, s.b, k) for k in range(1, s.d + 1)) for s in ss)
    flops_distinct = sum(2.0 * 2 * s.p * at.distinct_elements(s.n, s.d) for s in ss)
    rng = np.random.default_rng(5)
    for i in range(0, 64, 8):
        s = ss[i]
        record_check("batched.stream%02d" % i, ctxs[i], rows[i][w * s.p:w * s.p + s.t], s.n, s.b, s.d, rng,
                     count=6, tol=TOL[prec])
    cum.cum_batch_free(bt)
    for c in ctxs:
        cum.cum_free(c)
    return {"streams": 64, "steps": steps, "warmup": warmup, "prec": prec, "timed_blocks": reps,
            "rows_per_s": rows_per_step * steps / el, "updates_per_s": 64 * steps / el,
            "ms_per_step": el / steps * 1e3, "rows_per_step": rows_per_step,
            "ms_per_step_blocks": [r / steps * 1e3 for r in runs],
            "spread": (max(runs) - min(runs)) / el,
            "tflops_algorithmic": flops * steps / el / 1e12,
            "tflops_distinct_elements": flops_distinct * steps / el / 1e12,
            "b_choice": {str(b): sum(1 for s in ss if s.b == b) for b in (1, 2, 4, 8)},
            "autotune_s": tune_s, "tol": TOL[prec]}


def run_order6(steps=50, warmup=1, paths=("fp32", "fp64", "bf16x3", "fp32-recursion")):
    """The high-order precision sweep: mixed Exp(1) sources, n=48, d=6, b=4,
    t=50000, p=2000, sliding mode, `steps` updates per path (FP32, FP64 and
    split-BF16x3 contractions with Alg. 4's combine, and FP32 with the
    recursion combine); per-kernel times from the event profiler, sampled
    errors against the oracle (cpu_baseline leg), and the norms beside their
    population values: the sources' cumulant tensors are diagonal with
    (k-1)! entries and the mixing is orthogonal, so ||C_k||_F tends to
    sqrt(48) (k-1)! (sampling noise is large at k = 5, 6)."""
    import math

    import torch

    import paper_1701_06446_amd as cum
    import streams

    n, d, b, t, p = 48, 6, 4, 50000, 2000
    s = streams.mixed_exp_stream(steps=warmup + steps)
    out = {"workload": "mixed Exp(1) sources S W, n=48 d=6 b=4 t=50000 p=2000, sliding",
           "steps": steps, "population_fro": [None, None] + [math.sqrt(n) * math.factorial(k - 1)
                                                             for k in range(2, d + 1)]}
    elems = [cum.cum_num_elems(n, b, k) for k in range(1, d + 1)]
    flops = 2.0 * 2 * p * sum(elems)
    out["flops_per_update"] = flops
    out["stored_elements"] = sum(elems)
    for path in paths:
        prec, _, method = path.partition("-")
        rows = np.ascontiguousarray(s.rows.astype(np.float64 if prec == "fp64" else np.float32))
        dev = torch.from_numpy(rows).to("cuda")
        t0 = time.perf_counter()
        ctx = cum.cum_init(n, d, b, dev[:t], prec=prec)
        cum.cum_sync(ctx)
        init_s = time.perf_counter() - t0
        if method:
            cum.cum_set_combine(ctx, method)
        w = 0

        def step():
            nonlocal w
            w += 1
            cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        cum.cum_profile_enable(ctx, True)
        t1 = time.perf_counter()
        for _ in range(steps):
            step()
        cum.cum_sync(ctx)  # the last step's norms
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        prof = cum.cum_profile_read(ctx)
        cum.cum_profile_enable(ctx, False)
        upd_ms = prof["update"][1] / prof["update"][0]
        fro, nu = cum.cum_norms(ctx)
        record_check("order6." + path, ctx, rows[w * p:w * p + t], n, b, d, np.random.default_rng(17), count=12,
                     tol=TOL[prec])
        out[path] = {"ms_per_step": el / steps * 1e3, "rows_per_s": steps * p / el,
                     # launches per step: one update; the combine order by order (6)
                     "kernel_ms_per_step": {k: v[1] / steps for k, v in prof.items() if v[0]},
                     "launches_per_step": {k: v[0] / steps for k, v in prof.items() if v[0]},
                     "update_ms": upd_ms,
                     "update_tflops": flops / (upd_ms * 1e-3) / 1e12,
                     "update_frac_peak": flops / (upd_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                     "init_s": init_s, "fro": [None if not np.isfinite(f) else f for f in fro],
                     "tol": TOL[prec]}
        cum.cum_free(ctx)
        del dev
        torch.cuda.empty_cache()
    return out


def run_trajectory(s, steps=200, switch=100, prec="fp32"):
    """The regime-change stream's 200 steps (the first `switch` Gaussian,
    the rest copula rows) with every step's norms read back synchronously
    (the emit of Alg. 1, Sec. 2.2): ||C_3||, ||C_4||, nu_3, nu_4 per step,
    the synchronous step latency, and sampled oracle checks at the last
    Gaussian step and the last step."""
    import torch

    import paper_1701_06446_amd as cum

    rows = np.ascontiguousarray(s.rows[:T + steps * P].astype(np.float32))
    dev = torch.from_numpy(rows).to("cuda")
    ctx = cum.cum_init(N, D, B, dev[:T], prec=prec)
    traj = {"fro3": [], "fro4": [], "nu3": [], "nu4": []}
    t0 = time.perf_counter()
    for w in range(1, steps + 1):
        cum.cum_update(ctx, dev[T + (w - 1) * P:T + w * P], dev[(w - 1) * P:w * P])
        fro, nu = cum.cum_norms(ctx)
        traj["fro3"].append(float("%.6g" % fro[3]))
        traj["fro4"].append(float("%.6g" % fro[4]))
        traj["nu3"].append(float("%.6g" % nu[3]))
        traj["nu4"].append(float("%.6g" % nu[4]))
        if w in (switch, steps):
            t0 -= time.perf_counter()
            record_check("trajectory.step%d" % w, ctx, rows[w * P:w * P + T], N, B, D, np.random.default_rng(w),
                         count=30, tol=TOL[prec])
            t0 += time.perf_counter()
    el = time.perf_counter() - t0
    cum.cum_free(ctx)
    nu4 = np.array(traj["nu4"])
    return {"workload": "regime-change stream n=60 d=4 b=4 t=20000 p=1000, %d steps, copula rows after "
                        "step %d" % (steps, switch), "prec": prec,
            "ms_per_step_with_norms_readback": el / steps * 1e3,
            "nu4_gaussian_steps_mean": float(nu4[:switch].mean()),
            "nu4_after_window_turnover_mean": float(nu4[switch + T // P:].mean()) if steps > switch + T // P else None,
            "turnover_steps": T // P, **traj}


def run_nu4_study(runs=100, n=100, t=1_000_000, tup=25_000, windows=61):
    """The paper's stream statistics study (Sec. 4.3) at its scale: n = 100,
    t = 10^6, t_up = 2.5 10^4, 61 windows, the first Gaussian, the updates
    from a Student-t copula (nu = 10) with the first window's Gaussian
    marginals, `runs` seeded repetitions on the fp32 path (d = 4, b = 4).
    nu_3 and nu_4 per window for the first run; the 5th, 50th and 95th
    percentiles of nu_4 at window 1 (Gaussian) and window 61 (no Gaussian
    row left after window 41) over the runs, beside the paper's (its
    covariance is not given: context only)."""
    import math

    import paper_1701_06446_amd as cum
    import streams

    from tests.noise_floor import gaussian_noise_floor

    nu_first, nu_last, curve = [], [], {"nu3": [], "nu4": []}
    t0 = time.perf_counter()
    for r in range(runs):
        if r and r % 10 == 0:
            print("[bench] nu_4 study: run %d" % r, file=sys.stderr, flush=True)
        X, S = streams.tcopula_study_rows(r, n=n, t=t, tup=tup, windows=windows)
        ctx = cum.cum_init(n, 4, 4, X[:t], prec="fp32")
        _, nu = cum.cum_norms(ctx)
        nu_first.append(nu[4])
        if r == 0:
            curve["nu3"].append(float("%.5g" % nu[3]))
            curve["nu4"].append(float("%.5g" % nu[4]))
        for w in range(2, windows + 1):
            lo = (w - 2) * tup
            cum.cum_update(ctx, X[t + lo:t + lo + tup], X[lo:lo + tup])
            if r == 0:
                _, nu = cum.cum_norms(ctx)
                curve["nu3"].append(float("%.5g" % nu[3]))
                curve["nu4"].append(float("%.5g" % nu[4]))
        _, nu = cum.cum_norms(ctx)
        nu_last.append(nu[4])
        if r == 0:
            t0 -= time.perf_counter()
            record_check("nu4_study.run0.window%d" % windows, ctx, X[-t:].double().cpu().numpy(), n, 4, 4,
                         np.random.default_rng(61), count=6, tol=TOL["fp32"])
            t0 += time.perf_counter()
        cum.cum_free(ctx)
        del X
    el = time.perf_counter() - t0
    q = lambda v: [float("%.4g" % x) for x in np.percentile(np.array(v), [5, 50, 95])]
    return {"workload": "n=%d t=%d t_up=%d, %d windows: Gaussian, then Student-t copula (nu=10) with "
                        "Gaussian marginals; d=4 b=4 fp32" % (n, t, tup, windows),
            "runs": runs, "seconds": el, "first_run": curve,
            "nu4_quantiles_5_50_95": {"window_1": q(nu_first), "window_%d" % windows: q(nu_last)},
            # the Gaussian window's expected nu_4: sqrt of the closed-form
            # E||C_4||^2 of Gaussian sampling noise over ||Sigma||_F^2
            "nu4_window_1_gaussian_noise_floor": math.sqrt(gaussian_noise_floor(S, t, 4)) / float(np.sum(S * S)),
            "paper_nu4_quantiles_5_50_95": {"gaussian": [0.004, 0.006, 0.011], "t_copula": [0.199, 0.209, 0.220]}}


def run_adjoint(reps=5):
    """The adjoint workload: L = ||C_3(X W^T)||^2 + ||C_4(X W^T)||^2 with
    X 10000 x 32 and W 32 x 32 (d=4, b=4); loss and both gradients per call."""
    import torch

    import paper_1701_06446_amd as cum
    import streams

    X, W = streams.adjoint_workload()
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(np.float32))).cuda()
    Wd = torch.from_numpy(np.ascontiguousarray(W.astype(np.float32))).cuda()
    L, _, _ = cum.cum_loss_grad(Xd, Wd, 4, 4, {3: 1.0, 4: 1.0})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        cum.cum_loss_grad(Xd, Wd, 4, 4, {3: 1.0, 4: 1.0})
    torch.cuda.synchronize()
    return {"workload": "X 10000x32, W 32x32, d=4 b=4, weights {3: 1, 4: 1}", "loss": L,
            "ms_per_call": (time.perf_counter() - t0) / reps * 1e3}


def cpu_baseline(s, budget_s=12.0):
    """The oracle (as it stands) on the host cores: sliding steps of p=1000 rows
    at n=60, d=4, b=4 from a 2000-row start window, each step = compensated
    sums + Alg. 4 combine + Alg. 5 norms; on all the cores the oracle's
    OpenMP loops use, and on one core (in a child process)."""
    import subprocess

    import oracle

    rows = s.rows.astype(np.float32).astype(np.float64)
    n_steps, el = cpu_timed(rows, budget_s, 30)
    out = {"value": n_steps * P / el, "unit": "rows/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": "%d sliding steps of p=1000 rows (n=60,d=4,b=4) from a 2000-row start window; "
                     "per step: FP64 compensated sums of orders 1..4, Alg.4 combine, Alg.5 norms; "
                     "%.1f s" % (n_steps, el)}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, json, time; sys.path.insert(0, %r); import numpy as np; import bench, streams; "
            "s = streams.regime_change_stream(steps=8, switch=8); "
            "rows = s.rows.astype(np.float32).astype(np.float64); "
            "import oracle; n, el = bench.cpu_timed(rows, 2, 6); "
            "print(json.dumps([n, el, oracle.num_threads()]))" % ROOT)
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        n1, el1, th1 = json.loads(res.stdout.strip().splitlines()[-1])
        out["one_core"] = {"value": n1 * P / el1, "unit": "rows/s", "cores": th1,
                           "sample": "%d sliding steps, the same per-step work; %.1f s" % (n1, el1)}
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        out["one_core"] = {"error": str(e)}
    return out


def cpu_timed(rows, budget, max_steps):
    """Oracle sliding steps on `rows` for about `budget` seconds (at least 2
    steps, at most max_steps): (steps, seconds)."""
    import oracle

    o = oracle.SlidingOracle(rows[:2000], N, D, B)
    n_steps, t0 = 0, time.perf_counter()
    while n_steps < 2 or (time.perf_counter() - t0 < budget and n_steps < max_steps):
        n_steps += 1
        lo, hi = (n_steps - 1) * P, n_steps * P
        o.update(rows[2000 + lo:2000 + hi], rows[lo:hi])
        oracle.norms(o.cumulants(), N, B)
    return n_steps, time.perf_counter() - t0


def oracle_checks():
    """The deferred checks against the oracle: for every recorded sample, the
    oracle's cumulant at each sampled element (Alg. 4 on moments taken from
    the same window) and the relative error over the sample."""
    from oracle.element import cumulant_at, indices_of

    out = {}
    for label, window, n, b, d, samples, tol in CHECKS:
        cache, worst = {}, 0.0
        for k, (offs, vals) in samples.items():
            idxs = indices_of(n, b, k, offs)
            keep = [i for i, x in enumerate(idxs) if x is not None]
            if not keep:
                continue
            ref = np.array([cumulant_at(window, idxs[i], cache) for i in keep])
            err = np.linalg.norm(vals[keep] - ref) / max(np.linalg.norm(ref), 1e-300)
            worst = max(worst, float(err))
        out[label] = {"err_sampled": worst, "tol": tol}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--paths", default="fp64,fp32,bf16x3,fp32-fifo,bf16x3-fifo",
                    help="paths to measure: a precision (sliding mode) or <precision>-fifo")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB three times (for scaling HBM counters)")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-stream batched leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the order-6 and adjoint legs")
    ap.add_argument("--no-trajectory", action="store_true", help="skip the 200-step trajectory leg")
    ap.add_argument("--order6-steps", type=int, default=50)
    ap.add_argument("--nu4-runs", type=int, default=100,
                    help="repetitions of the paper-scale nu_4 study (0 skips it)")
    ap.add_argument("--adjoint-only", type=int, default=0, metavar="CALLS",
                    help="only time CALLS adjoint calls and print their figures (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import streams

    if args.adjoint_only:
        print(json.dumps({"adjoint": run_adjoint(reps=args.adjoint_only)}))
        return
    total_steps = max(200, args.warmup + SETTLE_STEPS + 2 * args.steps + 30)
    s = streams.regime_change_stream(n=N, d=D, b=B, t=T, p=P, steps=total_steps, switch=100)
    paths = [p for p in args.paths.split(",") if p and p != args.prec] + [args.prec]
    res = {}
    for prec in paths:
        print("[bench] path %s: warmup %d + %d settle steps, %d timed steps"
              % (prec, args.warmup, SETTLE_STEPS, args.steps),
              file=sys.stderr, flush=True)
        res[prec] = run_path(prec, s, args.warmup, args.steps, not args.no_check, host_leg=(prec == args.prec))
        print("[bench] path %s: %.3f ms/step" % (prec, res[prec]["ms_per_step"]), file=sys.stderr, flush=True)
    for path, r in res.items():
        rows_contracted = P if path.endswith("-fifo") else 2 * P
        f = algorithmic_flops_per_update(P) * rows_contracted / (2 * P)
        r["update_kernel_tflops"] = f / (r["kernel_ms"]["update"] * 1e-3) / 1e12
    main = res[args.prec]
    flops = algorithmic_flops_per_update(P)
    upd_ms = main["kernel_ms"]["update"]
    achieved = flops / (upd_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": main["rows_per_s"],
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_steps": SETTLE_STEPS,
        "ms_per_step": main["ms_per_step"],
        "updates_per_s": main["updates_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (f32 accumulate)"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "regime-change stream n=60 d=4 b=4 t=20000 p=1000 (Gaussian, then "
                               "Gaussian copula with t6/Exp marginals after step 100)",
                   "n": N, "d": D, "b": B, "t": T, "p": P, "prec": args.prec},
        "roofline": {"bound": "mfma", "kernel": "k_update", "achieved": achieved,
                     "peak": PEAK_TFLOPS[args.prec], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS[args.prec],
                     "flops_per_launch": flops, "kernel_ms": upd_ms, "traffic": traffic_for(args.prec)},
        "paths": res,
        "device": torch.cuda.get_device_name(0),
    }
    if args.copy_calibration:
        line["copy_calibration"] = copy_calibration(args.copy_calibration)
    if not args.no_trajectory:
        print("[bench] trajectory: 200 steps with norms read back", file=sys.stderr, flush=True)
        line["trajectory"] = run_trajectory(s)
        print("[bench] trajectory: %.3f ms/step" % line["trajectory"]["ms_per_step_with_norms_readback"],
              file=sys.stderr, flush=True)
    if not args.no_extra:
        print("[bench] order 6: n=48 d=6 b=4 p=2000, %d steps per path" % args.order6_steps,
              file=sys.stderr, flush=True)
        line["order6"] = run_order6(steps=args.order6_steps)
        for k in ("fp32", "fp64", "bf16x3", "fp32-recursion"):
            print("[bench] order 6 %s: %.3f ms/step" % (k, line["order6"][k]["ms_per_step"]),
                  file=sys.stderr, flush=True)
        print("[bench] adjoint", file=sys.stderr, flush=True)
        line["adjoint"] = run_adjoint()
    if not args.no_batched:
        print("[bench] batched: 64 streams, 5 x 30 steps", file=sys.stderr, flush=True)
        line["batched"] = run_batched(steps=30, warmup=10, reps=5)
        print("[bench] batched: %.3f ms/step" % line["batched"]["ms_per_step"], file=sys.stderr, flush=True)
    if args.nu4_runs > 0:
        print("[bench] nu_4 study: %d runs" % args.nu4_runs, file=sys.stderr, flush=True)
        line["nu4_study"] = run_nu4_study(runs=args.nu4_runs)
        print("[bench] nu_4 study: %.1f s" % line["nu4_study"]["seconds"], file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(s)
        print("[bench] oracle checks: %d samples" % len(CHECKS), file=sys.stderr, flush=True)
        checks = oracle_checks()
        line["oracle_checks"] = checks
        for path, r in res.items():
            if "paths." + path in checks:
                r["err_sampled"] = checks["paths." + path]["err_sampled"]
        line["oracle_checks_pass"] = all(c["err_sampled"] <= c["tol"] for c in checks.values())
    print(json.dumps(line))


if __name__ == "__main__":
    main()
