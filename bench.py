"""Sliding-window cumulant update throughput on one MI355X.

Workload: the regime-change stream at n=60 columns, d=4, b=4, window t=20000
rows, p=1000 rows per update (Gaussian rows first, Gaussian-copula rows with
Student-t(6)/Exp(1) marginals after step 100).  One step = one cum_update:
the signed moment contraction of orders 1..4 with its compensated fold, the
FP64 moment->cumulant combine of every order and the norms / nu_k, all on the
GPU, with the stream's rows already resident in HBM.

Prints one JSON line: rows/s of the main path (--prec, default fp32) as
`value`, the per-path figures (fp64, fp32, split-bf16x3) with their sampled
error against the FP64 oracle, the dominant kernel's roofline, and the
oracle's own throughput on the host cores (cpu_baseline).
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
TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


# HBM bytes per k_update launch at this workload from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE; mean over the sliding-update dispatches),
# each scaled by the ratio of known bytes to the same counter on a plain
# device copy.  Valid only for the kernel source they were taken on.
TRAFFIC = {"prec": "fp32",
           "kernels_sha256": "2f11412f710bb2cfd1325968bf0d5c17c9c56e7c66e24a6e172bffb96bb6c4ba",
           "fetch_bytes": 6095.99 * 1024 * 1.99988,   # FETCH_SIZE KiB x (256 MiB / 131078.5 KiB)
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


def sampled_error(ctx, window: np.ndarray, rng, count: int = 40):
    """Relative error of the GPU cumulants against the per-element FP64 oracle
    on sampled stored elements of orders 2..d (Frobenius over the sample)."""
    import paper_1701_06446_amd as cum
    from oracle.element import cumulant_at, sample_elements

    cache = {}
    worst = 0.0
    for k in range(2, D + 1):
        g = cum.cum_get(ctx, k)
        offs, idxs = sample_elements(N, B, k, count, rng)
        ref = np.array([cumulant_at(window, idx, cache) for idx in idxs])
        err = np.linalg.norm(g[offs] - ref) / max(np.linalg.norm(ref), 1e-300)
        worst = max(worst, float(err))
    return worst


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

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: HIP events on the context's stream bracket one update
    # kernel launch in EVENT_EVERY (each pair adds a gap of a few us)
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
        window = rows[w * P: w * P + T].astype(np.float64)
        out["err_sampled"] = sampled_error(ctx, window, np.random.default_rng(7))
        out["tol"] = TOL[prec]
    if mode == "fifo":
        out["fifo_slots"] = T // P
    cum.cum_free(ctx)
    del dev
    torch.cuda.empty_cache()
    return out


def run_batched(steps, warmup, prec="fp32", autotune=True):
    """64 uneven streams (n in 8..96, d in 3..4, t in 1000..20000, p = t/20)
    updated together by one captured graph; b per stream from the autotuner."""
    import torch

    import paper_1701_06446_amd as cum
    import streams
    from oracle.element import cumulant_at, sample_elements
    from paper_1701_06446_amd import autotune as at

    ss = streams.batched_streams(m=64, steps=warmup + steps)
    t0 = time.perf_counter()
    if autotune:
        cache = at.load_cache()
        for s in ss:
            s.b = at.choose_b(s.n, s.d, s.t, s.p, prec, cache=cache)
        at.save_cache(cache)
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
    t1 = time.perf_counter()
    for _ in range(steps):
        step()
    cum.cum_batch_sync(bt)
    el = time.perf_counter() - t1
    rows_per_step = sum(s.p for s in ss)
    flops = sum(2.0 * 2 * s.p * sum(cum.cum_num_elems(s.n, s.b, k) for k in range(1, s.d + 1)) for s in ss)
    flops_distinct = sum(2.0 * 2 * s.p * at.distinct_elements(s.n, s.d) for s in ss)
    rng = np.random.default_rng(5)
    worst = 0.0
    for i in range(0, 64, 8):
        s = ss[i]
        window = rows[i][w * s.p:w * s.p + s.t].astype(np.float64)
        cache = {}
        for k in range(2, s.d + 1):
            offs, idxs = sample_elements(s.n, s.b, k, 6, rng)
            ref = np.array([cumulant_at(window, idx, cache) for idx in idxs])
            g = cum.cum_get(ctxs[i], k)[offs]
            worst = max(worst, float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
    cum.cum_batch_free(bt)
    for c in ctxs:
        cum.cum_free(c)
    return {"streams": 64, "steps": steps, "warmup": warmup, "prec": prec,
            "rows_per_s": rows_per_step * steps / el, "updates_per_s": 64 * steps / el,
            "ms_per_step": el / steps * 1e3, "rows_per_step": rows_per_step,
            "tflops_algorithmic": flops * steps / el / 1e12,
            "tflops_distinct_elements": flops_distinct * steps / el / 1e12,
            "b_choice": {str(b): sum(1 for s in ss if s.b == b) for b in (1, 2, 4, 8)},
            "autotune_s": tune_s, "err_sampled_max": worst, "tol": TOL[prec]}


def run_order6(steps=4, warmup=1):
    """The order-6 workload: mixed Exp(1) sources, n=48, d=6, b=4, t=50000,
    p=2000, fp32 sliding mode; per-kernel times from the event profiler and
    the sampled error against the per-element FP64 oracle."""
    import torch

    import paper_1701_06446_amd as cum
    import streams
    from oracle.element import cumulant_at, sample_elements

    n, d, b, t, p = 48, 6, 4, 50000, 2000
    s = streams.mixed_exp_stream(steps=warmup + steps)
    rows = np.ascontiguousarray(s.rows.astype(np.float32))
    dev = torch.from_numpy(rows).to("cuda")
    t0 = time.perf_counter()
    ctx = cum.cum_init(n, d, b, dev[:t])
    init_s = time.perf_counter() - t0
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
    elems = [cum.cum_num_elems(n, b, k) for k in range(1, d + 1)]
    flops = 2.0 * 2 * p * sum(elems)
    upd_ms = prof["update"][1] / prof["update"][0]
    window = rows[w * p:w * p + t].astype(np.float64)
    rng = np.random.default_rng(17)
    cache, worst = {}, 0.0
    for k in range(2, d + 1):
        offs, idxs = sample_elements(n, b, k, 12, rng)
        ref = np.array([cumulant_at(window, idx, cache) for idx in idxs])
        worst = max(worst, float(np.linalg.norm(cum.cum_get(ctx, k)[offs] - ref) / np.linalg.norm(ref)))
    cum.cum_free(ctx)
    return {"workload": "mixed Exp(1) sources S W, n=48 d=6 b=4 t=50000 p=2000, fp32 sliding",
            "steps": steps, "ms_per_step": el / steps * 1e3, "rows_per_s": steps * p / el,
            "kernel_ms": {k: v[1] / v[0] for k, v in prof.items() if v[0]},
            "update_tflops": flops / (upd_ms * 1e-3) / 1e12, "update_frac_fp32_peak": flops / (upd_ms * 1e-3) / 1e12 / 157.3,
            "flops_per_update": flops, "stored_elements": sum(elems), "init_s": init_s,
            "err_sampled": worst, "tol": TOL["fp32"]}


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
    sums + Alg. 4 combine + Alg. 5 norms."""
    import oracle

    rows = s.rows.astype(np.float32).astype(np.float64)
    o = oracle.SlidingOracle(rows[:2000], N, D, B)
    n_steps, t0 = 0, time.perf_counter()
    while n_steps < 2 or (time.perf_counter() - t0 < budget_s and n_steps < 30):
        n_steps += 1
        lo, hi = (n_steps - 1) * P, n_steps * P
        o.update(rows[2000 + lo:2000 + hi], rows[lo:hi])
        oracle.norms(o.cumulants(), N, B)
    el = time.perf_counter() - t0
    return {"value": n_steps * P / el, "unit": "rows/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d sliding steps of p=1000 rows (n=60,d=4,b=4) from a 2000-row start window; "
                      "per step: FP64 compensated sums of orders 1..4, Alg.4 combine, Alg.5 norms; "
                      "%.1f s" % (n_steps, el)}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import streams

    total_steps = max(200, args.warmup + 2 * args.steps + 30)
    s = streams.regime_change_stream(n=N, d=D, b=B, t=T, p=P, steps=total_steps, switch=100)
    paths = [p for p in args.paths.split(",") if p and p != args.prec] + [args.prec]
    res = {}
    for prec in paths:
        print("[bench] path %s: warmup %d, %d timed steps" % (prec, args.warmup, args.steps),
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
    if not args.no_extra:
        print("[bench] order 6: n=48 d=6 b=4 p=2000", file=sys.stderr, flush=True)
        line["order6"] = run_order6()
        print("[bench] order 6: %.3f ms/step" % line["order6"]["ms_per_step"], file=sys.stderr, flush=True)
        print("[bench] adjoint", file=sys.stderr, flush=True)
        line["adjoint"] = run_adjoint()
    if not args.no_batched:
        print("[bench] batched: 64 streams, 40 steps", file=sys.stderr, flush=True)
        line["batched"] = run_batched(steps=40, warmup=3)
        print("[bench] batched: %.3f ms/step" % line["batched"]["ms_per_step"], file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
