#!/usr/bin/env python3
"""Benchmark of the low-precision GP solve on one MI355X.

Workload (mixed-precision solve): N = 100,000 points, d = 8, X ~ N(0, I)
column-standardised, right-hand sides [y, 15 Rademacher probes] (R = 16),
lengthscale 1, outputscale 1, noise 0.05; Matern-5/2 and RBF.  One step runs,
for each of the two kernels, the whole hot path: the rank-100 pivoted-Cholesky
preconditioner build and the enhanced-stability CG solve (binary16 fused
kernel-matrix product with float32 accumulation, logsumexp step sizes,
re-orthogonalisation, tolerance 1.0, at least 10 iterations) including the
float64 true residual at exit.  Inputs are resident in HBM before timing.

Printed metric: fused kernel-matrix-product entries (N^2 per product) per
second of whole-step wall time, in Gentries/s.  Alongside: the fused kernel's
own roofline (live per-launch HIP-event timing), time-to-tolerance of each
solve next to the standard float32 CG on the same GPU, and the float64 CPU
oracle's product rate on a bounded sample of rows.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak figures (MI355X public specification) used for roofline fractions.
PEAK_FP32_VECTOR_TFLOPS = 157.3      # 78.6 T FMA lane-ops/s
PEAK_FP16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# VALU issue slots per kernel entry in the fused product, counted in
# float32-FMA units: a transcendental (v_exp_f32, v_sqrt_f32) issues at a quarter
# of the FMA rate (4 slots); one packed float32->binary16 conversion covers two
# entries (0.5 slot).  RBF: exp2 + conversion.  Matern-5/2: sqrt + exp2 + two
# FMAs and one multiply for the polynomial + conversion.
VALU_SLOTS = {0: 4.0 + 0.5, 1: 4.0 + 4.0 + 3.0 + 0.5}
KIND_NAME = {0: "rbf", 1: "matern52"}

N, D, R, RANK = 100_000, 8, 16, 100

# HBM bytes per launch of the fused kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes on this workload, each scaled by the same counter's reading for a
# 1 GiB device copy (FETCH x2.0, WRITE x1.0), per column-split count (the
# split partial sums are most of the traffic); valid only for the kernel
# source they were measured on (sha256 prefix of csrc/kmvm_f16.hip +
# csrc/fused_tile.h).
MEASURED_TRAFFIC = {"kernel_sha256_prefix": "e17a539ada7a4e3b",
                    "bytes_per_launch_by_splits": {8: 112.2e6, 16: 163.5e6}}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the standard float32 CG comparator solves")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-problem batched measurement")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served-request measurement")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests replayed from the served stream (arrivals Exp(5 ms))")
    ap.add_argument("--no-training", action="store_true",
                    help="skip the hyperparameter-training measurement")
    ap.add_argument("--no-truncation", action="store_true",
                    help="skip the truncated-product measurement")
    ap.add_argument("--no-prediction", action="store_true",
                    help="skip the cached-prediction measurement")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the number-format (bfloat16, summation ablation) measurement")
    ap.add_argument("--part", choices=("batched", "serve", "serve-stream", "training", "truncation",
                                       "prediction", "precision"),
                    default=None,
                    help="run only this measurement and print its figures (for profiling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch-shape rules instead of measuring them first")
    ap.add_argument("--splits", type=int, default=None,
                    help="fix the column splits of the single-problem product instead of tuning them "
                         "(used to take the HBM counters per split count)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("kmvm_f16.hip", "fused_tile.h"):
        h.update(open(os.path.join(ROOT, "paper_2207_06856_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def product_splits(tuned, n):
    """Column splits the single-problem product uses at n rows under `tuned`
    (the built-in rule when the bucket holds 0)."""
    n_pad = -(-n // 256) * 256
    stages = -(-n // 128)
    b = 0
    while b + 1 < 8 and tuned["f16_bucket_rows"][b + 1] <= n_pad:
        b += 1
    s = tuned["f16_splits"][b]
    if s <= 0:
        want = -(-2048 // (n_pad // 256))
        s = min(64, -(-max(want, 8) // 8) * 8)
    return max(1, min(s, stages))


def measured_traffic(splits):
    if kernel_sha() != MEASURED_TRAFFIC["kernel_sha256_prefix"]:
        return None
    return MEASURED_TRAFFIC["bytes_per_launch_by_splits"].get(splits)


def batched_measurement(gpmi, torch, dev):
    """256 independent problems (N log-uniform in [500, 20000], d in {2..16},
    8 right-hand sides, RBF, per-problem lengthscale and noise, rank
    min(100, N/5) preconditioner, tol 1.0): one batched binary16 solve vs the
    standard float32 CG solved problem by problem on the same GPU."""
    import numpy as np
    from paper_2207_06856_amd import synth
    probs = synth.batched()
    dp = []
    for q in probs:
        dp.append(dict(X=torch.from_numpy(q.X).to(dev), B=torch.from_numpy(q.B).to(dev),
                       kind=q.kind, lengthscale=q.lengthscale, outputscale=q.outputscale,
                       noise=q.noise, precond_rank=min(100, q.n // 5)))
    outs = [torch.empty_like(p["B"]) for p in dp]
    entries_per_mvm = np.array([float(q.n) ** 2 for q in probs])
    gpmi.cg_solve_batched(dp, outs=outs)
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = gpmi.cg_solve_batched(dp, outs=outs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    ent = float(sum(e * s["mvms"] for e, s in zip(entries_per_mvm, st)))
    conv = all(bool(s["converged"].all()) for s in st)
    its = [int(s["iters"].max()) for s in st]
    # baseline: standard float32 CG one problem after another, same preconditioner rank
    t0 = time.perf_counter()
    its32 = []
    for p, U in zip(dp, outs):
        P = gpmi.Precond(p["X"], p["kind"], p["lengthscale"], p["outputscale"], p["noise"],
                         p["precond_rank"])
        _, s32 = gpmi.cg_solve(p["X"], p["B"], p["kind"], p["lengthscale"], p["outputscale"],
                               p["noise"], tol=1.0, max_iter=100, min_iter=10,
                               algo=gpmi.CG_STANDARD, precision=gpmi.FP32, precond=P, out=U)
        P.close()
        its32.append(int(s32["iters"].max()))
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    return {"problems": len(probs), "rows_total": int(sum(q.n for q in probs)),
            "batched_s": round(tb, 4), "batched_solves_per_s": round(len(probs) / tb, 1),
            "batched_gentries_per_s": round(ent / tb / 1e9, 1), "all_converged": conv,
            "iters_median": int(np.median(its)), "plain_fp32_sequential_s": round(t32, 4),
            "plain_fp32_iters_median": int(np.median(its32)),
            "speedup_vs_plain_fp32": round(t32 / tb, 2)}


def serve_measurement(gpmi, count):
    """Served request stream: Poisson arrivals at 200/s, N log-uniform in
    [1e3, 2e5], d in {4..12}, R in {1..32}, RBF or Matern-5/2, tol 1.0 or 0.1,
    rank-100 preconditioner, at most 100 iterations; arena 200 GB, 64 slots.
    The first `count` requests are replayed in real time from a submitter
    thread; latency is finish minus submit.  The same requests are then run
    through a one-slot server (one request at a time, same kernels) to show
    what continuous batching adds."""
    import threading

    import numpy as np
    from paper_2207_06856_amd import synth
    descs = synth.served_requests(count=count)
    probs = [synth.materialise(q) for q in descs]

    def run(slots, realtime, count=len(probs), stretch=1.0):
        with gpmi.Server(hbm_budget_bytes=200 * 10**9, max_slots=slots, iters_per_round=5) as srv:
            tickets = [None] * count

            def submitter():
                t0 = time.perf_counter()
                for i, (q, p) in enumerate(zip(descs[:count], probs[:count])):
                    if realtime:
                        dt = q["arrival_s"] * stretch - (time.perf_counter() - t0)
                        if dt > 0:
                            time.sleep(dt)
                    tickets[i] = srv.submit(p.X, p.B, p.kind, p.lengthscale, p.outputscale,
                                            p.noise, tol=q["tol"], max_iter=100, precond_rank=100)

            th = threading.Thread(target=submitter)
            w0 = time.perf_counter()
            th.start()
            th.join()
            res = [srv.wait(t) for t in tickets]
            wall = time.perf_counter() - w0
            st = srv.stats()
        return res, wall, st

    run(64, False, 16)   # warm-up: code objects, arena first touch
    res, wall, st = run(64, True)
    lat = np.array([r["t_finish"] - r["t_submit"] for r in res])
    span = max(r["t_finish"] for r in res) - min(r["t_submit"] for r in res)
    ok = sum(r["status"] == 0 for r in res)
    conv = sum(r["converged"] == len(r["col_iters"]) for r in res if r["status"] == 0)
    ent = float(sum(float(p.X.shape[0]) ** 2 * r["iters"] for p, r in zip(probs, res)))
    # light load: the first requests again, arrivals stretched to half the measured capacity
    light = min(len(probs), 48)
    stretch = light / (0.5 * (len(res) / span) * descs[light - 1]["arrival_s"])
    stretch = max(stretch, 1.0)
    resl, _, stl = run(64, True, light, stretch)
    latl = np.array([r["t_finish"] - r["t_submit"] for r in resl])
    res1, wall1, _ = run(1, False)
    span1 = max(r["t_finish"] for r in res1) - min(r["t_submit"] for r in res1)
    same = all(np.array_equal(a["U"], b["U"]) for a, b in zip(res, res1) if a["status"] == 0)
    # the first requests once more, all at once, against the standard float32 CG
    # solved one request after another on the same GPU (same tolerance,
    # preconditioner rank and iteration cap; inputs copied to the device per
    # request, as the server does at admission)
    import torch
    cmp_n = min(16, len(probs))
    resc, _, _ = run(64, False, cmp_n)
    spanc = max(r["t_finish"] for r in resc) - min(r["t_submit"] for r in resc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, p in zip(descs[:cmp_n], probs[:cmp_n]):
        X = torch.from_numpy(p.X).to("cuda:0")
        B = torch.from_numpy(p.B).to("cuda:0")
        P = gpmi.Precond(X, p.kind, p.lengthscale, p.outputscale, p.noise, min(100, p.X.shape[0]))
        gpmi.cg_solve(X, B, p.kind, p.lengthscale, p.outputscale, p.noise, tol=q["tol"],
                      max_iter=100, min_iter=10, algo=gpmi.CG_STANDARD, precision=gpmi.FP32,
                      precond=P)
        P.close()
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    return {"requests": len(res), "offered_per_s": round(len(res) / descs[-1]["arrival_s"], 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "solves_per_s": round(len(res) / span, 1),
            "gentries_per_s": round(ent / span / 1e9, 1),
            "utilisation": round(st["busy_seconds"] / st["uptime_seconds"], 3),
            "status_ok": int(ok), "all_columns_converged": int(conv),
            "peak_arena_gb": round(st["peak_bytes"] / 1e9, 2),
            "light_load": {"requests": light,
                           "offered_per_s": round(light / (descs[light - 1]["arrival_s"] * stretch), 2),
                           "p50_ms": round(float(np.percentile(latl, 50)) * 1e3, 2),
                           "p99_ms": round(float(np.percentile(latl, 99)) * 1e3, 2),
                           "utilisation": round(stl["busy_seconds"] / stl["uptime_seconds"], 3)},
            "one_slot_solves_per_s": round(len(res1) / span1, 1),
            "speedup_vs_one_slot": round(span1 / span, 2),
            "results_equal_one_slot": bool(same),
            "plain_fp32_comparison": {"requests": cmp_n,
                                      "served_s": round(spanc, 3),
                                      "plain_fp32_sequential_s": round(t32, 3),
                                      "speedup_vs_plain_fp32": round(t32 / spanc, 2)}}


def serve_stream_measurement(gpmi, count, progress_s=30.0):
    """The served configuration at full length: `count` requests (10,000) of
    the served stream replayed at their Poisson arrival times into a 64-slot
    server with a 200 GB arena.  Inputs are drawn just in time by the
    submitter thread (a request's host arrays live from its arrival until its
    result is read), results are read as they finish, and a progress line goes
    to stderr every `progress_s` seconds.  Reports latency percentiles (finish
    minus submit), solves/s over the span, the offered rate actually achieved
    by the submitter and the status counts."""
    import collections
    import queue
    import threading

    import numpy as np
    from paper_2207_06856_amd import synth
    descs = synth.served_requests(count=count)
    rows = []                                       # (t_submit, t_admit, t_finish, status, conv, n, iters)
    t_last_submit = [0.0]
    with gpmi.Server(hbm_budget_bytes=200 * 10**9, max_slots=64, iters_per_round=5) as srv:
        sub_q = queue.Queue()

        def submitter():
            t0 = time.perf_counter()
            for q in descs:
                dt = q["arrival_s"] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                p = synth.materialise(q)
                sub_q.put((p.X.shape[0], srv.submit(p.X, p.B, p.kind, p.lengthscale,
                                                    p.outputscale, p.noise, tol=q["tol"],
                                                    max_iter=100, precond_rank=100)))
            t_last_submit[0] = time.perf_counter() - t0
            sub_q.put(None)

        th = threading.Thread(target=submitter)
        w0 = time.perf_counter()
        th.start()
        outstanding = collections.deque()
        submitted_all = False
        last = w0
        while not (submitted_all and not outstanding):
            while True:
                try:
                    item = sub_q.get_nowait()
                except queue.Empty:
                    break
                if item is None:
                    submitted_all = True
                else:
                    outstanding.append(item)
            if outstanding:
                n, t = outstanding[0]
                r = srv.wait(t, timeout_ms=50)
                if r is not None:
                    outstanding.popleft()
                    conv = r["status"] == 0 and r["converged"] == len(r["col_iters"])
                    rows.append((r["t_submit"], r["t_admit"], r["t_finish"], r["status"], conv, n,
                                 r["iters"]))
            else:
                time.sleep(0.01)
            now = time.perf_counter()
            if now - last >= progress_s:
                print(f"serve-stream: {len(rows)}/{count} finished, {len(outstanding)} read-pending,"
                      f" {now - w0:.0f} s", file=sys.stderr, flush=True)
                last = now
        th.join()
        st = srv.stats()
    a = np.array([(r[0], r[1], r[2]) for r in rows])
    lat = a[:, 2] - a[:, 0]
    span = a[:, 2].max() - a[:, 0].min()
    ok = sum(r[3] == 0 for r in rows)
    ent = float(sum(float(r[5]) ** 2 * r[6] for r in rows if r[3] == 0))
    return {"requests": len(rows), "offered_per_s_schedule": round(count / descs[-1]["arrival_s"], 1),
            "offered_per_s_achieved": round(count / t_last_submit[0], 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
            "p50_queue_ms": round(float(np.percentile(a[:, 1] - a[:, 0], 50)) * 1e3, 1),
            "solves_per_s": round(len(rows) / span, 2), "span_s": round(span, 1),
            "gentries_per_s": round(ent / span / 1e9, 1),
            "utilisation": round(st["busy_seconds"] / st["uptime_seconds"], 3),
            "status_ok": int(ok), "all_columns_converged": int(sum(r[4] for r in rows)),
            "peak_arena_gb": round(st["peak_bytes"] / 1e9, 2)}


# Work per evaluated entry of the gradient reduction, in the convention of
# VALU_SLOTS (float32-FMA issue slots, a transcendental counts 4, 2 flops a
# slot against the 157.3 TFLOP/s vector peak): per input dimension a
# difference, a square and the accumulation (3 slots; an isotropic lengthscale
# needs none); the RBF value (exp2 with its argument, 5); the unscaled W entry,
# kappa W, G W, the clamp of r^2 (4).  The squared distance is a float32
# matrix-core product of (d + 4)-long augmented vectors, 2 (d + 4) flops that
# run at the same float32 rate and do not overlap the vector work; the W tiles
# come from the binary16 matrix cores, which do, and are not counted.  With the
# symmetric tiling an entry (i, j) past the diagonal block stands for (j, i) as
# well, so about half of the N^2 logical entries are evaluated.
def grad_flops_per_entry(d, ard=True):
    dm = 4 if d <= 4 else 8 if d <= 8 else 16 if d <= 16 else 32
    slots = (3 * dm if ard else 0) + 5 + 4
    return 2 * slots + 2 * (dm + 4)


def grad_evaluated_entries(n, d):
    rb = 128 if d <= 16 else 64
    stages = -(-n // 64)
    total = 0
    for b in range(-(-n // rb)):
        total += (stages - (b * rb) // 64) * 64 * rb
    return float(total)


def training_measurement(gpmi, torch, dev, steps=8):
    """Hyperparameter training as in App. C: N = 100,000, d = 8 standardised
    synthetic regression data, RBF with ARD, 15 Rademacher probes, rank-100
    preconditioner rebuilt every step, binary16 product, CG tolerance 1.0
    (10 to 50 iterations), Gamma priors, Adam 0.1.  One training step = probes,
    preconditioner, mBCG solve, Eq. (approx) gradient, Adam update.  The
    gradient reduction is timed on its own with HIP events on the stream it
    runs on (the float64 oracle's gradient is timed by cpu_baseline_training)."""
    import numpy as np

    from paper_2207_06856_amd import synth
    n, d, M = 100_000, 8, 15
    X, y = synth.training(n=n, d=d)
    Xd = torch.from_numpy(X).to(dev)
    yd = torch.from_numpy(y).to(dev)
    with gpmi.Trainer(Xd, yd, probes=M, precond_rank=RANK, seed=1) as t:
        t.step()                                  # warm-up (code objects, workspace)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(t.step())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        B, U = t.blocks()
        theta = t.state()["theta"]
    # the gradient reduction alone, on the last step's blocks
    ls = theta[:d].astype(np.float32)
    a2 = float(theta[d])
    for _ in range(2):
        gpmi.mll_grad(Xd, B, U, gpmi.RBF, ls, a2, 1.0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 5
    ev[0].record()
    for _ in range(reps):
        gpmi.mll_grad(Xd, B, U, gpmi.RBF, ls, a2, 1.0)
    ev[1].record()
    torch.cuda.synchronize()
    grad_ms = ev[0].elapsed_time(ev[1]) / reps
    entries = float(n) * float(n)
    evaluated = grad_evaluated_entries(n, d)
    tflops = evaluated * grad_flops_per_entry(d) / (grad_ms / 1e3) / 1e12
    sec = lambda k: float(np.median([i[k] for i in infos]) * 1e3)
    return {"workload": f"App. C training: N={n}, d={d}, RBF-ARD, {M} probes, rank {RANK}, "
                        "binary16 product, CG tol 1.0 (10..50 iterations), priors, Adam 0.1",
            "steps": steps, "ms_per_step": round(wall / steps * 1e3, 2),
            "steps_per_s": round(steps / wall, 2),
            "median_ms": {"precond": round(sec("seconds_precond"), 2),
                          "solve": round(sec("seconds_solve"), 2),
                          "grad_and_adam": round(sec("seconds_grad"), 2)},
            "cg_iters_median": int(np.median([i["cg_iters"] for i in infos])),
            "theta_after": [round(float(v), 4) for v in theta],
            "grad_kernel": {"avg_ms": round(grad_ms, 3),
                            "logical_gentries_per_s": round(entries / (grad_ms / 1e3) / 1e9, 1),
                            "evaluated_entries": evaluated,
                            "bound": "alu", "achieved_tflops": round(tflops, 2),
                            "peak_tflops": PEAK_FP32_VECTOR_TFLOPS,
                            "frac": round(tflops / PEAK_FP32_VECTOR_TFLOPS, 4),
                            "flops_per_evaluated_entry": grad_flops_per_entry(d)}}


def truncation_measurement(gpmi, torch, dev, reps=3):
    """Truncated binary16 product (Sec. 4.1, Fig. 2c) on the support workload:
    N = 1,000,000 points uniform in [-10, 10]^2, RBF l = 1, R = 16 right-hand
    sides, K~ V with the noise term.  Times (HIP events, mean of `reps` calls)
    of gp_kmvm (caller's order, every tile), gp_kmvm_truncated without
    skipping (Z-order, every tile) and with skipping; outputs of the last two
    compared bit for bit."""
    from paper_2207_06856_amd import synth
    p = synth.compact_support()
    X = torch.from_numpy(p.X).to(dev)
    B = torch.from_numpy(p.B).to(dev)
    ls, a2, s2 = p.lengthscale, p.outputscale, p.noise

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            out = fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps, out

    t_full, _ = timed(lambda: gpmi.kmvm(X, X, B, 0, ls, a2, s2, add_noise=True))
    t_noskip, o0 = timed(lambda: gpmi.kmvm_truncated(X, X, B, 0, ls, a2, s2, add_noise=True, skip=False))
    t_skip, o1 = timed(lambda: gpmi.kmvm_truncated(X, X, B, 0, ls, a2, s2, add_noise=True, skip=True))
    _, st = gpmi.kmvm_truncated(X, X, B, 0, ls, a2, s2, add_noise=True, skip=True, stats=True)
    n = float(p.n)
    return {"workload": "K~V, N=1000000 uniform in [-10,10]^2, RBF l=1, R=16 (binary16)",
            "full_ms": round(t_full, 3), "ordered_no_skip_ms": round(t_noskip, 3),
            "truncated_ms": round(t_skip, 3), "speedup_vs_full": round(t_full / t_skip, 2),
            "tiles_visited_frac": round(st["tiles_visited"] / st["tiles_total"], 4),
            # the visited share of the full product's time over the truncated time
            "efficiency_vs_visited_share": round(st["tiles_visited"] / st["tiles_total"] * t_full
                                                 / t_skip, 3),
            "radius": round(st["radius"], 4),
            "logical_gentries_per_s": round(n * n / (t_skip / 1e3) / 1e9, 1),
            "bit_identical_to_no_skip": bool(torch.equal(o0, o1))}


def prediction_measurement(gpmi, torch, dev, reps=3, served=240):
    """Predictive means with a cached solve (Sec. 4.1): the cache
    v = K~^{-1} y of the mixed-precision workload (N = 100,000, d = 8, RBF
    l = 1, s^2 = 0.05, rank-100 preconditioner, binary16 CG to tol 1e-2), then
    mu = a^2 K(x*, X) v for 100,000 test points from the same distribution
    (binary16, float32 and truncated products; HIP events, mean of `reps`).
    Served: `served` prediction requests of 1,000 points (Poisson arrivals at
    400/s) replayed in real time into a server that is also running 24 solve
    requests of the served stream; latency = finish - submit."""
    import threading

    import numpy as np
    from paper_2207_06856_amd import synth
    p = synth.mixed_precision(n=N, kind=0)
    X = torch.from_numpy(p.X).to(dev)
    y = torch.from_numpy(np.ascontiguousarray(p.B[:, 0])).to(dev)
    g = np.random.default_rng(17)
    Xs_h = g.standard_normal((100_000, D)).astype(np.float32)
    Xs = torch.from_numpy(Xs_h).to(dev)
    torch.cuda.synchronize()
    a = time.perf_counter()
    m = gpmi.Model(X, y, 0, p.lengthscale, 1.0, p.noise, precond_rank=RANK)
    t_model = time.perf_counter() - a
    info = m.info()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    t16 = timed(lambda: m.predict(Xs))
    t32 = timed(lambda: m.predict(Xs, precision=gpmi.FP32))
    tt = timed(lambda: m.predict(Xs, truncate=True))
    ent = float(N) * 100_000.0
    # served predictions beside solves
    arrivals = np.cumsum(g.exponential(1.0 / 400.0, size=served))
    chunks = [Xs_h[(i * 1000) % 99_000:(i * 1000) % 99_000 + 1000] for i in range(served)]
    solves = [synth.materialise(q) for q in synth.served_requests(count=24)]
    with gpmi.Server(hbm_budget_bytes=100 * 10**9, max_slots=32, iters_per_round=5) as srv:
        tickets = [None] * served
        stickets = []

        def submitter():
            t0 = time.perf_counter()
            for q in solves:
                stickets.append(srv.submit(q.X, q.B, q.kind, q.lengthscale, q.outputscale, q.noise,
                                           tol=1.0, max_iter=100, precond_rank=100))
            for i in range(served):
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit_predict(m, chunks[i])

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        res = [srv.wait(t) for t in tickets]
        sres = [srv.wait(t) for t in stickets]
    m.close()
    lat = np.array([r["t_finish"] - r["t_submit"] for r in res])
    return {"workload": "cache: N=100000, d=8, RBF l=1, s2=0.05, rank 100, binary16 CG tol 1e-2; "
                        "100000 test points",
            "cache_solve_s": round(t_model, 3), "cache_iters": info["iters"],
            "cache_true_rel_res": round(info["true_rel_res"], 5),
            "predict_fp16_ms": round(t16, 3), "predict_fp32_ms": round(t32, 3),
            "predict_truncated_ms": round(tt, 3),
            "predict_fp16_gentries_per_s": round(ent / (t16 / 1e3) / 1e9, 1),
            "predictions_per_s_fp16": round(100_000 / (t16 / 1e3), 0),
            "served": {"requests": served, "points_per_request": 1000, "offered_per_s": 400,
                       "with_solves": len(solves),
                       "status_ok": int(sum(r["status"] == 0 for r in res)),
                       "solves_ok": int(sum(r["status"] == 0 for r in sres)),
                       "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2)}}


def precision_measurement(gpmi, torch, dev, reps=3):
    """Number-format variants on the mixed-precision workload (N = 100,000,
    d = 8, l = 1, s^2 = 0.05): K~V for R = 16 with binary16 and bfloat16
    operands (HIP events, mean of `reps`), the binary16 summation ablations
    (blocks of 32 summed in half or single, Kahan in half; paper's
    n^(-1/2) scale) for R = 1, each product's mean relative error against the
    float32 product on the same GPU (the comparison of Fig. 4b), and the
    bfloat16 CG solve (rank-100 preconditioner, tol 1.0) next to binary16's."""
    import numpy as np
    from paper_2207_06856_amd import synth

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            out = fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps, out

    def mean_rel(a, ref):
        a = a.double()
        ref = ref.double()
        return float((a - ref).abs().mean() / ref.abs().mean())

    res = {}
    ent = float(N) * float(N)
    for kind in (1, 0):
        p = synth.mixed_precision(n=N, kind=kind)
        X = torch.from_numpy(p.X).to(dev)
        B = torch.from_numpy(p.B).to(dev)
        y = B[:, :1].contiguous()
        ls, a2, s2 = p.lengthscale, p.outputscale, p.noise
        k = {}
        t, ref16 = timed(lambda: gpmi.kmvm(X, X, B, kind, ls, a2, s2, add_noise=True,
                                            precision=gpmi.FP32))
        k["fp32_r16_ms"] = round(t, 3)
        t, o16 = timed(lambda: gpmi.kmvm(X, X, B, kind, ls, a2, s2, add_noise=True))
        k["fp16_r16_ms"] = round(t, 3)
        k["fp16_r16_mean_rel_err"] = round(mean_rel(o16, ref16), 7)
        t, ob = timed(lambda: gpmi.kmvm(X, X, B, kind, ls, a2, s2, add_noise=True,
                                        precision=gpmi.BF16))
        k["bf16_r16_ms"] = round(t, 3)
        k["bf16_r16_gentries_per_s"] = round(ent / (t / 1e3) / 1e9, 1)
        # same vector-ALU slot model as the binary16 product (whole call incl.
        # quantisation and reduction, so a lower bound on the kernel's own)
        k["bf16_r16_valu_frac"] = round(ent * VALU_SLOTS[kind] * 2 / (t / 1e3) / 1e12
                                        / PEAK_FP32_VECTOR_TFLOPS, 4)
        k["bf16_r16_mean_rel_err"] = round(mean_rel(ob, ref16), 7)
        _, ref1 = timed(lambda: gpmi.kmvm(X, X, y, kind, ls, a2, s2, precision=gpmi.FP32))
        t, o = timed(lambda: gpmi.kmvm(X, X, y, kind, ls, a2, s2))
        k["fp16_r1_ms"] = round(t, 3)
        k["fp16_r1_mean_rel_err"] = round(mean_rel(o, ref1), 7)
        for name, sch in (("block_half", gpmi.SUM_BLOCK_HALF), ("block_single", gpmi.SUM_BLOCK_SINGLE),
                          ("kahan_half", gpmi.SUM_KAHAN_HALF)):
            t, o = timed(lambda: gpmi.kmvm_summation(X, X, y, kind, ls, a2, s2, sch, block=32))
            k[f"{name}_r1_ms"] = round(t, 3)
            k[f"{name}_r1_gentries_per_s"] = round(ent / (t / 1e3) / 1e9, 1)
            k[f"{name}_r1_mean_rel_err"] = round(mean_rel(o, ref1), 7)
        for prec, nm in ((gpmi.FP16, "fp16"), (gpmi.BF16, "bf16")):
            P = gpmi.Precond(X, kind, ls, a2, s2, RANK)
            torch.cuda.synchronize()
            a = time.perf_counter()
            _, st = gpmi.cg_solve(X, B, kind, ls, a2, s2, tol=1.0, max_iter=100, min_iter=10,
                                  precision=prec, precond=P)
            torch.cuda.synchronize()
            k[f"cg_{nm}_ms"] = round((time.perf_counter() - a) * 1e3, 2)
            k[f"cg_{nm}_iters"] = int(st["iters"].max())
            k[f"cg_{nm}_true_rel_res_max"] = round(float(st["true_rel_res"].max()), 5)
            P.close()
        res[KIND_NAME[kind]] = k
    res["workload"] = ("K~V, N=100000, d=8, l=1, s2=0.05 (mixed-precision workload); R=16 for the "
                       "matrix-core formats, R=1 (y) for the summation ablations, blocks of 32")
    return res


def _timed_oracle(fn):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        a = time.perf_counter()
        fn()
        return time.perf_counter() - a


def cpu_baseline_training(rows=96):
    """float64 oracle Eq. (approx) gradient on sampled rows of the training
    workload (one BLAS thread).  U and B are synthetic blocks of the solve's
    shape: the oracle's time does not depend on their values."""
    import numpy as np

    from oracle import train as otrain
    from paper_2207_06856_amd import synth
    n, d, M = 100_000, 8, 15
    X, y = synth.training(n=n, d=d)
    g = np.random.default_rng(3)
    B = np.concatenate([y[:, None], g.choice([-1.0, 1.0], (n, M))], axis=1)
    U = g.standard_normal((n, M + 1))
    ls = np.full(d, np.log(2.0))
    dt = _timed_oracle(lambda: otrain.pseudo_loss_grad(X, U, B, 0, ls, float(np.log(2.0)), True,
                                                       rows=np.arange(rows)))
    return {"value": round(rows * n / dt / 1e9, 4), "unit": "Gentries/s", "cores": 1,
            "kind": "oracle", "sample": f"Eq. (approx) gradient, {rows} rows x {n} columns, "
                                        f"RBF-ARD d={d}, float64 ({dt:.1f} s)"}


def cpu_baseline_truncation(rows=64):
    """float64-emulated truncated binary16 product of the oracle on sampled
    rows of the support workload (one BLAS thread)."""
    import numpy as np

    from oracle import support
    from paper_2207_06856_amd import synth
    p = synth.compact_support()
    sel = np.random.default_rng(4).choice(p.n, rows, replace=False)
    dt = _timed_oracle(lambda: support.kmvm_fp16_truncated(p.X[sel], p.X, p.B, 0, p.lengthscale,
                                                            p.outputscale, p.noise, False))
    return {"value": round(rows * p.n / dt / 1e9, 4), "unit": "Gentries/s (logical)", "cores": 1,
            "kind": "oracle", "sample": f"truncated binary16 emulation, {rows} sampled rows x "
                                        f"{p.n} columns x 16 right-hand sides ({dt:.1f} s)"}


def cpu_baseline_prediction(rows=512):
    """float64 oracle mean product a^2 K(x*, X) v for sampled test points of
    the prediction workload (one BLAS thread); the cache solve itself (a dense
    Cholesky of order 100,000) is beyond a bounded CPU sample.  v is synthetic:
    the time does not depend on its values."""
    import numpy as np

    from oracle import kmvm as okmvm
    from paper_2207_06856_amd import synth
    p = synth.mixed_precision(n=N, kind=0)
    g = np.random.default_rng(17)
    Xs = g.standard_normal((rows, D))
    v = g.standard_normal((N, 1))
    dt = _timed_oracle(lambda: okmvm.kmvm(Xs, p.X, v, 0, p.lengthscale, 1.0, p.noise, False))
    return {"value": round(rows * N / dt / 1e9, 4), "unit": "Gentries/s", "cores": 1,
            "kind": "oracle", "sample": f"predictive-mean product, {rows} test points x {N} "
                                        f"training points, float64 ({dt:.1f} s)"}


def cpu_baseline_precision(rows=256, sum_rows=16):
    """The oracle's bfloat16 emulation (R = 16) and binary16 summation schemes
    (R = 1, blocks of 32) on sampled rows of the mixed-precision workload (RBF,
    one BLAS thread)."""
    import numpy as np

    from oracle import precision as oprec
    from paper_2207_06856_amd import synth
    p = synth.mixed_precision(n=N, kind=0)
    sel = np.random.default_rng(5).choice(N, rows, replace=False)
    res = {}
    dt = _timed_oracle(lambda: oprec.kmvm_bf16_emulated(p.X, p.X, p.B, 0, p.lengthscale, 1.0,
                                                         p.noise, True, rows=sel))
    res["bf16_r16"] = {"value": round(rows * N / dt / 1e9, 4), "unit": "Gentries/s",
                       "sample": f"{rows} rows x {N} columns x 16 right-hand sides ({dt:.1f} s)"}
    sel = sel[:sum_rows]
    y = p.B[:, :1].copy()
    for scheme in oprec.SCHEMES:
        dt = _timed_oracle(lambda: oprec.kmvm_fp16_summation(p.X, p.X, y, 0, p.lengthscale, 1.0,
                                                             p.noise, True, scheme, block=32,
                                                             rows=sel))
        res[scheme + "_r1"] = {"value": round(sum_rows * N / dt / 1e9, 6), "unit": "Gentries/s",
                               "sample": f"{sum_rows} rows x {N} columns ({dt:.1f} s)"}
    return {"cores": 1, "kind": "oracle", **res}


def cpu_baseline(p, rows_per_kind=3072):
    """float64 oracle product on sampled rows (BLAS limited to one thread)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import kmvm as okmvm
    from paper_2207_06856_amd import synth
    rng = np.random.default_rng(0)
    rows = rng.choice(p.n, rows_per_kind, replace=False)
    total_entries = 0.0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for kind in (1, 0):
            q = synth.mixed_precision(n=N, kind=kind)
            okmvm.kmvm(q.X, q.X, q.B, kind, q.lengthscale, q.outputscale, q.noise, True, rows=rows)
            total_entries += rows.size * float(p.n)
    dt = time.perf_counter() - t0
    return {"value": total_entries / dt / 1e9, "unit": "Gentries/s", "cores": 1, "kind": "oracle",
            "sample": f"float64 oracle product, {rows_per_kind} sampled output rows x {p.n} "
                      f"columns x {R} right-hand sides, Matern-5/2 and RBF ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solve is "
              "single-GPU by design and no multi-GPU path is built", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_2207_06856_amd import gpmi, synth

    dev = "cuda:0"
    if args.copy_calibration:
        src = torch.ones(1 << 28, device=dev)          # 1 GiB of float32
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
        return 0
    if args.part is not None and not args.no_autotune:
        gpmi.autotune(max_bucket=5)
    if args.part == "batched":
        print(json.dumps({"batched": batched_measurement(gpmi, torch, dev)}), flush=True)
        return 0
    if args.part == "serve":
        print(json.dumps({"serve": serve_measurement(gpmi, args.serve_requests)}), flush=True)
        return 0
    if args.part == "serve-stream":
        print(json.dumps({"serve_stream": serve_stream_measurement(gpmi, args.serve_requests)}),
              flush=True)
        return 0
    part_cpu = {"training": cpu_baseline_training, "truncation": cpu_baseline_truncation,
                "prediction": cpu_baseline_prediction, "precision": cpu_baseline_precision}
    part_fn = {"training": training_measurement, "truncation": truncation_measurement,
               "prediction": prediction_measurement, "precision": precision_measurement}
    if args.part in part_fn:
        res = part_fn[args.part](gpmi, torch, dev)
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = part_cpu[args.part]()
        print(json.dumps({args.part: res}), flush=True)
        return 0
    # launch shapes of the binary16 product from the autotuner (outside every timed region)
    if args.splits is not None:
        gpmi.tune_set(f16_splits=[args.splits] * 8)
        tuned = gpmi.tune_info()
    else:
        tuned = gpmi.autotune(max_bucket=5) if not args.no_autotune else gpmi.tune_info()
    probs = {kind: synth.mixed_precision(n=N, kind=kind) for kind in (1, 0)}
    p0 = probs[1]
    X = torch.from_numpy(p0.X).to(dev)
    B = torch.from_numpy(p0.B).to(dev)
    U = torch.empty_like(B)
    torch.cuda.synchronize()

    def solve(kind, algo=gpmi.CG_ENHANCED, precision=gpmi.FP16):
        p = probs[kind]
        P = gpmi.Precond(X, kind, p.lengthscale, p.outputscale, p.noise, RANK)
        _, st = gpmi.cg_solve(X, B, kind, p.lengthscale, p.outputscale, p.noise, tol=1.0,
                              max_iter=100, min_iter=10, algo=algo, precision=precision,
                              precond=P, out=U, true_res_every=0)
        P.close()
        return st

    def step():
        return {kind: solve(kind) for kind in (1, 0)}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gpmi.profile_reset()
    gpmi.profile_enable(True)
    t0 = time.perf_counter()
    per_solve_ms = {1: [], 0: []}
    stats = []
    for _ in range(args.steps):
        for kind in (1, 0):
            a = time.perf_counter()
            st = solve(kind)
            per_solve_ms[kind].append((time.perf_counter() - a) * 1e3)
            stats.append((kind, st))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gpmi.profile_enable(False)
    ms, ent, kinds = gpmi.profile_read()
    gpmi.profile_reset()

    wall = t1 - t0
    entries_total = float(sum(st["mvms"] for _, st in stats)) * float(N) * float(N)
    value = entries_total / wall / 1e9
    # working launches (a launch after every column froze exits at once)
    work = ms > 0.05 * np.median(ms)
    roof = {}
    for kind in (1, 0):
        m = work & (kinds == kind)
        dur = ms[m].mean() / 1e3
        e = ent[m].mean()
        roof[kind] = dict(avg_ms=ms[m].mean(), gentries=e / dur / 1e9,
                          valu_tflops=e * VALU_SLOTS[kind] * 2 / dur / 1e12,
                          mfma_alg_tflops=e * (2 * D + 2 * R) / dur / 1e12, launches=int(m.sum()))
    # dominant kernel: the product launches of the whole step, both kernel kinds
    tot_dur = ms[work].sum() / 1e3
    valu_work = sum(ent[work & (kinds == k)].sum() * VALU_SLOTS[k] * 2 for k in (1, 0))
    achieved = valu_work / tot_dur / 1e12
    product_share = tot_dur / wall

    # comparators outside the timed region: standard CG with the float32 product
    cmp = {kind: dict(ms=float("nan"), iters=-1, converged=False) for kind in (1, 0)}
    for kind in ((1, 0) if not args.no_compare else ()):
        solve(kind)
        torch.cuda.synchronize()
        a = time.perf_counter()
        st32 = solve(kind, algo=gpmi.CG_STANDARD, precision=gpmi.FP32)
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - a) * 1e3
        cmp[kind] = dict(ms=t32, iters=int(st32["iters"].max()),
                         converged=bool(st32["converged"].all()))

    last = {k: st for k, st in stats}
    detail = {}
    for kind in (1, 0):
        st = last[kind]
        t = float(np.median(per_solve_ms[kind]))
        detail[KIND_NAME[kind]] = dict(
            time_to_tol_ms=round(t, 3), iters=int(st["iters"].max()),
            converged=bool(st["converged"].all()),
            true_rel_res_max=float(st["true_rel_res"].max()),
            plain_fp32_time_to_tol_ms=round(cmp[kind]["ms"], 3),
            plain_fp32_iters=cmp[kind]["iters"],
            speedup_vs_plain_fp32=(round(cmp[kind]["ms"] / t, 3)
                                   if cmp[kind]["iters"] >= 0 else None),
            kmvm_avg_ms=round(roof[kind]["avg_ms"], 4),
            kmvm_gentries_per_s=round(roof[kind]["gentries"], 1),
            kmvm_valu_frac=round(roof[kind]["valu_tflops"] / PEAK_FP32_VECTOR_TFLOPS, 4),
            kmvm_mfma_alg_frac=round(roof[kind]["mfma_alg_tflops"] / PEAK_FP16_MFMA_TFLOPS, 4))

    out = {
        "metric": "fused kernel-MVM Gentries/s; CG time-to-tol vs plain FP32; serve p50/p99",
        "value": round(value, 2),
        "unit": "Gentries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "mixed-precision CG: N=100000, d=8, R=16 (y + 15 Rademacher "
                               "probes), Matern-5/2 and RBF, l=1, noise 0.05, rank-100 pivoted "
                               "Cholesky, tol 1.0, min 10 / max 100 iterations",
                   "n": N, "d": D, "r": R, "precond_rank": RANK, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": measured_traffic(product_splits(tuned, N)),
                     "column_splits": product_splits(tuned, N),
                     "kernel": "kmvm_f16_main", "product_share_of_step": round(product_share, 4)},
        "solves": detail,
        "autotune": tuned,
    }
    if not args.no_batched:
        out["batched"] = batched_measurement(gpmi, torch, dev)
    if not args.no_serve:
        out["serve"] = serve_measurement(gpmi, args.serve_requests)
    if not args.no_training:
        out["training"] = training_measurement(gpmi, torch, dev)
    if not args.no_truncation:
        out["truncation"] = truncation_measurement(gpmi, torch, dev)
    if not args.no_prediction:
        out["prediction"] = prediction_measurement(gpmi, torch, dev)
    if not args.no_precision:
        out["precision"] = precision_measurement(gpmi, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p0)
        for name, fn in part_cpu.items():
            if name in out:
                out[name]["cpu_baseline"] = fn()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
