#!/usr/bin/env python3
"""Benchmark of the low-precision GP solve on one MI355X.

Headline workload (large single problem): N = 1,800,000 points, d = 11,
X ~ N(0, I) with three correlated pairs, right-hand sides [y, 15 Rademacher
probes] (R = 16), RBF lengthscale 1.5, outputscale 1, noise 0.01, rank-100
pivoted-Cholesky preconditioner, enhanced-stability CG (binary16 fused
kernel-matrix product with float32 accumulation, logsumexp step sizes,
re-orthogonalisation).  One step is one CG iteration of that solve: the fused
product, the logsumexp dots, the x / r update, the CGS2 re-orthogonalisation
(one coefficient and one update sweep through the basis Gram matrix), the
preconditioner apply, the direction and its binary16 requantisation.  K timed steps are one solve of exactly K iterations (after a
warm-up solve of W iterations); the preconditioner build and the float64 true
residual are timed separately and reported beside it.  Inputs are resident in
HBM before timing.

Printed metric: fused kernel-matrix-product entries (N^2 per iteration) per
second of wall time, in Gentries/s.  Alongside: the fused kernel's roofline
(live per-launch HIP-event timing; algorithmic binary16 matrix-core FLOP over
the matrix-core peak, and the vector-issue share of the kernel values at the
probed instruction rates), the chip probes, time-to-tolerance of the
100,000-point mixed-precision solves next to the standard float32 CG on the
same GPU, and the float64 CPU oracle's product rate on a bounded sample of
rows on all host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak figures used for roofline fractions: MI355X's published dense
# matrix-core and HBM figures.  Vector-unit figures are the probed issue rates
# (peaks_measurement) and the unit-count ceiling without packed FP32 (every
# source is built with packed FP32 disabled).
PEAK_FP16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
KIND_NAME = {0: "rbf", 1: "matern52"}

N, D, R, RANK = 100_000, 8, 16, 100          # mixed-precision solves (secondary)
NL, DL = 1_800_000, 11                        # headline: the large single problem

# HBM bytes per launch of the fused kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes on this workload, each scaled by the same counter's reading for a
# 1 GiB device copy (FETCH x2.0, WRITE x1.0), per column-split count (the
# split partial sums are most of the traffic); valid only for the kernel
# source they were measured on (sha256 prefix of csrc/kmvm_f16.hip +
# csrc/fused_tile.h).
MEASURED_TRAFFIC = {"kernel_sha256_prefix": "e17a539ada7a4e3b",
                    "bytes_per_launch_by_splits": {8: 112.2e6, 16: 163.5e6}}


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed CG iterations of the large problem")
    ap.add_argument("--warmup", type=int, default=3,
                    help="iterations of the untimed warm-up solve")
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
                                       "prediction", "precision", "peaks", "large-product",
                                       "solves", "plain"),
                    default=None,
                    help="run only this measurement and print its figures (for profiling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch-shape rules instead of measuring them first")
    ap.add_argument("--splits", type=int, default=None,
                    help="fix the column splits of the single-problem product instead of tuning them "
                         "(used to take the HBM counters per split count)")
    ap.add_argument("--one-sided", action="store_true",
                    help="--part large-product: also time the one-sided kernel on the same data")
    ap.add_argument("--reps", type=int, default=3,
                    help="repetitions of the --part large-product launch (for the counters)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def kernel_sha(files=("kmvm_f16.hip", "fused_tile.h")):
    import hashlib
    h = hashlib.sha256()
    for f in files:
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


# The same counters for the headline product (N = 1,800,000, d = 11, R = 16).
MEASURED_TRAFFIC_LARGE = {"kernel_sha256_prefix": "ccfba85fbdb92d26",
                          "bytes_per_launch_by_splits": {"sym": 154.39e9}}


def product_kernel(n, d, r):
    """Which fused kernel gp_kmvm and the solver run for one point set of n
    points: the symmetric form from 16384 points when the operand width is 32
    (d <= 14) and r <= 16, else the one-sided kernel."""
    return "sym_kernel" if n >= 16384 and 2 * d + 4 <= 32 and r <= 16 else "kmvm_f16_main"


def measured_traffic_large(splits):
    files = (("kmvm_sym.hip", "fused_tile.h") if product_kernel(NL, DL, 16) == "sym_kernel"
             else ("kmvm_f16.hip", "fused_tile.h"))
    if kernel_sha(files) != MEASURED_TRAFFIC_LARGE["kernel_sha256_prefix"]:
        return None
    return MEASURED_TRAFFIC_LARGE["bytes_per_launch_by_splits"].get(splits)


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
    conv_cols = int(sum(int(s["converged"].sum()) for s in st))
    cols = int(sum(s["converged"].size for s in st))
    true_max = max(float(s["true_rel_res"].max()) for s in st)
    true_med = float(np.median([float(s["true_rel_res"].max()) for s in st]))
    its = [int(s["iters"].max()) for s in st]
    # baseline: standard float32 CG one problem after another, same preconditioner rank
    t0 = time.perf_counter()
    its32, conv32, true32 = [], 0, []
    for p, U in zip(dp, outs):
        P = gpmi.Precond(p["X"], p["kind"], p["lengthscale"], p["outputscale"], p["noise"],
                         p["precond_rank"])
        _, s32 = gpmi.cg_solve(p["X"], p["B"], p["kind"], p["lengthscale"], p["outputscale"],
                               p["noise"], tol=1.0, max_iter=100, min_iter=10,
                               algo=gpmi.CG_STANDARD, precision=gpmi.FP32, precond=P, out=U)
        P.close()
        its32.append(int(s32["iters"].max()))
        conv32 += int(s32["converged"].sum())
        true32.append(float(s32["true_rel_res"].max()))
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    return {"problems": len(probs), "rows_total": int(sum(q.n for q in probs)),
            "batched_s": round(tb, 4), "batched_solves_per_s": round(len(probs) / tb, 1),
            "batched_gentries_per_s": round(ent / tb / 1e9, 1), "all_converged": conv,
            "converged_columns": conv_cols, "columns": cols,
            "true_rel_res_max": round(true_max, 4), "true_rel_res_median": round(true_med, 4),
            "iters_median": int(np.median(its)), "plain_fp32_sequential_s": round(t32, 4),
            "plain_fp32_iters_median": int(np.median(its32)),
            "plain_fp32_converged_columns": conv32,
            "plain_fp32_true_rel_res_max": round(max(true32), 4),
            "plain_fp32_true_rel_res_median": round(float(np.median(true32)), 4),
            "speedup_vs_plain_fp32": round(t32 / tb, 2),
            "note": "speed-up at the same tolerance (1.0) and iteration limits; both sides' "
                    "converged columns and float64 true residuals are given"}


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
    conv32, cols32, true32 = 0, 0, []
    for q, p in zip(descs[:cmp_n], probs[:cmp_n]):
        X = torch.from_numpy(p.X).to("cuda:0")
        B = torch.from_numpy(p.B).to("cuda:0")
        P = gpmi.Precond(X, p.kind, p.lengthscale, p.outputscale, p.noise, min(100, p.X.shape[0]))
        _, s32 = gpmi.cg_solve(X, B, p.kind, p.lengthscale, p.outputscale, p.noise, tol=q["tol"],
                               max_iter=100, min_iter=10, algo=gpmi.CG_STANDARD,
                               precision=gpmi.FP32, precond=P)
        P.close()
        conv32 += int(s32["converged"].sum())
        cols32 += int(s32["converged"].size)
        true32.append(float(s32["true_rel_res"].max()))
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    convc = sum(int(r["converged"]) for r in resc)
    colsc = sum(len(r.get("col_iters", ())) for r in resc)
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
                                      "served_converged_columns": convc, "columns": colsc,
                                      "served_true_rel_res_max": round(
                                          max(r["max_true_rel_res"] for r in resc), 4),
                                      "plain_fp32_sequential_s": round(t32, 3),
                                      "plain_fp32_converged_columns": conv32,
                                      "plain_fp32_true_rel_res_max": round(max(true32), 4),
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


# Vector instructions per evaluated entry of the gradient reduction's inner
# loop (gfx950 assembly: 245 vector instructions and 3 float32 MFMAs per 8
# entries a lane, for d = 8 with ARD): per input dimension a difference, a
# square and the accumulation, the RBF value, the W entry, kappa W, G W and the
# clamp of r^2.  With the symmetric tiling an entry (i, j) past the diagonal
# block stands for (j, i) as well, so about half of the N^2 logical entries
# are evaluated.  The roofline is the vector issue rate: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s (no packed FP32).
GRAD_VALU_PER_ENTRY_D8 = 245 / 8
PEAK_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9


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
    lane_instr = evaluated * GRAD_VALU_PER_ENTRY_D8 / (grad_ms / 1e3)
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
                            "bound": "alu",
                            "achieved_lane_instr_per_s": round(lane_instr, -9),
                            "peak_lane_instr_per_s": PEAK_LANE_INSTR_PER_S,
                            "frac": round(lane_instr / PEAK_LANE_INSTR_PER_S, 4),
                            "valu_instr_per_evaluated_entry": round(GRAD_VALU_PER_ENTRY_D8, 3)}}


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
        # algorithmic matrix-core FLOP of the whole call (incl. quantisation and
        # reduction, so a lower bound on the kernel's own)
        k["bf16_r16_mfma_alg_frac"] = round(ent * (2 * D + 2 * R) / (t / 1e3) / 1e12
                                            / PEAK_FP16_MFMA_TFLOPS, 4)
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


def cpu_baseline_training(rows_per_thread=24):
    """float64 oracle Eq. (approx) gradient on sampled rows of the training
    workload, on all host threads.  U and B are synthetic blocks of the
    solve's shape: the oracle's time does not depend on their values."""
    import numpy as np

    from oracle import train as otrain
    from paper_2207_06856_amd import synth
    n, d, M = 100_000, 8, 15
    X, y = synth.training(n=n, d=d)
    g = np.random.default_rng(3)
    B = np.concatenate([y[:, None], g.choice([-1.0, 1.0], (n, M))], axis=1)
    U = g.standard_normal((n, M + 1))
    ls = np.full(d, np.log(2.0))
    th = host_threads()
    rows = np.arange(rows_per_thread * th)
    dt = oracle_parallel(lambda ch: otrain.pseudo_loss_grad(X, U, B, 0, ls, float(np.log(2.0)),
                                                            True, rows=ch), rows, th)
    return {"value": round(rows.size * n / dt / 1e9, 4), "unit": "Gentries/s", "cores": th,
            "kind": "oracle", "sample": f"Eq. (approx) gradient, {rows.size} rows x {n} columns, "
                                        f"RBF-ARD d={d}, float64, {th} threads ({dt:.1f} s)"}


def cpu_baseline_truncation(rows_per_thread=16):
    """float64-emulated truncated binary16 product of the oracle on sampled
    rows of the support workload, on all host threads."""
    import numpy as np

    from oracle import support
    from paper_2207_06856_amd import synth
    p = synth.compact_support()
    th = host_threads()
    sel = np.random.default_rng(4).choice(p.n, rows_per_thread * th, replace=False)
    dt = oracle_parallel(lambda ch: support.kmvm_fp16_truncated(p.X[ch], p.X, p.B, 0,
                                                                p.lengthscale, p.outputscale,
                                                                p.noise, False), sel, th)
    return {"value": round(sel.size * p.n / dt / 1e9, 4), "unit": "Gentries/s (logical)",
            "cores": th, "kind": "oracle",
            "sample": f"truncated binary16 emulation, {sel.size} sampled rows x {p.n} columns x "
                      f"16 right-hand sides, {th} threads ({dt:.1f} s)"}


def cpu_baseline_prediction(rows_per_thread=128):
    """float64 oracle mean product a^2 K(x*, X) v for sampled test points of
    the prediction workload, on all host threads; the cache solve itself (a
    dense Cholesky of order 100,000) is beyond a bounded CPU sample.  v is
    synthetic: the time does not depend on its values."""
    import numpy as np

    from oracle import kmvm as okmvm
    from paper_2207_06856_amd import synth
    p = synth.mixed_precision(n=N, kind=0)
    th = host_threads()
    g = np.random.default_rng(17)
    Xs = g.standard_normal((rows_per_thread * th, D))
    v = g.standard_normal((N, 1))
    dt = oracle_parallel(lambda ch: okmvm.kmvm(Xs[ch], p.X, v, 0, p.lengthscale, 1.0, p.noise,
                                               False), np.arange(Xs.shape[0]), th)
    return {"value": round(Xs.shape[0] * N / dt / 1e9, 4), "unit": "Gentries/s", "cores": th,
            "kind": "oracle", "sample": f"predictive-mean product, {Xs.shape[0]} test points x "
                                        f"{N} training points, float64, {th} threads ({dt:.1f} s)"}


def cpu_baseline_precision(rows_per_thread=64, sum_rows_per_thread=2):
    """The oracle's bfloat16 emulation (R = 16) and binary16 summation schemes
    (R = 1, blocks of 32) on sampled rows of the mixed-precision workload
    (RBF), on all host threads."""
    import numpy as np

    from oracle import precision as oprec
    from paper_2207_06856_amd import synth
    p = synth.mixed_precision(n=N, kind=0)
    th = host_threads()
    sel = np.random.default_rng(5).choice(N, rows_per_thread * th, replace=False)
    res = {}
    dt = oracle_parallel(lambda ch: oprec.kmvm_bf16_emulated(p.X, p.X, p.B, 0, p.lengthscale,
                                                             1.0, p.noise, True, rows=ch), sel, th)
    res["bf16_r16"] = {"value": round(sel.size * N / dt / 1e9, 4), "unit": "Gentries/s",
                       "sample": f"{sel.size} rows x {N} columns x 16 right-hand sides "
                                 f"({dt:.1f} s)"}
    sel = sel[:sum_rows_per_thread * th]
    y = p.B[:, :1].copy()
    for scheme in oprec.SCHEMES:
        dt = oracle_parallel(lambda ch: oprec.kmvm_fp16_summation(p.X, p.X, y, 0, p.lengthscale,
                                                                  1.0, p.noise, True, scheme,
                                                                  block=32, rows=ch), sel, th)
        res[scheme + "_r1"] = {"value": round(sel.size * N / dt / 1e9, 6), "unit": "Gentries/s",
                               "sample": f"{sel.size} rows x {N} columns ({dt:.1f} s)"}
    return {"cores": th, "kind": "oracle", **res}


def host_threads():
    """Threads of the oracle legs: the host cores this process may use (at most
    16, the host share of one GPU on the benchmark machines)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_parallel(fn, rows, threads):
    """Run fn(rows_chunk) over `threads` contiguous chunks of `rows` on a thread
    pool, BLAS limited to one thread each (numpy releases the GIL in the
    oracle's array loops); returns the wall time."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    chunks = [c for c in np.array_split(np.asarray(rows), threads) if c.size]
    with threadpool_limits(limits=1):
        a = time.perf_counter()
        with ThreadPoolExecutor(len(chunks)) as ex:
            list(ex.map(fn, chunks))
        return time.perf_counter() - a


def peaks_measurement(gpmi):
    """Probed issue rates and bandwidth of this chip (gp_probe_rate)."""
    iters = {"exp": 20000, "sqrt": 20000, "fma": 20000, "mfma_f16_16x16x32": 20000,
             "mfma_f16_16x16x16": 20000, "mfma_f64_16x16x4": 20000, "copy": 8}
    r = {k: gpmi.probe_rate(k, iters[k]) for k in iters}
    # how far independent MFMA and vector streams overlap: the mixed loops
    # against the single-kind loops at the same occupancy (8 and 2 waves per
    # SIMD); per wave-iteration the mixed loop issues 4 binary16 MFMAs and 16
    # FMAs or 8 exponentials per lane
    overlap = {}
    for tw, tag in ((False, "8_waves_per_simd"), (True, "2_waves_per_simd")):
        one = (lambda k: r[k]) if not tw else (lambda k: gpmi.probe_rate(k, 20000, two_waves=True))
        t_m = 4 * 16384 / one("mfma_f16_16x16x32")
        t_vec = {"fma": 64 * 16 / one("fma"), "exp": 64 * 8 / one("exp")}
        for kind in ("fma", "exp"):
            t_mix = 4 * 16384 / gpmi.probe_rate("mix_" + kind, 20000, two_waves=tw)
            tv = t_vec[kind]
            overlap[f"mfma_with_{kind}_{tag}"] = {
                "vector_alone_over_mfma_alone": round(tv / t_m, 3),
                "mixed_over_sum": round(t_mix / (t_m + tv), 3),
                "mixed_over_max": round(t_mix / max(t_m, tv), 3)}
    return {"exp_lane_ops_per_s": r["exp"], "sqrt_lane_ops_per_s": r["sqrt"],
            "fma_lane_ops_per_s": r["fma"],
            "mfma_f16_16x16x32_flops": r["mfma_f16_16x16x32"],
            "mfma_f16_16x16x16_flops": r["mfma_f16_16x16x16"],
            "mfma_f64_flops": r["mfma_f64_16x16x4"], "copy_bytes_per_s": r["copy"],
            "lane_slot_ceiling_per_s": 256 * 4 * 16 * 2.4e9,
            "overlap": overlap,
            "note": "lane ops/s of one instruction kind alone (packed FP32 disabled); FLOP/s of "
                    "the matrix instruction alone; copy = bytes read + written per second; "
                    "overlap: time of the mixed loop over the sum and over the larger of its "
                    "two streams' times alone (1.0 over the sum: no overlap; 1.0 over the "
                    "larger: full overlap)"}


# vector instructions per kernel entry in the fused product's tile loop
# (gfx950 assembly): the transcendentals, and the other vector instructions
# (conversion to binary16 is one packed instruction per two entries)
# (1.60 and 5.61 vector lane-instructions per entry besides the MFMAs, RBF and
# Matern-5/2, from the SQ instruction counters of the product)
VALU_MIX = {0: {"exp": 1.0, "sqrt": 0.0, "other": 0.60},
            1: {"exp": 1.0, "sqrt": 1.0, "other": 3.61}}


def valu_issue_frac(kind, entries_per_s, peaks, evaluated_per_entry=1.0):
    """Share of the launch time the vector unit spends issuing the kernel-value
    instructions at the probed rates of each instruction kind alone.
    evaluated_per_entry: kernel values computed per entry of the product (0.5
    for the symmetric kernel, which evaluates each unique pair once)."""
    m = VALU_MIX[kind]
    t = (m["exp"] / peaks["exp_lane_ops_per_s"] + m["sqrt"] / peaks["sqrt_lane_ops_per_s"]
         + m["other"] / peaks["fma_lane_ops_per_s"])
    return entries_per_s * evaluated_per_entry * t


def large_problem(gpmi, torch, dev):
    from paper_2207_06856_amd import synth
    p = synth.large_single(n=NL)
    X = torch.from_numpy(p.X).to(dev)
    B = torch.from_numpy(p.B).to(dev)
    torch.cuda.synchronize()
    return p, X, B


def large_product_part(gpmi, torch, dev, reps, one_sided=False):
    """`reps` launches of the headline fused product K~V at full size (for the
    rocprofv3 kernel trace and counter passes)."""
    p, X, B = large_problem(gpmi, torch, dev)
    out = torch.empty_like(B)
    gpmi.kmvm(X, X, B, p.kind, p.lengthscale, p.outputscale, p.noise, add_noise=True, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        gpmi.kmvm(X, X, B, p.kind, p.lengthscale, p.outputscale, p.noise, add_noise=True, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res = {"workload": f"K~V, N={NL}, d={DL}, R=16, RBF l=1.5, binary16", "reps": reps,
           "kernel": product_kernel(NL, DL, 16),
           "ms": round(dt * 1e3, 3), "gentries_per_s": round(float(NL) ** 2 / dt / 1e9, 1)}
    if one_sided:
        # the same product through the one-sided kernel (a copy of X is not the same set)
        X2 = X.clone()
        gpmi.kmvm(X, X2, B, p.kind, p.lengthscale, p.outputscale, p.noise, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gpmi.kmvm(X, X2, B, p.kind, p.lengthscale, p.outputscale, p.noise, out=out)
        torch.cuda.synchronize()
        d1 = (time.perf_counter() - t0) / reps
        res.update(one_sided_ms=round(d1 * 1e3, 3),
                   one_sided_gentries_per_s=round(float(NL) ** 2 / d1 / 1e9, 1))
    return res


def headline_large(gpmi, torch, dev, steps, warmup, tuned, peaks):
    """K iterations of the large single problem's solve, timed; the product's
    own launches timed with HIP events on their stream."""
    import numpy as np
    p, X, B = large_problem(gpmi, torch, dev)
    U = torch.empty_like(B)
    kw = dict(tol=1.0, algo=gpmi.CG_ENHANCED, precision=gpmi.FP16, out=U)
    torch.cuda.synchronize()
    a = time.perf_counter()
    P = gpmi.Precond(X, p.kind, p.lengthscale, p.outputscale, p.noise, RANK)
    torch.cuda.synchronize()
    precond_s = time.perf_counter() - a
    if warmup > 0:
        gpmi.cg_solve(X, B, p.kind, p.lengthscale, p.outputscale, p.noise, max_iter=warmup,
                      min_iter=warmup, true_res_every=-1, precond=P, **kw)
    torch.cuda.synchronize()
    gpmi.profile_reset()
    gpmi.profile_enable(True)
    t0 = time.perf_counter()
    _, st = gpmi.cg_solve(X, B, p.kind, p.lengthscale, p.outputscale, p.noise, max_iter=steps,
                          min_iter=steps, true_res_every=-1, precond=P, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpmi.profile_enable(False)
    ms, ent, _ = gpmi.profile_read()
    gpmi.profile_reset()
    # the float64 true residual of the iterate (the solver's exit check), timed alone
    rows = torch.arange(NL, device=dev, dtype=torch.int64)
    torch.cuda.synchronize()
    a = time.perf_counter()
    res = gpmi.true_residual_rows(X, B, U, rows, p.kind, p.lengthscale, p.outputscale, p.noise)
    torch.cuda.synchronize()
    true_res_s = time.perf_counter() - a
    true_rel = (torch.linalg.norm(res, dim=0) / torch.linalg.norm(B.double(), dim=0)).cpu().numpy()
    del res
    # the product alone (gp_kmvm: operand preparation, quantisation, fused kernel, reduction)
    out = torch.empty_like(B)
    gpmi.kmvm(X, X, B, p.kind, p.lengthscale, p.outputscale, p.noise, add_noise=True, out=out)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(3):
        gpmi.kmvm(X, X, B, p.kind, p.lengthscale, p.outputscale, p.noise, add_noise=True, out=out)
    torch.cuda.synchronize()
    kmvm_s = (time.perf_counter() - a) / 3
    P.close()
    del out, U, X, B, P
    torch.cuda.empty_cache()
    gpmi.release_cached_memory()    # the large problem's workspace is not kept for the next parts

    entries = float(NL) ** 2
    value = steps * entries / wall / 1e9
    dur = float(ms.mean()) / 1e3                       # every launch is a working launch here
    flops = (2 * DL + 2 * 16) * entries                # algorithmic FLOP per launch
    achieved = flops / dur / 1e12
    splits = (product_splits(tuned, NL) if product_kernel(NL, DL, 16) == "kmvm_f16_main"
              else "sym")
    valu = valu_issue_frac(0, entries / dur, peaks, 0.5 if splits == "sym" else 1.0)
    issued = DL + 2 * 16 if splits == "sym" else 2 * DL + 2 * 16
    # what the matrix cores execute: the cross term padded to K = 32 (one
    # 16x16x32 MFMA per 256 evaluated pairs) and 32 FLOP per evaluated pair per
    # sum direction for each 16 right-hand sides
    issued_padded = 32 + 32 if splits == "sym" else 64 + 32
    mfma_probed = issued_padded * entries / dur / peaks["mfma_f16_16x16x32_flops"]
    return {
        "value": value, "ms_per_step": wall / steps * 1e3,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2),
                     "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP16_MFMA_TFLOPS, 4),
                     "traffic": measured_traffic_large(splits),
                     "kernel": product_kernel(NL, DL, 16), "launches": int(ms.size),
                     "avg_launch_ms": round(dur * 1e3, 3),
                     "launch_ms_p10_p50_p90": [round(float(np.percentile(ms, q)), 3)
                                               for q in (10, 50, 90)],
                     "flops_per_entry": 2 * DL + 2 * 16, "entries_per_launch": entries,
                     # the symmetric kernel evaluates each unique pair once: half the distance work
                     "issued_flops_per_entry": issued,
                     "issued_padded_flops_per_entry": issued_padded,
                     "column_splits": splits,
                     "valu_issue_frac": round(valu, 4),
                     "mfma_frac_of_probed_peak": round(mfma_probed, 4),
                     # the serial issue model: vector and matrix-core issue times added
                     # (independent streams overlap only partly, see peaks.overlap, and
                     # this loop's dependent ones not at all); the share of the launch
                     # that model explains
                     "serial_issue_model_frac": round(valu + mfma_probed, 4),
                     "product_share_of_step": round(float(ms.sum()) / 1e3 / wall, 4)},
        "large": {"precond_build_s": round(precond_s, 3),
                  "true_residual_s": round(true_res_s, 3),
                  "true_rel_res_after_steps": [round(float(v), 4) for v in true_rel],
                  "recursive_rel_res_after_steps": [round(float(v), 4) for v in st["rel_res"]],
                  "iters": steps,
                  "kmvm_call_ms": round(kmvm_s * 1e3, 3),
                  "kmvm_call_gentries_per_s": round(entries / kmvm_s / 1e9, 1),
                  "fused_kernel_gentries_per_s": round(entries / dur / 1e9, 1)},
    }


def cpu_baseline_large(rows_per_thread=64):
    """float64 oracle product K~V on sampled rows of the large problem, on all
    host threads (one BLAS thread each)."""
    import numpy as np

    from oracle import kmvm as okmvm
    from paper_2207_06856_amd import synth
    p = synth.large_single(n=NL)
    th = host_threads()
    rows = np.sort(np.random.default_rng(0).choice(NL, rows_per_thread * th, replace=False))
    dt = oracle_parallel(lambda ch: okmvm.kmvm(p.X, p.X, p.B, p.kind, p.lengthscale, 1.0,
                                               p.noise, True, rows=ch), rows, th)
    return {"value": round(rows.size * float(NL) / dt / 1e9, 4), "unit": "Gentries/s",
            "cores": th, "kind": "oracle",
            "sample": f"float64 oracle product, {rows.size} sampled output rows x {NL} columns x "
                      f"16 right-hand sides, RBF, d={DL}, {th} threads ({dt:.1f} s)"}


def mixed_precision_solves(gpmi, torch, dev, peaks, tuned, compare=True):
    """The mixed-precision solves to tolerance (N = 100,000, d = 8): three timed
    binary16 Alg. 1 solves per kernel, the product's rate from its own launch
    timing, and (compare) the standard float32 CG comparator."""
    import numpy as np

    from paper_2207_06856_amd import synth

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

    for kind in (1, 0):
        solve(kind)
    torch.cuda.synchronize()
    gpmi.profile_reset()
    gpmi.profile_enable(True)
    per_solve_ms = {1: [], 0: []}
    stats = []
    for _ in range(3):
        for kind in (1, 0):
            a = time.perf_counter()
            st = solve(kind)
            per_solve_ms[kind].append((time.perf_counter() - a) * 1e3)
            stats.append((kind, st))
    torch.cuda.synchronize()
    gpmi.profile_enable(False)
    ms, ent, kinds = gpmi.profile_read()
    gpmi.profile_reset()
    # working launches (a launch after every column froze exits at once)
    work = ms > 0.05 * np.median(ms)
    roof = {}
    for kind in (1, 0):
        m = work & (kinds == kind)
        dur = ms[m].mean() / 1e3
        e = ent[m].mean()
        roof[kind] = dict(avg_ms=ms[m].mean(), gentries=e / dur / 1e9,
                          mfma_alg_tflops=e * (2 * D + 2 * R) / dur / 1e12,
                          valu_issue=valu_issue_frac(
                              kind, e / dur, peaks,
                              0.5 if product_kernel(N, D, R) == "sym_kernel" else 1.0))

    # comparators: standard CG with the float32 product, same preconditioner
    cmp = {kind: dict(ms=float("nan"), iters=-1, converged=False, true=float("nan"))
           for kind in (1, 0)}
    for kind in ((1, 0) if compare else ()):
        solve(kind)
        torch.cuda.synchronize()
        a = time.perf_counter()
        st32 = solve(kind, algo=gpmi.CG_STANDARD, precision=gpmi.FP32)
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - a) * 1e3
        cmp[kind] = dict(ms=t32, iters=int(st32["iters"].max()),
                         converged=int(st32["converged"].sum()),
                         true=float(st32["true_rel_res"].max()))

    last = {k: st for k, st in stats}
    detail = {}
    for kind in (1, 0):
        st = last[kind]
        t = float(np.median(per_solve_ms[kind]))
        detail[KIND_NAME[kind]] = dict(
            time_to_tol_ms=round(t, 3), iters=int(st["iters"].max()),
            ms_per_iteration=round(t / max(1, int(st["iters"].max())), 4),
            converged_columns=int(st["converged"].sum()), columns=R,
            true_rel_res_max=round(float(st["true_rel_res"].max()), 5),
            plain_fp32_time_to_tol_ms=round(cmp[kind]["ms"], 3),
            plain_fp32_iters=cmp[kind]["iters"],
            plain_fp32_converged_columns=cmp[kind]["converged"],
            plain_fp32_true_rel_res_max=round(cmp[kind]["true"], 5),
            speedup_vs_plain_fp32=(round(cmp[kind]["ms"] / t, 3)
                                   if cmp[kind]["iters"] >= 0 else None),
            kmvm_avg_ms=round(roof[kind]["avg_ms"], 4),
            kmvm_gentries_per_s=round(roof[kind]["gentries"], 1),
            kmvm_mfma_alg_frac=round(roof[kind]["mfma_alg_tflops"] / PEAK_FP16_MFMA_TFLOPS, 4),
            kmvm_valu_issue_frac=round(roof[kind]["valu_issue"], 4),
            kmvm_kernel=product_kernel(N, D, R),
            kmvm_traffic=(measured_traffic(product_splits(tuned, N))
                          if kind == 0 and product_kernel(N, D, R) == "kmvm_f16_main" else None))

    return detail


def plain_solve_measurement(gpmi, torch, dev, reps=5):
    """The small plain solve to a tight tolerance (N = 2000, d = 3, R = 1, RBF
    l = 0.5, noise 0.01, float32 product, no preconditioner, relative residual
    1e-6, at most 500 iterations): median time-to-tol of `reps` solves with
    re-orthogonalised Alg. 1 and with standard CG (Alg. 2), and the time per
    iteration, which at this size is the launch sequence of one iteration."""
    import numpy as np

    from paper_2207_06856_amd import synth

    p = synth.plain_solve()
    X = torch.from_numpy(p.X).to(dev)
    B = torch.from_numpy(p.B).to(dev)
    U = torch.empty_like(B)
    out = {"workload": "N=2000, d=3 (X ~ U[-1,1]), R=1, RBF l=0.5, noise 0.01, float32 "
                       "product, no preconditioner, tol 1e-6, max 500 iterations, poll every 20"}
    for name, algo, cap in (("enhanced", gpmi.CG_ENHANCED, 500), ("standard", gpmi.CG_STANDARD,
                                                                  1500)):
        def solve():
            return gpmi.cg_solve(X, B, p.kind, p.lengthscale, 1.0, p.noise, tol=1e-6,
                                 max_iter=cap, min_iter=0, algo=algo, precision=gpmi.FP32,
                                 poll_every=20, out=U)[1]
        solve()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = time.perf_counter()
            st = solve()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - a) * 1e3)
        t = float(np.median(ts))
        it = int(st["iters"].max())
        out[name] = {"time_to_tol_ms": round(t, 3), "iters": it,
                     "us_per_iteration": round(1e3 * t / max(1, it), 2),
                     "converged": bool(st["converged"].all()),
                     "rel_res": float(st["rel_res"].max()),
                     "true_rel_res": round(float(st["true_rel_res"].max()), 7)}
        if name == "standard":
            out[name]["max_iter"] = cap
    return out


def cpu_baseline_plain():
    """The oracle's float64 Alg. 1 (re-orthogonalised) on the whole small plain
    solve, dense K~ products on all host threads (BLAS), to the same
    tolerance."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cg as ocg, direct
    from paper_2207_06856_amd import synth
    p = synth.plain_solve()
    th = host_threads()
    with threadpool_limits(limits=th):
        a = time.perf_counter()
        K = direct.ktilde(p.X, p.kind, p.lengthscale, 1.0, p.noise)
        _, st = ocg.solve(lambda V: K @ V, p.B, 1e-6, 500, algo="enhanced")
        dt = time.perf_counter() - a
    return {"value": round(dt * 1e3, 3), "unit": "ms time-to-tol", "cores": th, "kind": "oracle",
            "sample": f"the whole solve (N=2000, R=1): dense float64 K~ built once, then "
                      f"oracle Alg. 1 to 1e-6 in {int(np.max(st['iters']))} iterations, "
                      f"{th} BLAS threads"}


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
    if args.part == "peaks":
        print(json.dumps({"peaks": peaks_measurement(gpmi)}), flush=True)
        return 0
    if args.part == "solves":
        print(json.dumps({"solves": mixed_precision_solves(gpmi, torch, dev, peaks_measurement(gpmi),
                                                           gpmi.tune_info(), compare=False)}),
              flush=True)
        return 0
    if args.part == "large-product":
        print(json.dumps({"large_product": large_product_part(gpmi, torch, dev, args.reps,
                                                              args.one_sided)}), flush=True)
        return 0
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
    part_cpu = {"plain": cpu_baseline_plain, "training": cpu_baseline_training,
                "truncation": cpu_baseline_truncation, "prediction": cpu_baseline_prediction,
                "precision": cpu_baseline_precision}
    part_fn = {"plain": plain_solve_measurement, "training": training_measurement,
               "truncation": truncation_measurement, "prediction": prediction_measurement,
               "precision": precision_measurement}
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
    log("autotune done; probing peaks")
    peaks = peaks_measurement(gpmi)
    log("peaks done; large problem (1.8M points)")
    head = headline_large(gpmi, torch, dev, args.steps, args.warmup, tuned, peaks)
    log(f"large problem done: {head['value']:.1f} Gentries/s; mixed-precision solves")

    log("large problem done; mixed-precision solves")
    detail = mixed_precision_solves(gpmi, torch, dev, peaks, tuned, compare=not args.no_compare)

    out = {
        "metric": "fused kernel-MVM Gentries/s; CG time-to-tol vs plain FP32; serve p50/p99",
        "value": round(head["value"], 2),
        "unit": "Gentries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": f"large single problem: N={NL}, d={DL} (X ~ N(0, I), pairs 1-2, "
                               "3-4, 5-6 correlated at 0.8), R=16 (y from 512 random Fourier "
                               "features + 15 Rademacher probes), RBF l=1.5, outputscale 1, "
                               "noise 0.01, rank-100 pivoted Cholesky, binary16 Alg. 1; "
                               "one step = one CG iteration (fused product, logsumexp dots, "
                               "update, CGS2 re-orthogonalisation through the basis Gram "
                               "matrix, preconditioner apply, direction and requantisation)",
                   "n": NL, "d": DL, "r": 16, "precond_rank": RANK, "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "large": head["large"],
        "peaks": peaks,
        "mixed_precision_solves": {"workload": "N=100000, d=8, R=16 (y + 15 probes), l=1, noise "
                                               "0.05, rank 100, tol 1.0, min 10 / max 100 "
                                               "iterations, 3 timed solves per kernel",
                                   **detail},
        "autotune": tuned,
    }
    log("plain solve")
    out["plain_solve"] = plain_solve_measurement(gpmi, torch, dev)
    if not args.no_batched:
        log("batched")
        out["batched"] = batched_measurement(gpmi, torch, dev)
    if not args.no_serve:
        log("serve")
        out["serve"] = serve_measurement(gpmi, args.serve_requests)
    if not args.no_training:
        log("training")
        out["training"] = training_measurement(gpmi, torch, dev)
    if not args.no_truncation:
        log("truncation")
        out["truncation"] = truncation_measurement(gpmi, torch, dev)
    if not args.no_prediction:
        log("prediction")
        out["prediction"] = prediction_measurement(gpmi, torch, dev)
    if not args.no_precision:
        log("precision")
        out["precision"] = precision_measurement(gpmi, torch, dev)
    if not args.no_cpu_baseline:
        log("oracle legs on the host")
        out["cpu_baseline"] = cpu_baseline_large()
        for name, fn in part_cpu.items():
            key = "plain_solve" if name == "plain" else name
            if key in out:
                log(f"oracle leg: {name}")
                out[key]["cpu_baseline"] = fn()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
