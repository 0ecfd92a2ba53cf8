"""gp_serve_*: the serving loop.

* a request's result does not depend on what else is resident: every served
  solution is bit-identical to gp_cg_solve_batched on that problem alone (same
  kernels, per-problem reductions merged in a fixed order);
* the float64 true residual the server reports agrees with the oracle's for
  the returned solution;
* admission never holds more than the arena: a budget that fits only a few
  requests at a time still completes every request, with peak bytes within
  the budget;
* a request larger than the arena is refused at submit; cancel of a queued
  request; unknown tickets; concurrent submitters.
"""
import threading

import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import direct
from paper_2207_06856_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make_requests(count, seed, n_lo=300, n_hi=6000):
    g = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(g.integers(n_lo, n_hi))
        d = int(g.integers(2, 13))
        r = int([1, 5, 16, 23][i % 4])
        X = synth.random_points(n, d, 900 + 13 * i + seed)
        B = synth.random_rhs(n, r, 900 + 13 * i + seed)
        reqs.append(dict(X=X, B=B, kind=int(i % 2) if i % 3 else int(i % 4),
                         lengthscale=np.array([float(np.exp(g.uniform(np.log(0.7), np.log(2.5))))],
                                              np.float32),
                         outputscale=1.0, noise=float(np.float32(g.uniform(0.03, 0.1))),
                         tol=[1.0, 0.1][i % 2], max_iter=60, precond_rank=[0, 12, 40][i % 3]))
    return reqs


def solo_batched(gpu_lib, q, min_iter=10):
    p = dict(X=torch.from_numpy(q["X"]).to(DEV), B=torch.from_numpy(q["B"]).to(DEV),
             kind=q["kind"], lengthscale=q["lengthscale"], outputscale=q["outputscale"],
             noise=q["noise"], precond_rank=q["precond_rank"])
    U, st = gpu_lib.cg_solve_batched([p], tol=q["tol"], max_iter=q["max_iter"], min_iter=min_iter,
                                     poll_every=5)
    return U[0].cpu().numpy(), st[0]


def submit(srv, q):
    return srv.submit(q["X"], q["B"], q["kind"], q["lengthscale"], q["outputscale"], q["noise"],
                      tol=q["tol"], max_iter=q["max_iter"], precond_rank=q["precond_rank"])


def test_served_equals_alone(gpu_lib):
    reqs = make_requests(10, seed=1)
    with gpu_lib.Server(hbm_budget_bytes=2 << 30, max_slots=6, iters_per_round=3) as srv:
        tickets = [submit(srv, q) for q in reqs]
        res = [srv.wait(t, timeout_ms=60000) for t in tickets]
        stats = srv.stats()
    print("server stats", stats, flush=True)
    assert stats["completed"] == len(reqs) and stats["resident"] == 0 and stats["queued"] == 0
    for i, (q, r) in enumerate(zip(reqs, res)):
        print(f"request {i}: n={q['X'].shape[0]} d={q['X'].shape[1]} r={q['B'].shape[1]} "
              f"kind={q['kind']} rank={q['precond_rank']} tol={q['tol']} iters={r['iters']} "
              f"status={r['status']}", flush=True)
        assert r is not None and r["status"] == 0, r
        assert r["t_submit"] <= r["t_admit"] <= r["t_finish"]
        U_alone, st = solo_batched(gpu_lib, q)
        np.testing.assert_array_equal(r["U"], U_alone)
        np.testing.assert_array_equal(r["col_iters"], st["iters"])
        np.testing.assert_array_equal(r["col_converged"], st["converged"])
        A = direct.ktilde(q["X"], q["kind"], q["lengthscale"], 1.0, q["noise"])
        tr = ocg.true_relative_residual(lambda V: A @ V, q["B"], r["U"])
        np.testing.assert_allclose(r["true_rel_res"], tr, rtol=1e-4, atol=1e-7)


def test_admission_respects_budget(gpu_lib):
    reqs = make_requests(8, seed=2, n_lo=3000, n_hi=6000)
    # footprints and results with room for everything
    with gpu_lib.Server(hbm_budget_bytes=1 << 30, max_slots=16, iters_per_round=2) as srv:
        free = [srv.wait(submit(srv, q), timeout_ms=60000) for q in reqs]
    foot = sorted(r["footprint_bytes"] for r in free)
    # every request fits alone, at most two fit at once
    budget = foot[-1] + foot[1] - 256
    with gpu_lib.Server(hbm_budget_bytes=budget, max_slots=16, iters_per_round=2) as srv:
        tickets = [submit(srv, q) for q in reqs]
        res = [srv.wait(t, timeout_ms=60000) for t in tickets]
        stats = srv.stats()
    print("footprints", foot, "budget", budget, "stats", stats, flush=True)
    assert stats["peak_bytes"] <= budget
    for a, b in zip(free, res):
        assert b["status"] == 0
        assert b["footprint_bytes"] == a["footprint_bytes"]
        np.testing.assert_array_equal(b["U"], a["U"])


def test_too_large_cancel_unknown(gpu_lib):
    big = dict(X=np.zeros((200000, 8), np.float32), B=np.ones((200000, 32), np.float32), kind=0,
               lengthscale=np.array([1.0], np.float32), outputscale=1.0, noise=0.05, tol=1.0,
               max_iter=100, precond_rank=100)
    reqs = make_requests(4, seed=3)
    with gpu_lib.Server(hbm_budget_bytes=256 << 20, max_slots=1, iters_per_round=2) as srv:
        with pytest.raises(gpu_lib.GpError) as ei:
            submit(srv, big)
        assert ei.value.status == gpu_lib.GP_ERR_TOO_LARGE
        tickets = [submit(srv, q) for q in reqs]
        # one slot: the last request is still queued right after submission
        srv.cancel(tickets[-1])
        r = srv.wait(tickets[-1], timeout_ms=60000)
        assert r["status"] == gpu_lib.GP_ERR_CANCELLED and r["U"] is None
        with pytest.raises(gpu_lib.GpError) as ei:
            srv.poll(tickets[-1])
        assert ei.value.status == gpu_lib.GP_ERR_UNKNOWN_TICKET
        with pytest.raises(gpu_lib.GpError):
            srv.poll(987654321)
        for t in tickets[:-1]:
            assert srv.wait(t, timeout_ms=60000)["status"] == 0


def test_concurrent_submitters(gpu_lib):
    reqs = make_requests(12, seed=4, n_lo=200, n_hi=2000)
    out = {}
    with gpu_lib.Server(hbm_budget_bytes=1 << 30, max_slots=8, iters_per_round=4) as srv:
        lock = threading.Lock()

        def worker(idx):
            for i in idx:
                t = submit(srv, reqs[i])
                with lock:
                    out[i] = t

        ths = [threading.Thread(target=worker, args=(list(range(k, 12, 3)),)) for k in range(3)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        res = {i: srv.wait(t, timeout_ms=60000) for i, t in out.items()}
    assert len(res) == 12
    for i, r in res.items():
        assert r["status"] == 0
        U_alone, _ = solo_batched(gpu_lib, reqs[i])
        np.testing.assert_array_equal(r["U"], U_alone)
