"""gp_autotune: the launch-shape tuner.

The decisions come from the candidate sets, tuned products keep the binary16
parity bars against the float64 oracle, and tuned batched solves stay
bit-identical to each problem alone (the split rule depends only on the
problem's own size).  The test restores the built-in rules at the end.
"""
import numpy as np
import pytest
import torch

from oracle import kmvm as okmvm
from paper_2207_06856_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_autotune_decisions_and_parity(gpu_lib):
    try:
        info = gpu_lib.autotune(max_bucket=3)
        print("tune", info, flush=True)
        assert info["tuned"]
        for b in range(4):
            assert info["f16_splits"][b] in (0, 8, 16, 24, 32, 48, 64)
            assert info["f16_gain"][b] >= 1.0 - 1e-9
        assert info["batched_split_div"] in (8, 16, 32)
        assert gpu_lib.tune_info() == info
        # product parity with the tuned splits (n spans several buckets' tiles)
        n, d, r = 20000, 8, 16
        X = synth.random_points(n, d, 77)
        V = synth.random_rhs(n, r, 77)
        Xt, Vt = torch.from_numpy(X).to(DEV), torch.from_numpy(V).to(DEV)
        out = gpu_lib.kmvm(Xt, Xt, Vt, 0, [1.0], 1.0, 0.05, add_noise=True,
                           precision=gpu_lib.FP16).cpu().numpy()
        rows = np.arange(0, n, 97)
        ref = okmvm.kmvm(X, X, V, 0, [1.0], 1.0, 0.05, True, rows=rows)
        err = np.linalg.norm(out[rows] - ref) / np.linalg.norm(ref)
        assert err <= 5e-3, err
        # batched: each problem alone equals it inside the batch under tuned rules
        probs = []
        for i, nn in enumerate([700, 3000, 9000]):
            Xi = synth.random_points(nn, 6, 300 + i)
            Bi = synth.random_rhs(nn, 8, 300 + i)
            probs.append(dict(X=torch.from_numpy(Xi).to(DEV), B=torch.from_numpy(Bi).to(DEV), kind=0,
                              lengthscale=np.array([1.2], np.float32), outputscale=1.0, noise=0.05,
                              precond_rank=10))
        Us, _ = gpu_lib.cg_solve_batched(probs, tol=1.0, max_iter=40)
        for i, p in enumerate(probs):
            U1, _ = gpu_lib.cg_solve_batched([p], tol=1.0, max_iter=40)
            np.testing.assert_array_equal(U1[0].cpu().numpy(), Us[i].cpu().numpy())
    finally:
        gpu_lib.tune_reset()
    assert not gpu_lib.tune_info()["tuned"]
