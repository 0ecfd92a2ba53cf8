"""Parity of gp_pivchol_precond / gp_precond_apply with the float64 oracle."""
import numpy as np
import pytest
import torch

from oracle import pivchol
from paper_2207_06856_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,d,rank,kind", [(500, 2, 10, 0), (3000, 8, 50, 1), (1000, 5, 100, 0),
                                            (777, 3, 128, 1)])
def test_pivots_factor_and_apply_match_oracle(gpu_lib, n, d, rank, kind):
    print(f"precond n={n} d={d} rank={rank} kind={kind}", flush=True)
    X = synth.random_points(n, d, 100 + n, dist="uniform", scale=3.0)
    s2 = float(np.float32(0.05))
    ls = np.array([0.8], np.float32)        # both sides see the same float32 value
    Pref, L, piv, diag = pivchol.build(X, kind, ls, 1.0, s2, rank)
    tX = torch.from_numpy(X).to(DEV)
    P = gpu_lib.Precond(tX, kind, ls, 1.0, s2, rank)
    assert P.rank == L.shape[1]
    np.testing.assert_array_equal(P.pivots, piv)
    assert abs(P.trace_residual - diag.sum()) <= 1e-8 * max(1.0, diag.sum()) + 1e-10
    W = synth.random_rhs(n, 7, n)
    got = P.apply(torch.from_numpy(W).to(DEV)).cpu().numpy()
    assert rel(got, Pref(W)) <= 1e-5
    P.close()


def test_early_stop_on_repeated_points(gpu_lib):
    base = synth.random_points(6, 3, 7)
    X = np.repeat(base, 5, axis=0)
    P = gpu_lib.Precond(torch.from_numpy(X).to(DEV), 0, [1.0], 1.0, 0.1, 20)
    Lr, piv, _ = pivchol.pivoted_cholesky(X, 0, [1.0], 1.0, 20)
    assert P.rank == Lr.shape[1] == 6
    np.testing.assert_array_equal(P.pivots, piv)


def test_rank_zero_is_scaled_identity(gpu_lib):
    X = synth.random_points(100, 2, 8)
    P = gpu_lib.Precond(torch.from_numpy(X).to(DEV), 0, [1.0], 1.0, 0.25, 0)
    W = torch.from_numpy(synth.random_rhs(100, 3, 8)).to(DEV)
    np.testing.assert_allclose(P.apply(W).cpu().numpy(), 4.0 * W.cpu().numpy(), rtol=1e-6)


def test_bad_rank_rejected(gpu_lib):
    X = torch.from_numpy(synth.random_points(10, 2, 9)).to(DEV)
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.Precond(X, 0, [1.0], 1.0, 0.1, 11)
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.Precond(X, 0, [1.0], 1.0, 0.0, 3)      # noise must be > 0


def test_early_stop_with_several_work_groups(gpu_lib):
    # 40 distinct points repeated 16 times (n = 640: three work groups of the
    # step launch).  The residual diagonal is exhausted after the 40 distinct
    # pivots, so the step that finds it stops inside a launch that other
    # groups are still running; every group must take the same decision.
    base = synth.random_points(40, 3, 12)
    X = np.repeat(base, 16, axis=0)
    s2 = float(np.float32(0.1))
    Pref, L, piv, diag = pivchol.build(X, 0, [1.0], 1.0, s2, 60)
    assert L.shape[1] == 40
    P = gpu_lib.Precond(torch.from_numpy(X).to(DEV), 0, [1.0], 1.0, s2, 60)
    assert P.rank == 40
    np.testing.assert_array_equal(P.pivots, piv)
    assert abs(P.trace_residual - diag.sum()) <= 1e-8
    W = synth.random_rhs(640, 5, 13)
    got = P.apply(torch.from_numpy(W).to(DEV)).cpu().numpy()
    assert rel(got, Pref(W)) <= 1e-5
    P.close()


def test_release_cached_memory(gpu_lib):
    X = torch.from_numpy(synth.random_points(2000, 3, 14)).to(DEV)
    P = gpu_lib.Precond(X, 0, [1.0], 1.0, 0.1, 30)
    piv = P.pivots.copy()
    P.close()                                  # the block goes to the cache
    freed = gpu_lib.release_cached_memory()
    assert freed >= 12 * 2000 * 30             # at least the factor's block
    assert gpu_lib.release_cached_memory() == 0
    P = gpu_lib.Precond(X, 0, [1.0], 1.0, 0.1, 30)   # allocates again
    np.testing.assert_array_equal(P.pivots, piv)
    P.close()
