"""gp_kmvm_noalloc (the allocation-free product) against gp_kmvm and the oracle.

Two calls in a row through the C ABI, the second on a smaller input, each
compared with gp_kmvm on the same arguments and with the float64 oracle at
the product's bars (float32 1e-5, binary16 5e-3 relative); a product whose
scratch cannot fit the fixed block is refused before anything runs.
"""
import numpy as np
import pytest
import torch

from oracle import kmvm as okmvm
from paper_2207_06856_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision,bar", [(1, 5e-3), (0, 1e-5), (2, 5e-3)])
def test_noalloc_matches_kmvm_on_two_calls(gpu_lib, precision, bar):
    ls = np.array([0.9], np.float32)
    s2 = float(np.float32(0.05))
    cases = [(9000, 6, 17, 1), (1300, 3, 5, 0)]       # second call smaller
    for n, d, r, kind in cases:
        print(f"noalloc precision={precision} n={n} d={d} r={r} kind={kind}", flush=True)
        X = synth.random_points(n, d, 40 + n)
        V = synth.random_rhs(n, r, 41 + n)
        tX, tV = torch.from_numpy(X).to(DEV), torch.from_numpy(V).to(DEV)
        out = torch.full((n, r), float("nan"), device=DEV)
        gpu_lib.kmvm_noalloc(tX, tX, tV, kind, ls, 1.0, s2, add_noise=True, precision=precision,
                             out=out)
        ref_dev = gpu_lib.kmvm(tX, tX, tV, kind, ls, 1.0, s2, add_noise=True, precision=precision)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        # same arithmetic; the split count (order of float32 partial sums) may differ
        assert rel(got, ref_dev.cpu().numpy().astype(np.float64)) <= 1e-6
        rows = np.arange(0, n, 7)
        ref = okmvm.kmvm(X, X, V, kind, ls, 1.0, s2, True, rows=rows)
        assert rel(got[rows], ref) <= bar


def test_noalloc_rectangular_and_repeat_is_deterministic(gpu_lib):
    X1 = synth.random_points(700, 4, 51)
    X2 = synth.random_points(5000, 4, 52)
    V = synth.random_rhs(5000, 16, 53)
    t1, t2, tV = (torch.from_numpy(a).to(DEV) for a in (X1, X2, V))
    a = gpu_lib.kmvm_noalloc(t1, t2, tV, 0, [1.1], 1.0, 0.0).cpu().numpy()
    b = gpu_lib.kmvm_noalloc(t1, t2, tV, 0, [1.1], 1.0, 0.0).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    ref = okmvm.kmvm(X1, X2, V, 0, [1.1], 1.0, 0.0, False)
    assert rel(a, ref) <= 5e-3


def test_noalloc_refuses_a_product_beyond_its_block(gpu_lib):
    cap = gpu_lib.kmvm_noalloc_scratch_bytes()
    assert cap == 64 << 20
    # binary16, d = 8 (operand width 32), r = 16: with one split the scratch is
    # 64 n1 + 64 n2 + 32 n2 + 64 n1 bytes (+ a few KB): 400,000 points exceed it
    n = 400_000
    X = torch.zeros((n, 8), device=DEV)
    V = torch.zeros((n, 16), device=DEV)
    out = torch.full((n, 16), 7.0, device=DEV)
    with pytest.raises(gpu_lib.GpError) as e:
        gpu_lib.kmvm_noalloc(X, X, V, 0, [1.0], 1.0, 0.1, add_noise=True, out=out)
    assert e.value.status == gpu_lib.GP_ERR_TOO_LARGE
    assert float(out[0, 0]) == 7.0                  # nothing ran
