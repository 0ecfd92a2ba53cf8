"""Pins for oracle.support against values the paper prints."""
import math

import numpy as np
import pytest

from oracle import kernels, support
from golden_values import paper_values


def test_matern12_worked_example():
    pv = paper_values()
    eps = 2.0 ** pv["matern12_example_eps_log2"]
    d = pv["matern12_example_distance"]
    # the printed figure is -log(eps)/d
    assert abs(-math.log(eps) / d - pv["matern12_example_bound"]) < 5e-3
    # the App. C cut-off at the lengthscale where the pair is just unrepresentable
    ls = d / -math.log(eps)
    assert abs(support.cutoff_distance("matern12", ls, eps) - d) < 1e-12
    assert abs(kernels.kfun(kernels.MATERN12, (d / ls) ** 2) - eps) < 1e-15


def test_rbf_cutoff_is_where_kernel_reaches_eps():
    for ls in (0.3, 1.0, 4.0):
        for eps in (2.0 ** -24, 2.0 ** -149, 2.0 ** -1074):
            dcut = support.cutoff_distance("rbf", ls, eps)
            v = kernels.kfun(kernels.RBF, (dcut / ls) ** 2)
            assert abs(math.log(v) - math.log(eps)) < 1e-9


def test_binary16_constants():
    fi = np.finfo(np.float16)
    assert support.FP16_MAX == float(fi.max)
    assert support.FP16_MIN_NORMAL == float(fi.tiny)
    assert support.FP16_MIN_SUBNORMAL == float(np.nextafter(np.float16(0), np.float16(1)))
    assert support.FP16_UNIT_ROUNDOFF == float(fi.eps) / 2


def test_zero_radius_matches_closed_forms_and_ordering():
    """App. C closed forms at eps = 2^-25 for RBF and Matern-1/2; the Matern
    radii lie between them (App. C: 'somewhere between Matern-1/2 and RBF');
    the kernel value at each radius is the threshold."""
    eps = support.FP16_ZERO_THRESHOLD
    r_rbf = support.zero_radius(kernels.RBF)
    r_m12 = support.zero_radius(kernels.MATERN12)
    assert abs(r_rbf - support.cutoff_distance("rbf", 1.0, eps)) < 1e-12
    assert abs(r_m12 - support.cutoff_distance("matern12", 1.0, eps)) < 1e-12
    r_m52 = support.zero_radius(kernels.MATERN52)
    r_m32 = support.zero_radius(kernels.MATERN32)
    assert r_rbf < r_m52 < r_m32 < r_m12
    for kind, r in ((kernels.MATERN52, r_m52), (kernels.MATERN32, r_m32)):
        assert abs(kernels.kfun(kind, r * r) / eps - 1.0) < 1e-9


def _fp16_kernel_matrix(X1, X2, kind, ls):
    from oracle import kmvm
    A = kmvm.quantize_inputs_fp16(X1, ls)
    B = kmvm.quantize_inputs_fp16(X2, ls)
    r2 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
    return kernels.kfun(kind, r2).astype(np.float16), r2


@pytest.mark.parametrize("kind", [kernels.RBF, kernels.MATERN52, kernels.MATERN32, kernels.MATERN12])
def test_truncated_product_drops_only_exact_zeros(kind):
    """Fig. 2c / the sparsified-MVM figure: dropping the unrepresentable pairs
    changes nothing -- every dropped binary16 kernel value is exactly zero, every
    kept one is nonzero, and the product equals the full binary16 emulation."""
    from oracle import kmvm
    g = np.random.default_rng(40 + kind)
    n1, n2 = 90, 140
    X1 = g.uniform(-12, 12, (n1, 2)).astype(np.float32)
    X2 = g.uniform(-12, 12, (n2, 2)).astype(np.float32)
    V = g.standard_normal((n2, 3)).astype(np.float32)
    ls = np.array([0.7, 1.1], np.float32)
    K16, r2 = _fp16_kernel_matrix(X1, X2, kind, ls)
    R = support.zero_radius(kind)
    far = r2 >= R * R
    assert far.any() and (~far).any()
    assert np.all(K16[far] == 0)
    assert np.all(K16[~far] != 0)
    full = kmvm.kmvm_fp16_emulated(X1, X2, V, kind, ls, 1.3, 0.1, False)
    trunc, kept = support.kmvm_fp16_truncated(X1, X2, V, kind, ls, 1.3, 0.1, False)
    assert kept == int(np.count_nonzero(~far))
    np.testing.assert_allclose(trunc, full, rtol=1e-13, atol=1e-13 * np.abs(full).max())


def test_truncated_product_fig1_setting_drops_the_far_pairs():
    """Fig. 1 points (500 evenly spaced in [-10, 10]), RBF l = 1: the kept
    fraction equals the fraction of pairs within the radius (counted directly)."""
    pv = paper_values()
    n = int(pv["fig1_points"])
    x = np.linspace(pv["fig1_lo"], pv["fig1_hi"], n).astype(np.float32)[:, None]
    V = np.ones((n, 1), np.float32)
    _, kept = support.kmvm_fp16_truncated(x, x, V, kernels.RBF, [1.0], 1.0, 0.0, False)
    xh = x.astype(np.float16).astype(np.float64)[:, 0]
    R = support.zero_radius(kernels.RBF)
    assert kept == int(np.count_nonzero(np.abs(xh[:, None] - xh[None, :]) < R))
    assert 0.3 < kept / n ** 2 < 0.7
