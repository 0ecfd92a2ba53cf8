"""Pins for oracle.support against values the paper prints."""
import math

import numpy as np

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
