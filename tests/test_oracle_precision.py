"""Pins for oracle.precision: bfloat16 rounding and the bfloat16 product
(Sec. 2.1), and the binary16 summation schemes (Sec. 5.1, Fig. 4; App. B).

Independent references: torch's float32 -> bfloat16 conversion, Python's
struct module (binary16 'e' and binary32 'f' packing, both round to nearest
even), closed forms of binary16 stagnation, and the recursive-summation error
bound gamma_k = k u / (1 - k u) (Higham, Accuracy and Stability of Numerical
Algorithms, Eq. 4.4).
"""
import math
import struct

import numpy as np
import pytest
import torch

from oracle import kernels, kmvm, precision


def _h(x):
    return struct.unpack("<e", struct.pack("<e", x))[0]


def _f(x):
    return struct.unpack("<f", struct.pack("<f", x))[0]


# ---- bfloat16 rounding ------------------------------------------------------

def test_round_bf16_matches_torch_on_float32_values():
    g = np.random.default_rng(3)
    bits = g.integers(0, 2 ** 32, 200_000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    # ties, halfway-plus-one, subnormals, the overflow boundary
    special = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -23, 2 ** -130,
                        3 * 2 ** -134, 2 ** -134, precision.BF16_MAX,
                        precision.BF16_MAX * (1 + 2 ** -9), 2 ** 127 * (2 - 2 ** -8),
                        -2.5e-40, 65504.0, 3.14159265], dtype=np.float32)
    x = np.concatenate([x, special, -special])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = precision.round_bf16(x.astype(np.float64))
    same = (got == ref) | (np.isnan(got) & np.isnan(ref))
    assert np.all(same), (x[~same][:5], got[~same][:5], ref[~same][:5])


def test_round_bf16_closed_forms():
    r = precision.round_bf16
    assert r(1 + 2 ** -8) == 1.0                       # tie -> even
    assert r(1 + 3 * 2 ** -8) == 1 + 2 ** -6           # tie -> even (upwards)
    # rounded directly from float64: just above a tie goes up, although the
    # float32 rounding of the same value is the tie itself
    assert r(1 + 2 ** -8 + 2 ** -40) == 1 + 2 ** -7
    assert r(math.pi) == 3.140625
    assert r(precision.BF16_MAX) == precision.BF16_MAX
    assert r(2.0 ** 128 * (1 - 2 ** -9)) == math.inf    # halfway above the largest finite
    assert r(2.0 ** -133) == 2.0 ** -133 and r(2.0 ** -134) == 0.0 and r(3 * 2.0 ** -134) == 2.0 ** -132
    assert r(-0.0) == 0.0 and math.isnan(r(float("nan")))


def test_round_bf16_error_and_significand():
    g = np.random.default_rng(4)
    x = g.standard_normal(100_000) * np.exp(g.uniform(-80, 80, 100_000))
    y = precision.round_bf16(x)
    assert np.all(np.abs(y - x) <= precision.BF16_UNIT_ROUNDOFF * np.abs(x))
    m, _ = np.frexp(y)
    assert np.all(np.ldexp(m, 8) == np.rint(np.ldexp(m, 8)))     # at most 8 significant bits


# ---- bfloat16 product -------------------------------------------------------

def test_bf16_product_exact_when_entries_are_representable():
    """Points in two far clusters (kernel values exactly 1 or 0) and right-hand
    sides on the bfloat16 grid: nothing rounds, so the emulation is the plain
    product."""
    g = np.random.default_rng(5)
    n, d = 60, 3
    X = np.where(np.arange(n)[:, None] % 2 == 0, 0.0, 100.0) * np.ones((1, d))
    V = precision.round_bf16(g.standard_normal((n, 3)))
    for kind in (kernels.RBF, kernels.MATERN52, kernels.MATERN12, kernels.MATERN32):
        ref = kmvm.kmvm(X, X, V, kind, [0.7], 1.5, 0.1, True)
        got = precision.kmvm_bf16_emulated(X, X, V, kind, [0.7], 1.5, 0.1, True)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_bf16_input_rounding_merges_close_points():
    """With l = 2^-6 the scaled inputs are 64 and 64.125: the same bfloat16
    value (spacing 0.5 there), so their kernel value is 1, while binary16
    (spacing 1/16) keeps them 0.125 apart: exp(-1/128) in binary16."""
    X1 = np.array([[1.0]])
    X2 = np.array([[1.0 + 2 ** -9]])
    V = np.array([[1.0]])
    ls = [2.0 ** -6]
    assert precision.kmvm_bf16_emulated(X1, X2, V, kernels.RBF, ls, 1.0, 0.0, False)[0, 0] == 1.0
    want = float(np.float16(math.exp(-1 / 128)))
    assert kmvm.kmvm_fp16_emulated(X1, X2, V, kernels.RBF, ls, 1.0, 0.0, False)[0, 0] == want < 1.0


def test_bf16_product_brute_force_with_torch_rounding():
    g = np.random.default_rng(6)
    n1, n2, d = 4, 7, 2
    X1 = g.uniform(-2, 2, (n1, d)).astype(np.float32)
    X2 = g.uniform(-2, 2, (n2, d)).astype(np.float32)
    V = g.standard_normal((n2, 2)).astype(np.float32)
    ls = np.array([0.8, 1.3], np.float32)

    def bf(v):
        return float(torch.tensor(float(v), dtype=torch.float32).to(torch.bfloat16).float())

    s = kmvm.column_scales(V, n2, 0)
    for kind in (kernels.RBF, kernels.MATERN52):
        got = precision.kmvm_bf16_emulated(X1, X2, V, kind, ls, 0.9, 0.0, False)
        for i in range(n1):
            for c in range(2):
                acc = 0.0
                for j in range(n2):
                    r2 = sum((bf(np.float32(X1[i, m]) / ls[m]) - bf(np.float32(X2[j, m]) / ls[m])) ** 2
                             for m in range(d))
                    kv = math.exp(-r2 / 2) if kind == kernels.RBF else \
                        (1 + math.sqrt(5 * r2) + 5 * r2 / 3) * math.exp(-math.sqrt(5 * r2))
                    acc += bf(kv) * bf(np.float32(V[j, c]) * s[c])
                assert abs(got[i, c] - 0.9 * acc / float(s[c])) <= 1e-12 * (1 + abs(got[i, c]))


def test_bf16_error_bound_on_grid_inputs():
    """Inputs on the bfloat16 grid with unit lengthscales: each term k_hat v_hat
    is within (2u + u^2)|k v| of k v (u = 2^-8), so each output entry is within
    (2u + u^2) a^2 sum_j |k_ij v_j| of the exact product, and the rounding is
    not a no-op (the error is a visible fraction of that bound)."""
    g = np.random.default_rng(7)
    n, d = 400, 3
    X = precision.round_bf16(g.uniform(-3, 3, (n, d)))
    V = g.standard_normal((n, 2))
    u = precision.BF16_UNIT_ROUNDOFF
    for kind in (kernels.RBF, kernels.MATERN32):
        got = precision.kmvm_bf16_emulated(X, X, V, kind, [1.0], 1.2, 0.0, False)
        ref = kmvm.kmvm(X, X, V, kind, [1.0], 1.2, 0.0, False)
        absK = 1.2 * kernels.kfun(kind, kernels.scaled_sqdist(X, X, [1.0]))
        bound = (2 * u + u * u) * (absK @ np.abs(V))
        err = np.abs(got - ref)
        assert np.all(err <= bound)
        assert np.median(err / bound) > 0.01


# ---- binary16 summation schemes --------------------------------------------

def _stagnation_case(n2):
    X = np.zeros((3, 2))
    X2 = np.zeros((n2, 2))
    V = np.ones((n2, 1))
    return X, X2, V


def test_half_sum_stagnation_closed_form():
    """4096 terms of 2^-6 (kernel value 1, v = 1, s_c = 4096^(-1/2) = 2^-6):
    the plain binary16 sum stops at 2^11 * 2^-6 = 32, where adding 2^-6 is a tie
    that rounds back to 32, so out = 32 / 2^-6 = 2048 instead of 4096; blocks
    of 256 sum exactly (4 per block, 64 in total), and so does Kahan's sum."""
    X1, X2, V = _stagnation_case(4096)
    f = precision.kmvm_fp16_summation
    assert np.all(f(X1, X2, V, kernels.RBF, [1.0], 1.0, 0.0, False, "block_half", block=4096) == 2048.0)
    assert np.all(f(X1, X2, V, kernels.RBF, [1.0], 1.0, 0.0, False, "block_half", block=1) == 2048.0)
    assert np.all(f(X1, X2, V, kernels.RBF, [1.0], 1.0, 0.0, False, "block_half", block=256) == 4096.0)
    assert np.all(f(X1, X2, V, kernels.RBF, [1.0], 1.0, 0.0, False, "block_single", block=4096) == 2048.0)
    assert np.all(f(X1, X2, V, kernels.RBF, [1.0], 1.0, 0.0, False, "block_single", block=256) == 4096.0)
    assert np.all(f(X1, X2, V, kernels.MATERN52, [1.0], 1.0, 0.0, False, "kahan_half") == 4096.0)


def _brute(P, scheme, block):
    n1, n2, R = P.shape
    out = np.zeros((n1, R))
    for i in range(n1):
        for c in range(R):
            p = [float(P[i, j, c]) for j in range(n2)]
            if scheme == "kahan_half":
                s = comp = 0.0
                for x in p:
                    y = _h(x - comp)
                    t = _h(s + y)
                    comp = _h(_h(t - s) - y)
                    s = t
                out[i, c] = s
                continue
            tot = 0.0
            for j0 in range(0, n2, block):
                bs = 0.0
                for x in p[j0:j0 + block]:
                    bs = _h(bs + x)
                tot = _h(tot + bs) if scheme == "block_half" else _f(tot + bs)
            out[i, c] = tot if scheme == "block_half" else _h(tot)
    return out


@pytest.mark.parametrize("scheme", precision.SCHEMES)
def test_half_sum_brute_force_struct_rounding(scheme):
    g = np.random.default_rng(8)
    n1, n2, d = 5, 203, 2
    X1 = g.uniform(-2, 2, (n1, d))
    X2 = g.uniform(-2, 2, (n2, d))
    V = g.standard_normal((n2, 2))
    P, s = precision.half_terms(X1, X2, V, kernels.RBF, [0.9])
    # the terms themselves: fp16(fp16(k) * fp16(v s))
    Xh1 = kmvm.quantize_inputs_fp16(X1, [0.9])
    Xh2 = kmvm.quantize_inputs_fp16(X2, [0.9])
    for (i, j, c) in [(0, 0, 0), (3, 101, 1), (4, 202, 0)]:
        r2 = float(np.sum((Xh1[i] - Xh2[j]) ** 2))
        want = _h(_h(math.exp(-r2 / 2)) * _h(float(np.float32(V[j, c]) * s[c])))
        assert float(P[i, j, c]) == want
    for block in (1, 16, 64, 500):
        got = precision.half_sum(P, scheme, block)
        assert np.array_equal(got, _brute(P, scheme, block)), (scheme, block)


def test_block_sizes_one_and_all_are_the_plain_sum():
    g = np.random.default_rng(9)
    P, _ = precision.half_terms(g.uniform(-2, 2, (6, 3)), g.uniform(-2, 2, (300, 3)),
                                g.standard_normal((300, 3)), kernels.MATERN32, [1.1])
    a = precision.half_sum(P, "block_half", 1)
    assert np.array_equal(a, precision.half_sum(P, "block_half", 300))
    assert np.array_equal(a, precision.half_sum(P, "block_half", 10_000))


def _gamma(k, u):
    return k * u / (1 - k * u)


@pytest.mark.parametrize("block", [32, 256])
def test_block_sums_within_recursive_summation_bounds(block):
    """Terms fixed, only the sums round: block_half is a recursive sum of depth
    (block - 1) + (nb - 1) in binary16; block_single has depth block - 1 in
    binary16, nb - 1 in float32 and one final rounding to binary16."""
    g = np.random.default_rng(10)
    n2 = 3000
    P, _ = precision.half_terms(g.uniform(-2, 2, (20, 2)), g.uniform(-2, 2, (n2, 2)),
                                g.standard_normal((n2, 2)), kernels.RBF, [0.6])
    exact = P.astype(np.float64).sum(axis=1)
    absum = np.abs(P.astype(np.float64)).sum(axis=1)
    u16, u32 = 2.0 ** -11, 2.0 ** -24
    nb = -(-n2 // block)
    e_half = np.abs(precision.half_sum(P, "block_half", block) - exact)
    assert np.all(e_half <= _gamma(block - 1 + nb - 1, u16) * absum)
    e_single = np.abs(precision.half_sum(P, "block_single", block) - exact)
    b = (1 + _gamma(block - 1, u16)) * (1 + _gamma(nb - 1, u32)) * (1 + u16) - 1
    assert np.all(e_single <= b * absum)


def test_summation_accuracy_ordering_of_fig4():
    """Fig. 4b's finding on synthetic data (positive right-hand side, blocks of
    32): binary16 block sums accumulated in single precision average below
    0.1% relative error against the exact product; accumulating them in half
    is clearly worse; Kahan's sum in half is nearly as accurate as the
    single-precision accumulation."""
    g = np.random.default_rng(11)
    n, d = 4096, 3
    X = g.uniform(0, 4, (n, d))
    V = g.uniform(0, 1, (n, 1))
    rows = np.arange(0, n, 16)
    ref = kmvm.kmvm(X, X, V, kernels.RBF, [0.5], 1.0, 0.0, False, rows=rows)

    def err(scheme):
        got = precision.kmvm_fp16_summation(X, X, V, kernels.RBF, [0.5], 1.0, 0.0, False, scheme,
                                            block=32, rows=rows)
        return float(np.mean(np.abs(got - ref)) / np.mean(np.abs(ref)))

    e_half, e_single, e_kahan = err("block_half"), err("block_single"), err("kahan_half")
    print("mean relative error: block_half", e_half, "block_single", e_single, "kahan_half", e_kahan)
    assert e_single < 1e-3
    assert e_half > 2.0 * e_single
    assert e_kahan < 1.5 * e_single


def test_summation_argument_errors():
    P = np.zeros((1, 2, 1), np.float16)
    with pytest.raises(ValueError):
        precision.half_sum(P, "pairwise", 4)
    with pytest.raises(ValueError):
        precision.half_sum(P, "block_half", 0)


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
@pytest.mark.parametrize("kind", [0, 1, 3])
def test_operator16_equals_the_emulated_products(fmt, kind):
    """Operator16 applies exactly the emulated 16-bit product (same rounded
    inputs, kernel values, right-hand sides and scales): equal to
    kmvm_fp16_emulated / kmvm_bf16_emulated up to float64 summation order, for
    several right-hand sides (each with its own column scale), including a
    column with tiny entries and a single vector."""
    from oracle import kmvm
    g = np.random.default_rng(7)
    X = g.standard_normal((300, 3)) * 2.0
    V = g.standard_normal((300, 5))
    V[:, 2] *= 1e-6
    ls, a2, s2 = [0.7], 1.3, 0.05
    op = precision.Operator16(X, kind, ls, a2, s2, fmt=fmt, block=128)
    want = (kmvm.kmvm_fp16_emulated(X, X, V, kind, ls, a2, s2, True) if fmt == "fp16"
            else precision.kmvm_bf16_emulated(X, X, V, kind, ls, a2, s2, True))
    got = op(V)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    np.testing.assert_allclose(op(V[:, 1]), want[:, 1], rtol=1e-12,
                               atol=1e-12 * np.abs(want).max())
    # the rounding is not a no-op: it differs from the exact product
    exact = kmvm.kmvm(X, X, V, kind, ls, a2, s2, True)
    assert np.linalg.norm(got - exact) > 1e-6 * np.linalg.norm(exact)
