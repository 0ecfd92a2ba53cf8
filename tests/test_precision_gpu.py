"""Number-format variants on the GPU: the bfloat16-operand product (gp_kmvm /
gp_cg_solve with GP_PREC_BF16) and the binary16 summation ablations
(gp_kmvm_summation) against the oracle's emulations (oracle.precision).

Bars.
* bfloat16 product: <= 5e-4 relative to the bfloat16 emulation (same rounded
  operands, exact accumulation).  The device forms the exponent argument in
  float32 and the kernel value with the hardware exp2, so a kernel value whose
  float32 value sits next to a bfloat16 rounding boundary can round one ulp
  (2^-8 relative) the other way; with float32 accumulation that stays far
  below 5e-4 over thousands of terms.  Against the exact product the device
  error must be that of the emulation: <= 1.2 x emulation error + 2e-4.
* Summation ablations: bit-identical to the emulation where every kernel
  value is exactly 0 or 1 (duplicate points in two far clusters), so that the
  rounding sequence of the sums is checked operation by operation; on general
  data <= max(5e-4, 0.25 x the emulation's own error) relative to the
  emulation (a one-ulp binary16 flip of a kernel value changes one term by
  2^-11 relative and the rest of that row's rounding sequence a little) and
  the device's error against the exact product within 1.25 x the
  emulation's + 2e-4.
"""
import numpy as np
import pytest
import torch

from oracle import kmvm as okmvm
from oracle import direct, precision
from paper_2207_06856_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


BF16_CASES = [
    # n1, n2, d, r, kind, ard, noise, scale_mode
    (1000, 1000, 3, 1, 0, False, True, 0),
    (777, 777, 8, 16, 1, False, True, 0),
    (300, 300, 9, 17, 0, True, True, 1),
    (1500, 1500, 16, 33, 1, True, True, 0),
    (129, 129, 1, 8, 2, False, True, 0),
    (257, 257, 2, 15, 3, False, True, 0),
    (200, 200, 30, 4, 0, True, True, 0),
    (150, 150, 51, 2, 3, False, True, 0),
    (100, 100, 64, 2, 1, False, True, 0),
    (333, 333, 5, 70, 0, False, True, 0),
    (500, 1200, 5, 3, 0, False, False, 1),
    (1, 300, 4, 1, 1, False, False, 0),
    (300, 1, 4, 1, 0, False, False, 0),
]


@pytest.mark.parametrize("case", BF16_CASES, ids=lambda c: "n%d_%d_d%d_r%d_k%d%s_s%d" % (
    c[0], c[1], c[2], c[3], c[4], "_ard" if c[5] else "", c[7]))
def test_bf16_product_parity(gpu_lib, case):
    n1, n2, d, r, kind, ard, noise, sm = case
    seed = 2000 + n1 + 7 * d + 13 * r
    print(f"bf16 case n1={n1} n2={n2} d={d} r={r} kind={kind} scale_mode={sm}", flush=True)
    X1 = synth.random_points(n1, d, seed)
    X2 = X1 if noise else synth.random_points(n2, d, seed + 1)
    V = synth.random_rhs(n2, r, seed)
    ls = np.linspace(0.7, 1.6, d).astype(np.float32) if ard else np.array([1.1], np.float32)
    a2, s2 = 1.3, 0.05
    t1 = dev(X1)
    t2 = t1 if noise else dev(X2)
    out = gpu_lib.kmvm(t1, t2, dev(V), kind, ls, a2, s2, add_noise=noise, precision=gpu_lib.BF16,
                       scale_mode=sm).cpu().numpy()
    ref = okmvm.kmvm(X1, X2, V, kind, ls, a2, s2, noise)
    emu = precision.kmvm_bf16_emulated(X1, X2, V, kind, ls, a2, s2, noise, scale_mode=sm)
    e_dev, e_emu, gap = rel(out, ref), rel(emu, ref), rel(out, emu)
    print(f"  rel vs exact {e_dev:.3e} (emulation {e_emu:.3e}), vs emulation {gap:.3e}", flush=True)
    assert gap <= 5e-4
    assert e_dev <= 1.2 * e_emu + 2e-4


def test_bf16_far_field_keeps_small_values(gpu_lib):
    """bfloat16 has float32's exponent range: pairs 9 lengthscales apart give
    RBF values near exp(-40.5) ~ 2.6e-18, zero in binary16 but kept here."""
    X1 = np.zeros((256, 1), np.float32)
    X2 = np.full((128, 1), 9.0, np.float32)
    V = np.ones((128, 1), np.float32)
    t = gpu_lib.kmvm(dev(X1), dev(X2), dev(V), 0, [1.0], 1.0, 0.0, precision=gpu_lib.BF16).cpu().numpy()
    h = gpu_lib.kmvm(dev(X1), dev(X2), dev(V), 0, [1.0], 1.0, 0.0, precision=gpu_lib.FP16).cpu().numpy()
    emu = precision.kmvm_bf16_emulated(X1, X2, V, 0, [1.0], 1.0, 0.0, False)
    assert np.all(h == 0.0)
    assert np.all(t > 0.0)
    assert rel(t, emu) <= 1e-6


def test_bf16_solve_converges_and_floor_is_above_binary16(gpu_lib):
    """CG with the bfloat16 product reaches a loose tolerance, and its float64
    true-residual floor lies above the binary16 one on the same problem (the
    bfloat16 operator is about 8 times less accurate)."""
    p = synth.materialise(synth.served_requests(count=1, n_hi=3000, seed=21)[0])
    X, B = dev(p.X), dev(p.B)
    P = gpu_lib.Precond(X, p.kind, p.lengthscale, p.outputscale, p.noise, 50)
    res = {}
    for prec in (gpu_lib.FP16, gpu_lib.BF16):
        U, st = gpu_lib.cg_solve(X, B, p.kind, p.lengthscale, p.outputscale, p.noise, tol=1e-4,
                                 max_iter=300, min_iter=10, precision=prec, precond=P)
        res[prec] = (U.cpu().numpy(), st)
        print("precision", prec, "iters", st["iters"], "true rel res", st["true_rel_res"], flush=True)
    U_ref = direct.solve(p.X, p.B, p.kind, p.lengthscale, p.outputscale, p.noise)
    for prec in (gpu_lib.FP16, gpu_lib.BF16):
        assert np.all(np.isfinite(res[prec][0]))
    tb = np.max(res[gpu_lib.BF16][1]["true_rel_res"])
    th = np.max(res[gpu_lib.FP16][1]["true_rel_res"])
    assert tb > th
    assert tb <= 0.1
    assert rel(res[gpu_lib.BF16][0], U_ref) <= 0.2


def test_bf16_errors(gpu_lib):
    X = dev(np.zeros((10, 3)))
    V = dev(np.zeros((10, 1)))
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.kmvm(X, X, V, 0, [1.0], 1.0, 0.1, precision=3)


# ---- binary16 summation ablations -------------------------------------------

def _clusters(n, d, seed):
    """Duplicate points in two clusters 100 apart: kernel values exactly 1
    (same cluster) or 0 (the other cluster) in every format."""
    g = np.random.default_rng(seed)
    which = g.integers(0, 2, n)
    return (which[:, None] * 100.0 * np.ones((1, d))).astype(np.float32)


def _expected_bits(T, n2, a2=1.0):
    """Device output for a binary16 total T: the float32 product of T with the
    float32 factor a^2 * fl32(sqrt(n2)) (the inverse of the paper's scale)."""
    f = np.float32(np.float32(a2) * np.float32(np.sqrt(float(n2))))
    return (f * T.astype(np.float32)).astype(np.float32)


SUM_EXACT_CASES = [
    # n1, n2, d, r, kind, scheme, block
    (300, 1000, 2, 1, 0, "block_half", 1),
    (300, 1000, 2, 3, 1, "block_half", 7),
    (513, 1000, 3, 5, 2, "block_half", 32),
    (100, 2999, 2, 16, 3, "block_half", 1000),
    (300, 1000, 2, 21, 0, "block_single", 32),
    (300, 777, 9, 2, 1, "block_single", 128),
    (257, 1000, 2, 4, 0, "kahan_half", 1),
    (64, 4095, 2, 17, 3, "kahan_half", 1),
]
SCHEME_ID = {"block_half": 0, "block_single": 1, "kahan_half": 2}


@pytest.mark.parametrize("case", SUM_EXACT_CASES, ids=lambda c: "n%d_%d_d%d_r%d_k%d_%s_b%d" % c)
def test_summation_bit_exact_on_unit_kernel_values(gpu_lib, case):
    n1, n2, d, r, kind, scheme, block = case
    print(f"summation exact case {case}", flush=True)
    X1 = _clusters(n1, d, 31 + n1)
    X2 = _clusters(n2, d, 37 + n2)
    V = synth.random_rhs(n2, r, 41 + r)
    out = gpu_lib.kmvm_summation(dev(X1), dev(X2), dev(V), kind, [0.8], 1.0, 0.0,
                                 SCHEME_ID[scheme], block=block).cpu().numpy()
    P, s = precision.half_terms(X1, X2, V, kind, [0.8])
    T = precision.half_sum(P, scheme, block)
    want = _expected_bits(T, n2)
    assert np.array_equal(out, want), np.argwhere(out != want)[:5]


def test_summation_stagnation_on_gpu(gpu_lib):
    """4096 terms of 2^-6: the plain binary16 sum stops at 32 (out 2048), blocks
    of 256 and Kahan's sum reach 64 (out 4096)."""
    X1 = np.zeros((300, 2), np.float32)
    X2 = np.zeros((4096, 2), np.float32)
    V = np.ones((4096, 1), np.float32)
    run = lambda sch, b: gpu_lib.kmvm_summation(dev(X1), dev(X2), dev(V), 0, [1.0], 1.0, 0.0, sch,
                                               block=b).cpu().numpy()
    assert np.all(run(gpu_lib.SUM_BLOCK_HALF, 4096) == 2048.0)
    assert np.all(run(gpu_lib.SUM_BLOCK_HALF, 256) == 4096.0)
    assert np.all(run(gpu_lib.SUM_BLOCK_SINGLE, 256) == 4096.0)
    assert np.all(run(gpu_lib.SUM_KAHAN_HALF, 1) == 4096.0)


SUM_CASES = [
    # n1, n2, d, r, kind, scheme, block, noise
    (400, 2000, 3, 3, 0, "block_half", 32, False),
    (400, 2000, 3, 3, 0, "block_single", 32, False),
    (400, 2000, 3, 3, 0, "kahan_half", 1, False),
    (700, 700, 8, 5, 1, "block_single", 256, True),
    (300, 1500, 12, 2, 2, "block_half", 64, False),
    (300, 1500, 2, 4, 3, "kahan_half", 1, False),
]


@pytest.mark.parametrize("case", SUM_CASES, ids=lambda c: "n%d_%d_d%d_r%d_k%d_%s_b%d_noise%d" % c)
def test_summation_parity(gpu_lib, case):
    n1, n2, d, r, kind, scheme, block, noise = case
    print(f"summation case {case}", flush=True)
    seed = 3000 + n1 + 7 * d + r
    X1 = synth.random_points(n1, d, seed)
    X2 = X1 if noise else synth.random_points(n2, d, seed + 1)
    V = synth.random_rhs(n2, r, seed)
    ls, a2, s2 = [0.9], 1.2, 0.07
    t1 = dev(X1)
    t2 = t1 if noise else dev(X2)
    out = gpu_lib.kmvm_summation(t1, t2, dev(V), kind, ls, a2, s2, SCHEME_ID[scheme], block=block,
                                 add_noise=noise).cpu().numpy()
    emu = precision.kmvm_fp16_summation(X1, X2, V, kind, ls, a2, s2, noise, scheme, block=block)
    ref = okmvm.kmvm(X1, X2, V, kind, ls, a2, s2, noise)
    e_emu, gap, e_dev = rel(emu, ref), rel(out, emu), rel(out, ref)
    print(f"  emulation vs exact {e_emu:.3e}, device vs emulation {gap:.3e}, device vs exact {e_dev:.3e}",
          flush=True)
    assert gap <= max(5e-4, 0.25 * e_emu)
    assert e_dev <= 1.25 * e_emu + 2e-4


def test_summation_full_size_sampled_rows(gpu_lib):
    """N = 100,000 points of the mixed-precision workload (d = 8, RBF): sampled
    rows of each scheme against the emulation of those rows."""
    p = synth.mixed_precision(n=100_000, kind=0)
    X = dev(p.X)
    V = p.B[:, :1].copy()
    rows = np.random.default_rng(5).choice(p.X.shape[0], 24, replace=False)
    for scheme in ("block_half", "block_single", "kahan_half"):
        out = gpu_lib.kmvm_summation(X, X, dev(V), 0, p.lengthscale, 1.0, p.noise, SCHEME_ID[scheme],
                                     block=32, add_noise=True).cpu().numpy()
        emu = precision.kmvm_fp16_summation(p.X, p.X, V, 0, p.lengthscale, 1.0, p.noise, True, scheme,
                                            block=32, rows=rows)
        ref = okmvm.kmvm(p.X, p.X, V, 0, p.lengthscale, 1.0, p.noise, True, rows=rows)
        e_emu, gap = rel(emu, ref), rel(out[rows], emu)
        print(f"  {scheme}: emulation vs exact {e_emu:.3e}, device vs emulation {gap:.3e}", flush=True)
        assert np.all(np.isfinite(out))
        assert gap <= max(5e-4, 0.25 * e_emu)


def test_summation_argument_errors(gpu_lib):
    X = dev(np.zeros((10, 3)))
    V = dev(np.zeros((10, 1)))
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.kmvm_summation(X, X, V, 0, [1.0], 1.0, 0.1, 3)
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.kmvm_summation(X, X, V, 0, [1.0], 1.0, 0.1, gpu_lib.SUM_BLOCK_HALF, block=0)
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.kmvm_summation(X, X, V, 0, [1.0], 1.0, 0.1, gpu_lib.SUM_BLOCK_SINGLE, scale_mode=2)


def test_bf16_model_cache_and_predictions(gpu_lib):
    """A predictive-mean model whose cache solve and predictions both use the
    bfloat16 product.  In the oracle's bfloat16 emulation of this problem
    (dense solve with the rounded kernel matrix) the cache has a float64 true
    residual of 1.8e-2 (the bfloat16 operator's floor, above the 2e-3 the
    converged flag would need at tol 1e-3), the bfloat16 means are 8.8e-3 from
    the exact means and 1.8e-2 from float32 means of the same cache; bars
    5e-2, 2e-2 and 3e-2."""
    g = np.random.default_rng(12)
    X = g.uniform(-3, 3, (1500, 3)).astype(np.float32)
    y = (np.sin(2 * X[:, 0]) + 0.1 * g.standard_normal(1500)).astype(np.float32)
    Xs = g.uniform(-3, 3, (300, 3)).astype(np.float32)
    ls, a2, s2 = [0.8], 1.0, float(np.float32(0.1))
    mu_ref, _ = direct.predictive_mean(X, y, Xs, 0, ls, a2, s2)
    with gpu_lib.Model(dev(X), dev(y), 0, ls, a2, s2, precond_rank=40, tol=1e-3, max_iter=500,
                       precision=gpu_lib.BF16) as m:
        info = m.info()
        print("bf16 cache solve", info, flush=True)
        assert info["iters"] < 500 and info["true_rel_res"] <= 5e-2
        mub = m.predict(dev(Xs), precision=gpu_lib.BF16).cpu().numpy()
        mu32 = m.predict(dev(Xs), precision=gpu_lib.FP32).cpu().numpy()
    print("rel bf16", rel(mub, mu_ref), "fp32 from bf16 cache", rel(mu32, mu_ref), flush=True)
    assert rel(mub, mu_ref) <= 2e-2
    assert rel(mub, mu32) <= 3e-2


def test_empty_sets_bf16_and_summation(gpu_lib):
    """n2 = 0 gives zeros, n1 = 0 an empty output, for the bfloat16 product and
    every summation scheme."""
    X = torch.from_numpy(synth.random_points(10, 3, 8)).to(DEV)
    V = torch.from_numpy(synth.random_rhs(10, 2, 8)).to(DEV)
    e = torch.empty((0, 3), device=DEV)
    ev = torch.empty((0, 2), device=DEV)
    out = gpu_lib.kmvm(X, e, ev, 0, [1.0], 1.0, 0.1, precision=gpu_lib.BF16)
    assert out.shape == (10, 2) and torch.all(out == 0)
    assert gpu_lib.kmvm(e, X, V, 0, [1.0], 1.0, 0.1, precision=gpu_lib.BF16).shape == (0, 2)
    for sch in (gpu_lib.SUM_BLOCK_HALF, gpu_lib.SUM_BLOCK_SINGLE, gpu_lib.SUM_KAHAN_HALF):
        out = gpu_lib.kmvm_summation(X, e, ev, 0, [1.0], 1.0, 0.1, sch)
        assert out.shape == (10, 2) and torch.all(out == 0)
        assert gpu_lib.kmvm_summation(e, X, V, 0, [1.0], 1.0, 0.1, sch).shape == (0, 2)


def test_summation_single_column_and_tiny_blocks(gpu_lib):
    """n2 = 1 (one term: every scheme returns fp16(k v) exactly) and a block
    longer than n2, against the emulation bit for bit on unit kernel values."""
    X1 = _clusters(70, 2, 3)
    X2 = np.zeros((1, 2), np.float32)
    V = np.array([[0.3, -1.7, 2.5]], np.float32)
    for scheme in ("block_half", "block_single", "kahan_half"):
        out = gpu_lib.kmvm_summation(dev(X1), dev(X2), dev(V), 0, [0.8], 1.0, 0.0,
                                     SCHEME_ID[scheme], block=5).cpu().numpy()
        P, _ = precision.half_terms(X1, X2, V, 0, [0.8])
        want = _expected_bits(precision.half_sum(P, scheme, 5), 1)
        assert np.array_equal(out, want)


@pytest.mark.parametrize("kind,rank", [(1, 20), (0, 0)])
def test_bf16_enhanced_matched_iteration_parity(gpu_lib, kind, rank):
    """Alg. 1 with the bfloat16 product at tol 1.0 against the oracle's Alg. 1
    run for the same per-column iteration counts, whose operator is the
    bfloat16 model: a^2 k_hat(x_hat_i, x_hat_j) applied to the direction
    rounded to bfloat16 (power-of-two column scales leave that rounding
    unchanged) plus s^2 times the direction (oracle.precision.Operator16,
    pinned against the emulated bfloat16 product).  What remains is
    float32 accumulation, the float32 exponent argument and float32 CG
    arithmetic against float64 over 10 iterations (~3e-4 at these sizes):
    bar 3e-3, a tenth of the gap to the exact solve's 0.13-0.32."""
    from oracle import cg as ocg
    from oracle import pivchol
    p = synth.mixed_precision(n=2000, kind=kind)
    tX, tB = dev(p.X), dev(p.B)
    P = gpu_lib.Precond(tX, kind, p.lengthscale, 1.0, p.noise, rank) if rank else None
    U, st = gpu_lib.cg_solve(tX, tB, kind, p.lengthscale, 1.0, p.noise, tol=1.0, max_iter=100,
                             min_iter=10, precond=P, precision=gpu_lib.BF16)
    print("bf16 iters", st["iters"], "true", st["true_rel_res"].max(), flush=True)
    assert not st["breakdown"].any()
    mvm = precision.Operator16(p.X, kind, p.lengthscale, 1.0, p.noise, fmt="bf16")
    Pc = pivchol.build(p.X, kind, p.lengthscale, 1.0, p.noise, rank)[0] if rank else None
    ref, _ = ocg.solve(mvm, p.B.astype(np.float64), tol=0.0, max_iter=st["iters"], precond=Pc)
    got = U.cpu().numpy()
    exact_op = np.linalg.solve(direct.ktilde(p.X, kind, p.lengthscale, 1.0, p.noise), p.B)
    print("vs bf16-model oracle", rel(got, ref), "vs exact solve", rel(got, exact_op), flush=True)
    assert rel(got, ref) <= 3e-3


def _random_shapes(seed, count):
    g = np.random.default_rng(seed)
    for _ in range(count):
        yield (int(g.integers(1, 700)), int(g.integers(1, 700)), int(g.integers(1, 65)),
               int(g.integers(1, 41)), int(g.integers(0, 4)), int(g.integers(0, 2 ** 31)))


@pytest.mark.parametrize("case", list(_random_shapes(77, 12)),
                         ids=lambda c: "n%d_%d_d%d_r%d_k%d" % c[:5])
def test_bf16_random_shapes(gpu_lib, case):
    """Seeded random shapes (ragged n1, n2 < 700, d up to 64, r up to 40, all
    kernels) against the bfloat16 emulation, bars as above."""
    n1, n2, d, r, kind, seed = case
    print(f"bf16 random case {case}", flush=True)
    X1 = synth.random_points(n1, d, seed % 100000)
    X2 = synth.random_points(n2, d, seed % 100000 + 1)
    V = synth.random_rhs(n2, r, seed % 100000)
    ls = np.array([1.3 * np.sqrt(d / 4.0)], np.float32)
    out = gpu_lib.kmvm(dev(X1), dev(X2), dev(V), kind, ls, 0.8, 0.0,
                       precision=gpu_lib.BF16).cpu().numpy()
    emu = precision.kmvm_bf16_emulated(X1, X2, V, kind, ls, 0.8, 0.0, False)
    ref = okmvm.kmvm(X1, X2, V, kind, ls, 0.8, 0.0, False)
    gap, e_emu, e_dev = rel(out, emu), rel(emu, ref), rel(out, ref)
    print(f"  vs emulation {gap:.3e}, emulation vs exact {e_emu:.3e}", flush=True)
    assert gap <= 5e-4
    assert e_dev <= 1.2 * e_emu + 2e-4


@pytest.mark.parametrize("case", list(_random_shapes(78, 12)),
                         ids=lambda c: "n%d_%d_d%d_r%d_k%d" % c[:5])
def test_summation_random_shapes(gpu_lib, case):
    """Seeded random shapes for the summation schemes (scheme and block length
    drawn too): bit-identical on unit kernel values (two far clusters)."""
    n1, n2, d, r, kind, seed = case
    g = np.random.default_rng(seed)
    scheme = ("block_half", "block_single", "kahan_half")[int(g.integers(0, 3))]
    block = int(g.integers(1, 300))
    print(f"summation random case {case} {scheme} block {block}", flush=True)
    X1 = _clusters(n1, d, seed % 1000)
    X2 = _clusters(n2, d, seed % 1000 + 1)
    V = synth.random_rhs(n2, r, seed % 100000)
    out = gpu_lib.kmvm_summation(dev(X1), dev(X2), dev(V), kind, [0.8], 1.0, 0.0,
                                 SCHEME_ID[scheme], block=block).cpu().numpy()
    P, _ = precision.half_terms(X1, X2, V, kind, [0.8])
    want = _expected_bits(precision.half_sum(P, scheme, block), n2)
    assert np.array_equal(out, want)
