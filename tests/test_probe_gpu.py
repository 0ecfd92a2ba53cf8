"""gp_probe_rate: the issue-rate and bandwidth probes the roofline figures use.

Sanity bounds only (the figures themselves are measurements): every rate is
positive and below the chip's unit-count ceiling, and the orderings that the
instruction timings fix hold (a transcendental issues no faster than an FMA;
the 16x16x32 binary16 matrix instruction does twice the work of 16x16x16; a
loop with MFMAs and vector work is no faster than its MFMAs alone)."""
import pytest

pytestmark = pytest.mark.gpu

# 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz
LANE_CEIL = 256 * 4 * 16 * 2.4e9


def test_probe_rates_are_plausible(gpu_lib):
    r = {name: gpu_lib.probe_rate(name, 2000 if name != "copy" else 2)
         for name in gpu_lib.PROBES}
    print({k: f"{v:.3e}" for k, v in r.items()}, flush=True)
    for k in ("exp", "sqrt", "fma"):
        assert 0 < r[k] <= 2.0 * LANE_CEIL
    assert r["exp"] <= 1.05 * r["fma"] and r["sqrt"] <= 1.05 * r["fma"]
    assert 0 < r["mfma_f16_16x16x32"] <= 2.6e15
    assert 0 < r["mfma_f16_16x16x16"] <= 1.05 * r["mfma_f16_16x16x32"]
    assert 0 < r["mfma_f64_16x16x4"] <= 8.2e13
    assert 5e11 < r["copy"] <= 8.2e12
    # a mixed loop does the MFMA work of the MFMA loop plus vector work: it
    # cannot beat the MFMA loop's rate at the same occupancy
    for k in ("mix_fma", "mix_exp"):
        assert 0 < r[k] <= 1.05 * r["mfma_f16_16x16x32"]
    m2 = gpu_lib.probe_rate("mfma_f16_16x16x32", 2000, two_waves=True)
    for k in ("mix_fma", "mix_exp"):
        assert 0 < gpu_lib.probe_rate(k, 2000, two_waves=True) <= 1.05 * m2
    with pytest.raises(gpu_lib.GpError):
        gpu_lib.lib()  # library loaded
        import ctypes
        gpu_lib._check(gpu_lib.lib().gp_probe_rate(99, 10, None, ctypes.byref(ctypes.c_double())))
    with pytest.raises(gpu_lib.GpError):
        # the occupancy flag applies to the loop probes only
        gpu_lib._check(gpu_lib.lib().gp_probe_rate(gpu_lib.PROBES["copy"] | gpu_lib.PROBE_TWO_WAVES, 1,
                                                   None, ctypes.byref(ctypes.c_double())))
