"""Python binding of libgpmi.so (ctypes; argument marshalling only).

Every computation happens in the HIP library.  PyTorch supplies device memory
and the current stream; tensors must be contiguous float32 CUDA tensors.  If
the library has not been built this module raises on first use: there is no
CPU fallback.
"""

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpmi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gpmi.h")

GP_OK = 0
GP_PENDING = 1
GP_ERR_ARG = -1
GP_ERR_NOMEM = -2
GP_ERR_HIP = -3
GP_ERR_NOT_PD = -4
GP_ERR_BREAKDOWN = -5
GP_ERR_TOO_LARGE = -6
GP_ERR_UNKNOWN_TICKET = -7
GP_ERR_CANCELLED = -8
GP_ERR_STOPPED = -9

RBF = 0
MATERN52 = 1
MATERN12 = 2
MATERN32 = 3

FP32 = 0
FP16 = 1
BF16 = 2

SUM_BLOCK_HALF = 0
SUM_BLOCK_SINGLE = 1
SUM_KAHAN_HALF = 2

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_f32 = ctypes.c_float
c_vp = ctypes.c_void_p


class GpKernel(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("ard", c_i32), ("lengthscale", ctypes.POINTER(c_f32)),
                ("outputscale", c_f32), ("noise", c_f32)]


CG_STANDARD = 0
CG_ENHANCED = 1


class GpCgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", c_i32), ("min_iter", c_i32),
                ("algo", c_i32), ("reorth", c_i32), ("use_lse", c_i32), ("precision", c_i32),
                ("scale_mode", c_i32), ("x0_given", c_i32), ("true_res_every", c_i32),
                ("poll_every", c_i32), ("P", c_vp)]


class GpCgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(c_i32)), ("rel_res", ctypes.POINTER(c_f32)),
                ("true_rel_res", ctypes.POINTER(ctypes.c_double)),
                ("converged", ctypes.POINTER(ctypes.c_int8)),
                ("breakdown", ctypes.POINTER(ctypes.c_int8)),
                ("history", ctypes.POINTER(c_f32)), ("true_history", ctypes.POINTER(ctypes.c_double)),
                ("total_iters", c_i32), ("mvms", c_i32)]


class GpProblem(ctypes.Structure):
    _fields_ = [("k", GpKernel), ("X", c_vp), ("n", c_i64), ("d", c_i32), ("B", c_vp),
                ("r", c_i32), ("U", c_vp), ("precond_rank", c_i32)]


class GpServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", c_i32), ("device", c_i32),
                ("iters_per_round", c_i32), ("min_iter", c_i32), ("algo", c_i32),
                ("reorth", c_i32), ("use_lse", c_i32), ("scale_mode", c_i32)]


class GpRequest(ctypes.Structure):
    _fields_ = [("k", GpKernel), ("X", c_vp), ("n", c_i64), ("d", c_i32), ("B", c_vp),
                ("r", c_i32), ("U_out", c_vp), ("tol", ctypes.c_double), ("max_iter", c_i32),
                ("precond_rank", c_i32), ("stats", ctypes.POINTER(GpCgStats))]


class GpResult(ctypes.Structure):
    _fields_ = [("status", c_i32), ("iters", c_i32), ("converged", c_i32), ("breakdown", c_i32),
                ("max_rel_res", ctypes.c_double), ("max_true_rel_res", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_finish", ctypes.c_double), ("footprint_bytes", ctypes.c_uint64),
                ("message", ctypes.c_char * 128)]


class GpServeStats(ctypes.Structure):
    _fields_ = [("queued", c_i32), ("resident", c_i32), ("submitted", c_i64),
                ("completed", c_i64), ("rounds", c_i64), ("iterations", c_i64),
                ("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("busy_seconds", ctypes.c_double), ("uptime_seconds", ctypes.c_double)]


class GpTuneInfo(ctypes.Structure):
    _fields_ = [("tuned", c_i32), ("f16_splits", c_i32 * 8), ("f16_bucket_rows", c_i64 * 8),
                ("f16_gain", ctypes.c_double * 8), ("batched_split_div", c_i32),
                ("batched_persistent", c_i32), ("batched_gain", ctypes.c_double)]


TRAIN_MAX_DIM = 32
TRAIN_MAX_PARAMS = TRAIN_MAX_DIM + 2
_dvec = ctypes.c_double * TRAIN_MAX_PARAMS


class GpTrainConfig(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("ard", c_i32), ("probes", c_i32), ("precond_rank", c_i32),
                ("use_priors", c_i32), ("pad_", c_i32), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("cg", GpCgOpts)]


class GpTrainStepInfo(ctypes.Structure):
    _fields_ = [("step", c_i32), ("cg_iters", c_i32), ("cg_converged", c_i32),
                ("precond_rank", c_i32), ("max_rel_res", ctypes.c_double), ("theta", _dvec),
                ("grad", _dvec), ("raw_grad", _dvec), ("theta_next", _dvec),
                ("data_fit", ctypes.c_double), ("seconds_precond", ctypes.c_double),
                ("seconds_solve", ctypes.c_double), ("seconds_grad", ctypes.c_double)]


class GpTrainState(ctypes.Structure):
    _fields_ = [("nparams", c_i32), ("step", c_i32), ("raw", _dvec), ("m", _dvec), ("v", _dvec),
                ("theta", _dvec)]


class GpModelInfo(ctypes.Structure):
    _fields_ = [("n", c_i64), ("d", c_i32), ("iters", c_i32), ("converged", c_i32),
                ("rel_res", c_f32), ("true_rel_res", ctypes.c_double)]


class GpPredictRequest(ctypes.Structure):
    _fields_ = [("model", c_vp), ("Xs", c_vp), ("ns", c_i64), ("mu_out", c_vp), ("truncate", c_i32)]


class GpTruncStats(ctypes.Structure):
    _fields_ = [("tiles_total", c_i64), ("tiles_visited", c_i64), ("radius", ctypes.c_double)]


class GpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"gpmi status {status}: {message}")
        self.status = status


_lib = None


def _declare(L):
    L.gp_last_error.restype = ctypes.c_char_p
    L.gp_last_error.argtypes = []
    L.gp_version.restype = ctypes.c_char_p
    L.gp_version.argtypes = []
    L.gp_release_cached_memory.restype = c_i32
    L.gp_release_cached_memory.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
    L.gp_kmvm.restype = c_i32
    L.gp_kmvm.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_vp, c_i64, c_i32, c_vp, c_i32,
                          c_vp, c_i32, c_i32, c_i32, c_vp]
    L.gp_kmvm_noalloc.restype = c_i32
    L.gp_kmvm_noalloc.argtypes = L.gp_kmvm.argtypes
    L.gp_kmvm_noalloc_scratch_bytes.restype = ctypes.c_uint64
    L.gp_kmvm_noalloc_scratch_bytes.argtypes = []
    L.gp_true_residual_rows.restype = c_i32
    L.gp_true_residual_rows.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_i32, c_vp, c_vp,
                                        c_i32, c_vp, c_i64, c_vp, c_vp]
    L.gp_probe_rate.restype = c_i32
    L.gp_probe_rate.argtypes = [c_i32, c_i64, c_vp, ctypes.POINTER(ctypes.c_double)]
    L.gp_pivchol_precond.restype = c_i32
    L.gp_pivchol_precond.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_i32, c_i32,
                                     ctypes.POINTER(c_vp), c_vp]
    L.gp_precond_apply.restype = c_i32
    L.gp_precond_apply.argtypes = [c_vp, c_vp, c_i32, c_vp, c_vp]
    L.gp_precond_info.restype = c_i32
    L.gp_precond_info.argtypes = [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64),
                                  ctypes.POINTER(ctypes.c_double)]
    L.gp_precond_destroy.restype = c_i32
    L.gp_precond_destroy.argtypes = [c_vp]
    L.gp_cg_solve_batched.restype = c_i32
    L.gp_cg_solve_batched.argtypes = [c_i32, ctypes.POINTER(GpProblem), ctypes.POINTER(GpCgOpts),
                                      ctypes.POINTER(GpCgStats), c_vp]
    L.gp_profile_enable.restype = c_i32
    L.gp_profile_enable.argtypes = [c_i32]
    L.gp_profile_read.restype = c_i32
    L.gp_profile_read.argtypes = [c_i64, ctypes.POINTER(c_f32), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(c_i32), ctypes.POINTER(c_i64)]
    L.gp_profile_reset.restype = c_i32
    L.gp_profile_reset.argtypes = []
    L.gp_cg_default_opts.restype = None
    L.gp_cg_default_opts.argtypes = [ctypes.POINTER(GpCgOpts)]
    L.gp_serve_default_config.restype = None
    L.gp_serve_default_config.argtypes = [ctypes.POINTER(GpServeConfig)]
    L.gp_serve_create.restype = c_i32
    L.gp_serve_create.argtypes = [ctypes.POINTER(GpServeConfig), ctypes.POINTER(c_vp)]
    L.gp_serve_submit.restype = c_i32
    L.gp_serve_submit.argtypes = [c_vp, ctypes.POINTER(GpRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.gp_serve_poll.restype = c_i32
    L.gp_serve_poll.argtypes = [c_vp, ctypes.c_uint64, ctypes.POINTER(GpResult)]
    L.gp_serve_wait.restype = c_i32
    L.gp_serve_wait.argtypes = [c_vp, ctypes.c_uint64, c_i64, ctypes.POINTER(GpResult)]
    L.gp_serve_cancel.restype = c_i32
    L.gp_serve_cancel.argtypes = [c_vp, ctypes.c_uint64]
    L.gp_serve_stats_read.restype = c_i32
    L.gp_serve_stats_read.argtypes = [c_vp, ctypes.POINTER(GpServeStats)]
    L.gp_serve_destroy.restype = c_i32
    L.gp_serve_destroy.argtypes = [c_vp]
    L.gp_autotune.restype = c_i32
    L.gp_autotune.argtypes = [c_i32, c_vp, ctypes.POINTER(GpTuneInfo)]
    L.gp_tune_get.restype = c_i32
    L.gp_tune_get.argtypes = [ctypes.POINTER(GpTuneInfo)]
    L.gp_tune_reset.restype = c_i32
    L.gp_tune_reset.argtypes = []
    L.gp_tune_set.restype = c_i32
    L.gp_tune_set.argtypes = [ctypes.POINTER(GpTuneInfo)]
    L.gp_model_default_opts.restype = None
    L.gp_model_default_opts.argtypes = [ctypes.POINTER(GpCgOpts)]
    L.gp_model_create.restype = c_i32
    L.gp_model_create.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_i32, c_vp,
                                  ctypes.POINTER(GpCgOpts), c_i32, c_vp, ctypes.POINTER(c_vp)]
    L.gp_model_predict.restype = c_i32
    L.gp_model_predict.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i32, c_i32, c_vp]
    L.gp_model_info_read.restype = c_i32
    L.gp_model_info_read.argtypes = [c_vp, ctypes.POINTER(GpModelInfo)]
    L.gp_model_weights.restype = c_i32
    L.gp_model_weights.argtypes = [c_vp, c_vp, c_vp]
    L.gp_model_device.restype = c_i32
    L.gp_model_device.argtypes = [c_vp]
    L.gp_model_destroy.restype = c_i32
    L.gp_model_destroy.argtypes = [c_vp]
    L.gp_serve_submit_predict.restype = c_i32
    L.gp_serve_submit_predict.argtypes = [c_vp, ctypes.POINTER(GpPredictRequest),
                                          ctypes.POINTER(ctypes.c_uint64)]
    L.gp_kmvm_summation.restype = c_i32
    L.gp_kmvm_summation.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_vp, c_i64, c_i32, c_vp,
                                    c_i32, c_vp, c_i32, c_i32, c_i32, c_i32, c_vp]
    L.gp_kmvm_truncated.restype = c_i32
    L.gp_kmvm_truncated.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_vp, c_i64, c_i32, c_vp,
                                    c_i32, c_vp, c_i32, c_i32, ctypes.POINTER(GpTruncStats), c_vp]
    L.gp_mll_grad.restype = c_i32
    L.gp_mll_grad.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_i32, c_vp, c_vp, c_i32, c_i64,
                              c_i64, ctypes.POINTER(ctypes.c_double), c_vp]
    L.gp_rademacher.restype = c_i32
    L.gp_rademacher.argtypes = [ctypes.c_uint64, ctypes.c_uint64, c_i64, c_i32, c_vp, c_i64, c_vp]
    L.gp_train_default_config.restype = None
    L.gp_train_default_config.argtypes = [ctypes.POINTER(GpTrainConfig)]
    L.gp_trainer_create.restype = c_i32
    L.gp_trainer_create.argtypes = [ctypes.POINTER(GpTrainConfig), c_vp, c_vp, c_i64, c_i32,
                                    ctypes.POINTER(ctypes.c_double), c_vp, ctypes.POINTER(c_vp)]
    L.gp_trainer_step.restype = c_i32
    L.gp_trainer_step.argtypes = [c_vp, ctypes.POINTER(GpTrainStepInfo)]
    L.gp_trainer_get_state.restype = c_i32
    L.gp_trainer_get_state.argtypes = [c_vp, ctypes.POINTER(GpTrainState)]
    L.gp_trainer_set_state.restype = c_i32
    L.gp_trainer_set_state.argtypes = [c_vp, ctypes.POINTER(GpTrainState)]
    L.gp_trainer_blocks.restype = c_i32
    L.gp_trainer_blocks.argtypes = [c_vp, c_vp, c_vp]
    L.gp_trainer_destroy.restype = c_i32
    L.gp_trainer_destroy.argtypes = [c_vp]
    L.gp_cg_solve.restype = c_i32
    L.gp_cg_solve.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_i32, c_vp, c_i32, c_vp,
                              ctypes.POINTER(GpCgOpts), ctypes.POINTER(GpCgStats), c_vp]


def lib():
    """Load libgpmi.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2207_06856_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def header_exports():
    """Names of the functions include/gpmi.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z0-9_]+)\s*\(", text)))


def _check(status):
    if status < 0:
        raise GpError(status, lib().gp_last_error().decode())
    return status


def make_kernel(kind, lengthscale, outputscale, noise):
    """Build the gp_kernel struct; returns (struct, keep-alive array)."""
    ls = np.ascontiguousarray(np.asarray(lengthscale, dtype=np.float32).reshape(-1))
    arr = (c_f32 * ls.size)(*ls.tolist())
    k = GpKernel(int(kind), 1 if ls.size > 1 else 0, ctypes.cast(arr, ctypes.POINTER(c_f32)),
                 float(outputscale), float(noise))
    return k, arr


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def _ptr_typed(t, dtype):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def version():
    return lib().gp_version().decode()


def kmvm(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise=False, precision=FP16,
         scale_mode=0, out=None, stream=None):
    """out = a^2 K(X1, X2) V + [add_noise] s^2 V on the GPU (gp_kmvm)."""
    import torch
    n1, d = X1.shape
    n2 = X2.shape[0]
    r = V.shape[1]
    if out is None:
        out = torch.empty((n1, r), device=X1.device, dtype=torch.float32)
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    _check(lib().gp_kmvm(ctypes.byref(k), _ptr(X1), n1, _ptr(X2), n2, d, _ptr(V), r, _ptr(out),
                         int(add_noise), int(precision), int(scale_mode), _stream(stream)))
    del keep
    return out


def kmvm_noalloc(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise=False,
                 precision=FP16, scale_mode=0, out=None, stream=None):
    """gp_kmvm with the library's fixed per-device scratch block (gp_kmvm_noalloc);
    `out` should be preallocated by callers that cannot allocate."""
    import torch
    n1, d = X1.shape
    n2 = X2.shape[0]
    r = V.shape[1]
    if out is None:
        out = torch.empty((n1, r), device=X1.device, dtype=torch.float32)
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    _check(lib().gp_kmvm_noalloc(ctypes.byref(k), _ptr(X1), n1, _ptr(X2), n2, d, _ptr(V), r,
                                 _ptr(out), int(add_noise), int(precision), int(scale_mode),
                                 _stream(stream)))
    del keep
    return out


def true_residual_rows(X, B, U, rows, kind, lengthscale, outputscale, noise, stream=None):
    """float64 rows of b - K~ u (gp_true_residual_rows); rows: int64 device tensor."""
    import torch
    n, d = X.shape
    r = B.shape[1]
    res = torch.empty((rows.shape[0], r), device=X.device, dtype=torch.float64)
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    _check(lib().gp_true_residual_rows(ctypes.byref(k), _ptr(X), n, d, _ptr(B), _ptr(U), r,
                                       _ptr_typed(rows, torch.int64), rows.shape[0],
                                       _ptr_typed(res, torch.float64), _stream(stream)))
    del keep
    return res


PROBES = {"exp": 0, "sqrt": 1, "fma": 2, "mfma_f16_16x16x32": 3, "mfma_f16_16x16x16": 4,
          "mfma_f64_16x16x4": 5, "copy": 6, "mix_fma": 7, "mix_exp": 8}
PROBE_TWO_WAVES = 256


def probe_rate(name, iters, stream=None, two_waves=False):
    """Measured issue rate or bandwidth of one probe (gp_probe_rate); two_waves
    runs a loop probe at 2 waves per SIMD instead of 8."""
    rate = ctypes.c_double(0.0)
    which = PROBES[name] | (PROBE_TWO_WAVES if two_waves else 0)
    _check(lib().gp_probe_rate(which, int(iters), _stream(stream), ctypes.byref(rate)))
    return rate.value


def kmvm_noalloc_scratch_bytes():
    return int(lib().gp_kmvm_noalloc_scratch_bytes())


def kmvm_truncated(X1, X2, V, kind, lengthscale, outputscale, noise, add_noise=False, skip=True,
                   out=None, stats=False, stream=None):
    """The binary16 product over the finite binary16 support (gp_kmvm_truncated);
    with stats=True returns (out, dict of tile counts and radius)."""
    import torch
    n1, d = X1.shape
    n2 = X2.shape[0]
    r = V.shape[1]
    if out is None:
        out = torch.empty((n1, r), device=X1.device, dtype=torch.float32)
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    st = GpTruncStats() if stats else None
    _check(lib().gp_kmvm_truncated(ctypes.byref(k), _ptr(X1), n1, _ptr(X2), n2, d, _ptr(V), r,
                                   _ptr(out), int(add_noise), int(bool(skip)),
                                   ctypes.byref(st) if stats else None, _stream(stream)))
    del keep
    if stats:
        return out, {f: getattr(st, f) for f, _ in GpTruncStats._fields_}
    return out


def kmvm_summation(X1, X2, V, kind, lengthscale, outputscale, noise, scheme, block=32,
                   add_noise=False, scale_mode=1, out=None, stream=None):
    """The product with binary16 terms and binary16 (or blocked float32) sums
    (gp_kmvm_summation): the summation ablations."""
    import torch
    n1, d = X1.shape
    n2 = X2.shape[0]
    r = V.shape[1]
    if out is None:
        out = torch.empty((n1, r), device=X1.device, dtype=torch.float32)
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    _check(lib().gp_kmvm_summation(ctypes.byref(k), _ptr(X1), n1, _ptr(X2), n2, d, _ptr(V), r,
                                   _ptr(out), int(add_noise), int(scheme), int(block),
                                   int(scale_mode), _stream(stream)))
    del keep
    return out


class Precond:
    """Pivoted-Cholesky preconditioner handle (gp_pivchol_precond)."""

    def __init__(self, X, kind, lengthscale, outputscale, noise, rank, stream=None):
        n, d = X.shape
        k, keep = make_kernel(kind, lengthscale, outputscale, noise)
        h = c_vp()
        _check(lib().gp_pivchol_precond(ctypes.byref(k), _ptr(X), n, d, int(rank),
                                        ctypes.byref(h), _stream(stream)))
        self.handle = h
        self.n = n
        rk = c_i32()
        tr = ctypes.c_double()
        _check(lib().gp_precond_info(h, ctypes.byref(rk), None, ctypes.byref(tr)))
        self.rank = rk.value
        self.trace_residual = tr.value
        piv = (c_i64 * max(self.rank, 1))()
        _check(lib().gp_precond_info(h, None, piv, None))
        self.pivots = np.array(piv[:self.rank], dtype=np.int64)

    def apply(self, R, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(R)
        _check(lib().gp_precond_apply(self.handle, _ptr(R), R.shape[1], _ptr(out),
                                      _stream(stream)))
        return out

    def close(self):
        if self.handle:
            lib().gp_precond_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_cg_opts():
    o = GpCgOpts()
    lib().gp_cg_default_opts(ctypes.byref(o))
    return o


def cg_solve(X, B, kind, lengthscale, outputscale, noise, tol=1.0, max_iter=100, min_iter=10,
             algo=CG_ENHANCED, reorth=True, use_lse=True, precision=FP16, scale_mode=0, x0=None,
             true_res_every=0, poll_every=10, precond=None, history=False, out=None,
             stream=None):
    """Solve (a^2 K + s^2 I) U = B on the GPU (gp_cg_solve); returns (U, stats)."""
    import torch
    n, d = X.shape
    r = B.shape[1]
    U = out if out is not None else torch.empty_like(B)
    if x0 is not None:
        U.copy_(x0)
    o = default_cg_opts()
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.min_iter = int(min_iter)
    o.algo = int(algo)
    o.reorth = int(bool(reorth))
    o.use_lse = int(bool(use_lse))
    o.precision = int(precision)
    o.scale_mode = int(scale_mode)
    o.x0_given = int(x0 is not None)
    o.true_res_every = int(true_res_every)
    o.poll_every = int(poll_every)
    o.P = precond.handle if precond is not None else None
    iters = (c_i32 * r)()
    rel = (c_f32 * r)()
    trel = (ctypes.c_double * r)()
    conv = (ctypes.c_int8 * r)()
    brk = (ctypes.c_int8 * r)()
    hist = (c_f32 * ((max_iter + 1) * r))() if history else None
    trows = max_iter // true_res_every if true_res_every > 0 else 0
    thist = (ctypes.c_double * (trows * r))() if trows else None
    st = GpCgStats(iters, rel, trel, conv, brk,
                   ctypes.cast(hist, ctypes.POINTER(c_f32)) if history else None,
                   ctypes.cast(thist, ctypes.POINTER(ctypes.c_double)) if trows else None, 0, 0)
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    status = lib().gp_cg_solve(ctypes.byref(k), _ptr(X), n, d, _ptr(B), r, _ptr(U),
                               ctypes.byref(o), ctypes.byref(st), _stream(stream))
    stats = dict(iters=np.array(iters[:], dtype=np.int64), rel_res=np.array(rel[:]),
                 true_rel_res=np.array(trel[:]), converged=np.array(conv[:], dtype=bool),
                 breakdown=np.array(brk[:], dtype=bool), total_iters=st.total_iters,
                 mvms=st.mvms, status=status)
    if history:
        stats["history"] = np.array(hist[:], dtype=np.float32).reshape(max_iter + 1, r)
    if trows:
        stats["true_history"] = np.array(thist[:]).reshape(trows, r)
    if status < 0 and status != GP_ERR_BREAKDOWN:
        _check(status)
    return U, stats


def profile_enable(on=True):
    _check(lib().gp_profile_enable(int(bool(on))))


def profile_reset():
    _check(lib().gp_profile_reset())


def profile_read():
    """Per-launch (ms, entries, kind) arrays of the fused product kernel."""
    cnt = c_i64()
    _check(lib().gp_profile_read(0, None, None, None, ctypes.byref(cnt)))
    m = cnt.value
    ms = (c_f32 * max(m, 1))()
    ent = (ctypes.c_double * max(m, 1))()
    kinds = (c_i32 * max(m, 1))()
    _check(lib().gp_profile_read(m, ms, ent, kinds, ctypes.byref(cnt)))
    return (np.array(ms[:m], dtype=np.float64), np.array(ent[:m], dtype=np.float64),
            np.array(kinds[:m], dtype=np.int64))


def cg_solve_batched(problems, tol=1.0, max_iter=100, min_iter=10, algo=CG_ENHANCED, reorth=True,
                     use_lse=True, scale_mode=0, x0=None, true_res_every=0, poll_every=10,
                     outs=None, stream=None):
    """Solve many independent systems in one batched call (gp_cg_solve_batched).

    problems: list of dicts with X, B (CUDA tensors), kind, lengthscale,
    outputscale, noise and optional precond_rank.  Returns (list of U, list of stats).
    """
    import torch
    nprob = len(problems)
    arr = (GpProblem * nprob)()
    keep = []
    Us = []
    st_arr = (GpCgStats * nprob)()
    host = []
    for i, p in enumerate(problems):
        X, B = p["X"], p["B"]
        n, d = X.shape
        r = B.shape[1]
        U = outs[i] if outs is not None else torch.empty_like(B)
        if x0 is not None:
            U.copy_(x0[i])
        Us.append(U)
        k, kk = make_kernel(p["kind"], p["lengthscale"], p["outputscale"], p["noise"])
        keep.append(kk)
        arr[i] = GpProblem(k, _ptr(X), n, d, _ptr(B), r, _ptr(U), int(p.get("precond_rank", 0)))
        h = dict(iters=(c_i32 * r)(), rel=(c_f32 * r)(), trel=(ctypes.c_double * r)(),
                 conv=(ctypes.c_int8 * r)(), brk=(ctypes.c_int8 * r)())
        host.append(h)
        st_arr[i] = GpCgStats(h["iters"], h["rel"], h["trel"], h["conv"], h["brk"], None, None, 0, 0)
    o = default_cg_opts()
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.min_iter = int(min_iter)
    o.algo = int(algo)
    o.reorth = int(bool(reorth))
    o.use_lse = int(bool(use_lse))
    o.precision = FP16
    o.scale_mode = int(scale_mode)
    o.x0_given = int(x0 is not None)
    o.true_res_every = int(true_res_every)
    o.poll_every = int(poll_every)
    o.P = None
    status = lib().gp_cg_solve_batched(nprob, arr, ctypes.byref(o), st_arr, _stream(stream))
    if status < 0 and status != GP_ERR_BREAKDOWN:
        _check(status)
    stats = []
    for i, h in enumerate(host):
        stats.append(dict(iters=np.array(h["iters"][:], dtype=np.int64),
                          rel_res=np.array(h["rel"][:]), true_rel_res=np.array(h["trel"][:]),
                          converged=np.array(h["conv"][:], dtype=bool),
                          breakdown=np.array(h["brk"][:], dtype=bool),
                          total_iters=st_arr[i].total_iters, mvms=st_arr[i].mvms, status=status))
    del keep
    return Us, stats


class Server:
    """Serving loop (gp_serve_*).  Requests take HOST float32 arrays; the
    binding keeps them alive until the request completes."""

    def __init__(self, hbm_budget_bytes=8 << 30, max_slots=64, device=0, iters_per_round=5,
                 min_iter=10, algo=CG_ENHANCED, reorth=True, use_lse=True, scale_mode=0):
        c = GpServeConfig()
        lib().gp_serve_default_config(ctypes.byref(c))
        c.hbm_budget_bytes = int(hbm_budget_bytes)
        c.max_slots = int(max_slots)
        c.device = int(device)
        c.iters_per_round = int(iters_per_round)
        c.min_iter = int(min_iter)
        c.algo = int(algo)
        c.reorth = int(bool(reorth))
        c.use_lse = int(bool(use_lse))
        c.scale_mode = int(scale_mode)
        h = c_vp()
        _check(lib().gp_serve_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self._pending = {}

    def submit(self, X, B, kind, lengthscale, outputscale, noise, tol=1.0, max_iter=100,
               precond_rank=0):
        """Queue one solve; returns its ticket."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        B = np.ascontiguousarray(B, dtype=np.float32)
        n, d = X.shape
        r = B.shape[1]
        U = np.zeros((n, r), np.float32)
        k, kk = make_kernel(kind, lengthscale, outputscale, noise)
        h = dict(iters=(c_i32 * r)(), rel=(c_f32 * r)(), trel=(ctypes.c_double * r)(),
                 conv=(ctypes.c_int8 * r)(), brk=(ctypes.c_int8 * r)())
        st = GpCgStats(h["iters"], h["rel"], h["trel"], h["conv"], h["brk"], None, None, 0, 0)
        q = GpRequest(k, X.ctypes.data_as(c_vp), n, d, B.ctypes.data_as(c_vp), r,
                      U.ctypes.data_as(c_vp), float(tol), int(max_iter), int(precond_rank),
                      ctypes.pointer(st))
        t = ctypes.c_uint64()
        _check(lib().gp_serve_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        self._pending[t.value] = (X, B, U, h, st, kk)
        return t.value

    def submit_predict(self, model, Xs, truncate=False):
        """Queue one prediction against a Model on the server's device; returns
        its ticket (the result dict carries `mu`)."""
        Xs = np.ascontiguousarray(Xs, dtype=np.float32)
        mu = np.zeros(Xs.shape[0], np.float32)
        q = GpPredictRequest(model.handle, Xs.ctypes.data_as(c_vp), Xs.shape[0],
                             mu.ctypes.data_as(c_vp), int(bool(truncate)))
        t = ctypes.c_uint64()
        _check(lib().gp_serve_submit_predict(self._h, ctypes.byref(q), ctypes.byref(t)))
        self._pending[t.value] = ("predict", Xs, mu, model)
        return t.value

    def _result(self, ticket, status, res):
        if status == GP_PENDING:
            return None
        if status == GP_ERR_UNKNOWN_TICKET or ticket not in self._pending:
            _check(status)
        if isinstance(self._pending[ticket][0], str):      # a prediction request
            _, Xs, mu, _ = self._pending.pop(ticket)
            return dict(status=status, t_submit=res.t_submit, t_admit=res.t_admit,
                        t_finish=res.t_finish, message=res.message.decode(),
                        mu=mu if status == GP_OK else None)
        X, B, U, h, st, _ = self._pending.pop(ticket)
        out = dict(status=status, iters=res.iters, converged=res.converged,
                   breakdown=res.breakdown, max_rel_res=res.max_rel_res,
                   max_true_rel_res=res.max_true_rel_res, t_submit=res.t_submit,
                   t_admit=res.t_admit, t_finish=res.t_finish,
                   footprint_bytes=res.footprint_bytes, message=res.message.decode(),
                   U=U if status in (GP_OK, GP_ERR_BREAKDOWN) else None)
        if status in (GP_OK, GP_ERR_BREAKDOWN):
            out.update(col_iters=np.array(h["iters"][:], dtype=np.int64),
                       rel_res=np.array(h["rel"][:]), true_rel_res=np.array(h["trel"][:]),
                       col_converged=np.array(h["conv"][:], dtype=bool),
                       col_breakdown=np.array(h["brk"][:], dtype=bool))
        return out

    def poll(self, ticket):
        """None while pending, else a result dict (status, U, stats, timestamps)."""
        res = GpResult()
        return self._result(ticket, lib().gp_serve_poll(self._h, ticket, ctypes.byref(res)), res)

    def wait(self, ticket, timeout_ms=-1):
        res = GpResult()
        return self._result(ticket, lib().gp_serve_wait(self._h, ticket, int(timeout_ms),
                                                        ctypes.byref(res)), res)

    def cancel(self, ticket):
        _check(lib().gp_serve_cancel(self._h, ticket))

    def stats(self):
        s = GpServeStats()
        _check(lib().gp_serve_stats_read(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in GpServeStats._fields_}

    def close(self):
        if self._h:
            lib().gp_serve_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tune_dict(t):
    return dict(tuned=bool(t.tuned), f16_splits=list(t.f16_splits),
                f16_bucket_rows=list(t.f16_bucket_rows), f16_gain=[round(g, 4) for g in t.f16_gain],
                batched_split_div=t.batched_split_div,
                batched_persistent=bool(t.batched_persistent),
                batched_gain=round(t.batched_gain, 4))


def autotune(max_bucket=5, stream=None):
    """Measure and install the fused product's launch shapes (gp_autotune)."""
    t = GpTuneInfo()
    _check(lib().gp_autotune(int(max_bucket), _stream(stream), ctypes.byref(t)))
    return _tune_dict(t)


def tune_info():
    t = GpTuneInfo()
    _check(lib().gp_tune_get(ctypes.byref(t)))
    return _tune_dict(t)


def tune_reset():
    _check(lib().gp_tune_reset())


def tune_set(f16_splits=None, batched_split_div=16, batched_persistent=False, tuned=True):
    """Install launch-shape decisions (gp_tune_set); f16_splits: 8 values, 0 = built-in rule."""
    t = GpTuneInfo()
    vals = list(f16_splits) if f16_splits is not None else [0] * 8
    for b in range(8):
        t.f16_splits[b] = int(vals[b])
    t.batched_split_div = int(batched_split_div)
    t.batched_persistent = int(bool(batched_persistent))
    t.tuned = int(bool(tuned))
    _check(lib().gp_tune_set(ctypes.byref(t)))


def release_cached_memory():
    """Free the library's kept workspaces and preconditioner blocks (gp_release_cached_memory);
    returns the bytes freed."""
    b = ctypes.c_uint64(0)
    _check(lib().gp_release_cached_memory(ctypes.byref(b)))
    return int(b.value)


# ---------------------------------------------------------------- training
def mll_grad(X, B, U, kind, lengthscale, outputscale, noise=1.0, rows=None, stream=None):
    """Eq. (approx) gradient estimate from B = [y, Z] and U = K~^{-1} B
    (gp_mll_grad).  Returns float64 [dL/dl.., dL/da^2, dL/ds^2, 1/2 y^T u_0]."""
    n, d = X.shape
    r = B.shape[1]
    if U.shape != B.shape:
        raise ValueError("U and B must have the same shape")
    k, keep = make_kernel(kind, lengthscale, outputscale, noise)
    nl = d if k.ard else 1
    out = (ctypes.c_double * (nl + 3))()
    i0, i1 = (0, n) if rows is None else (int(rows[0]), int(rows[1]))
    _check(lib().gp_mll_grad(ctypes.byref(k), _ptr(X), n, d, _ptr(B), _ptr(U), r, i0, i1, out,
                             _stream(stream)))
    del keep
    return np.array(out[:], dtype=np.float64)


def rademacher(rows, cols, seed, first=0, out=None, ld=None, device="cuda", stream=None):
    """+-1 probes from the SplitMix64 counter stream (gp_rademacher)."""
    import torch
    if out is None:
        out = torch.empty((rows, cols), device=device, dtype=torch.float32)
    ld = out.shape[1] if ld is None else ld
    _check(lib().gp_rademacher(ctypes.c_uint64(seed), ctypes.c_uint64(first), rows, cols, _ptr(out),
                               ld, _stream(stream)))
    return out


def default_train_config():
    c = GpTrainConfig()
    lib().gp_train_default_config(ctypes.byref(c))
    return c


class Trainer:
    """Hyperparameter training with the Eq. (approx) gradient and Adam
    (gp_trainer_*).  X (n x d) and y (n) are float32 CUDA tensors."""

    def __init__(self, X, y, kind=RBF, ard=True, probes=15, precond_rank=100, use_priors=True,
                 lr=0.1, seed=0, theta0=None, tol=1.0, max_iter=50, min_iter=10, precision=FP16,
                 true_res_every=-1, stream=None):
        n, d = X.shape
        c = default_train_config()
        c.kind = int(kind)
        c.ard = int(bool(ard))
        c.probes = int(probes)
        c.precond_rank = int(precond_rank)
        c.use_priors = int(bool(use_priors))
        c.lr = float(lr)
        c.seed = int(seed)
        c.cg.tol = float(tol)
        c.cg.max_iter = int(max_iter)
        c.cg.min_iter = int(min_iter)
        c.cg.precision = int(precision)
        c.cg.true_res_every = int(true_res_every)
        self.n, self.d = n, d
        self.nl = d if ard else 1
        self.r = probes + 1
        self._stream = stream
        th = None
        if theta0 is not None:
            th = (ctypes.c_double * (self.nl + 2))(*[float(v) for v in theta0])
        h = c_vp()
        _check(lib().gp_trainer_create(ctypes.byref(c), _ptr(X), _ptr(y.reshape(-1)), n, d, th,
                                       _stream(stream), ctypes.byref(h)))
        self.handle = h

    def step(self):
        info = GpTrainStepInfo()
        _check(lib().gp_trainer_step(self.handle, ctypes.byref(info)))
        p = self.nl + 2
        return dict(step=info.step, cg_iters=info.cg_iters, cg_converged=info.cg_converged,
                    precond_rank=info.precond_rank, max_rel_res=info.max_rel_res,
                    theta=np.array(info.theta[:p]), grad=np.array(info.grad[:p]),
                    raw_grad=np.array(info.raw_grad[:p]), theta_next=np.array(info.theta_next[:p]),
                    data_fit=info.data_fit, seconds_precond=info.seconds_precond,
                    seconds_solve=info.seconds_solve, seconds_grad=info.seconds_grad)

    def state(self):
        s = GpTrainState()
        _check(lib().gp_trainer_get_state(self.handle, ctypes.byref(s)))
        p = s.nparams
        return dict(step=s.step, raw=np.array(s.raw[:p]), m=np.array(s.m[:p]),
                    v=np.array(s.v[:p]), theta=np.array(s.theta[:p]))

    def set_state(self, st):
        s = GpTrainState()
        s.nparams = self.nl + 2
        s.step = int(st["step"])
        for name in ("raw", "m", "v"):
            arr = getattr(s, name)
            for i, val in enumerate(st[name]):
                arr[i] = float(val)
        _check(lib().gp_trainer_set_state(self.handle, ctypes.byref(s)))

    def blocks(self):
        """Copies of the last step's [y, Z] and U (n x (M + 1) CUDA tensors)."""
        import torch
        B = torch.empty((self.n, self.r), device="cuda", dtype=torch.float32)
        U = torch.empty_like(B)
        _check(lib().gp_trainer_blocks(self.handle, _ptr(B), _ptr(U)))
        return B, U

    def close(self):
        if self.handle:
            lib().gp_trainer_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- prediction
def default_model_opts():
    o = GpCgOpts()
    lib().gp_model_default_opts(ctypes.byref(o))
    return o


class Model:
    """Cached predictive-mean weights v = K~^{-1} y (gp_model_*).  X (n x d) and
    y (n) are float32 CUDA tensors."""

    def __init__(self, X, y, kind, lengthscale, outputscale, noise, precond_rank=0, tol=1e-2,
                 max_iter=1000, precision=FP16, stream=None):
        n, d = X.shape
        k, keep = make_kernel(kind, lengthscale, outputscale, noise)
        o = default_model_opts()
        o.tol = float(tol)
        o.max_iter = int(max_iter)
        o.precision = int(precision)
        h = c_vp()
        _check(lib().gp_model_create(ctypes.byref(k), _ptr(X), n, d, _ptr(y.reshape(-1)),
                                     ctypes.byref(o), int(precond_rank), _stream(stream),
                                     ctypes.byref(h)))
        del keep
        self.handle = h
        self.n, self.d = n, d

    def predict(self, Xs, precision=FP16, truncate=False, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(Xs.shape[0], device=Xs.device, dtype=torch.float32)
        _check(lib().gp_model_predict(self.handle, _ptr(Xs), Xs.shape[0], _ptr(out),
                                      int(precision), int(bool(truncate)), _stream(stream)))
        return out

    def info(self):
        i = GpModelInfo()
        _check(lib().gp_model_info_read(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in GpModelInfo._fields_}

    def weights(self, stream=None):
        import torch
        v = torch.empty(self.n, device="cuda", dtype=torch.float32)
        _check(lib().gp_model_weights(self.handle, _ptr(v), _stream(stream)))
        return v

    def close(self):
        if self.handle:
            lib().gp_model_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
