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

RBF = 0
MATERN52 = 1
MATERN12 = 2
MATERN32 = 3

FP32 = 0
FP16 = 1

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_f32 = ctypes.c_float
c_vp = ctypes.c_void_p


class GpKernel(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("ard", c_i32), ("lengthscale", ctypes.POINTER(c_f32)),
                ("outputscale", c_f32), ("noise", c_f32)]


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
    L.gp_kmvm.restype = c_i32
    L.gp_kmvm.argtypes = [ctypes.POINTER(GpKernel), c_vp, c_i64, c_vp, c_i64, c_i32, c_vp, c_i32,
                          c_vp, c_i32, c_i32, c_i32, c_vp]


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
