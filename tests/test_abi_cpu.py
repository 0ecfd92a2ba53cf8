"""Host-side checks of the C ABI library: it loads, exports what the header
declares, and rejects bad arguments before touching a device."""
import ctypes
import os

import numpy as np
import pytest

from paper_2207_06856_amd import gpmi

pytestmark = pytest.mark.skipif(not os.path.exists(gpmi.LIB_PATH),
                                reason="libgpmi.so not built (run __graft_entry__.build())")


def test_library_exports_every_header_symbol():
    L = gpmi.lib()
    names = gpmi.header_exports()
    assert "gp_kmvm" in names and "gp_last_error" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []


def test_version_string():
    assert "gfx950" in gpmi.version()


def _call_kmvm(k, n1=4, n2=4, d=2, r=1, add_noise=0, precision=1, scale_mode=0,
               X1=1, X2=1, V=1, out=2):
    # fake non-null device addresses: every call below must fail validation
    # before any HIP call dereferences them
    p = lambda v: ctypes.c_void_p(0x10000 * v) if v else None
    return gpmi.lib().gp_kmvm(ctypes.byref(k), p(X1), n1, p(X2), n2, d, p(V), r, p(out),
                              add_noise, precision, scale_mode, None)


def test_argument_errors_are_reported():
    L = gpmi.lib()
    k, keep = gpmi.make_kernel(gpmi.RBF, [1.0], 1.0, 0.1)
    assert _call_kmvm(k, d=0) == gpmi.GP_ERR_ARG
    assert b"d=0" in L.gp_last_error()
    assert _call_kmvm(k, d=65) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, r=0) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, precision=7) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, scale_mode=3) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, n1=-1) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, X1=None) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, add_noise=1, X2=3) == gpmi.GP_ERR_ARG     # different point sets
    assert _call_kmvm(k, out=1) == gpmi.GP_ERR_ARG                 # out aliases inputs
    bad, keep2 = gpmi.make_kernel(gpmi.RBF, [-1.0], 1.0, 0.1)
    assert _call_kmvm(bad) == gpmi.GP_ERR_ARG
    bad, keep3 = gpmi.make_kernel(7, [1.0], 1.0, 0.1)
    assert _call_kmvm(bad) == gpmi.GP_ERR_ARG
    bad, keep4 = gpmi.make_kernel(gpmi.RBF, [1.0], 0.0, 0.1)
    assert _call_kmvm(bad) == gpmi.GP_ERR_ARG
    bad, keep5 = gpmi.make_kernel(gpmi.RBF, [1.0], 1.0, float("nan"))
    assert _call_kmvm(bad) == gpmi.GP_ERR_ARG
    # an empty output is a no-op that succeeds without a device
    assert _call_kmvm(k, n1=0, X1=None, out=None) == gpmi.GP_OK
