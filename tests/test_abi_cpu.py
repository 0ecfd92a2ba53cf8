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


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a host C compiler."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    body = "\n".join(f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields)
    src = f"""#include <stddef.h>
#include <stdio.h>
#include "gpmi.h"
int main(void) {{ printf("%zu\\n", sizeof({struct})); {body} return 0; }}
"""
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "l.c")
        exe = os.path.join(tmp, "l")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", inc, c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("struct,cls", [("gp_train_config", gpmi.GpTrainConfig),
                                        ("gp_train_step_info", gpmi.GpTrainStepInfo),
                                        ("gp_train_state", gpmi.GpTrainState),
                                        ("gp_cg_opts", gpmi.GpCgOpts)])
def test_struct_layouts_match_header(struct, cls):
    fields = [f for f, _ in cls._fields_]
    got = _c_layout(struct, fields)
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, f).offset for f in fields]


def test_training_argument_errors_are_reported():
    L = gpmi.lib()
    p = lambda v: ctypes.c_void_p(0x10000 * v) if v else None
    k, keep = gpmi.make_kernel(gpmi.RBF, [1.0, 1.0], 1.0, 0.1)
    g = (ctypes.c_double * 8)()
    call = lambda **a: L.gp_mll_grad(ctypes.byref(k), p(a.get("X", 1)), a.get("n", 10), a.get("d", 2),
                                     p(a.get("B", 2)), p(a.get("U", 3)), a.get("r", 4),
                                     a.get("i0", 0), a.get("i1", 10), g, None)
    assert call(r=1) == gpmi.GP_ERR_ARG          # no probes
    assert call(r=65) == gpmi.GP_ERR_ARG
    assert call(d=33) == gpmi.GP_ERR_ARG
    assert call(i1=11) == gpmi.GP_ERR_ARG
    assert call(i0=5, i1=4) == gpmi.GP_ERR_ARG
    assert call(U=None) == gpmi.GP_ERR_ARG
    assert L.gp_rademacher(1, 0, 4, 3, p(1), 2, None) == gpmi.GP_ERR_ARG     # ld < cols
    assert L.gp_rademacher(1, 0, 0, 3, None, 3, None) == gpmi.GP_OK         # empty
    c = gpmi.default_train_config()
    assert (c.kind, c.ard, c.probes, c.precond_rank, c.use_priors) == (gpmi.RBF, 1, 15, 100, 1)
    assert (c.lr, c.beta1, c.beta2, c.eps) == (0.1, 0.9, 0.999, 1e-8)
    assert (c.cg.tol, c.cg.max_iter, c.cg.min_iter) == (1.0, 50, 10)
    h = ctypes.c_void_p()
    for field, val in (("probes", 0), ("probes", 64), ("precond_rank", 129), ("lr", 0.0),
                       ("beta2", 1.0), ("kind", 9)):
        c = gpmi.default_train_config()
        setattr(c, field, val)
        assert L.gp_trainer_create(ctypes.byref(c), p(1), p(2), 200, 3, None, None,
                                   ctypes.byref(h)) == gpmi.GP_ERR_ARG, field
    c = gpmi.default_train_config()
    bad = (ctypes.c_double * 5)(1.0, 1.0, 1.0, 1.0, 5e-5)     # noise below its floor
    assert L.gp_trainer_create(ctypes.byref(c), p(1), p(2), 200, 3, bad, None, ctypes.byref(h)) == gpmi.GP_ERR_ARG
    assert L.gp_trainer_create(ctypes.byref(c), p(1), p(2), 200, 33, None, None, ctypes.byref(h)) == gpmi.GP_ERR_ARG
    assert not h.value


def test_number_format_argument_errors_are_reported():
    """gp_kmvm with bfloat16 and gp_kmvm_summation reject bad arguments before
    any device work (fake non-null addresses, as above)."""
    L = gpmi.lib()
    k, keep = gpmi.make_kernel(gpmi.RBF, [1.0], 1.0, 0.1)
    assert _call_kmvm(k, precision=gpmi.BF16, d=0) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, precision=gpmi.BF16, scale_mode=2) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, precision=3) == gpmi.GP_ERR_ARG
    assert _call_kmvm(k, precision=gpmi.BF16, n1=0, X1=None, out=None) == gpmi.GP_OK
    p = lambda v: ctypes.c_void_p(0x10000 * v) if v else None

    def summ(scheme=gpmi.SUM_BLOCK_HALF, block=32, scale_mode=1, n1=4, n2=4, d=2, r=1,
             X1=1, X2=1, V=1, out=2, add_noise=0):
        return L.gp_kmvm_summation(ctypes.byref(k), p(X1), n1, p(X2), n2, d, p(V), r, p(out),
                                   add_noise, scheme, block, scale_mode, None)

    assert summ(scheme=3) == gpmi.GP_ERR_ARG
    assert b"scheme" in L.gp_last_error()
    assert summ(scheme=-1) == gpmi.GP_ERR_ARG
    assert summ(block=0) == gpmi.GP_ERR_ARG
    assert summ(scheme=gpmi.SUM_BLOCK_SINGLE, block=(1 << 30) + 1) == gpmi.GP_ERR_ARG
    assert summ(scale_mode=2) == gpmi.GP_ERR_ARG
    assert summ(r=0) == gpmi.GP_ERR_ARG
    assert summ(d=65) == gpmi.GP_ERR_ARG
    assert summ(X1=None) == gpmi.GP_ERR_ARG
    assert summ(V=None) == gpmi.GP_ERR_ARG
    assert summ(out=1) == gpmi.GP_ERR_ARG                           # out aliases an input
    assert summ(add_noise=1, X2=3) == gpmi.GP_ERR_ARG               # different point sets
    # Kahan's sum ignores the block length; an empty output is a no-op
    assert summ(scheme=gpmi.SUM_KAHAN_HALF, block=0, n1=0, X1=None, out=None) == gpmi.GP_OK
