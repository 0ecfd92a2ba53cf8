"""The library's host code under AddressSanitizer (CPU only, no device calls).

The host sources (argument checks, option defaults, workspace plans, the
serving, training and tuning front ends) are rebuilt with the sanitizer on
their host side (``paper_2207_06856_amd.build.build_host_asan``) and linked
with the kernel objects of the regular build.  The host-side ABI checks of
``test_abi_cpu.py`` and a few handle-free entry points then run against that
library in a child process that loads the sanitizer runtime first; any
sanitizer report fails the child.
"""
import os
import subprocess
import sys

import pytest

from paper_2207_06856_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_KERNEL_OBJECTS = [os.path.join(B.BUILD, os.path.basename(f) + ".o") for f in B.sources()
                   if f.endswith(".hip")]

pytestmark = pytest.mark.skipif(not all(os.path.exists(o) for o in _KERNEL_OBJECTS),
                                reason="kernel objects not built (run __graft_entry__.build())")

# The child: ABI argument checks, then entry points that need no device.
_CHILD = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
from paper_2207_06856_amd import gpmi
gpmi.LIB_PATH = {lib!r}
import pytest
rc = pytest.main(["-q", "-p", "no:cacheprovider", {abi!r}])
L = gpmi.lib()
assert L._name == {lib!r}
assert b"gfx950" in L.gp_version()
L.gp_precond_destroy(None)
L.gp_model_destroy(None)
print("children done", int(rc), flush=True)
sys.exit(int(rc))
"""


@pytest.fixture(scope="module")
def asan_lib():
    return B.build_host_asan()


def test_host_objects_are_instrumented(asan_lib):
    out = subprocess.run(["nm", "-D", "--undefined-only", asan_lib], capture_output=True,
                         text=True, check=True).stdout
    assert "__asan_report_load" in out and "__asan_init" in out


def test_abi_checks_clean_under_address_sanitizer(asan_lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = B.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:exitcode=23"
    code = _CHILD.format(root=ROOT, lib=asan_lib,
                         abi=os.path.join(ROOT, "tests", "test_abi_cpu.py"))
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=300)
    log = p.stdout[-3000:] + p.stderr[-3000:]
    assert "AddressSanitizer" not in p.stderr, log
    assert p.returncode == 0, log
    assert "children done 0" in p.stdout, log
