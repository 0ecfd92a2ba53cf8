"""Build libgpmi.so (HIP, gfx950) in-tree with hipcc.

Every call recompiles every source: this is the "does it build" step, and the
tests, the smoke check and the benchmark load the library it leaves next to
this file.
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgpmi.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-x", "hip", "-c", "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs: the kernel value is computed
    # straight from the MFMA result without accumulator-register copies
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + [src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{out}")
    return obj, out


def build(jobs=None, verbose=False):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found; the gfx950 library cannot be built")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs = []
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for obj, out in ex.map(_compile, srcs):
            objs.append(obj)
            if verbose and out.strip():
                print(out, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


# Host AddressSanitizer build: the host sources (*.cpp: argument checks,
# workspace planning, the serving scheduler, the tuner) are compiled with the
# sanitizer on their host side only; the kernel sources (*.hip) are linked from
# the objects of the last build().  The sanitizer runtime is not linked in: a
# process loads it first (LD_PRELOAD of the runtime named by asan_runtime()).
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libgpmi_asan.so")


def asan_runtime():
    """Path of clang's shared AddressSanitizer runtime next to hipcc."""
    p = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = p.stdout.strip()
    if p.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the clang AddressSanitizer runtime was not found")
    return path


def _compile_asan(src):
    obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g",
                                               "-Xarch_host", "-fsanitize=address",
                                               "-Xarch_host", "-fno-omit-frame-pointer"]
    p = subprocess.run([HIPCC] + flags + [src, "-o", obj], capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc (host sanitizer) failed on {os.path.basename(src)}:\n"
                           + p.stdout + p.stderr)
    return obj


def build_host_asan(jobs=None):
    """libgpmi_asan.so under _build/asan; needs the kernel objects of build()."""
    kernels = [os.path.join(BUILD, os.path.basename(f) + ".o") for f in sources()
               if f.endswith(".hip")]
    missing = [k for k in kernels if not os.path.exists(k)]
    if missing:
        raise RuntimeError("run build() first: missing " + ", ".join(map(os.path.basename, missing)))
    os.makedirs(ASAN_DIR, exist_ok=True)
    hosts = [f for f in sources() if f.endswith(".cpp")]
    with concurrent.futures.ThreadPoolExecutor(jobs or min(len(hosts), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile_asan, hosts))
    tmp = ASAN_LIB + ".tmp"
    p = subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + kernels,
                       capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link (host sanitizer) failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
