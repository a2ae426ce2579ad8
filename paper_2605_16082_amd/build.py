"""Build libslimdg.so (HIP, gfx950) in the package directory.

    python -m paper_2605_16082_amd.build [--sanitize]

--sanitize builds _build/asan/libslimdg_asan.so instead, with the host code
under AddressSanitizer and UndefinedBehaviorSanitizer (device code as usual).

Every HIP source is compiled with hipcc for gfx950 only, with packed FP32
instructions disabled, then linked into one shared library next to this file.
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libslimdg.so")

ARCH = "gfx950"
HIPFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build (device code
# unchanged): every -fsanitize applies to the host pass only.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
ASAN_LIB = os.path.join(BUILD, "asan", "libslimdg_asan.so")


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime (it also carries the UBSan
    handlers), to LD_PRELOAD into the Python process that loads ASAN_LIB."""
    clang = os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    path = _run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"]).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def build_sanitized(verbose: bool = False, jobs: int = 8) -> str:
    """Compile the library with host-side ASan/UBSan into _build/asan."""
    return build(verbose, jobs, extra=SANITIZE_FLAGS, out=ASAN_LIB, objdir=os.path.join(BUILD, "asan"))


def build(verbose: bool = False, jobs: int = 8, extra=(), out: str = LIB, objdir: str = BUILD) -> str:
    """Compile every csrc/*.hip for gfx950 and link libslimdg.so; returns its path."""
    hipcc = _hipcc()
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]

    def compile_one(pair):
        src, obj = pair
        cmd = [hipcc, *HIPFLAGS, *extra, "-c", src, "-o", obj]
        r = _run(cmd)
        if verbose:
            print(" ".join(cmd), flush=True)
            if r.stderr.strip():
                print(r.stderr, flush=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    tmp = out + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, out)
    if verbose:
        print("built", out, flush=True)
    return out


C_EXAMPLE_SRC = os.path.join(ROOT, "tests", "c_abi", "c_abi_step.cpp")
C_EXAMPLE = os.path.join(ROOT, "tests", "c_abi", "c_abi_step")


def build_c_example(verbose: bool = False) -> str:
    """Compile the C-ABI example program (host code only) against the built
    library; it finds libslimdg.so through its run path."""
    tmp = C_EXAMPLE + ".tmp"
    cmd = [_hipcc(), "-O2", "-std=c++17", "-I", INCLUDE, C_EXAMPLE_SRC, "-L", PKG, "-lslimdg",
           "-Wl,-rpath,$ORIGIN/../../paper_2605_16082_amd", "-o", tmp]
    _run(cmd)
    os.replace(tmp, C_EXAMPLE)
    if verbose:
        print("built", C_EXAMPLE, flush=True)
    return C_EXAMPLE


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized(verbose="-v" in sys.argv)
    else:
        build(verbose="-v" in sys.argv)
        build_c_example(verbose="-v" in sys.argv)
