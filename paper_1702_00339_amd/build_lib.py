"""Build the HIP library liblhf.so for gfx950 (in-tree, next to this file).

Each source under csrc/ is compiled by hipcc into _build/, in parallel, then
linked into lib/liblhf.so.  All device code is built with packed FP32
instructions disabled.

build_sanitized() makes a test variant, _build_san/liblhf_san.so: the host
sources (descriptor validation, planning, step sequencing, Toeplitz set-up)
recompiled with AddressSanitizer and UndefinedBehaviorSanitizer on the host
side only, linked with the regular objects of the HIP sources.  It is loaded
through LHF_LIB with the sanitizer runtime preloaded, by the host tests only.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "liblhf.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]

SOURCES = ["plan.cpp", "api.cpp", "step.cpp", "factors.hip", "gram.hip", "combine.hip", "blockdft.hip",
           "heev.hip", "toeplitz.hip", "toeplitz.cpp", "lobpcg.hip", "noalloc.hip", "eigvec.hip", "toeplitz3.hip", "rrsyev.hip"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


HOST_SOURCES = ["plan.cpp", "api.cpp", "step.cpp", "toeplitz.cpp"]
SAN_DIR = os.path.join(os.path.dirname(HERE), "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "liblhf_san.so")
SAN_FLAGS = ["-O1", "-g", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Wno-unused-command-line-argument",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
CLANG = os.environ.get("LHF_CLANG", "/opt/rocm/llvm/bin/clang++")


def sanitizer_runtime() -> str | None:
    """The shared AddressSanitizer runtime of the ROCm clang (to preload)."""
    root = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(root):
        return None
    for ver in sorted(os.listdir(root), reverse=True):
        p = os.path.join(root, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def build_sanitized(verbose: bool = False) -> str:
    hip_objs = [os.path.join(OBJ, s + ".o") for s in SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in hip_objs):
        build()
    os.makedirs(SAN_DIR, exist_ok=True)

    def comp(src: str) -> str:
        obj = os.path.join(SAN_DIR, src + ".o")
        cmd = [HIPCC, *SAN_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(comp, HOST_SOURCES))
    tmp = SAN_LIB + ".tmp"
    # a host-only link (no device code is compiled here), by clang with the
    # shared sanitizer runtime
    cmd = [CLANG, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan", "-o", tmp, *objs, *hip_objs,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
