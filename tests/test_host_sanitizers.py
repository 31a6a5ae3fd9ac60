"""The host C++ of the library (descriptor validation, planning, step
sequencing, Toeplitz set-up) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

build_lib.build_sanitized() recompiles the host sources with both
sanitizers (host side only) and links them with the regular objects of the
HIP sources; the host ABI tests then run in a child process that loads that
build through LHF_LIB with the sanitizer runtime preloaded.  Any sanitizer
report aborts the child.  The shared Sturm-count header is compiled the same
way into the host driver of test_sturm_host and run on split and unsplit
matrices.
"""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from paper_1702_00339_amd import build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")


def _env(runtime):
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"   # the HIP runtime keeps its allocations
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


@pytest.fixture(scope="module")
def runtime():
    if not (os.path.exists(build_lib.HIPCC) or shutil.which(build_lib.HIPCC)) or not os.path.exists(build_lib.CLANG):
        pytest.skip("hipcc or clang not found")
    rt = build_lib.sanitizer_runtime()
    if rt is None:
        pytest.skip("no shared AddressSanitizer runtime")
    return rt


def test_host_abi_under_asan_and_ubsan(runtime):
    lib = build_lib.build_sanitized()
    env = _env(runtime)
    env["LHF_LIB"] = lib
    probe = "from paper_1702_00339_amd import lhf; l = lhf.load(); print(l._name)"
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().endswith("liblhf_san.so")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi_host.py",
                        "tests/test_abi_layout.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]


def test_sturm_counts_under_asan_and_ubsan(runtime, tmp_path):
    exe = str(tmp_path / "sturm_san")
    r = subprocess.run([build_lib.HIPCC, "--offload-host-only", "-x", "hip", "-O1", "-g", "-std=c++17",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-Xarch_host", "-fno-sanitize-recover=undefined",
                        os.path.join(HERE, "sturm_check.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    rng = np.random.default_rng(5)
    lines = ["3"]
    for n, split in ((1, False), (9, True), (33, False)):
        d = rng.uniform(-1, 1, n)
        e2 = rng.uniform(0.01, 0.2, n)
        e2[0] = 0.0
        if split:
            e2[4] = 0.0
        xs = rng.uniform(-1.5, 1.5, 7)
        fmt = lambda a: " ".join(repr(float(v)) for v in a)   # noqa: E731
        lines += [str(n), fmt(d), fmt(e2), str(len(xs)), fmt(xs)]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr
    assert len(r.stdout.split()) == 2 * 3 * 7
