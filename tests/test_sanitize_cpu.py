"""Memory and undefined-behaviour checks on the CPU (no GPU): the oracle and the host
side of libnbody.so (argument checks, workspace layout of contexts and batches) built
with AddressSanitizer and UndefinedBehaviorSanitizer and driven by small C programs
in tests/sanitize/. Device code is built as usual; only host code is instrumented."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
CSRC = os.path.join(ROOT, "paper_1812_00367_amd", "csrc")
SOURCES = ["nbody_abi.hip", "nbody_kernels.hip", "nbody_batch.hip", "nbody_crackle.hip",
           "nbody_sym.hip", "nbody_group.hip"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fopenmp", "-ffp-contract=off", "-o", exe,
          os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
          os.path.join(ROOT, "oracle", "nbody_oracle.c"), "-lm"])
    assert _run([exe], env=ENV).strip() == "ok"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not installed")
def test_host_library_under_sanitizers(tmp_path):
    lib = str(tmp_path / "libnbody_asan.so")
    # host code instrumented only: each -fsanitize= follows -Xarch_host
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-omit-frame-pointer",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-o", lib]
         + [os.path.join(CSRC, s) for s in SOURCES])
    exe = str(tmp_path / "abi_check")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "abi_check.c"),
          "-L" + str(tmp_path), "-lnbody_asan", "-Wl,-rpath," + str(tmp_path),
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    # the HIP runtime's own allocations are not this library's: no leak report there
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0")
    assert _run([exe], env=env).strip() == "ok"
