"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the library with the host side of every source instrumented
(``-Xarch_host -fsanitize=address``, ``-Xarch_host -fsanitize=undefined``;
the device code compiled as in the product build) and the oracle with both
sanitizers, then runs the rest of the CPU suite against those builds
(``RIPK_LIB``, ``RIPK_ORACLE_LIB``) with the sanitizer runtime preloaded,
stopping at the first report.  That covers the host runtime's descriptor
validation and derived geometry, the polygon checks and per-cell edge lists
(``ripk_plan_check`` builds them for a polygon), the server's argument checks,
and the oracle with its pins.  No GPU is touched.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_cpu_suite_under_host_sanitizers(tmp_path):
    rt = _asan_runtime()
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and rt):
        pytest.skip("hipcc, clang or the clang sanitizer runtime is missing")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan"]
    lib = str(tmp_path / "libripk_san.so")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1912_04753_amd", "csrc", "*.hip")) +
                  glob.glob(os.path.join(ROOT, "paper_1912_04753_amd", "csrc", "*.cpp")))
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include")] + san + srcs + ["-o", lib],
                   check=True, capture_output=True)
    olib = str(tmp_path / "liboracle_san.so")
    subprocess.run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-shared-libsan",
                    "-fno-omit-frame-pointer", "-fopenmp", "-fPIC", "-shared",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", olib],
                   check=True, capture_output=True)
    # the sanitizer runtime first; anything already preloaded stays, after it
    pre = ":".join([rt] + ([os.environ["LD_PRELOAD"]] if os.environ.get("LD_PRELOAD") else []))
    env = dict(os.environ, LD_PRELOAD=pre, RIPK_LIB=lib, RIPK_ORACLE_LIB=olib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x",
           "-q", "-p", "no:cacheprovider",
           "--ignore", os.path.join(ROOT, "tests", "test_host_sanitizers.py")]
    if shutil.which("nproc") and (os.cpu_count() or 1) >= 4:
        try:
            import xdist  # noqa: F401
            cmd += ["-n", "4"]
        except ImportError:
            pass
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=1500, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
