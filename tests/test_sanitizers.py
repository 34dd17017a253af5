"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The C oracle is built with both sanitizers and driven through every entry
point (valid and invalid calls, traces with short buffers, threaded runs).
The HIP library is built with the sanitizers on its host code only (device
code is unchanged) and driven through the host-only paths of its C ABI:
parameter validation, workspace sizing, and the argument checks that return
before any device work.  Neither run needs a GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPERS = os.path.join(ROOT, "tests", "helpers")
CSRC = os.path.join(ROOT, "paper_1208_0961_amd", "csrc")

pytestmark = pytest.mark.slow

ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, (" ".join(cmd) + "\n" + res.stdout + res.stderr)[-4000:]
    return res.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "san_oracle")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "cuba_oracle.c"),
          os.path.join(HELPERS, "sanitize_oracle.c"), "-o", exe, "-lm", "-lpthread"])
    assert "oracle sanitizer run ok" in _run([exe], env=ENV)


def test_library_host_paths_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "san_api")
    _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address,undefined",
          "-Xarch_host", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "api.hip"),
          os.path.join(HELPERS, "sanitize_api.cpp"), "-o", exe])
    assert "api sanitizer run ok" in _run([exe], env=ENV)
