"""Builds libcuba.so (the HIP kernels and the C ABI) for gfx950, in-tree.

hipcc flags that define the library's arithmetic:
  -ffp-contract=off   no fused multiply-add: every FP64 expression rounds
                      exactly as written (the determinism contract);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions are generated.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcuba.so")
SOURCES = ["kernels.hip", "api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def source_files() -> list[str]:
    """Every file the library is compiled from, in a fixed order."""
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".hpp", ".h")))
    return files + [os.path.join(INCLUDE, "cuba.h")]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the library's sources and build
    flags; compiled into libcuba.so (cuba_build_info) so that a loaded
    library can be matched to the sources it was built from."""
    h = hashlib.sha256()
    for path in source_files():
        h.update(os.path.relpath(path, ROOT).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
    # flags with the checkout's location removed, so that a copy of the
    # tree elsewhere hashes alike
    h.update(" ".join(flags(with_hash=False)).replace(ROOT, ".").encode())
    return h.hexdigest()[:16]


def flags(with_hash: bool = True) -> list[str]:
    extra = ['-DCUBA_SOURCE_HASH="' + source_hash() + '"'] if with_hash else []
    return extra + ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-I", INCLUDE, "-I", CSRC,
            "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + flags() + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


def sources_newer_than_lib() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in source_files())


if __name__ == "__main__":
    print(build(verbose=True))
