"""The C-ABI library loads, exports every function include/cuba.h declares,
and its host-side validation behaves as documented (no device work)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cuba.h")


@pytest.fixture(scope="module")
def C():
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import cuba
    return cuba


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cuba_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(C):
    names = declared_functions()
    assert len(names) >= 11
    out = subprocess.run(["nm", "-D", "--defined-only", C.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (cuba_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(C.library_path())
    for n in names:
        getattr(lib, n)


def test_code_object_targets_gfx950(C, tmp_path):
    fatbin = str(tmp_path / "fatbin.bin")
    r = subprocess.run(["/opt/rocm/llvm/bin/llvm-objcopy", "--dump-section=.hip_fatbin=" + fatbin,
                        C.library_path(), str(tmp_path / "copy.so")], capture_output=True)
    if r.returncode != 0:
        pytest.skip("llvm-objcopy cannot read the library")
    out = subprocess.run(["/opt/rocm/llvm/bin/clang-offload-bundler", "--list", "--type=o",
                          "--input=" + fatbin], capture_output=True, text=True, check=True)
    targets = [t for t in out.stdout.split() if "amdgcn" in t]
    assert targets == ["hipv4-amdgcn-amd-amdhsa--gfx950"], out.stdout


def test_workspace_bytes_and_parameter_checks(C):
    p = C.make_params((10, 2, 2), (100, 10, 10), 0.4, 2500, 0.02, 1, cell_capacity=256)
    n = 1020851
    ws = C.cuba_workspace_bytes(p, n)
    # two buffers of cells x capacity slots of 52 B, each with n spill slots
    # (52 B + their cell, 4 B) and an overflowing-cell list; scratch for
    # overflowing cells of 3 n + 3 cells words; per-cell arrays (two counts,
    # two overflow lists, trace offsets, 4 observe sums, three scratch
    # words: 64 B) and small pieces
    slots = 10000 * 256
    want = 104 * slots + (2 * 56 + 12) * n + 64 * 10000
    assert want <= ws <= want + 64 * 1024
    p2 = C.make_params((10, 2, 2), (100, 10, 10), 0.4, 2500, 0.02, 1, cell_capacity=512)
    assert C.cuba_workspace_bytes(p2, n) > ws
    # default: twice the mean occupancy (102.1) plus 32, rounded up to 32
    p0 = C.make_params((10, 2, 2), (100, 10, 10), 0.4, 2500, 0.02, 1)
    assert C.cuba_workspace_bytes(p0, n) == ws
    for cap in (-1, 1025):
        bad = C.make_params((10, 2, 2), (100, 10, 10), 0.4, 2500, 0.02, 1, cell_capacity=cap)
        assert C.cuba_workspace_bytes(bad, n) == 0
    bad = [
        C.make_params((10, 2, 2), (100, 10, 10), 0.4, 2500, 0.1, 1),     # dt >= dx
        C.make_params((10, 2, 2), (100, 10, 10), -0.4, 2500, 0.02, 1),   # sigma < 0
        C.make_params((10, 2, 2), (100, 10, 10), 0.4, 0.0, 0.02, 1),     # r_test = 0
        C.make_params((10, 2, 2), (0, 10, 10), 0.4, 2500, 0.02, 1),      # no cells
        C.make_params((float("nan"), 2, 2), (100, 10, 10), 0.4, 2500, 0.02, 1),
        C.make_params((10, 2, 2), (100, 10, 10), 400.0, 1.0, 0.02, 1),   # 2K > 1
    ]
    for b in bad:
        assert C.cuba_workspace_bytes(b, 10) == 0
        assert C.cuba_last_error() != ""


def test_init_rejects_before_touching_the_device(C):
    ctx = ctypes.c_void_p()
    L = C._lib
    bad = C.make_params((10, 1, 1), (100, 1, 1), 0.4, 100, 0.5, 1)
    rc = L.cuba_init(ctypes.byref(ctx), ctypes.byref(bad), 10, *([None] * 6), None, 0, None)
    assert rc == C.CUBA_EINVAL and ctx.value is None
    good = C.make_params((10, 1, 1), (100, 1, 1), 0.4, 100, 0.02, 1)
    rc = L.cuba_init(ctypes.byref(ctx), ctypes.byref(good), 10, *([None] * 6), None, 0, None)
    assert rc == C.CUBA_EINVAL and "NULL" in C.cuba_last_error()
    # misaligned workspace and a too-small one are refused by the host code
    rc = L.cuba_init(ctypes.byref(ctx), ctypes.byref(good), 0, *([None] * 6), 8, 1 << 20, None)
    assert rc == C.CUBA_EINVAL and "aligned" in C.cuba_last_error()
    rc = L.cuba_init(ctypes.byref(ctx), ctypes.byref(good), 0, *([None] * 6), 256, 16, None)
    assert rc == C.CUBA_ENOMEM
    for code in (0, -1, -2, -3, -4):
        assert C.cuba_strerror(code).startswith("CUBA_")


def test_lanes_and_batch_arguments_checked_on_the_host(C):
    L = C._lib
    out = ctypes.c_int32()
    assert L.cuba_set_cell_lanes(None, 8) == C.CUBA_EINVAL
    assert L.cuba_get_cell_lanes(None, ctypes.byref(out)) == C.CUBA_EINVAL
    assert L.cuba_batch_set_cell_lanes(None, 0, 8) == C.CUBA_EINVAL
    assert L.cuba_batch_set_observe(None, 0, 7, None, 1) == C.CUBA_EINVAL
    assert L.cuba_timing_begin_sampled(None, 8, 10) == C.CUBA_EINVAL
    # batch table: the event descriptors plus four work-space index arrays,
    # 256-byte aligned pieces, growing with the slot count
    assert C.cuba_batch_workspace_bytes(0) == 0
    prev = 0
    for slots in (1, 2, 64, 65, 1000):
        nb = C.cuba_batch_workspace_bytes(slots)
        assert nb % 256 == 0 and nb > prev and nb >= slots * (200 + 16)
        prev = nb
    # the slot count is bounded by the grid's y dimension (65535)
    assert C.cuba_batch_workspace_bytes(65535) > 0
    assert C.cuba_batch_workspace_bytes(65536) == 0
    b = ctypes.c_void_p()
    rc = L.cuba_batch_create(ctypes.byref(b), 65536, 256, 1 << 30, None)
    assert rc == C.CUBA_EINVAL and b.value is None
    rc = L.cuba_batch_create(ctypes.byref(b), 4, 8, 1 << 20, None)
    assert rc == C.CUBA_EINVAL and b.value is None
    rc = L.cuba_batch_create(ctypes.byref(b), 4, 256, 16, None)
    assert rc == C.CUBA_ENOMEM and b.value is None


def test_capacity_suggestion_checked_on_the_host(C):
    """cuba_suggest_cell_capacity: its scratch size (one word a cell plus
    one, 256-byte aligned) and the argument checks made before any device
    work."""
    L = C._lib
    good = C.make_params((10.0, 1.0, 1.0), (100, 1, 1), 0.4, 100.0, 0.02, 7)
    assert C.cuba_capacity_scratch_bytes(good) == 512
    big = C.make_params((10.0, 2.0, 2.0), (100, 10, 10), 0.4, 2500.0, 0.02, 7)
    assert C.cuba_capacity_scratch_bytes(big) == (10001 * 4 + 255) // 256 * 256
    bad = C.make_params((10.0, 1.0, 1.0), (0, 1, 1), 0.4, 100.0, 0.02, 7)
    assert C.cuba_capacity_scratch_bytes(bad) == 0
    cap = ctypes.c_int32()
    rc = L.cuba_suggest_cell_capacity(ctypes.byref(good), 0, None, None, None, 256, 512,
                                      None, None)
    assert rc == C.CUBA_EINVAL and "cap" in C.cuba_last_error()
    rc = L.cuba_suggest_cell_capacity(ctypes.byref(bad), 0, None, None, None, 256, 512,
                                      None, ctypes.byref(cap))
    assert rc == C.CUBA_EINVAL
    rc = L.cuba_suggest_cell_capacity(ctypes.byref(good), 5, None, None, None, 256, 512,
                                      None, ctypes.byref(cap))
    assert rc == C.CUBA_EINVAL and "NULL" in C.cuba_last_error()
    rc = L.cuba_suggest_cell_capacity(ctypes.byref(good), -1, None, None, None, 256, 512,
                                      None, ctypes.byref(cap))
    assert rc == C.CUBA_EINVAL
    for scratch, nbytes in ((256, 256), (8, 512), (None, 512)):
        rc = L.cuba_suggest_cell_capacity(ctypes.byref(good), 0, None, None, None, scratch,
                                          nbytes, None, ctypes.byref(cap))
        assert rc == C.CUBA_EINVAL and "scratch" in C.cuba_last_error()
