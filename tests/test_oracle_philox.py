"""Pins of the oracle's Philox4x32-10 and of its 53-bit uniform.

The library pin is rocRAND's header-only Philox4x32-10 engine run on the
host (tests/helpers/rocrand_philox_ref.cpp), an implementation independent
of the oracle's.  The uniform map U53 is pinned by its exact end points and
by monotonicity; the generator's output by equidistribution tests.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HELPERS = os.path.join(os.path.dirname(__file__), "helpers")


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists(
            "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.run([hipcc, "-O1", os.path.join(HELPERS, "rocrand_philox_ref.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def _ref_blocks(exe, rows):
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                         check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand_library(orc, rocrand_ref):
    rng = np.random.default_rng(7)
    rows = []
    # edge counters/keys plus random ones (counter word 1 < 2^30: the
    # library's offset argument counts 4 outputs per counter value)
    rows.append([0, 0, 0, 0, 0, 0])
    rows.append([0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF])
    rows.append([1, 2, 3, 4, 5, 6])
    for _ in range(300):
        r = rng.integers(0, 2**32, size=6, dtype=np.uint64)
        r[1] %= 2**30
        rows.append([int(v) for v in r])
    ref = _ref_blocks(rocrand_ref, rows)
    for r, want in zip(rows, ref):
        got = orc.philox4x32_10(r[:4], r[4:])
        assert [int(v) for v in got] == [int(v) for v in want], r


def test_u53_endpoints_and_order(orc):
    assert orc.u53(0, 0) == 0.0
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    # only the top 53 of the 64 bits count: the low 11 bits are dropped
    assert orc.u53(0x7FF, 0) == 0.0
    assert orc.u53(0x800, 0) == 2.0**-53
    assert orc.u53(0, 1) == 2.0**-32
    assert orc.u53(0, 0x80000000) == 0.5
    vals = [orc.u53(lo, hi) for hi in (0, 1, 77, 2**31) for lo in (0, 2048, 2**31)]
    assert vals == sorted(vals)


def test_philox_equidistribution(orc):
    """Counters differing only in the pair index (as in one cell) give words
    that are uniform (chi-square over 256 bins) and serially uncorrelated."""
    key = [0x12080961, 0x1]
    words = np.array([orc.philox4x32_10([k, 17, 3, 0], key) for k in range(20000)],
                     dtype=np.uint64)
    for j in range(4):
        h = np.bincount((words[:, j] >> 24).astype(np.int64), minlength=256)
        chi2 = ((h - h.mean()) ** 2 / h.mean()).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4, (j, chi2)
    u = (((words[:, 1] << np.uint64(32)) | words[:, 0]) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5.0 / np.sqrt(len(u))


def test_philox_key_and_counter_sensitivity(orc):
    base = orc.philox4x32_10([5, 6, 7, 0], [1, 2])
    for ctr, key in (([5, 6, 7, 1], [1, 2]), ([5, 6, 8, 0], [1, 2]),
                     ([5, 7, 7, 0], [1, 2]), ([4, 6, 7, 0], [1, 2]),
                     ([5, 6, 7, 0], [1, 3]), ([5, 6, 7, 0], [0, 2])):
        other = orc.philox4x32_10(ctr, key)
        # avalanche: about half of the 128 bits flip
        flips = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, other))
        assert 30 < flips < 98
