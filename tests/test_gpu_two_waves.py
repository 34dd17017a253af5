"""Two waves per cell (cuba_set_cell_lanes(ctx, 128)): the pair range of a
cell split over a workgroup of two waves, the second filtering its half
into its own buffer and the first resolving and claiming every filtered pair
in increasing pair order.  The decisions and the arithmetic are those of one
wave per cell, so:

* fused steps (and the collide-only step that ends a run) match one oracle
  step from the GPU's previous state, on a dense tube, on ragged cells (the
  counting rank below 64 particles, fewer pairs than one 128-pair block),
  and on a cell at the 1024 cap with 2K = 1, where every pair passes the
  Philox filter and the second wave's buffer fills, so that the first wave
  resumes the tests where it stopped;
* 30 steps give states and work counters identical to one wave per cell.
"""
import numpy as np
import pytest

from paper_1208_0961_amd import workload as W
from test_gpu_parity import _cells_box, say, lib  # noqa: F401
from test_gpu_small_cells import _fused_step_check

pytestmark = pytest.mark.gpu

TWO = 128


def test_two_waves_dense_tube(orc, lib):  # noqa: F811
    w = W.TUBE_1D
    state = W.riemann_state(w, seed=14)
    assert _fused_step_check(orc, lib, w.params(), state, 3, TWO, "tube1d") > 20


def test_two_waves_ragged_cells(orc, lib):  # noqa: F811
    occ = [0, 1, 2, 3, 9, 17, 23, 33, 48, 63, 64, 65, 120, 200, 300] + [4] * 49
    state = _cells_box(occ, seed=8)
    params = dict(box=(1.0, 1.0, 1.0), cells=(4, 4, 4), sigma=2.0, r_test=1.0,
                  dt=0.001, seed=3)
    assert _fused_step_check(orc, lib, params, state, 3, TWO, "ragged") > 20


@pytest.mark.parametrize("sigma", (500.0, 2.0))
def test_two_waves_full_cell(orc, lib, sigma):  # noqa: F811
    # K = sigma / r_test * dt / V = 0.5 at sigma = 500: 2K = 1
    state = _cells_box([1024], m=1, seed=17)
    params = dict(box=(1.0, 1.0, 1.0), cells=(1, 1, 1), sigma=sigma, r_test=1.0,
                  dt=0.001, seed=99)
    claims = _fused_step_check(orc, lib, params, state, 2, TWO, f"cap1024 sigma={sigma}")
    assert claims > (400 if sigma == 500.0 else 0)


def test_two_waves_bit_identical_to_one(lib):  # noqa: F811
    from paper_1208_0961_amd import cuba as C
    w = W.Workload("tw", (10.0, 2.0, 2.0), (100, 10, 10), 600.0, 0.4, 0.02, 0.45, 0.36,
                   seed=23)
    state = W.riemann_state(w, seed=24)
    out = {}
    for lanes in (0, TWO):
        s = lib.Sim(w.params(), state, cell_lanes=lanes)
        assert s.cell_lanes == lanes
        s.step(13)
        s.step(17)
        out[lanes] = (s.get_state(), C.cuba_counters(s.ctx))
        s.close()
    for d in range(6):
        assert np.array_equal(out[0][0][d], out[TWO][0][d]), d
    assert out[0][1] == out[TWO][1]
    assert out[0][1]["claims"] > 1000


def test_two_waves_not_for_batches(lib):  # noqa: F811
    import torch
    from paper_1208_0961_amd import batch
    from paper_1208_0961_amd import cuba as C
    w = W.TUBE_1D
    B = batch.Batch(1)
    B.admit(0, w.params(), [torch.from_numpy(a).cuda() for a in W.riemann_state(w)])
    with pytest.raises(C.CubaError) as e:
        B.set_cell_lanes(0, TWO)
    assert e.value.code == C.CUBA_EINVAL
    B.close()
