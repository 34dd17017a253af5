"""Stage timing through the C-ABI: HIP events around every launch
(cuba_timing_begin), or around every launch of the rare stages and every
n-th fused step only (cuba_timing_begin_sampled), which keeps the events'
own delay out of a timed run."""
import pytest

from paper_1208_0961_amd import workload as W
from test_gpu_parity import lib, say  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lanes", (128, 0, 8, 1))
def test_stage_timing_every_launch_and_sampled(lib, lanes):  # noqa: F811
    # one-kernel launches (two waves or one wave per cell) carry the events
    # on their dispatch; the small-cell and packed launches (two kernels,
    # forked) are bracketed
    from paper_1208_0961_amd import cuba as C
    w = W.TUBE_1D
    s = lib.Sim(w.params(), W.riemann_state(w), cell_lanes=lanes)
    # a call of 25 steps: one stream-bin launch, 24 fused steps, one
    # collide-only launch
    say(f"[timing] every launch, lanes {lanes}")
    C.cuba_timing_begin(s.ctx, 100)
    s.step(25)
    s.observe_async()
    st = C.cuba_timing_end(s.ctx)
    assert [st[k][1] for k in ("bin", "step", "collide", "observe")] == [1, 24, 1, 1]
    assert all(st[k][0] > 0 for k in ("bin", "step", "collide", "observe"))
    say("[timing] every 10th fused step")
    C.cuba_timing_begin_sampled(s.ctx, 100, 10)
    s.step(25)       # fused launches 0..23 of the timing: 0, 10, 20 timed
    s.step(25)       # 24..47: 30, 40
    st = C.cuba_timing_end(s.ctx)
    assert [st[k][1] for k in ("bin", "step", "collide")] == [2, 5, 2]
    assert st["step"][0] > 0
    # the cap on timed launches still holds
    C.cuba_timing_begin_sampled(s.ctx, 3, 1)
    s.step(25)
    st = C.cuba_timing_end(s.ctx)
    assert sum(st[k][1] for k in C.STAGES) == 3
    s.close()
