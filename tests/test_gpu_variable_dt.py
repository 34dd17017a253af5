"""Variable time step on the GPU (cuba_set_dt, cuba_batch_set_dt; Sec. 6).

* After a change of dt, the next steps stream with the new dt and test
  pairs with the new K: a GPU run that stops one step short, followed by
  one oracle step at the dt of that step, equals the full GPU run
  (positions and unscattered momenta bit-exact, scattered momenta within
  1e-12 of the pair energy), at every step of a schedule that changes dt
  twice, for one wave per cell and for 8 lanes per cell.
* A batched event whose dt changes between runs equals the same event run
  alone with the same schedule, bit for bit.
* Invalid values are rejected and leave dt as it was.
* The collision-limited policy reaches t_end exactly, keeps every dt
  within its limits, and conserves particle number and energy.
"""
import math

import numpy as np
import pytest

from paper_1208_0961_amd import timestep as TS
from paper_1208_0961_amd import workload as W
from test_gpu_parity import _orc_params, _rows, say, lib  # noqa: F401

pytestmark = pytest.mark.gpu

SCHEDULE = ((3, 0.02), (2, 0.035), (2, 0.01))


def _workload():
    """A 10 x 1 x 1 fm Riemann tube of 100 x 5 x 5 cells, ~9 / ~5
    particles per cell, K = 0.09 at dt = 0.02."""
    return W.Workload("vdt", (10.0, 1.0, 1.0), (100, 5, 5), 100.0, 1.8, 0.02, 0.45, 0.36,
                      seed=41)


def _gpu_run(lib, params, state, schedule, lanes):  # noqa: F811
    sim = lib.Sim(params, state, cell_lanes=lanes)
    for k, dt in schedule:
        sim.dt = dt
        sim.step(k)
    out = sim.get_state()
    sim.close()
    return out


def _truncate(schedule, m):
    out, left = [], m
    for k, dt in schedule:
        if left == 0:
            break
        out.append((min(k, left), dt))
        left -= min(k, left)
    return out


@pytest.mark.parametrize("lanes", (0, 8, 1))
def test_dt_changes_match_oracle(orc, lib, lanes):  # noqa: F811
    w = _workload()
    params = w.params()
    state = W.riemann_state(w, seed=42)
    total = sum(k for k, _ in SCHEDULE)
    scattered_total = 0
    for m in range(2, total + 1):
        prev = _gpu_run(lib, params, state, _truncate(SCHEDULE, m - 1), lanes)
        got = _gpu_run(lib, params, state, _truncate(SCHEDULE, m), lanes)
        dt_m = _truncate(SCHEDULE, m)[-1][1]
        say(f"[vdt] lanes={lanes} step {m - 1} dt={dt_m}")
        st = orc.State(*prev)
        tr = orc.step(_orc_params(orc, dict(params, dt=dt_m)), st, m - 1, trace=True)
        for d in range(3):
            assert np.array_equal(got[d], st[d]), (m, d)
        scattered = np.zeros(len(state[0]), bool)
        pair_e = np.zeros(len(state[0]))
        offs = tr["offsets"].astype(np.int64)
        E = np.sqrt(st[3] ** 2 + st[4] ** 2 + st[5] ** 2)
        for c, i, j in _rows(tr["claim"]):
            ia, ib = tr["perm"][offs[c] + i], tr["perm"][offs[c] + j]
            scattered[[ia, ib]] = True
            pair_e[[ia, ib]] = E[ia] + E[ib]
        for d in range(3, 6):
            assert np.array_equal(got[d][~scattered], st[d][~scattered]), (m, d)
            assert np.all(np.abs(got[d][scattered] - st[d][scattered])
                          <= 1e-12 * pair_e[scattered]), (m, d)
        scattered_total += int(scattered.sum())
    assert scattered_total > 500


def test_batched_dt_change_equals_alone(lib):  # noqa: F811
    import torch
    from paper_1208_0961_amd import batch
    ws = [_workload(), W.Workload("vdt2", (10.0, 1.0, 1.0), (100, 4, 4), 60.0, 0.9, 0.02,
                                  0.4, 0.32, seed=43)]
    states = [W.riemann_state(w, seed=50 + i) for i, w in enumerate(ws)]
    B = batch.Batch(len(ws), use_graphs=True)
    for i, (w, st) in enumerate(zip(ws, states)):
        B.admit(i, w.params(), st)
    B.step(3)
    B.set_dt(0, 0.035)
    B.step(3)
    B.set_dt(0, 0.01)
    B.set_dt(1, 0.03)
    B.step(3)
    assert B.dt(0) == 0.01 and B.dt(1) == 0.03
    got = [B.get_state(i) for i in range(len(ws))]
    B.close()
    torch.cuda.synchronize()
    sched = [((3, 0.02), (3, 0.035), (3, 0.01)), ((3, 0.02), (3, 0.02), (3, 0.03))]
    for i, (w, st) in enumerate(zip(ws, states)):
        want = _gpu_run(lib, w.params(), st, sched[i], None)
        for d in range(6):
            assert np.array_equal(got[i][d], want[d]), (w.name, d)


def test_invalid_dt_is_rejected(lib):  # noqa: F811
    from paper_1208_0961_amd import cuba as C
    w = _workload()
    sim = lib.Sim(w.params(), W.riemann_state(w, seed=1))
    # not finite, not positive, not below the 0.1 fm cell edge
    for bad in (0.0, -0.01, math.nan, math.inf, 0.1, 0.2):
        with pytest.raises(C.CubaError) as e:
            sim.dt = bad
        assert e.value.code == C.CUBA_EINVAL, bad
        assert sim.dt == 0.02 and C.cuba_get_dt(sim.ctx) == 0.02
    sim.dt = 0.05
    assert C.cuba_get_dt(sim.ctx) == 0.05
    sim.close()
    # sigma = 9 fm^2: K = 9 / 100 * dt / 0.004 = 22.5 dt, so 2K <= 1 needs
    # dt <= 1 / 45
    params = dict(w.params(), sigma=9.0)
    sim = lib.Sim(params, W.riemann_state(w, seed=1))
    with pytest.raises(C.CubaError) as e:
        sim.dt = 0.03
    assert e.value.code == C.CUBA_EINVAL and sim.dt == 0.02
    sim.dt = 0.022
    assert C.cuba_get_dt(sim.ctx) == 0.022
    sim.close()


def test_collision_limited_schedule(lib):  # noqa: F811
    w = _workload()
    state = W.riemann_state(w, seed=44)
    sim = lib.Sim(w.params(), state)
    e0 = float(sim.observe_moments()["T00"].sum())
    t_end = 0.5
    sched = TS.run_to(sim, t_end, p_max=0.2, every=10)
    say(f"[vdt] schedule {sched}")
    edge, k_max = TS.dt_limits(w.params())
    assert abs(sim.time - t_end) < 1e-12
    assert abs(sum(k * dt for k, dt in sched) - t_end) < 1e-12
    assert all(0 < dt <= 0.5 * edge and dt < k_max for _, dt in sched)
    # the densest slab sets dt: n sigma dt = p_max, n a little above the
    # hot side's mean (~230 particles per slab)
    n_hot = W.gluon_density(0.45)
    assert 0.2 / (1.4 * n_hot * 1.8) < sched[0][1] < 0.2 / (n_hot * 1.8)
    # the log holds the step index at which each dt took effect (the
    # policy's first dt replaces the initial one at step 0)
    starts = np.cumsum([0] + [k for k, _ in sched[:-1]])
    assert sim.dt_log == [(int(t), dt) for t, (_, dt) in zip(starts, sched)]
    m = sim.observe_moments()
    assert float(m["T00"].sum()) == pytest.approx(e0, rel=1e-12)
    dx = 10.0 / 100
    assert int(round(float((m["n"] * w.r_test * dx * 1.0 * 1.0).sum()))) == w.n
    sim.close()
