"""Batched events: every event advanced in a batch (mixed with other events,
admitted and retired at different times, under any launch shape) ends in
exactly the state it reaches when run alone through cuba_step."""
import sys

import numpy as np
import pytest

from paper_1208_0961_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import batch, sim
    return batch, sim


def small_events():
    """Heterogeneous events: the 1-D tube and four small ensemble-style events
    of different r_test, sigma, temperature and box size."""
    evs = [W.TUBE_1D]
    for i, (rt, sig, TL, L) in enumerate(((50.0, 0.9, 0.45, 1.0), (400.0, 0.1, 0.31, 1.0),
                                          (150.0, 0.5, 0.38, 2.0), (60.0, 0.05, 0.5, 2.0))):
        n = int(round(5 * L))
        evs.append(W.Workload(f"small{i}", (10.0, L, L), (100, n, n), rt, sig, 0.02, TL,
                              0.8 * TL, seed=1000 + i))
    return evs


def alone(sim, w, state, nsteps):
    s = sim.Sim(w.params(), state)
    s.step(nsteps)
    out = s.get_state()
    s.close()
    return out


def assert_same(a, b, label):
    for d in range(6):
        assert np.array_equal(a[d], b[d]), f"{label}: array {d} differs"


def test_batch_equals_alone(mods):
    batch, sim = mods
    evs = small_events()
    states = [W.riemann_state(w, seed=77 + i) for i, w in enumerate(evs)]
    say(f"[batch] {len(evs)} events, n = {[w.n for w in evs]}")
    B = batch.Batch(8)
    for i, (w, st) in enumerate(zip(evs, states)):
        B.admit(i, w.params(), st)
    for k in (7, 1, 12):
        B.step(k)
    B.sync()
    for i, (w, st) in enumerate(zip(evs, states)):
        assert B.next_step(i) == 20
        assert_same(B.get_state(i), alone(sim, w, st, 20), w.name)
    B.close()


@pytest.mark.parametrize("cpi,persistent,graphs", [(1, 0, False), (3, 97, False),
                                                   (64, 0, True), (2, 300, True)])
def test_batch_launch_shapes(mods, cpi, persistent, graphs):
    batch, sim = mods
    evs = small_events()[1:]
    states = [W.riemann_state(w, seed=5 + i) for i, w in enumerate(evs)]
    say(f"[batch] cpi={cpi} persistent={persistent} graphs={graphs}")
    B = batch.Batch(4, persistent_waves=persistent, use_graphs=graphs)
    for i, (w, st) in enumerate(zip(evs, states)):
        B.admit(i, w.params(), st)
        B.set_cells_per_item(i, cpi)
    # repeated replays of the same run shape, with eager work in between
    for r in range(3):
        B.step(5)
        B.observe(r % len(evs))
    B.step(2)
    B.sync()
    for i, (w, st) in enumerate(zip(evs, states)):
        assert_same(B.get_state(i), alone(sim, w, st, 17), w.name)
    B.close()


def test_batch_staggered_admission_and_slot_reuse(mods):
    batch, sim = mods
    a, b, c = small_events()[1:4]
    sa, sb, sc = (W.riemann_state(w, seed=s) for w, s in ((a, 1), (b, 2), (c, 3)))
    B = batch.Batch(2, use_graphs=True)
    B.admit(0, a.params(), sa)
    B.step(10)
    B.admit(1, b.params(), sb)
    B.step(10)
    got_a = B.get_state(0)
    ws = B.retire(0)
    need = batch.event_workspace_bytes(batch.with_capacity(c.params(), sc), c.n)
    B.admit(0, c.params(), sc, workspace=ws if ws.numel() >= need else None)
    B.step(5)
    B.sync()
    assert_same(got_a, alone(sim, a, sa, 20), "A")
    assert_same(B.get_state(1), alone(sim, b, sb, 15), "B")
    assert_same(B.get_state(0), alone(sim, c, sc, 5), "C")
    B.close()


def test_batch_reports_the_failing_slot(mods):
    """A device-side error of one event (a cell past the 32-bit pair-index
    bound) names its slot; the other events keep their results."""
    batch, sim = mods
    from paper_1208_0961_amd import cuba as C
    ok = small_events()[1]
    n = C.CUBA_MAX_CELL_PARTICLES + 1
    rng = np.random.default_rng(4)
    bad_state = [0.2 + 0.6 * rng.random(n), 0.2 + 0.6 * rng.random(n),
                 0.2 + 0.6 * rng.random(n)] + list(W.sample_gas(rng, n, 0.4, (0, 0, 0),
                                                               (1, 1, 1))[3:])
    bad = dict(box=(1.0, 1.0, 1.0), cells=(1, 1, 1), sigma=1e-6, r_test=1.0, dt=0.001,
               seed=1, cell_capacity=256)
    ok_state = W.riemann_state(ok)
    B = batch.Batch(3)
    B.admit(0, ok.params(), ok_state)
    B.admit(2, bad, bad_state)
    B.step(2)
    with pytest.raises(C.CubaError) as e:
        B.sync()
    assert e.value.code == C.CUBA_ERANGE and e.value.slot == 2
    B.sync()       # reported once
    got = B.get_state(0)
    B.close()
    assert_same(got, alone(sim, ok, ok_state, 2), "healthy event beside a failing one")


def test_batch_mixed_lanes_per_cell(mods):
    """Events stepped with different lanes-per-cell settings in one batch,
    with items that end inside a group of cells, equal the events run alone
    (with the library's default setting)."""
    batch, sim = mods
    evs = small_events()
    states = [W.riemann_state(w, seed=40 + i) for i, w in enumerate(evs)]
    settings = [(0, 5), (8, 3), (16, 7), (32, 5), (64, 2)]
    B = batch.Batch(len(evs), use_graphs=True)
    for i, ((lanes, cpi), w, st) in enumerate(zip(settings, evs, states)):
        B.admit(i, w.params(), st)
        B.set_cell_lanes(i, lanes)
        B.set_cells_per_item(i, cpi)
        assert B.cell_lanes(i) == lanes
    say(f"[batch] lanes/cpi {settings}")
    for k in (6, 1, 6):
        B.step(k)
        B.observe(0)
    B.sync()
    for i, (w, st) in enumerate(zip(evs, states)):
        assert_same(B.get_state(i), alone(sim, w, st, 13), w.name)
    B.close()


def test_batch_mixed_cell_capacities(mods):
    """Events of cell capacity <= 512 and > 512 are stepped by kernels of
    different LDS size in one batch step (dense events in two one-wave-per-
    cell spaces; a small-cell event with a large capacity takes the large
    oversize scan); all equal the events run alone."""
    batch, sim = mods
    evs = small_events()
    states = [W.riemann_state(w, seed=60 + i) for i, w in enumerate(evs)]
    settings = [(0, 640), (0, 256), (16, 768), (0, 1024), (8, 128)]
    B = batch.Batch(len(evs), use_graphs=True)
    for i, ((lanes, cap), w, st) in enumerate(zip(settings, evs, states)):
        B.admit(i, {**w.params(), "cell_capacity": cap}, st)
        B.set_cell_lanes(i, lanes)
    say(f"[batch] lanes/capacity {settings}")
    for k in (5, 3):
        B.step(k)
    B.sync()
    for i, (w, st) in enumerate(zip(evs, states)):
        assert_same(B.get_state(i), alone(sim, w, st, 8), w.name)
    B.close()


def test_held_events_keep_their_state(mods):
    """cuba_batch_set_active: an event held out of some runs keeps its state
    and step index, and once resumed ends as its lone run of the steps it
    took part in; held with graphs on, so the table and graphs are rebuilt."""
    batch, sim = mods
    evs = small_events()[1:4]
    states = [W.riemann_state(w, seed=21 + i) for i, w in enumerate(evs)]
    B = batch.Batch(3, use_graphs=True)
    for i, (w, st) in enumerate(zip(evs, states)):
        B.admit(i, w.params(), st)
    B.step(4)                     # all: 4
    B.set_active(1, False)
    B.step(4)                     # 0 and 2: 8
    held = B.get_state(1)
    B.set_active(0, False)
    B.set_active(2, False)
    B.set_active(1, True)
    B.step(4)                     # 1: 8
    B.set_active(0, True)
    B.step(3)                     # 0: 11, 1: 11
    B.sync()
    assert [B.next_step(i) for i in range(3)] == [11, 11, 8]
    assert_same(held, alone(sim, evs[1], states[1], 4), "held")
    for i, n in enumerate((11, 11, 8)):
        assert_same(B.get_state(i), alone(sim, evs[i], states[i], n), evs[i].name)
    B.close()


def test_full_ensemble_sampled_parity(mods, orc):
    """The 256-event ensemble of the batched benchmark, admitted and tuned as
    it is there (graph-captured runs): after 4 steps, one more batched step
    of each sampled event (the smallest, the median, the largest below 2 M
    particles, and one stepped with several cells per wave if the tuning
    gives one) equals one oracle step from its state: positions and
    unscattered momenta bit-exact, scattered momenta within 1e-12 of the
    pair energy."""
    import torch
    from paper_1208_0961_amd import autotune as AT
    from test_gpu_parity import _orc_params, _rows
    batch, sim = mods
    events = W.ensemble_events(256)
    B = batch.Batch(len(events))
    for i, w in enumerate(events):
        st = W.riemann_state_torch(w, 100000 + i)
        B.admit(i, {**w.params(), "cell_capacity": W.capacity_for(w)}, st)
        del st
    table = AT.load() or AT.tune(events)
    AT.apply(B, table, dict(enumerate(events)), use_graphs=True)
    order = sorted(range(len(events)), key=lambda i: events[i].n)
    small = [i for i in order if events[i].n < 2_000_000]
    sample = {order[0], order[len(order) // 2], small[-1]}
    lanes = [i for i in small if B.cell_lanes(i) > 0]
    if lanes:
        sample.add(lanes[len(lanes) // 2])
    B.step(4)
    prev = {i: B.get_state(i) for i in sample}
    B.step(1)
    got = {i: B.get_state(i) for i in sample}
    B.close()
    torch.cuda.synchronize()
    scattered_total = 0
    for i in sorted(sample):
        w = events[i]
        say(f"[ensemble] event {i}: n={w.n}, lanes={lanes and i in lanes}")
        st = orc.State(*prev[i])
        tr = orc.step(_orc_params(orc, w.params()), st, 4, trace=True)
        for d in range(3):
            assert np.array_equal(got[i][d], st[d]), (i, d)
        scattered = np.zeros(w.n, bool)
        pair_e = np.zeros(w.n)
        offs = tr["offsets"].astype(np.int64)
        E = np.sqrt(st[3] ** 2 + st[4] ** 2 + st[5] ** 2)
        for c, a, b in _rows(tr["claim"]):
            ia, ib = tr["perm"][offs[c] + a], tr["perm"][offs[c] + b]
            scattered[[ia, ib]] = True
            pair_e[[ia, ib]] = E[ia] + E[ib]
        for d in range(3, 6):
            assert np.array_equal(got[i][d][~scattered], st[d][~scattered]), (i, d)
            assert np.all(np.abs(got[i][d][scattered] - st[d][scattered])
                          <= 1e-12 * pair_e[scattered]), (i, d)
        scattered_total += int(scattered.sum())
    assert scattered_total > 1000


@pytest.mark.parametrize("graphs", (False, True))
def test_observation_inside_runs(mods, graphs):
    """Observations written by the runs' own launches (cuba_batch_set_observe)
    equal the plain path's cuba_observe at the same steps: every 7 steps of
    each event, in runs of 10 steps that do not stop there (the last launch
    of a run observing too), for events stepped a wave per cell, with 8, 16
    and 32 lanes per cell, and one whose cells overflow their blocks; an
    event without observation and a held event are left alone."""
    import torch
    batch, sim = mods
    evs = small_events()
    states = [W.riemann_state(w, seed=60 + i) for i, w in enumerate(evs)]
    settings = [0, 8, 16, 32, 0]
    every, rows = 7, 4
    B = batch.Batch(len(evs) + 1, use_graphs=graphs)
    outs = []
    for i, (lanes, w, st) in enumerate(zip(settings, evs, states)):
        params = w.params()
        if i == 4:
            params = {**params, "cell_capacity": 8}   # overflowing cells
        B.admit(i, params, st)
        B.set_cell_lanes(i, lanes)
        outs.append(B.set_observe(i, every, rows))
    # a held event and an unobserved one beside them
    B.admit(5, evs[1].params(), states[1])
    B.set_active(5, False)
    for k in (10, 10, 10):
        B.step(k)
    B.sync()
    torch.cuda.synchronize()
    for i, (w, st) in enumerate(zip(evs, states)):
        params = w.params() if i != 4 else {**w.params(), "cell_capacity": 8}
        s = sim.Sim(params, st)
        done = 0
        for t in (7, 14, 21, 28):
            s.step(t - done)
            done = t
            T00, T0x = s.observe()
            got = outs[i][(t // every) % rows].cpu().numpy()
            say(f"[obs] event {i} after step {t}")
            assert np.allclose(got[0], T00, rtol=1e-12, atol=0), (i, t)
            assert np.allclose(got[1], T0x, rtol=1e-12, atol=1e-12 * np.abs(T00).max()), (i, t)
        s.close()
    assert B.next_step(5) == 0
    B.close()
