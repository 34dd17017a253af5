"""Host-side logic of the serving loop (no device work)."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def serve():
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import serve
    return serve


def test_fifo_replay_recurrence(serve):
    reqs = [serve.Request(i, None, a, 0) for i, a in enumerate((0.0, 0.5, 0.6, 5.0))]
    fin = serve.fifo_replay(reqs, {0: 1.0, 1: 1.0, 2: 1.0, 3: 1.0})
    assert fin == {0: 1.0, 1: 2.0, 2: 3.0, 3: 6.0}


def test_request_stream_sizes_and_poisson_arrivals(serve):
    reqs = serve.request_stream(2000, 10.0, seed=5)
    ns = np.array([r.work.n for r in reqs])
    assert len(reqs) == 2000 and ns.min() >= 1e4 and ns.max() <= 4e6
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert np.all(gaps >= 0)
    # exponential inter-arrival times with mean 1/rate
    assert abs(gaps.mean() - 0.1) < 4 * 0.1 / np.sqrt(len(gaps))
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.1
    # deterministic
    again = serve.request_stream(2000, 10.0, seed=5)
    assert [r.arrival for r in again] == [r.arrival for r in reqs]


def test_footprint_matches_workspace_formula(serve):
    from paper_1208_0961_amd import workload as W
    r = serve.request_stream(3, 1.0, seed=1)[0]
    cap = W.capacity_for(r.work)
    slots = r.work.n_cells * cap
    fp = serve.footprint(r)
    # blocks (104 B a slot), spill slots and overflow scratch (124 B a
    # particle), per-cell arrays (64 B a cell)
    want = 104 * slots + 124 * r.work.n + 64 * r.work.n_cells
    assert want <= fp <= want + 64 * 1024


def test_percentiles(serve):
    p50, p99 = serve.percentiles(np.arange(1, 101, dtype=float))
    assert p50 == pytest.approx(50.5) and p99 == pytest.approx(99.01)


class _FakeBatch:
    """Records set_active calls; stands in for the device batch."""

    def __init__(self):
        self.calls = []

    def set_active(self, slot, active):
        self.calls.append((slot, bool(active)))


class _FakeLane:
    """A lane as Server.run keeps it: live events and a fake batch."""

    def __init__(self, live):
        self.live = live
        self.B = _FakeBatch()


def _server(serve, policy, live, **attrs):
    srv = serve.Server.__new__(serve.Server)
    srv.policy, srv.peak_held = policy, 0
    srv.lanes = [_FakeLane(live)]
    for k, v in attrs.items():
        setattr(srv, k, v)
    return srv, srv.lanes[0]


def _live(serve, specs):
    """live dict as Server.run keeps it: slot -> request of equal size with
    (steps done, arrival), active flag."""
    from paper_1208_0961_amd import workload as W
    live = {}
    for slot, (done, arrival) in enumerate(specs):
        w = W.Workload(f"r{slot}", (10.0, 1.0, 1.0), (100, 5, 5), 100.0, 0.5, 0.02, 0.4, 0.32,
                       steps=200)
        req = serve.Request(slot, w, arrival, 0)
        live[slot] = {"req": req, "need": 0, "done": done, "admitted": 0.0, "active": True}
    return live


def test_srpt_policy_choice(serve):
    """The oldest event always runs; the others join by least remaining work
    (particles x steps left) while they fit the particle budget; set_active
    is called only for events whose state changes."""
    live = _live(serve, [(0, 0.5), (150, 0.1), (0, 0.2), (100, 0.3)])
    n = {s: ev["req"].work.n for s, ev in live.items()}
    # room for the oldest (slot 1) and one more
    srv, lane = _server(serve, "srpt", live, run_particles=n[1] + n[3])
    act = srv._choose(lane)
    left = {s: n[s] * (200 - live[s]["done"]) for s in live}
    assert 1 in act                           # oldest arrival
    # the event with the least remaining work besides the oldest is slot 3
    assert min((s for s in live if s != 1), key=left.get) == 3
    assert act == {1, 3}
    assert sorted(lane.B.calls) == [(0, False), (2, False)]
    assert srv.peak_held == 2
    # nothing changes: no calls
    lane.B.calls.clear()
    assert srv._choose(lane) == {1, 3} and lane.B.calls == []
    # a budget below the oldest's size still runs the oldest alone
    srv.run_particles = 1
    assert srv._choose(lane) == {1}
    assert lane.B.calls == [(3, False)]
    # policy all: every live event, no calls
    live2 = _live(serve, [(0, 0.5), (150, 0.1), (0, 0.2), (100, 0.3)])
    srv2, lane2 = _server(serve, "all", live2)
    assert srv2._choose(lane2) == set(live2) and lane2.B.calls == []


def test_fifo_policy_choice(serve):
    """fifo: the oldest events in arrival order while they fit the particle
    budget (the oldest always), then others by least remaining work while
    they fit the fill budget."""
    live = _live(serve, [(0, 0.5), (150, 0.1), (0, 0.2), (100, 0.3)])
    n = {s: ev["req"].work.n for s, ev in live.items()}
    # arrival order: 1, 2, 3, 0; room for two in arrival order, no fill
    srv, lane = _server(serve, "fifo", live, run_particles=n[1] + n[2], fill_particles=0)
    assert srv._choose(lane) == {1, 2}
    assert sorted(lane.B.calls) == [(0, False), (3, False)]
    # a fill of one event: the least remaining work among the rest (slot 3,
    # 100 steps done, before slot 0 with none)
    srv.fill_particles = n[3]
    assert srv._choose(lane) == {1, 2, 3}
    # the oldest runs even past the budget
    srv.run_particles, srv.fill_particles = 1, 0
    assert srv._choose(lane) == {1}


def test_classes_policy_lanes(serve):
    """classes: requests up to short_particles go to the short lane, whose
    runs take every live event there to its end; the long lane is stepped
    as under fifo."""
    from paper_1208_0961_amd import workload as W
    long_live = _live(serve, [(0, 0.5), (150, 0.1), (0, 0.2)])
    short_live = _live(serve, [(0, 0.6), (0, 0.7)])
    n = long_live[0]["req"].work.n
    srv, long_lane = _server(serve, "classes", long_live, run_particles=n, fill_particles=0,
                             short_particles=n, run_steps=25, final_only=True)
    short_lane = _FakeLane(short_live)
    short_lane.run_steps = 1 << 30
    long_lane.run_steps = 25
    srv.lanes.append(short_lane)
    assert srv._choose(long_lane) == {1}          # fifo head, no room for more
    assert sorted(long_lane.B.calls) == [(0, False), (2, False)]
    assert srv._choose(short_lane) == {0, 1} and short_lane.B.calls == []
    # a short run goes to the end of its events, a long one stops at run_steps
    w = short_live[0]["req"].work
    assert srv.steps_to_stop(w, 0, short_lane.run_steps) == w.steps
    assert srv.steps_to_stop(w, 0, long_lane.run_steps) == 25
    # lane by size
    small = serve.Request(9, W.Workload("s", (10.0, 1.0, 1.0), (100, 5, 5), 50.0, 0.5, 0.02,
                                        0.3, 0.24), 0.0, 0)
    big = serve.Request(10, W.Workload("b", (10.0, 4.0, 4.0), (100, 20, 20), 2500.0, 0.5,
                                       0.02, 0.5, 0.4), 0.0, 0)
    srv.short_particles = 300_000
    assert small.work.n <= 300_000 < big.work.n
    assert srv._lane_for(small) is short_lane and srv._lane_for(big) is long_lane


def test_server_rejects_unknown_policy(serve):
    with pytest.raises(ValueError):
        serve.Server(policy="lifo", hbm_budget=1 << 20)


def test_runs_stop_at_ends_and_observations(serve):
    """A run never takes an event past its last step, nor (when every
    profile is wanted) past its next observation."""
    from paper_1208_0961_amd import workload as W
    w = W.Workload("r", (10.0, 1.0, 1.0), (100, 5, 5), 100.0, 0.5, 0.02, 0.4, 0.32,
                   steps=130, observe_every=50)
    srv = serve.Server.__new__(serve.Server)
    srv.run_steps, srv.final_only = 40, False
    seq, done = [], 0
    while done < w.steps:
        k = srv.steps_to_stop(w, done)
        seq.append(k)
        done += k
    assert seq == [40, 10, 40, 10, 30] and done == 130
    srv.final_only = True
    seq, done = [], 0
    while done < w.steps:
        k = srv.steps_to_stop(w, done)
        seq.append(k)
        done += k
    assert seq == [40, 40, 40, 10]
    srv.run_steps = 200
    assert srv.steps_to_stop(w, 0) == 130 and srv.steps_to_stop(w, 125) == 5
    srv.final_only = False
    assert srv.steps_to_stop(w, 0) == 50 and srv.steps_to_stop(w, 120) == 10
    # observations written inside the runs: only the end and run_steps stop
    srv.observe_in_runs = True
    srv.run_steps = 40
    assert srv.steps_to_stop(w, 0) == 40 and srv.steps_to_stop(w, 120) == 10


def test_server_rejects_empty_runs(serve):
    with pytest.raises(ValueError):
        serve.Server(run_steps=0, hbm_budget=1 << 20)


class _FakeEvent:
    def __init__(self, done):
        self.done = done
        self.waited = False

    def query(self):
        return self.done

    def synchronize(self):
        self.waited = True
        self.done = True


def test_results_are_collected_out_of_order(serve):
    """A result whose copy has completed is collected even when one queued
    before it (the long lane's) is still on the GPU; block waits for the
    oldest."""
    import torch
    from collections import deque
    h = torch.zeros(2, dtype=torch.float64)
    long_ev, short_ev, later_ev = _FakeEvent(False), _FakeEvent(True), _FakeEvent(False)
    fields = lambda rid: dict(rid=rid, n=1, arrival=0.0, admitted=0.0)
    pending = deque([(long_ev, fields(0), h, h), (short_ev, fields(1), h, h),
                     (later_ev, fields(2), h, h)])
    results = []
    serve.collect_ready(pending, results, lambda: 1.0)
    assert [r.rid for r in results] == [1]
    assert [p[1]["rid"] for p in pending] == [0, 2]
    serve.collect_ready(pending, results, lambda: 2.0, block=True)
    assert long_ev.waited and not later_ev.waited
    assert [r.rid for r in results] == [1, 0] and results[1].finished == 2.0
    assert [p[1]["rid"] for p in pending] == [2]
