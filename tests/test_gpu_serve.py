"""Serving: each request's result is the same when served in the mix (with
continuous batching, staggered admission and HBM-footprint admission) as
when run alone through the plain path."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import serve
    return serve


# run lengths: 25 and 50 divide the 100 steps and the 50-step observations;
# 40 does not: with the observations written inside the runs, runs of 40
# steps observe in their middle; with observations from the host between
# runs (in_runs False), runs stop early at every observation (40, 10, 40, 10)
@pytest.mark.parametrize("policy,final_only,run_steps,in_runs",
                         (("all", False, 25, True), ("srpt", False, 25, False),
                          ("srpt", True, 50, True), ("all", False, 40, True),
                          ("all", False, 40, False), ("fifo", True, 25, True),
                          ("classes", True, 25, True), ("classes", False, 40, True)))
def test_results_same_alone_and_in_the_mix(serve, policy, final_only, run_steps, in_runs):
    reqs = serve.request_stream(10, 0.0, seed=8, nmin=1e4, nmax=8e4, steps=100)
    budget = 3 * max(serve.footprint(r) for r in reqs)
    # srpt: a run holds about two of the requests, so events wait, are held
    # and resume between runs
    run_particles = 2 * max(r.work.n for r in reqs)
    # classes: about half the requests in each lane
    short = int(np.median([r.work.n for r in reqs]))
    # (fifo without the fill of small requests, so that events are held)
    srv = serve.Server(max_slots=4, hbm_budget=budget, run_steps=run_steps,
                       keep_states=True, policy=policy, run_particles=run_particles,
                       final_only=final_only, fill_particles=0, short_particles=short,
                       observe_in_runs=in_runs)
    res = srv.run(reqs, realtime=False)
    assert srv.peak_live <= 4 and srv.peak_bytes <= budget
    assert srv.peak_live >= 2          # the requests overlapped on the device
    if policy in ("srpt", "fifo"):
        assert srv.peak_held >= 1
    if policy == "classes":
        assert min(srv.lane_runs) >= 1   # both lanes ran
    srv.close()
    assert sorted(r.rid for r in res) == list(range(len(reqs)))
    by_id = {r.rid: r for r in reqs}
    for r in res:
        print(f"[serve] request {r.rid} n={r.n}", flush=True)
        _, T00, T0x, state = serve.run_alone(by_id[r.rid], keep_state=True,
                                             final_only=final_only)
        for d in range(6):
            assert np.array_equal(r.state[d], state[d]), (r.rid, d)
        # profile sums run in storage order: equal to rounding
        assert np.allclose(r.T00, T00, rtol=1e-12, atol=0)
        assert np.allclose(r.T0x, T0x, rtol=1e-12, atol=1e-12 * np.abs(T00).max())


def _anchor_requests(serve, steps):
    """Six requests of the served distribution (1e4 .. 4e6 test particles):
    the smallest, the largest and four between, arriving at runs 0, 0, 1,
    2, 3 and 4 of the server's logical clock, so that later requests are
    admitted while earlier ones are on the device."""
    pool = serve.request_stream(80, 0.0, seed=21, nmin=1e4, nmax=4e6, steps=steps)
    pool = sorted(pool, key=lambda r: r.work.n)
    picks = [pool[0], pool[-1], pool[20], pool[40], pool[60], pool[-2]]
    out = []
    for i, (r, run) in enumerate(zip(picks, (0, 0, 1, 2, 3, 4))):
        out.append(serve.Request(i, r.work, float(run), r.state_seed))
    return out


def test_served_requests_anchor_to_the_oracle(serve, orc):
    """Requests served with staggered admission, once with S - 1 = 7 steps
    and once with S = 8 (runs of 3 steps): one traced oracle step from each
    request's S - 1 result reproduces its S result at the parity contract's
    tolerance (positions and unscattered momenta bit-exact, the scattered set
    equal to the oracle's claims, scattered momenta within 1e-12 (Ea + Eb)).
    The S result also equals the request run alone, bit for bit."""
    import dataclasses
    import parity
    S = 8
    results = {}
    for steps in (S - 1, S):
        reqs = [dataclasses.replace(r, work=dataclasses.replace(r.work, steps=steps))
                for r in _anchor_requests(serve, S)]
        assert max(r.work.n for r in reqs) > 3_000_000
        srv = serve.Server(max_slots=8, run_steps=3, keep_states=True, final_only=True)
        res = srv.run(reqs, realtime="runs")
        srv.close()
        assert sorted(r.rid for r in res) == list(range(len(reqs)))
        by = {r.rid: r for r in res}
        # a request admitted while others were still on the device
        assert any(by[j].admitted_run > by[i].admitted_run
                   and by[j].admitted_run < by[i].finished_run
                   for i in by for j in by if i != j)
        results[steps] = by
    reqs = {r.rid: r for r in _anchor_requests(serve, S)}
    for rid, req in reqs.items():
        prev, got = results[S - 1][rid].state, results[S][rid].state
        print(f"[serve-anchor] request {rid}: n={req.work.n}", flush=True)
        n_sc = parity.full_step_check(orc, prev, got, req.work.params(), S - 1,
                                      f"request {rid}", threads=16)
        assert n_sc > 0
        _, _, _, alone = serve.run_alone(dataclasses.replace(
            req, work=dataclasses.replace(req.work, steps=S)), keep_state=True,
            final_only=True)
        for d in range(6):
            assert np.array_equal(got[d], alone[d]), (rid, d)


def test_async_admission_reports_a_bad_state_at_sync(serve):
    """An event admitted without waiting for the GPU whose initial state has
    a particle outside the box is reported by the next sync, with its slot;
    the event beside it keeps its result."""
    from paper_1208_0961_amd import batch, cuba as C, sim
    from paper_1208_0961_amd import workload as W
    w = W.TUBE_1D
    good = W.riemann_state(w, seed=3)
    bad = [a.copy() for a in W.riemann_state(w, seed=4)]
    bad[0][17] = 10.5   # outside [0, 10]
    B = batch.Batch(4)
    B.admit_async(1, w.params(), good, lanes=0)
    B.admit_async(3, w.params(), bad, lanes=0)
    with pytest.raises(C.CubaError) as e:
        B.sync()
    assert e.value.code == C.CUBA_ERANGE and e.value.slot == 3
    B.retire(3)
    B.step(5)
    got = B.get_state(1)
    B.close()
    s = sim.Sim(w.params(), good)
    s.step(5)
    want = s.get_state()
    s.close()
    for d in range(6):
        assert np.array_equal(got[d], want[d]), d
