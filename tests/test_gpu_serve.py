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
# 40 does not, so runs stop early at every observation (40, 10, 40, 10)
@pytest.mark.parametrize("policy,final_only,run_steps",
                         (("all", False, 25), ("srpt", False, 25), ("srpt", True, 50),
                          ("all", False, 40)))
def test_results_same_alone_and_in_the_mix(serve, policy, final_only, run_steps):
    reqs = serve.request_stream(10, 0.0, seed=8, nmin=1e4, nmax=8e4, steps=100)
    budget = 3 * max(serve.footprint(r) for r in reqs)
    # srpt: a run holds about two of the requests, so events wait, are held
    # and resume between runs
    run_particles = 2 * max(r.work.n for r in reqs)
    srv = serve.Server(max_slots=4, hbm_budget=budget, run_steps=run_steps,
                       keep_states=True, policy=policy, run_particles=run_particles,
                       final_only=final_only)
    res = srv.run(reqs, realtime=False)
    assert srv.peak_live <= 4 and srv.peak_bytes <= budget
    assert srv.peak_live >= 2          # the requests overlapped on the device
    if policy == "srpt":
        assert srv.peak_held >= 1
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
