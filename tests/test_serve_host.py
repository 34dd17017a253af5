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
    assert 104 * slots <= fp <= 104 * slots + 48 * r.work.n_cells + 64 * 1024


def test_percentiles(serve):
    p50, p99 = serve.percentiles(np.arange(1, 101, dtype=float))
    assert p50 == pytest.approx(50.5) and p99 == pytest.approx(99.01)
