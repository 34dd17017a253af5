"""cuba_suggest_cell_capacity: the largest initial cell occupancy counted on
the device, against the same count in numpy (cell index of Sec. 2:
floor(x / dx) per axis, clamped to the grid, x-major)."""
import numpy as np
import pytest

from paper_1208_0961_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import sim
    return sim


def _max_occupancy(params, state):
    box = np.asarray(params["box"], np.float64)
    cells = np.asarray(params["cells"], np.int64)
    r = [np.asarray(state[d], np.float64) for d in range(3)]
    ok = np.isfinite(r[0]) & np.isfinite(r[1]) & np.isfinite(r[2])
    idx = [np.clip(np.floor(r[d][ok] / (box[d] / cells[d])), 0, cells[d] - 1).astype(np.int64)
           for d in range(3)]
    flat = (idx[0] * cells[1] + idx[1]) * cells[2] + idx[2]
    return int(np.bincount(flat).max()) if len(flat) else 0


def _want(m):
    if m == 0:
        return 64
    return max(64, min(1024, -(-(2 * m + 32) // 32) * 32))


def test_capacity_counts_on_the_device(mods):
    sim = mods
    w = W.TUBE_1D
    st = W.riemann_state(w)
    m = _max_occupancy(w.params(), st)
    assert sim.suggest_cell_capacity(w.params(), st) == _want(m)
    # known occupancies: the largest cell holds 300, one holds a particle at
    # x = L (clamped into the last cell), and NaN positions are skipped
    rng = np.random.default_rng(3)
    params = dict(box=(1.0, 1.0, 1.0), cells=(4, 4, 4), sigma=0.5, r_test=1.0, dt=0.01, seed=1)
    occ = rng.integers(0, 40, 64)
    occ[17] = 300
    cell = np.repeat(np.arange(64), occ)
    ijk = np.stack([cell // 16, (cell // 4) % 4, cell % 4], 1)
    r = (ijk + rng.random((len(cell), 3))) / 4.0
    x, y, z = [np.ascontiguousarray(r[:, d]) for d in range(3)]
    x[:3] = 1.0
    y[3:5] = np.nan
    st = [x, y, z] + [np.ones(len(x))] * 3
    m = _max_occupancy(params, st)
    assert m >= 298
    assert sim.suggest_cell_capacity(params, st) == _want(m)
    # beyond the largest block: clamped; no particles: the smallest block
    big = [np.full(700, 0.1)] * 3 + [np.ones(700)] * 3
    assert sim.suggest_cell_capacity(params, big) == 1024
    empty = [np.zeros(0)] * 6
    assert sim.suggest_cell_capacity(params, empty) == 64


def test_paper_set_capacity_matches_numpy(mods):
    """The 32^3 fm^3 set's 24.9 M particles: the device count agrees with
    numpy's."""
    import torch
    sim = mods
    w = W.PAPER_32
    st = W.riemann_state_torch(w, seed=77, device="cuda")
    host = [a.cpu().numpy() for a in st[:3]]
    assert sim.suggest_cell_capacity(w.params(), st) == _want(_max_occupancy(w.params(), host))
    del st
    torch.cuda.empty_cache()
