"""Parity of the small-cell kernels (several cells per wave, one particle per
lane, larger cells stepped by the whole wave) with the CPU oracle, for every
lanes-per-cell setting.

cuba_trace_step runs the collision kernel of the context's setting, so the
trace comparison checks that kernel's decisions (cells, canonical order,
candidate and claimed pairs) bit for bit.  The fused kernel (collisions of
step t, then streaming and binning of step t+1) is checked by running
n - 1 and n steps from the same state: one oracle step from the first
result must reproduce the second.
"""
import numpy as np
import pytest

from paper_1208_0961_amd import workload as W
from test_gpu_parity import compare_step, _cells_box, _orc_params, _rows, say, lib  # noqa: F401

pytestmark = pytest.mark.gpu

LANES = (8, 16, 32, 64)
PACKED = 1                  # whole cells packed into waves of up to 64 particles
SETTINGS = (PACKED,) + LANES


def sparse_workload(mean_scale=1.0, seed=31):
    """A 10 x 1 x 1 fm Riemann tube, 100 x 5 x 5 cells, about 3.8 / 1.9
    particles per cell on the two sides (scaled by mean_scale), K = 0.09."""
    return W.Workload("sparse", (10.0, 1.0, 1.0), (100, 5, 5), 50.0 * mean_scale,
                      0.9 * mean_scale, 0.02, 0.45, 0.36, seed=seed)


@pytest.mark.parametrize("lanes", SETTINGS)
def test_small_cells_trace_parity_sparse(orc, lib, lanes):  # noqa: F811
    w = sparse_workload()
    state = W.riemann_state(w, seed=5)
    n_claim = 0
    for t in range(3):
        state, tr = compare_step(orc, lib, w.params(), state, t, "sparse", lanes=lanes)
        n_claim += len(tr["claim"])
    assert n_claim > 300


@pytest.mark.parametrize("lanes", SETTINGS)
def test_small_cells_trace_parity_ragged(orc, lib, lanes):  # noqa: F811
    # occupancies on both sides of every group size, the 64-lane limit, and
    # cells the whole wave must take over
    occ = ([0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 300]
           + [2] * 20 + [5] * 16 + [12] * 10)
    state = _cells_box(occ)
    params = dict(box=(1.0, 1.0, 1.0), cells=(4, 4, 4), sigma=2.0, r_test=1.0,
                  dt=0.001, seed=777)
    for t in range(2):
        state, tr = compare_step(orc, lib, params, state, t, "ragged", lanes=lanes)
    assert len(tr["claim"]) > 50


@pytest.mark.parametrize("lanes", SETTINGS)
def test_small_cells_every_pair_passes_filter(orc, lib, lanes):  # noqa: F811
    # 2K = 1: the w1 filter passes every pair, so every pair takes the exact
    # test and many claims compete inside each cell (packed: cells of up to
    # 64 particles, whose 2016 pairs fill the filtered-pair list many times)
    occ = [lanes, lanes - 1, 3, 2] * 2 if lanes != PACKED else [64, 63, 40, 2] * 2
    state = _cells_box(occ, m=2)
    V = 1.0 / 8.0
    params = dict(box=(1.0, 1.0, 1.0), cells=(2, 2, 2), sigma=0.5 * V / 0.001,
                  r_test=1.0, dt=0.001, seed=4242)
    _, tr = compare_step(orc, lib, params, state, 9, "K=1/2", lanes=lanes)
    assert len(tr["claim"]) >= (lanes if lanes != PACKED else 64) // 2


def _fused_step_check(orc, lib, params, state, nsteps, lanes, label):  # noqa: F811
    """GPU runs of nsteps - 1 and nsteps steps from state (the later steps of
    a run use the fused kernel); one oracle step from the first result must
    give the second (positions and unscattered momenta bit-exact, scattered
    momenta within 1e-12 of the pair energy)."""
    say(f"[fused] {label} lanes={lanes} nsteps={nsteps}")
    a = lib.Sim(params, state, cell_lanes=lanes)
    a.step(nsteps - 1)
    prev = a.get_state()
    a.close()
    b = lib.Sim(params, state, cell_lanes=lanes)
    b.step(nsteps)
    got = b.get_state()
    b.close()
    st = orc.State(*prev)
    t = (params.get("step0", 0) + nsteps - 1) & 0xFFFFFFFF
    tr = orc.step(_orc_params(orc, params), st, t, trace=True)
    for d in range(3):
        assert np.array_equal(got[d], st[d]), f"positions differ on axis {d}"
    scattered = np.zeros(len(state[0]), bool)
    pair_e = np.zeros(len(state[0]))
    offs = tr["offsets"].astype(np.int64)
    E = np.sqrt(st[3] ** 2 + st[4] ** 2 + st[5] ** 2)
    for c, i, j in _rows(tr["claim"]):
        ia = tr["perm"][offs[c] + i]
        ib = tr["perm"][offs[c] + j]
        scattered[[ia, ib]] = True
        pair_e[[ia, ib]] = E[ia] + E[ib]
    for d in range(3, 6):
        assert np.array_equal(got[d][~scattered], st[d][~scattered]), "unscattered p differs"
        assert np.all(np.abs(got[d][scattered] - st[d][scattered]) <= 1e-12 * pair_e[scattered])
    return len(tr["claim"])


@pytest.mark.parametrize("lanes", (0,) + SETTINGS)
def test_fused_small_cell_steps_match_oracle(orc, lib, lanes):  # noqa: F811
    w = sparse_workload(seed=11)
    state = W.riemann_state(w, seed=12)
    assert _fused_step_check(orc, lib, w.params(), state, 4, lanes, "sparse") > 50
    occ = [0, 1, 2, 3, 9, 17, 33, 65, 120] + [4] * 55
    state = _cells_box(occ, seed=8)
    params = dict(box=(1.0, 1.0, 1.0), cells=(4, 4, 4), sigma=2.0, r_test=1.0,
                  dt=0.001, seed=3)
    assert _fused_step_check(orc, lib, params, state, 3, lanes, "ragged") > 20


def test_lanes_settings_agree_bit_for_bit(lib):  # noqa: F811
    """Every setting runs the same decisions and the same arithmetic: after
    30 steps the states are identical, and so are the work counters."""
    from paper_1208_0961_amd import cuba as C
    w = sparse_workload(mean_scale=2.0, seed=21)
    state = W.riemann_state(w, seed=22)
    ref = None
    for lanes in (0,) + SETTINGS:
        s = lib.Sim(w.params(), state, cell_lanes=lanes)
        assert s.cell_lanes == lanes
        s.step(13)
        s.step(17)
        out = s.get_state()
        cnt = C.cuba_counters(s.ctx)
        s.close()
        if ref is None:
            ref = (out, cnt)
            assert cnt["claims"] > 1000
            continue
        for d in range(6):
            assert np.array_equal(out[d], ref[0][d]), f"lanes={lanes}: array {d}"
        assert cnt == ref[1], f"lanes={lanes}: counters {cnt} vs {ref[1]}"


def test_lanes_setting_is_validated(lib):  # noqa: F811
    from paper_1208_0961_amd import cuba as C
    w = sparse_workload()
    s = lib.Sim(w.params(), W.riemann_state(w))
    assert s.cell_lanes in (0,) + SETTINGS
    for bad in (-1, 2, 4, 12, 256):
        with pytest.raises(C.CubaError) as e:
            s.cell_lanes = bad
        assert e.value.code == C.CUBA_EINVAL
    s.close()


def _grid_state(occ, m=32, T=0.4, seed=9):
    """Cell j of an m^3 grid of unit edge holds occ[j] particles, uniform in
    the cell."""
    rng = np.random.default_rng(seed)
    occ = np.asarray(occ, dtype=np.int64)
    cell = np.repeat(np.arange(m ** 3), occ)
    ijk = np.stack([cell // (m * m), (cell // m) % m, cell % m], 1)
    r = (ijk + 0.05 + 0.9 * rng.random((len(cell), 3))) / m
    _, _, _, px, py, pz = W.sample_gas(rng, len(cell), T, (0, 0, 0), (1, 1, 1))
    return [np.ascontiguousarray(a) for a in (r[:, 0], r[:, 1], r[:, 2], px, py, pz)]


def test_default_lanes_rule(lib):  # noqa: F811
    """cuba_init's choice from the initial occupancy and K (32^3 cells), and
    the batch's, which never leaves a large share of the cells oversize."""
    import torch
    from paper_1208_0961_amd import batch
    m = 32
    C = m ** 3
    half = np.where(np.arange(C) < C // 2, 40, 3)
    # 2K = 6.6 % (sigma 0.1), or 0.066 % (sigma 0.001)
    cases = [("all 3", np.full(C, 3), 0.1, PACKED, 8),
             ("all 12", np.full(C, 12), 0.1, PACKED, 16),
             ("all 12, small K", np.full(C, 12), 0.001, 16, 16),
             ("all 25", np.full(C, 25), 0.1, 32, 32), ("all 40", np.full(C, 40), 0.1, 0, 0),
             ("dense and sparse halves", half, 0.1, PACKED, 0)]
    params = dict(box=(1.0, 1.0, 1.0), cells=(m, m, m), sigma=0.1, r_test=100.0,
                  dt=0.001, seed=5, cell_capacity=64)
    for label, occ, sigma, want_plain, want_batch in cases:
        state = _grid_state(occ)
        params = dict(params, sigma=sigma)
        s = lib.Sim(params, state)
        got = s.cell_lanes
        s.close()
        B = batch.Batch(1)
        B.admit(0, params, [torch.from_numpy(a).cuda() for a in state])
        got_b = B.cell_lanes(0)
        B.close()
        say(f"[lanes] {label}: plain {got}, batch {got_b}")
        assert (got, got_b) == (want_plain, want_batch), label
    # fewer cells than SIMDs, dense: two waves per cell on the plain path
    m = 8
    params_small = dict(params, cells=(m, m, m))
    for occ, want in ((40, 128), (20, 0)):
        state = _grid_state(np.full(m ** 3, occ), m=m)
        s = lib.Sim(params_small, state)
        got = s.cell_lanes
        s.close()
        B = batch.Batch(1)
        B.admit(0, params_small, [torch.from_numpy(a).cuda() for a in state])
        got_b = B.cell_lanes(0)
        B.close()
        say(f"[lanes] 512 cells of {occ}: plain {got}, batch {got_b}")
        assert (got, got_b) == (want, 0)


@pytest.mark.parametrize("two_k", (1.0, 0.3))
def test_fused_claimed_momenta_in_lds_or_written_back(orc, lib, two_k):  # noqa: F811
    # one wave per cell, fused: a cell keeps the new momenta of up to
    # cap / 12 claims (42 at 512 slots) in LDS for its binning and writes
    # more back to its block first; at 2K = 1 every pair passes the filter,
    # so the cells below hold claims on both sides of that bound
    occ = [200, 96, 88, 60, 30, 2, 1, 0]
    state = _cells_box(occ, m=2)
    V = 1.0 / 8.0
    params = dict(box=(1.0, 1.0, 1.0), cells=(2, 2, 2), sigma=two_k * 0.5 * V / 0.001,
                  r_test=1.0, dt=0.001, seed=31)
    claims = _fused_step_check(orc, lib, params, state, 3, 0, f"claim momenta 2K={two_k}")
    assert claims > (150 if two_k == 1.0 else 20)


def test_fused_full_cell_one_wave(orc, lib):  # noqa: F811
    # the 1024-slot kernel (85 claims in LDS) with a cell at the occupancy
    # limit and 2K = 1: hundreds of claims, written back
    state = _cells_box([1024], m=1, seed=17)
    params = dict(box=(1.0, 1.0, 1.0), cells=(1, 1, 1), sigma=500.0, r_test=1.0,
                  dt=0.001, seed=99)
    assert _fused_step_check(orc, lib, params, state, 2, 0, "cap1024 one wave") > 400
