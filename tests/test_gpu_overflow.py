"""Cells that hold more particles than their block (cell_capacity): the
surplus goes to spill slots and the collision kernels' overflow path
steps the cell.
Nothing is dropped, and every step keeps the parity contract with the
oracle: cells, canonical order, candidates and claims identical, positions
and unscattered momenta bit-exact, scattered momenta within 1e-12 (Ea + Eb).
Overflow is forced with small capacities: at init, mid-run (a cell filling
past its block during a step), under every launch shape, in a batch, and
for a cell past the 32-bit pair-index bound."""
import sys

import numpy as np
import pytest

import parity
from paper_1208_0961_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1208_0961_amd import build
    if build.sources_newer_than_lib():
        build.build()
    from paper_1208_0961_amd import sim
    return sim


def cells_box(occupancies, L=1.0, m=4, T=0.4, seed=3):
    """Particles placed so that cell j of an m x m x m grid (edge L/m) holds
    occupancies[j] of them, ids shuffled."""
    rng = np.random.default_rng(seed)
    dxc = L / m
    xs, ys, zs = [], [], []
    for j, k in enumerate(occupancies):
        ix, iy, iz = j // (m * m), (j // m) % m, j % m
        lo = np.array([ix, iy, iz]) * dxc + 0.1 * dxc
        r = lo + 0.8 * dxc * rng.random((k, 3))
        xs.append(r[:, 0]); ys.append(r[:, 1]); zs.append(r[:, 2])
    n = int(sum(occupancies))
    _, _, _, px, py, pz = W.sample_gas(rng, n, T, (0, 0, 0), (1, 1, 1))
    perm = rng.permutation(n)
    return [np.concatenate(xs)[perm], np.concatenate(ys)[perm], np.concatenate(zs)[perm],
            px[perm], py[perm], pz[perm]]


def traced_step(orc, lib, params, state, t, label, lanes=None):
    """One traced step on both sides from the same state; the parity
    contract.  Returns the GPU state after the step."""
    say(f"[overflow] {label} n={len(state[0])} t={t} lanes={lanes}")
    st = orc.State(*state)
    tr_o = orc.step(parity.orc_params(orc, params), st, t, trace=True)
    sim = lib.Sim({**params, "step0": t}, state, cell_lanes=lanes)
    tr_g = sim.trace_step(cand_cap=len(tr_o["cand"]) + 1024)
    gs = sim.get_state()
    T00, T0x = sim.observe()
    sim.close()
    assert np.array_equal(tr_g["cell"], tr_o["cell"]), f"{label}: cells"
    assert np.array_equal(tr_g["offsets"], tr_o["offsets"]), f"{label}: offsets"
    assert np.array_equal(tr_g["perm"], tr_o["perm"]), f"{label}: canonical order"
    assert np.array_equal(parity.rows(tr_g["cand"]), parity.rows(tr_o["cand"])), \
        f"{label}: candidates"
    assert np.array_equal(parity.rows(tr_g["claim"]), parity.rows(tr_o["claim"])), \
        f"{label}: claims"
    for d in range(3):
        assert np.array_equal(gs[d], st[d]), f"{label}: positions, axis {d}"
    scattered = np.zeros(len(state[0]), bool)
    pair_e = np.zeros(len(state[0]))
    offs = tr_o["offsets"].astype(np.int64)
    E = np.sqrt(st[3] ** 2 + st[4] ** 2 + st[5] ** 2)
    for c, a, b in parity.rows(tr_o["claim"]):
        ia, ib = tr_o["perm"][offs[c] + a], tr_o["perm"][offs[c] + b]
        scattered[[ia, ib]] = True
        pair_e[[ia, ib]] = E[ia] + E[ib]
    for d in range(3, 6):
        assert np.array_equal(gs[d][~scattered], st[d][~scattered]), f"{label}: unscattered p"
        dev = np.abs(gs[d][scattered] - st[d][scattered])
        assert np.all(dev <= 1e-12 * pair_e[scattered]), (label, d, float(dev.max()))
    # profiles of the (partly spilled) state: within the rounding of the sums
    p = parity.orc_params(orc, params)
    oT00, oT0x = orc.observe(p, orc.State(*gs))
    dx = p.box[0] / p.cells[0]
    vol = p.r_test * dx * p.box[1] * p.box[2]
    ix = np.clip(np.floor(gs[0] / dx).astype(np.int64), 0, p.cells[0] - 1)
    cnt = np.bincount(ix, minlength=p.cells[0])
    Eg = np.sqrt(gs[3] ** 2 + gs[4] ** 2 + gs[5] ** 2)
    eps = 2.0 ** -53
    assert np.all(np.abs(T00 - oT00) <= 2 * (cnt + 2) * eps * np.bincount(ix, Eg, p.cells[0]) / vol + 1e-300)
    assert np.all(np.abs(T0x - oT0x) <= 2 * (cnt + 2) * eps * np.bincount(ix, np.abs(gs[3]), p.cells[0]) / vol + 1e-300)
    return gs, tr_o


def test_overflowing_cell_from_init(orc, lib):
    # one cell of 1100 particles in blocks of 64: the whole cell past its
    # block from the start; K = sigma dt / V = 0.004 gives ~2 400 candidates
    # over 148 claim rounds of 4 096 pairs
    state = cells_box([1100], m=1)
    params = dict(box=(1.0, 1.0, 1.0), cells=(1, 1, 1), sigma=4.0, r_test=1.0,
                  dt=0.001, seed=11, cell_capacity=64)
    gs, tr = traced_step(orc, lib, params, state, 0, "one cell 1100 / 64")
    assert len(tr["claim"]) > 300
    # and beyond the largest block
    params["cell_capacity"] = 1024
    state = cells_box([1500], m=1, seed=4)
    traced_step(orc, lib, params, state, 3, "one cell 1500 / 1024")


@pytest.mark.parametrize("lanes,cap", [(0, 32), (16, 32), (128, 32), (64, 16), (1, 32)])
def test_mixed_overflowing_and_normal_cells(orc, lib, lanes, cap):
    # 64 cells, a third of them past a block of 32 (up to 300 members), the
    # rest below it, some empty; several steps, traced.  With blocks of 16
    # and 64 lanes per cell, cells of 17 .. 64 overflow while fitting the
    # small-cell kernel's lanes
    rng = np.random.default_rng(7)
    occ = rng.integers(0, 30, 64)
    occ[rng.choice(64, 22, replace=False)] = rng.integers(33, 300, 22)
    occ[:3] = [0, 1, 2]
    state = cells_box(list(occ), m=4, seed=8)
    params = dict(box=(1.0, 1.0, 1.0), cells=(4, 4, 4), sigma=0.002, r_test=1.0,
                  dt=0.01, seed=5, cell_capacity=cap)
    for t in range(4):
        state, _ = traced_step(orc, lib, params, state, t, f"mixed lanes {lanes}", lanes)


def test_fused_steps_with_overflow(orc, lib):
    # a fused step (collisions of step t, then the binning of t + 1, with
    # the overflow path for the overflowing cells) from the traced state
    rng = np.random.default_rng(9)
    occ = list(rng.integers(40, 140, 27))
    state = cells_box(occ, m=3, seed=10)
    params = dict(box=(1.0, 1.0, 1.0), cells=(3, 3, 3), sigma=0.004, r_test=1.0,
                  dt=0.01, seed=6, cell_capacity=64)
    g1, _ = traced_step(orc, lib, params, state, 0, "fused: first step")
    sim = lib.Sim(params, state)
    sim.step(3)
    g3 = sim.get_state()
    sim.close()
    sim = lib.Sim(params, state)
    sim.step(2)
    g2 = sim.get_state()
    sim.close()
    parity.full_step_check(orc, g1, g2, params, 1, "fused step 1 with overflow")
    parity.full_step_check(orc, g2, g3, params, 2, "fused step 2 with overflow")


def test_cell_fills_past_its_block_during_a_run(orc, lib):
    # the right half of the box streams into the left cell: after one step
    # it holds ~120 particles in blocks of 64
    n = 60
    rng = np.random.default_rng(4)
    x = np.concatenate([0.1 + 0.3 * rng.random(n), 0.5 + 0.004 * rng.random(n)])
    y = rng.random(2 * n)
    z = rng.random(2 * n)
    px = np.concatenate([np.ones(n), -np.ones(n)]) * (1 + 0.1 * rng.random(2 * n))
    py = 0.05 * rng.standard_normal(2 * n)
    pz = 0.05 * rng.standard_normal(2 * n)
    state = [x, y, z, px, py, pz]
    params = dict(box=(1.0, 1.0, 1.0), cells=(2, 1, 1), sigma=0.5, r_test=1.0,
                  dt=0.01, seed=1, cell_capacity=64)
    st = state
    for t in range(3):
        st, tr = traced_step(orc, lib, params, st, t, "filling")
    assert np.bincount(tr["cell"], minlength=2)[0] > 64
    # nothing lost over a longer run: particle number and energy kept
    sim = lib.Sim(params, state)
    sim.step(40)
    sim.sync()
    gs = sim.get_state()
    sim.close()
    E0 = np.sqrt(px ** 2 + py ** 2 + pz ** 2).sum()
    E1 = np.sqrt(gs[3] ** 2 + gs[4] ** 2 + gs[5] ** 2).sum()
    assert abs(E1 - E0) <= 1e-12 * E0
    assert np.all(np.isfinite(gs[0]))


def test_batch_event_with_overflow_equals_alone(lib):
    from paper_1208_0961_amd import batch
    rng = np.random.default_rng(12)
    occ = list(rng.integers(20, 160, 27))
    state = cells_box(occ, m=3, seed=13)
    params = dict(box=(1.0, 1.0, 1.0), cells=(3, 3, 3), sigma=0.004, r_test=1.0,
                  dt=0.01, seed=2, cell_capacity=64)
    other = W.riemann_state(W.TUBE_1D, seed=5)
    B = batch.Batch(4)
    B.admit(0, params, state)
    B.admit(1, W.TUBE_1D.params(), other)
    B.step(6)
    B.sync()
    got = B.get_state(0)
    got_other = B.get_state(1)
    B.close()
    for label, p, s0, g in (("overflowing event", params, state, got),
                            ("tube", W.TUBE_1D.params(), other, got_other)):
        sim = lib.Sim(p, s0)
        sim.step(6)
        want = sim.get_state()
        sim.close()
        for d in range(6):
            assert np.array_equal(g[d], want[d]), f"{label}: column {d}"


def test_cell_past_the_pair_index_bound(lib):
    from paper_1208_0961_amd import cuba as C
    # 92 682 particles in one cell: its pair indices overflow the counter
    # word, so its collisions are skipped and the sync reports it; its
    # particles still stream
    n = C.CUBA_MAX_CELL_PARTICLES + 1
    rng = np.random.default_rng(3)
    state = [0.2 + 0.6 * rng.random(n), 0.2 + 0.6 * rng.random(n),
             0.2 + 0.6 * rng.random(n)] + list(W.sample_gas(rng, n, 0.4, (0, 0, 0),
                                                           (1, 1, 1))[3:])
    params = dict(box=(1.0, 1.0, 1.0), cells=(1, 1, 1), sigma=1e-6, r_test=1.0,
                  dt=0.001, seed=1, cell_capacity=256)
    sim = lib.Sim(params, state)
    sim.step(1)
    with pytest.raises(C.CubaError) as e:
        sim.sync()
    assert e.value.code == C.CUBA_ERANGE and "pair" in str(e.value)
    gs = sim.get_state()
    sim.close()
    for d in range(3):
        v = state[d + 3] / np.sqrt(state[3] ** 2 + state[4] ** 2 + state[5] ** 2)
        assert np.array_equal(gs[d], state[d] + v * 0.001), f"streaming, axis {d}"
    for d in range(3, 6):
        assert np.array_equal(gs[d], state[d]), "momenta changed"
