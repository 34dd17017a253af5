"""Pins of free streaming (Eq. (2)), wall reflection and binning.

Special cases with exact answers, an independently computed unfolded
(triangle-wave) trajectory for sigma = 0, and brute-force sorting for the
counting sort.
"""
import numpy as np
import pytest

from paper_1208_0961_amd import workload as W


def _params(orc, box=(10.0, 1.0, 1.0), cells=(100, 1, 1), sigma=0.0, r_test=100.0,
            dt=0.02, seed=1):
    return orc.make_params(box, cells, sigma, r_test, dt, seed)


def test_axis_aligned_particle_moves_exactly_dt(orc):
    p = _params(orc)
    st = orc.State([1.0, 2.5], [0.5, 0.25], [0.5, 0.75],
                   [0.7, -2.0], [0.0, 0.0], [0.0, 0.0])
    orc.step(p, st, 0)
    # p along +-x: p_x / E = +-1 exactly, so x moves by exactly +-dt
    assert st[0][0] == 1.0 + 0.02
    assert st[0][1] == 2.5 - 0.02
    assert st[1].tolist() == [0.5, 0.25] and st[2].tolist() == [0.5, 0.75]
    assert st[3].tolist() == [0.7, -2.0]


def test_reflection_at_each_wall(orc):
    p = _params(orc, box=(1.0, 1.0, 1.0), cells=(4, 4, 4), dt=0.1)
    # six particles, each 0.05 from a wall and moving into it along one axis
    x = [0.05, 0.95, 0.5, 0.5, 0.5, 0.5]
    y = [0.5, 0.5, 0.05, 0.95, 0.5, 0.5]
    z = [0.5, 0.5, 0.5, 0.5, 0.05, 0.95]
    px = [-1.0, 1.0, 0, 0, 0, 0]
    py = [0, 0, -2.0, 2.0, 0, 0]
    pz = [0, 0, 0, 0, -3.0, 3.0]
    st = orc.State(x, y, z, px, py, pz)
    orc.step(p, st, 0)
    # mirrored overshoot: 0.05 - 0.1 = -0.05 -> 0.05; 0.95 + 0.1 -> 2 - 1.05
    assert st[0][0] == -(0.05 - 0.1) and st[3][0] == 1.0
    assert st[0][1] == 2.0 - (0.95 + 0.1) and st[3][1] == -1.0
    assert st[1][2] == -(0.05 - 0.1) and st[4][2] == 2.0
    assert st[1][3] == 2.0 - (0.95 + 0.1) and st[4][3] == -2.0
    assert st[2][4] == -(0.05 - 0.1) and st[5][4] == 3.0
    assert st[2][5] == 2.0 - (0.95 + 0.1) and st[5][5] == -3.0


def test_particle_landing_on_wall_stays(orc):
    p = _params(orc, box=(1.0, 1.0, 1.0), cells=(4, 4, 4), dt=0.125)
    st = orc.State([0.125, 0.875], [0.5, 0.5], [0.5, 0.5], [-1.0, 1.0], [0, 0], [0, 0])
    tr = orc.step(p, st, 0, trace=True)
    assert st[0].tolist() == [0.0, 1.0]          # exactly on the walls: no flip
    assert st[3].tolist() == [-1.0, 1.0]
    # x = L maps to the last cell
    assert tr["cell"][1] // 16 == 3 and tr["cell"][0] // 16 == 0


def _unfold(x0, v, t, L):
    """Free motion with specular walls: the triangle wave of the unfolded
    straight line (an independent form of stream + reflect)."""
    u = np.mod(x0 + v * t, 2.0 * L)
    return np.where(u > L, 2.0 * L - u, u)


def test_sigma0_matches_unfolded_trajectories(orc):
    box = (3.0, 2.0, 1.0)
    x, y, z, px, py, pz = W.thermal_box(box, 2000, 0.3, seed=11)
    p = _params(orc, box=box, cells=(10, 8, 4), dt=0.05)
    st = orc.State(x, y, z, px, py, pz)
    nsteps = 400   # 20 fm/c: many reflections on every axis
    orc.run(p, st, 0, nsteps)
    E0 = np.sqrt(px**2 + py**2 + pz**2)
    t = nsteps * 0.05
    for d, (r0, q0) in enumerate(((x, px), (y, py), (z, pz))):
        want = _unfold(r0, q0 / E0, t, box[d])
        assert np.max(np.abs(st[d] - want)) < 1e-11
        # the momentum component's magnitude is preserved, its sign follows
        # the parity of the number of wall hits
        assert np.array_equal(np.abs(st[3 + d]), np.abs(q0))
    E1 = np.sqrt(st[3]**2 + st[4]**2 + st[5]**2)
    assert np.array_equal(E1, E0)


def test_binning_is_stable_counting_sort(orc):
    w = W.TUBE_1D
    x, y, z, px, py, pz = W.riemann_state(w, seed=5)
    box, cells = (10.0, 2.0, 2.0), (20, 5, 4)
    p = orc.make_params(box, cells, 0.4, 100.0, 0.02, 3)
    st = orc.State(x, 2 * y, 2 * z, px, py, pz)
    tr = orc.step(p, st, 0, trace=True)
    # cells computed independently from the streamed positions
    dx = np.array(box) / np.array(cells)
    idx = [np.clip(np.floor(st[d] / dx[d]).astype(np.int64), 0, cells[d] - 1)
           for d in range(3)]
    cell = (idx[0] * cells[1] + idx[1]) * cells[2] + idx[2]
    assert np.array_equal(tr["cell"].astype(np.int64), cell)
    ids = np.arange(len(x))
    assert np.array_equal(tr["perm"], np.lexsort((ids, cell)).astype(np.uint32))
    counts = np.bincount(cell, minlength=np.prod(cells))
    assert np.array_equal(tr["offsets"][1:], np.cumsum(counts).astype(np.uint32))
    assert tr["offsets"][0] == 0 and tr["offsets"][-1] == len(x)


def test_check_rejects_bad_input(orc):
    p = _params(orc)
    good = orc.State([1.0], [0.5], [0.5], [1.0], [0.0], [0.0])
    assert orc.check(p, good) == orc.OK
    assert orc.check(p, orc.State([10.5], [0.5], [0.5], [1.0], [0.0], [0.0])) == orc.ERANGE
    assert orc.check(p, orc.State([1.0], [0.5], [0.5], [0.0], [0.0], [0.0])) == orc.ERANGE
    assert orc.check(p, orc.State([np.nan], [0.5], [0.5], [1.0], [0.0], [0.0])) == orc.ERANGE
    # dt not below the cell edge (Sec. 5)
    assert orc.check(_params(orc, dt=0.1), good) == orc.EINVAL
    # P22 bound 2K > 1
    assert orc.check(_params(orc, sigma=1e4, r_test=1.0), good) == orc.EINVAL
    assert orc.check(_params(orc, sigma=-1.0), good) == orc.EINVAL
