"""Variable time step (Sec. 6): pins of the oracle under a changing dt and
of the dt policy (paper_1208_0961_amd/timestep.py).

* Without collisions (sigma = 0) two steps of dt1 and dt2 move every
  particle exactly as one step of dt1 + dt2 (free streaming with specular
  walls composes), up to rounding.
* The policy's dt is the smaller of its closed forms: p_max / (n sigma),
  cfl times the smallest cell edge, and the 2K <= 1 bound.
* At the policy's dt the oracle's thermal box scatters the fraction of its
  particles per step that kinetic theory gives: n sigma <v_rel> dt with
  <v_rel> = 1 for an isotropic massless gas, times (N_cell - 1) / N_cell
  for the pairs a particle has in its own cell.
"""
import math

import numpy as np
import pytest

from paper_1208_0961_amd import timestep as TS
from paper_1208_0961_amd import workload as W


def test_free_streaming_composes_over_a_dt_schedule(orc):
    n = 20000
    st0 = W.thermal_box((10.0, 1.0, 1.0), n, 0.4, seed=8)
    a = orc.State(*st0)
    b = orc.State(*st0)
    box, cells = (10.0, 1.0, 1.0), (100, 10, 10)
    for t, dt in enumerate((0.03, 0.05)):
        orc.step(orc.make_params(box, cells, 0.0, 1.0, dt, 3), a, t)
    orc.step(orc.make_params(box, cells, 0.0, 1.0, 0.08, 3), b, 0)
    for d in range(3):
        assert np.allclose(a[d], b[d], rtol=0, atol=1e-13 * box[d])
        assert np.array_equal(a[d + 3], b[d + 3])
    # some particles met a wall on the way
    assert np.sum(a[3] != st0[3]) + np.sum(a[4] != st0[4]) > 100


def test_collision_dt_closed_forms():
    p = dict(box=(10.0, 2.0, 2.0), cells=(100, 10, 10), sigma=0.4, r_test=2500.0)
    edge, k_max = TS.dt_limits(p)
    assert edge == pytest.approx(0.1, rel=1e-15)
    assert k_max == pytest.approx(2500.0 * 0.004 / 0.8, rel=1e-14)
    n = 13.5
    assert TS.collision_dt(n, p, 0.05) == pytest.approx(0.05 / (n * 0.4), rel=1e-15)
    assert TS.collision_dt(n, p, 10.0, cfl=0.3) == pytest.approx(0.03, rel=1e-15)
    # a cross section so large that P22 <= 1 binds
    q = dict(p, sigma=4000.0)
    assert TS.collision_dt(1e-9, q, 1e9) == pytest.approx(2500 * 0.004 / 8000, rel=1e-8)
    assert TS.collision_dt(1e-9, q, 1e9) * 4000.0 / 2500.0 / 0.004 * 2 <= 1.0
    # a bound on the largest pair probability 2K
    assert TS.collision_dt(n, p, 10.0, cfl=0.9, p22_max=0.001) == pytest.approx(
        0.001 * 2500 * 0.004 / 0.8, rel=1e-8)
    # no cross section: only the cell edge limits dt
    assert TS.collision_dt(n, dict(p, sigma=0.0), 0.05) == pytest.approx(0.05, rel=1e-15)
    for bad in (dict(p_max=0.0), dict(cfl=1.0), dict(p22_max=1.5)):
        with pytest.raises(ValueError):
            TS.collision_dt(n, p, **bad)


def test_policy_dt_gives_the_kinetic_scattering_fraction(orc):
    T, sigma, p_max = 0.4, 0.4, 0.05
    box, cells, r_test = (2.0, 2.0, 2.0), (10, 10, 10), 300.0
    n_phys = W.gluon_density(T)
    params = dict(box=box, cells=cells, sigma=sigma, r_test=r_test)
    dt = TS.collision_dt(n_phys, params, p_max)
    assert dt == pytest.approx(p_max / (n_phys * sigma), rel=1e-15)
    N = int(round(r_test * n_phys * 8.0))
    st = orc.State(*W.thermal_box(box, N, T, seed=33))
    p = orc.make_params(box, cells, sigma, r_test, dt, 17)
    steps, claims = 5, 0
    for t in range(steps):
        claims += len(orc.step(p, st, t, trace=True)["claim"])
    frac = 2.0 * claims / (N * steps)
    n_cell = N / 1000.0
    want = p_max * (n_cell - 1.0) / n_cell
    # binomial noise of ~1.6 % on ~4000 claims, and a particle scatters at
    # most once per step (a ~p_max / 2 relative loss)
    sd = math.sqrt(claims) / claims
    assert abs(frac / want - 1.0) < 4 * sd + p_max / 2, (frac, want)


class _FakeSim:
    """The parts of Sim that timestep.run_to uses, with a density that
    halves every 0.1 fm/c (an expanding gas)."""

    def __init__(self, params, n0):
        self.params, self.n0 = params, n0
        self.time, self._dt, self.calls = 0.0, params["dt"], []

    def observe_moments(self):
        return {"n": np.array([self.n0 * 0.5 ** (self.time / 0.1), 1.0])}

    @property
    def dt(self):
        return self._dt

    @dt.setter
    def dt(self, dt):
        self._dt = dt

    def step(self, k):
        self.calls.append((k, self._dt))
        self.time += k * self._dt


def test_run_to_schedule_follows_the_density():
    params = dict(box=(10.0, 1.0, 1.0), cells=(100, 5, 5), sigma=0.4, r_test=100.0, dt=0.02)
    sim = _FakeSim(params, n0=50.0)
    sched = TS.run_to(sim, 0.5, p_max=0.05, every=4)
    assert sched == sim.calls
    assert abs(sim.time - 0.5) < 1e-12
    edge, k_max = TS.dt_limits(params)
    assert all(0 < dt <= 0.5 * edge for _, dt in sched)
    # dt grows as the gas thins (until the cell-edge limit) and each dt is
    # the policy's value at the start of its run, except the shortened last
    t = 0.0
    for i, (k, dt) in enumerate(sched):
        n = 50.0 * 0.5 ** (t / 0.1)
        want = TS.collision_dt(n, params, 0.05)
        if i < len(sched) - 1:
            assert dt == pytest.approx(want, rel=1e-12)
        else:
            assert dt <= want * (1 + 1e-12)
        t += k * dt
    assert sched[-2][1] > sched[0][1]
