"""Variable time step: the paper's Sec. 6 names a variable dt as the next
step of the method.  The library takes a new dt between steps
(cuba_set_dt); this module chooses it.

Limits on dt, all from the method:
* dt below every cell edge, so a particle crosses at most one cell per step
  (Sec. 5);
* 2K <= 1, K = sigma / r_test * dt / V_cell, so that P22 = K v_rel <= 1
  (Eq. (3), v_rel <= 2 for massless particles);
* accuracy: a test particle in a gas of physical density n collides at the
  rate n sigma <v_rel> per unit time, <v_rel> = 1 for an isotropic massless
  gas, and scatters at most once per step.  The expected number of
  collisions per particle and step, n sigma dt, must stay small for that
  limit not to cut the rate; `collision_dt` keeps it at p_max in the densest
  x-slab.

The density is the slab density of cuba_observe_moments, i.e. averaged over
y and z: a box that is inhomogeneous transversely needs a smaller p_max.
"""
from __future__ import annotations

import math

import numpy as np


def dt_limits(params: dict) -> tuple[float, float]:
    """(largest dt below every cell edge, largest dt with 2K <= 1)."""
    dx = [float(params["box"][d]) / int(params["cells"][d]) for d in range(3)]
    vcell = dx[0] * dx[1] * dx[2]
    sigma = float(params["sigma"])
    k_max = math.inf if sigma == 0.0 else float(params["r_test"]) * vcell / (2.0 * sigma)
    return min(dx), k_max


def collision_dt(n_max: float, params: dict, p_max: float = 0.05,
                 cfl: float = 0.5, p22_max: float = 1.0) -> float:
    """The largest dt with n_max sigma dt <= p_max, at most cfl times the
    smallest cell edge, and with the largest pair probability 2K at most
    p22_max (1: the bound P22 <= 1; less by a margin of 1e-9 relative, for
    the rounding of K)."""
    if not (0.0 < p_max and 0.0 < cfl < 1.0 and 0.0 < p22_max <= 1.0):
        raise ValueError("p_max must be > 0, 0 < cfl < 1 and 0 < p22_max <= 1")
    edge, k_max = dt_limits(params)
    dt = cfl * edge
    sigma = float(params["sigma"])
    if n_max > 0.0 and sigma > 0.0:
        dt = min(dt, p_max / (n_max * sigma))
    return min(dt, p22_max * k_max * (1.0 - 1e-9))


def run_to(sim, t_end: float, p_max: float = 0.05, every: int = 10, cfl: float = 0.5,
           p22_max: float = 1.0):
    """Advances `sim` (a Sim) from sim.time to t_end, choosing dt every
    `every` steps from the observed densest slab; the last run shortens dt
    so that the run ends at t_end.  Returns the schedule as a list of
    (steps, dt); sim.dt_log records the step index at which each dt took
    effect."""
    schedule = []
    while True:
        left = t_end - sim.time
        if left <= 1e-12 * max(1.0, abs(t_end)):
            return schedule
        n_max = float(np.max(sim.observe_moments()["n"]))
        dt = collision_dt(n_max, sim.params, p_max, cfl, p22_max)
        k = min(every, int(math.ceil(left / dt)))
        if k * dt > left:
            dt = left / k
        sim.dt = dt
        sim.step(k)
        schedule.append((k, dt))
