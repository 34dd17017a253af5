"""Cross-section scan of the Riemann tube: the approach to ideal
hydrodynamics as sigma grows (the paper's Sec. 5 and Fig. 3).

For each sigma an ensemble of independent events (own seed, own initial
state) is advanced in one batch to the same time, then every event's slab
moments are observed: T00, T0x, Txx, density n and the rest-frame e and v
(cuba_observe_moments).  The ensemble means are what Fig. 3 plots against
the ideal-fluid solution.  Every step runs in libcuba.so; this module only
sets up events and averages the observed profiles.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import cuba as C
from . import workload as W
from .batch import Batch

# The tube of the scan: 10 x 1 x 1 fm, 100 x 4 x 4 cells, r_test = 400
# (about 34 / 17 test particles per cell), T = 0.40 / 0.32 GeV.
BOX = (10.0, 1.0, 1.0)
CELLS = (100, 4, 4)
R_TEST = 400.0
T_LEFT, T_RIGHT = 0.40, 0.32
# sigma [fm^2] and dt [fm/c]; dt shrinks with sigma so that the collision
# probability per particle and step n sigma dt stays small
SCAN = ((0.4, 0.005), (1.6, 0.005), (4.0, 0.002))


def event(sigma: float, dt: float, seed: int) -> W.Workload:
    return W.Workload(f"sigma{sigma:g}-seed{seed}", BOX, CELLS, R_TEST, sigma, dt, T_LEFT,
                      T_RIGHT, seed=seed)


def run(sigma: float, dt: float, seeds, t_end: float = 4.0, run_steps: int = 50,
        device: str = "cuda") -> dict:
    """Advances len(seeds) events of cross section sigma to t_end in one
    batch; returns the per-event moments [events, 6, nx] (rows as
    cuba_observe_moments), their ensemble means, the step count and the
    wall time of the stepping."""
    nsteps = int(round(t_end / dt))
    evs = [event(sigma, dt, s) for s in seeds]
    B = Batch(len(evs), device=device, use_graphs=True)
    for slot, w in enumerate(evs):
        state = W.riemann_state_torch(w, seed=7000 + int(w.seed), device=device)
        B.admit(slot, {**w.params(), "cell_capacity": W.capacity_for(w)}, state)
    B.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        k = min(run_steps, nsteps - done)
        B.step(k)
        done += k
    outs = [B.observe_moments_async(slot) for slot in range(len(evs))]
    B.sync()
    elapsed = time.perf_counter() - t0
    per_event = np.stack([o.cpu().numpy() for o in outs])
    B.close()
    return {"sigma": sigma, "dt": dt, "steps": nsteps, "events": len(evs),
            "particles": sum(w.n for w in evs), "seconds": elapsed,
            "per_event": per_event,
            "mean": {k: per_event[:, i].mean(0) for i, k in enumerate(C.MOMENTS)}}
