"""Autotuner for batched steps: lanes per cell and cells per work item by
occupancy class, and the launch shape (one workgroup per item, or a
persistent grid).

Tuning runs on a probe batch of representative events with fresh states, so
it never advances the events being simulated.  Results are kept in a small
JSON table (per device name) that later batches reuse.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import workload as W
from .batch import Batch

# classes of mean particles per cell (upper bounds)
OCC_BOUNDS = (2.0, 8.0, 32.0, 128.0, math.inf)
CPI_CANDIDATES = (1, 2, 4, 8, 16, 32, 64)
# lanes-per-cell settings worth trying per occupancy class (0: one wave per cell)
LANES_CANDIDATES = {0: (8, 16, 0), 1: (16, 32, 8, 0), 2: (32, 64, 0), 3: (64, 0), 4: (0,)}
PERSISTENT_CANDIDATES = (0, 256 * 16, 256 * 32)
DEFAULT_TABLE = os.path.join(os.path.expanduser("~"), ".cache", "cuba_mi355x", "tuning.json")


def occupancy_class(mean_occupancy: float) -> int:
    for k, ub in enumerate(OCC_BOUNDS):
        if mean_occupancy < ub:
            return k
    return len(OCC_BOUNDS) - 1


def heuristic_cpi(mean_occupancy: float) -> int:
    if mean_occupancy <= 0:
        return 64
    return max(1, min(64, int(64.0 / mean_occupancy)))


def heuristic_lanes(mean_occupancy: float) -> int:
    """Lanes per cell for a class: groups that hold the typical cell."""
    for ub, lanes in ((2.0, 8), (5.0, 16), (14.0, 32), (36.0, 64)):
        if mean_occupancy <= ub:
            return lanes
    return 0


def cpi_candidates(lanes: int) -> list:
    """Cells per item, in whole groups of 64 / lanes cells."""
    per = 64 // lanes if lanes else 1
    return sorted({-(-c // per) * per for c in CPI_CANDIDATES})


def _time_run(B: Batch, steps: int, repeats: int) -> float:
    B.step(steps)                       # warm (and graph capture if enabled)
    B.sync()
    best = math.inf
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(B.stream)
        B.step(steps)
        e1.record(B.stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(events: list, per_class: int = 3, steps: int = 3, repeats: int = 2,
         device: str = "cuda", seed: int = 9) -> dict:
    """Tunes on up to per_class probe events of each occupancy class present
    in `events` (Workloads).  Returns the tuning table."""
    by_class: dict[int, list] = {}
    for w in events:
        by_class.setdefault(occupancy_class(W.max_mean_occupancy(w)), []).append(w)
    probes = []
    for k in sorted(by_class):
        ws = sorted(by_class[k], key=lambda w: w.n)
        # the smallest, median and largest event of the class
        pick = [ws[0], ws[len(ws) // 2], ws[-1]][:per_class]
        probes += [(k, w) for w in pick]
    B = Batch(len(probes), device=device)
    for slot, (k, w) in enumerate(probes):
        state = W.riemann_state_torch(w, seed + slot, device=device)
        B.admit(slot, {**w.params(), "cell_capacity": W.capacity_for(w)}, state)
    lanes = {k: heuristic_lanes(W.max_mean_occupancy(by_class[k][0])) for k in by_class}
    cpi = {k: cpi_candidates(lanes[k])[0] if lanes[k] else
           heuristic_cpi(W.max_mean_occupancy(by_class[k][0])) for k in by_class}

    def apply_settings():
        for slot, (k, w) in enumerate(probes):
            B.set_cell_lanes(slot, lanes[k])
            B.set_cells_per_item(slot, cpi[k])

    t0 = time.perf_counter()
    for k in sorted(by_class):
        # lanes per cell (each with its smallest whole-group item), then cells per item
        best_t, best = math.inf, (lanes[k], cpi[k])
        for g in LANES_CANDIDATES[k]:
            lanes[k] = g
            cpi[k] = (cpi_candidates(g)[0] if g else
                      heuristic_cpi(W.max_mean_occupancy(by_class[k][0])))
            apply_settings()
            dt = _time_run(B, steps, repeats)
            if dt < best_t:
                best_t, best = dt, (g, cpi[k])
        lanes[k] = best[0]
        for c in cpi_candidates(lanes[k]):
            cpi[k] = c
            apply_settings()
            dt = _time_run(B, steps, repeats)
            if dt < best_t:
                best_t, best = dt, (lanes[k], c)
        lanes[k], cpi[k] = best
    apply_settings()
    best_t, best_p = math.inf, 0
    for pw in PERSISTENT_CANDIDATES:
        B.set_launch(pw, False)
        dt = _time_run(B, steps, repeats)
        if dt < best_t:
            best_t, best_p = dt, pw
    B.close()
    return {"device": torch.cuda.get_device_name(device),
            "cells_per_item": {str(k): v for k, v in cpi.items()},
            "cell_lanes": {str(k): v for k, v in lanes.items()},
            "persistent_waves": best_p,
            "tuning_seconds": time.perf_counter() - t0}


def save(table: dict, path: str = DEFAULT_TABLE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(path: str = DEFAULT_TABLE) -> dict | None:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply(B: Batch, table: dict, events_by_slot: dict, use_graphs: bool = True) -> None:
    """Sets each slot's lanes per cell and cells per item from its occupancy
    class and the batch's launch shape from the table."""
    for slot, w in events_by_slot.items():
        m = W.max_mean_occupancy(w)
        k = occupancy_class(m)
        g = table.get("cell_lanes", {}).get(str(k))
        g = int(g) if g is not None else heuristic_lanes(m)
        c = table["cells_per_item"].get(str(k))
        c = int(c) if c else heuristic_cpi(m)
        B.set_cell_lanes(slot, g)
        B.set_cells_per_item(slot, c)
    B.set_launch(int(table.get("persistent_waves", 0)), use_graphs)
