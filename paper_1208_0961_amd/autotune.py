"""Autotuner for batched steps: cells per work item by occupancy class, and
the launch shape (one workgroup per item, or a persistent grid).

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
    cpi = {k: heuristic_cpi(W.max_mean_occupancy(by_class[k][0])) for k in by_class}

    def apply_cpi():
        for slot, (k, w) in enumerate(probes):
            B.set_cells_per_item(slot, cpi[k])

    t0 = time.perf_counter()
    for k in sorted(by_class):
        best_t, best_c = math.inf, cpi[k]
        for c in CPI_CANDIDATES:
            cpi[k] = c
            apply_cpi()
            dt = _time_run(B, steps, repeats)
            if dt < best_t:
                best_t, best_c = dt, c
        cpi[k] = best_c
    apply_cpi()
    best_t, best_p = math.inf, 0
    for pw in PERSISTENT_CANDIDATES:
        B.set_launch(pw, False)
        dt = _time_run(B, steps, repeats)
        if dt < best_t:
            best_t, best_p = dt, pw
    B.close()
    return {"device": torch.cuda.get_device_name(device),
            "cells_per_item": {str(k): v for k, v in cpi.items()},
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
    """Sets each slot's cells per item from its occupancy class and the
    batch's launch shape from the table."""
    for slot, w in events_by_slot.items():
        k = occupancy_class(W.max_mean_occupancy(w))
        c = table["cells_per_item"].get(str(k))
        B.set_cells_per_item(slot, int(c) if c else heuristic_cpi(W.max_mean_occupancy(w)))
    B.set_launch(int(table.get("persistent_waves", 0)), use_graphs)
