"""Autotuner for batched steps: lanes per cell and cells per binning item
by occupancy class, and the binning launch shape (one wave per item, or a
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
# lanes-per-cell settings tried per class; AUTO keeps each event's own
# library default (chosen at admission from its occupancy histogram)
AUTO = -1
LANES_CANDIDATES = (AUTO, 0, 8, 16, 32, 64)
PERSISTENT_CANDIDATES = (0, 256 * 16, 256 * 32)
DEFAULT_TABLE = os.path.join(os.path.expanduser("~"), ".cache", "cuba_mi355x", "tuning.json")
# the table measured on an MI355X and shipped with the package: used when no
# table of the user's own has been saved
PACKAGED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")


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


def _probe_batch(ws: list, device: str, seed: int) -> Batch:
    B = Batch(len(ws), device=device)
    for slot, w in enumerate(ws):
        state = W.riemann_state_torch(w, seed + slot, device=device)
        B.admit(slot, {**w.params(), "cell_capacity": W.capacity_for(w)}, state)
    return B


def tune(events: list, per_class: int = 3, steps: int = 8, repeats: int = 3,
         device: str = "cuda", seed: int = 9) -> dict:
    """Tunes each occupancy class present in `events` (Workloads) on a probe
    batch of up to per_class of its events (the smallest, median and
    largest), so that a setting's effect is timed on the work it changes:
    first lanes per cell, then cells per binning item; then the binning
    launch shape on all probe events together.  Returns the tuning table."""
    by_class: dict[int, list] = {}
    for w in events:
        by_class.setdefault(occupancy_class(W.max_mean_occupancy(w)), []).append(w)
    picks = {}
    for k in sorted(by_class):
        ws = sorted(by_class[k], key=lambda w: w.n)
        picks[k] = [ws[0], ws[len(ws) // 2], ws[-1]][:per_class]
    t0 = time.perf_counter()
    lanes, cpi = {}, {}
    for k in sorted(picks):
        B = _probe_batch(picks[k], device, seed)
        own = {slot: B.cell_lanes(slot) for slot in range(len(picks[k]))}

        def apply_settings(g, c):
            for slot, w in enumerate(picks[k]):
                gl = own[slot] if g == AUTO else g
                B.set_cell_lanes(slot, gl)
                if c is None:   # default binning item for the lanes setting
                    c_slot = 64 if gl > 0 else heuristic_cpi(W.max_mean_occupancy(w))
                else:
                    c_slot = c
                B.set_cells_per_item(slot, c_slot)

        best_t, best = math.inf, (AUTO, None)
        for g in LANES_CANDIDATES:
            apply_settings(g, None)
            dt = _time_run(B, steps, repeats)
            if dt < best_t:
                best_t, best = dt, (g, None)
        for c in CPI_CANDIDATES:
            apply_settings(best[0], c)
            dt = _time_run(B, steps, repeats)
            if dt < best_t:
                best_t, best = dt, (best[0], c)
        lanes[k], cpi[k] = best
        B.close()
    # the binning launch shape, all classes together
    probes = [w for k in sorted(picks) for w in picks[k]]
    B = _probe_batch(probes, device, seed)
    apply(B, {"cells_per_item": {str(k): v for k, v in cpi.items()},
              "cell_lanes": {str(k): v for k, v in lanes.items()}},
          dict(enumerate(probes)), use_graphs=False)
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


def load(path: str | None = None) -> dict | None:
    """The tuning table at path; by default the user's saved table, else the
    packaged MI355X table, else None."""
    for p in ([path] if path else [DEFAULT_TABLE, PACKAGED_TABLE]):
        if os.path.exists(p):
            with open(p) as f:
                return json.load(f)
    return None


def apply(B: Batch, table: dict, events_by_slot: dict, use_graphs: bool = True) -> None:
    """Sets each slot's lanes per cell and cells per binning item from its
    occupancy class (AUTO or no entry: the event's own library default) and
    the batch's launch shape from the table."""
    for slot, w in events_by_slot.items():
        settings_for(B, slot, w, table)
    B.set_launch(int(table.get("persistent_waves", 0)), use_graphs)


def settings_for(B: Batch, slot: int, w, table: dict) -> None:
    """Applies the table's class settings to one admitted event."""
    m = W.max_mean_occupancy(w)
    k = str(occupancy_class(m))
    g = table.get("cell_lanes", {}).get(k)
    if g is not None and int(g) != AUTO:
        B.set_cell_lanes(slot, int(g))
    c = table.get("cells_per_item", {}).get(k)
    if c is None:
        c = 64 if B.cell_lanes(slot) > 0 else heuristic_cpi(m)
    B.set_cells_per_item(slot, int(c))
