"""Batch: many independent events advanced together by libcuba.so, with
PyTorch supplying device memory (each event's workspace and the event
table) and the stream.  Every step runs inside the library; this class only
allocates, marshals and keeps the per-slot bookkeeping.
"""
from __future__ import annotations

import numpy as np
import torch

from . import cuba as C
from .sim import _dev, suggest_cell_capacity


def event_workspace_bytes(params: dict, n: int) -> int:
    """Device bytes one event needs (the admission footprint)."""
    nbytes = C.cuba_workspace_bytes(C.make_params(**params), n)
    if nbytes == 0:
        raise C.CubaError(C.CUBA_EINVAL, "cuba_workspace_bytes", C.cuba_last_error())
    return nbytes


def with_capacity(params: dict, state, device=None, stream=None) -> dict:
    """params with a cell_capacity chosen from the initial state if unset
    (counted on the device, on `stream`)."""
    q = dict(params)
    if not q.get("cell_capacity"):
        q["cell_capacity"] = suggest_cell_capacity(q, state, device=device or "cuda",
                                                   stream=stream)
    return q


class Batch:
    def __init__(self, max_slots: int, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, persistent_waves: int = 0,
                 use_graphs: bool = False):
        self.device = torch.device(device)
        # a dedicated stream (graph capture needs one that is not the null stream)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.max_slots = int(max_slots)
        nbytes = C.cuba_batch_workspace_bytes(self.max_slots)
        with torch.cuda.stream(self.stream):
            self.table = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.b = C.cuba_batch_create(self.max_slots, self.table.data_ptr(), nbytes,
                                     self.stream.cuda_stream)
        self.slots: dict[int, dict] = {}
        self.set_launch(persistent_waves, use_graphs)

    # -- admission ------------------------------------------------------------
    def free_slot(self) -> int | None:
        for s in range(self.max_slots):
            if s not in self.slots:
                return s
        return None

    def admit(self, slot: int, params: dict, state, workspace: torch.Tensor | None = None):
        """Admits an event (params as for Sim; state: six id-ordered arrays)."""
        params = with_capacity(params, state, self.device, self.stream)
        n = int(len(state[0]))
        p = C.make_params(**params)
        nbytes = C.cuba_workspace_bytes(p, n)
        if nbytes == 0:
            raise C.CubaError(C.CUBA_EINVAL, "cuba_workspace_bytes", C.cuba_last_error())
        # the inputs may have been produced on another stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            if workspace is None:
                workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            arrs = [_dev(a, self.device) for a in state]
            nx = int(params["cells"][0])
            T00 = torch.empty(nx, dtype=torch.float64, device=self.device)
            T0x = torch.empty(nx, dtype=torch.float64, device=self.device)
        C.cuba_batch_admit(self.b, slot, p, n, *[a.data_ptr() for a in arrs],
                           workspace.data_ptr(), nbytes)
        self.slots[slot] = {"params": params, "n": n, "workspace": workspace,
                            "T00": T00, "T0x": T0x}

    def admit_async(self, slot: int, params: dict, state, lanes: int = 0,
                    workspace: torch.Tensor | None = None):
        """As admit, without waiting for the stream (cuba_batch_admit_async):
        errors of the initial state surface at the next sync; lanes: the
        event's lanes per cell."""
        params = with_capacity(params, state, self.device, self.stream)
        n = int(len(state[0]))
        p = C.make_params(**params)
        nbytes = C.cuba_workspace_bytes(p, n)
        if nbytes == 0:
            raise C.CubaError(C.CUBA_EINVAL, "cuba_workspace_bytes", C.cuba_last_error())
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            if workspace is None:
                workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            arrs = [_dev(a, self.device) for a in state]
            nx = int(params["cells"][0])
            T00 = torch.empty(nx, dtype=torch.float64, device=self.device)
            T0x = torch.empty(nx, dtype=torch.float64, device=self.device)
        C.cuba_batch_admit_async(self.b, slot, p, n, *[a.data_ptr() for a in arrs],
                                 workspace.data_ptr(), nbytes, lanes)
        self.slots[slot] = {"params": params, "n": n, "workspace": workspace,
                            "T00": T00, "T0x": T0x}

    def retire(self, slot: int) -> torch.Tensor:
        """Frees the slot without waiting for the stream (the queued steps
        still use the workspace; a tensor allocated on this batch's stream is
        reused by later allocations on it in stream order); returns the
        event's workspace."""
        C.cuba_batch_retire(self.b, slot)
        return self.slots.pop(slot)["workspace"]

    def ctx(self, slot: int):
        return C.cuba_batch_slot(self.b, slot)

    # -- stepping -------------------------------------------------------------
    def set_cells_per_item(self, slot: int, cells: int) -> None:
        C.cuba_batch_set_cells_per_item(self.b, slot, cells)

    def set_cell_lanes(self, slot: int, lanes: int) -> None:
        C.cuba_batch_set_cell_lanes(self.b, slot, lanes)

    def cell_lanes(self, slot: int) -> int:
        return C.cuba_get_cell_lanes(self.ctx(slot))

    def set_active(self, slot: int, active: bool) -> None:
        """Holds the slot's event out of the steps (False) or lets it take
        part again (cuba_batch_set_active)."""
        C.cuba_batch_set_active(self.b, slot, active)

    def set_observe(self, slot: int, every: int, rows: int = 1) -> torch.Tensor | None:
        """Observation inside runs (cuba_batch_set_observe): after every
        `every` steps of the slot's event its T00 and T0x profiles go to row
        (step / every) % rows of the returned device tensor [rows, 2, nx]
        (T00, T0x), written by the run's own launches; every = 0 turns it
        off (returns None)."""
        s = self.slots[slot]
        if every <= 0:
            C.cuba_batch_set_observe(self.b, slot, 0, None, 0)
            s.pop("obs", None)
            return None
        nx = int(s["params"]["cells"][0])
        with torch.cuda.stream(self.stream):
            out = torch.zeros((rows, 2, nx), dtype=torch.float64, device=self.device)
        C.cuba_batch_set_observe(self.b, slot, every, out.data_ptr(), rows)
        s["obs"] = out   # kept alive with the slot
        return out

    def set_dt(self, slot: int, dt: float) -> None:
        """The slot's time step from its next step on (cuba_batch_set_dt)."""
        C.cuba_batch_set_dt(self.b, slot, dt)

    def dt(self, slot: int) -> float:
        return C.cuba_get_dt(self.ctx(slot))

    def set_launch(self, persistent_waves: int = 0, use_graphs: bool = False) -> None:
        C.cuba_batch_set_launch(self.b, persistent_waves, use_graphs)

    def step(self, nsteps: int) -> None:
        C.cuba_batch_step(self.b, nsteps)

    def sync(self) -> None:
        C.cuba_batch_sync(self.b)

    # -- outputs --------------------------------------------------------------
    def observe_async(self, slot: int):
        s = self.slots[slot]
        C.cuba_batch_observe(self.b, slot, s["T00"].data_ptr(), s["T0x"].data_ptr())
        return s["T00"], s["T0x"]

    def observe(self, slot: int):
        T00, T0x = self.observe_async(slot)
        self.sync()
        return T00.cpu().numpy().copy(), T0x.cpu().numpy().copy()

    def observe_moments_async(self, slot: int) -> torch.Tensor:
        """Launches the moments of a slot's event; returns the device tensor
        [6, nx] (rows T00, T0x, Txx, n, e, v)."""
        nx = int(self.slots[slot]["params"]["cells"][0])
        with torch.cuda.stream(self.stream):
            out = torch.empty((6, nx), dtype=torch.float64, device=self.device)
        C.cuba_batch_observe_moments(self.b, slot, out.data_ptr())
        return out

    def get_state(self, slot: int):
        n = self.slots[slot]["n"]
        with torch.cuda.stream(self.stream):
            out = [torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(6)]
        C.cuba_get_state(self.ctx(slot), *[o.data_ptr() for o in out])
        self.sync()
        return [o.cpu().numpy() for o in out]

    def next_step(self, slot: int) -> int:
        return C.cuba_info(self.ctx(slot))[0]

    def counters(self, slot: int):
        return C.cuba_counters(self.ctx(slot))

    def close(self) -> None:
        if getattr(self, "b", None):
            C.cuba_batch_destroy(self.b)
            self.b = None
            self.slots.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
