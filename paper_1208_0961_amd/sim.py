"""Sim: one simulation context on a GPU, with PyTorch supplying the device
memory (particle arrays, workspace, outputs) and the stream.  Every step of
the method runs inside libcuba.so; this class only allocates and marshals.
"""
from __future__ import annotations

import numpy as np
import torch

from . import cuba as C


def _dev(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


def suggest_cell_capacity(params: dict, state, headroom: float = 2.0, margin: int = 32,
                          device: str | torch.device = "cuda",
                          stream: torch.cuda.Stream | None = None) -> int:
    """Slots per cell for the workspace, counted on the device by
    cuba_suggest_cell_capacity: twice the largest initial cell occupancy
    plus 32, rounded up to 32, within [64, 1024].  A layout choice only: a
    cell that later holds more keeps the surplus in spill slots and is
    stepped on the library's slower overflow path.  (headroom and margin
    are those of the library and kept for callers that name them.)"""
    if (headroom, margin) != (2.0, 32):
        raise ValueError("the library's rule is 2 x the largest occupancy + 32")
    device = torch.device(device)
    p = C.make_params(**{**params, "cell_capacity": 0})
    n = int(len(state[0]))
    stream = stream if stream is not None else torch.cuda.current_stream(device)
    with torch.cuda.stream(stream):
        pos = [_dev(state[d], device) for d in range(3)]
        nbytes = C.cuba_capacity_scratch_bytes(p)
        if nbytes == 0:
            raise C.CubaError(C.CUBA_EINVAL, "cuba_capacity_scratch_bytes", C.cuba_last_error())
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return C.cuba_suggest_cell_capacity(p, n, *[a.data_ptr() for a in pos],
                                        scratch.data_ptr(), nbytes, stream.cuda_stream)


class Sim:
    """A box of test particles advanced by libcuba.so.

    params: dict with box, cells, sigma, r_test, dt, seed and optionally
    step0 and cell_capacity (default: suggest_cell_capacity of the initial
    state).  state: six arrays (x, y, z, px, py, pz) indexed by particle id.
    cell_lanes: lanes per cell of the cell kernels (None: the library's
    choice from the initial occupancy; see cuba_set_cell_lanes).
    `dt` may be changed between steps (cuba_set_dt); `time` is the time
    advanced since construction, sum of dt over the steps taken, and
    `dt_log` lists (step index, dt) for the initial dt and every change.
    """

    def __init__(self, params: dict, state, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, cell_lanes: int | None = None):
        self.device = torch.device(device)
        self.params = dict(params)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(self.stream):
            arrs = [_dev(a, self.device) for a in state]
        if not self.params.get("cell_capacity"):
            self.params["cell_capacity"] = suggest_cell_capacity(self.params, arrs,
                                                                 device=self.device,
                                                                 stream=self.stream)
        self.p = C.make_params(**self.params)
        self.n = int(len(state[0]))
        self.nx = int(self.params["cells"][0])
        self.n_cells = int(np.prod(self.params["cells"]))
        with torch.cuda.stream(self.stream):
            self.ws_bytes = C.cuba_workspace_bytes(self.p, self.n)
            if self.ws_bytes == 0:
                raise C.CubaError(C.CUBA_EINVAL, "cuba_workspace_bytes",
                                  C.cuba_last_error())
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            self.T00 = torch.empty(self.nx, dtype=torch.float64, device=self.device)
            self.T0x = torch.empty(self.nx, dtype=torch.float64, device=self.device)
            self.ctx = C.cuba_init(self.p, self.n, *[a.data_ptr() for a in arrs],
                                   self.workspace.data_ptr(), self.ws_bytes,
                                   self.stream.cuda_stream)
            # the inputs are copied on the stream; keep them until it passes
            self._inputs = arrs
        if cell_lanes is not None:
            C.cuba_set_cell_lanes(self.ctx, cell_lanes)
        self._dt = C.cuba_get_dt(self.ctx)
        self.time = 0.0
        self.dt_log = [(C.cuba_info(self.ctx)[0], self._dt)]

    @property
    def cell_lanes(self) -> int:
        return C.cuba_get_cell_lanes(self.ctx)

    @property
    def dt(self) -> float:
        return self._dt

    @dt.setter
    def dt(self, dt: float) -> None:
        C.cuba_set_dt(self.ctx, dt)
        self._dt = C.cuba_get_dt(self.ctx)
        t = C.cuba_info(self.ctx)[0]
        if self.dt_log[-1][0] == t:
            self.dt_log[-1] = (t, self._dt)
        else:
            self.dt_log.append((t, self._dt))

    @cell_lanes.setter
    def cell_lanes(self, lanes: int) -> None:
        C.cuba_set_cell_lanes(self.ctx, lanes)

    # -- stepping -------------------------------------------------------------
    def step(self, nsteps: int = 1) -> None:
        C.cuba_step(self.ctx, nsteps)
        self.time += nsteps * self._dt

    def sync(self) -> None:
        C.cuba_sync(self.ctx)
        self._inputs = None

    @property
    def next_step(self) -> int:
        return C.cuba_info(self.ctx)[0]

    # -- outputs --------------------------------------------------------------
    def observe_async(self):
        """Launches the profile reduction; returns the device tensors."""
        C.cuba_observe(self.ctx, self.T00.data_ptr(), self.T0x.data_ptr())
        return self.T00, self.T0x

    def observe(self):
        T00, T0x = self.observe_async()
        self.sync()
        return T00.cpu().numpy().copy(), T0x.cpu().numpy().copy()

    def observe_moments(self):
        """Per-slab T00, T0x, Txx, n, e, v (see cuba_observe_moments), as a
        dict of numpy arrays."""
        with torch.cuda.stream(self.stream):
            out = torch.empty(6 * self.nx, dtype=torch.float64, device=self.device)
        C.cuba_observe_moments(self.ctx, out.data_ptr())
        self.sync()
        a = out.cpu().numpy().reshape(6, self.nx)
        return {k: a[i].copy() for i, k in enumerate(C.MOMENTS)}

    def get_state(self):
        with torch.cuda.stream(self.stream):
            out = [torch.empty(self.n, dtype=torch.float64, device=self.device)
                   for _ in range(6)]
        C.cuba_get_state(self.ctx, *[o.data_ptr() for o in out])
        self.sync()
        return [o.cpu().numpy() for o in out]

    def trace_step(self, cand_cap: int | None = None, claim_cap: int | None = None):
        """One step with its decision record (see cuba_trace_step)."""
        cand_cap = cand_cap if cand_cap is not None else max(1024, self.n)
        claim_cap = claim_cap if claim_cap is not None else max(1, self.n // 2)
        with torch.cuda.stream(self.stream):
            u32 = dict(dtype=torch.int32, device=self.device)
            cell = torch.empty(max(1, self.n), **u32)
            perm = torch.empty(max(1, self.n), **u32)
            offs = torch.empty(self.n_cells + 1, **u32)
            cand = torch.empty((cand_cap, 3), **u32)
            claim = torch.empty((claim_cap, 3), **u32)
            counts = torch.zeros(2, **u32)
        tr = C.cuba_trace(cell.data_ptr(), perm.data_ptr(), offs.data_ptr(),
                          cand.data_ptr(), cand_cap, claim.data_ptr(), claim_cap,
                          counts.data_ptr())
        C.cuba_trace_step(self.ctx, tr)
        self.sync()
        nc, ncl = [int(v) for v in counts.cpu().numpy().view(np.uint32)]
        as_u32 = lambda t: t.cpu().numpy().view(np.uint32)
        return {"cell": as_u32(cell)[:self.n], "perm": as_u32(perm)[:self.n],
                "offsets": as_u32(offs), "cand": as_u32(cand)[:nc].copy(),
                "claim": as_u32(claim)[:ncl].copy()}

    def close(self) -> None:
        if getattr(self, "ctx", None):
            C.cuba_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
