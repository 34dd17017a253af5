"""ctypes binding of libcuba.so -- the functions of include/cuba.h under the
same names, argument marshalling only.  Pointers are passed as integers
(device addresses, e.g. ``tensor.data_ptr()``); a non-zero return code
raises :class:`CubaError` carrying the library's detail message.

Importing this module loads libcuba.so and raises if it has not been built
(``python -c "import __graft_entry__ as g; g.build()"``): there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcuba.so")

CUBA_OK = 0
CUBA_EINVAL = -1
CUBA_ERANGE = -2
CUBA_ENOMEM = -3
CUBA_EDEVICE = -4
CUBA_MAX_CELL_CAPACITY = 1024      # largest cell_capacity (a layout bound)
CUBA_MAX_CELL_PARTICLES = 92681    # most particles a cell may hold


class CubaError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {cuba_strerror(code)} ({detail})")
        self.code = code


class cuba_params(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double * 3),
                ("cells", ctypes.c_int32 * 3),
                ("sigma", ctypes.c_double),
                ("r_test", ctypes.c_double),
                ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64),
                ("step0", ctypes.c_uint32),
                ("cell_capacity", ctypes.c_int32)]


class cuba_trace(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_void_p),
                ("perm", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p),
                ("cand", ctypes.c_void_p),
                ("cand_cap", ctypes.c_int64),
                ("claim", ctypes.c_void_p),
                ("claim_cap", ctypes.c_int64),
                ("counts", ctypes.c_void_p)]


def _load() -> ctypes.CDLL:
    # torch's ROCm build ships its own HIP runtime, which its libraries name
    # "libamdhip64.so"; libcuba.so names the soname "libamdhip64.so.7".
    # Loaded first, torch's copy satisfies both and the process holds one
    # runtime.  Loaded the other way round, the process would hold two, and
    # the second finds no device.
    import torch  # noqa: F401
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built: the HIP library is required "
                          "(build it with paper_1208_0961_amd.build.build())")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    P = ctypes.POINTER(cuba_params)
    L.cuba_workspace_bytes.argtypes = [P, i64]
    L.cuba_workspace_bytes.restype = ctypes.c_size_t
    L.cuba_capacity_scratch_bytes.argtypes = [P]
    L.cuba_capacity_scratch_bytes.restype = ctypes.c_size_t
    L.cuba_suggest_cell_capacity.argtypes = [P, i64, vp, vp, vp, vp, ctypes.c_size_t, vp,
                                             ctypes.POINTER(i32)]
    L.cuba_suggest_cell_capacity.restype = ctypes.c_int
    L.cuba_init.argtypes = [ctypes.POINTER(vp), P, i64] + [vp] * 6 + [vp, ctypes.c_size_t, vp]
    L.cuba_init.restype = ctypes.c_int
    L.cuba_init_static.argtypes = [ctypes.POINTER(vp), P, i64] + [vp] * 6 + [vp]
    L.cuba_init_static.restype = ctypes.c_int
    L.cuba_step.argtypes = [vp, i32]
    L.cuba_step.restype = ctypes.c_int
    L.cuba_observe.argtypes = [vp, vp, vp]
    L.cuba_observe.restype = ctypes.c_int
    L.cuba_get_state.argtypes = [vp] + [vp] * 6
    L.cuba_get_state.restype = ctypes.c_int
    L.cuba_trace_step.argtypes = [vp, ctypes.POINTER(cuba_trace)]
    L.cuba_trace_step.restype = ctypes.c_int
    L.cuba_sync.argtypes = [vp]
    L.cuba_sync.restype = ctypes.c_int
    L.cuba_set_cell_lanes.argtypes = [vp, i32]
    L.cuba_set_cell_lanes.restype = ctypes.c_int
    L.cuba_get_cell_lanes.argtypes = [vp, ctypes.POINTER(i32)]
    L.cuba_get_cell_lanes.restype = ctypes.c_int
    L.cuba_set_dt.argtypes = [vp, ctypes.c_double]
    L.cuba_set_dt.restype = ctypes.c_int
    L.cuba_get_dt.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.cuba_get_dt.restype = ctypes.c_int
    L.cuba_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(i64),
                            ctypes.POINTER(i64)]
    L.cuba_info.restype = ctypes.c_int
    L.cuba_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.cuba_counters.restype = ctypes.c_int
    L.cuba_timing_begin.argtypes = [vp, i32]
    L.cuba_timing_begin.restype = ctypes.c_int
    L.cuba_timing_begin_sampled.argtypes = [vp, i32, i32]
    L.cuba_timing_begin_sampled.restype = ctypes.c_int
    L.cuba_timing_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]
    L.cuba_timing_end.restype = ctypes.c_int
    L.cuba_batch_workspace_bytes.argtypes = [i32]
    L.cuba_batch_workspace_bytes.restype = ctypes.c_size_t
    L.cuba_batch_create.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, vp]
    L.cuba_batch_create.restype = ctypes.c_int
    L.cuba_batch_admit.argtypes = [vp, i32, P, i64] + [vp] * 6 + [vp, ctypes.c_size_t]
    L.cuba_batch_admit.restype = ctypes.c_int
    L.cuba_batch_admit_async.argtypes = [vp, i32, P, i64] + [vp] * 6 + [vp, ctypes.c_size_t,
                                                                         i32]
    L.cuba_batch_admit_async.restype = ctypes.c_int
    L.cuba_batch_retire.argtypes = [vp, i32]
    L.cuba_batch_retire.restype = ctypes.c_int
    L.cuba_batch_slot.argtypes = [vp, i32]
    L.cuba_batch_slot.restype = vp
    L.cuba_batch_set_cells_per_item.argtypes = [vp, i32, i32]
    L.cuba_batch_set_cells_per_item.restype = ctypes.c_int
    L.cuba_observe_moments.argtypes = [vp, vp]
    L.cuba_observe_moments.restype = ctypes.c_int
    L.cuba_batch_observe_moments.argtypes = [vp, i32, vp]
    L.cuba_batch_observe_moments.restype = ctypes.c_int
    L.cuba_batch_observe.argtypes = [vp, i32, vp, vp]
    L.cuba_batch_observe.restype = ctypes.c_int
    L.cuba_batch_set_observe.argtypes = [vp, i32, i32, vp, i32]
    L.cuba_batch_set_observe.restype = ctypes.c_int
    L.cuba_batch_set_cell_lanes.argtypes = [vp, i32, i32]
    L.cuba_batch_set_cell_lanes.restype = ctypes.c_int
    L.cuba_batch_set_active.argtypes = [vp, i32, i32]
    L.cuba_batch_set_active.restype = ctypes.c_int
    L.cuba_batch_set_dt.argtypes = [vp, i32, ctypes.c_double]
    L.cuba_batch_set_dt.restype = ctypes.c_int
    L.cuba_batch_set_launch.argtypes = [vp, i32, i32]
    L.cuba_batch_set_launch.restype = ctypes.c_int
    L.cuba_batch_step.argtypes = [vp, i32]
    L.cuba_batch_step.restype = ctypes.c_int
    L.cuba_batch_sync.argtypes = [vp, ctypes.POINTER(i32)]
    L.cuba_batch_sync.restype = ctypes.c_int
    L.cuba_batch_timing_begin.argtypes = [vp, i32]
    L.cuba_batch_timing_begin.restype = ctypes.c_int
    L.cuba_batch_timing_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]
    L.cuba_batch_timing_end.restype = ctypes.c_int
    L.cuba_batch_destroy.argtypes = [vp]
    L.cuba_batch_destroy.restype = None
    L.cuba_destroy.argtypes = [vp]
    L.cuba_destroy.restype = None
    L.cuba_build_info.argtypes = []
    L.cuba_build_info.restype = ctypes.c_char_p
    L.cuba_strerror.argtypes = [ctypes.c_int]
    L.cuba_strerror.restype = ctypes.c_char_p
    L.cuba_last_error.argtypes = []
    L.cuba_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()


def library_path() -> str:
    return _LIB_PATH


def _check(rc: int, where: str) -> None:
    if rc != CUBA_OK:
        raise CubaError(rc, where, cuba_last_error())


def make_params(box, cells, sigma, r_test, dt, seed, step0=0,
                cell_capacity=0) -> cuba_params:
    p = cuba_params()
    for d in range(3):
        p.box[d] = float(box[d])
        p.cells[d] = int(cells[d])
    p.sigma, p.r_test, p.dt = float(sigma), float(r_test), float(dt)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    p.step0 = int(step0) & 0xFFFFFFFF
    p.cell_capacity = int(cell_capacity)
    return p


def cuba_strerror(code: int) -> str:
    return _lib.cuba_strerror(int(code)).decode()


def cuba_last_error() -> str:
    return _lib.cuba_last_error().decode()


def cuba_build_info() -> str:
    return _lib.cuba_build_info().decode()


def build_hash() -> str:
    """The source hash compiled into the loaded library."""
    info = cuba_build_info()
    return info.split()[1].rstrip(";") if info.startswith("sources ") else "unknown"


def cuba_workspace_bytes(params: cuba_params, n: int) -> int:
    return int(_lib.cuba_workspace_bytes(ctypes.byref(params), int(n)))


def cuba_capacity_scratch_bytes(params: cuba_params) -> int:
    return int(_lib.cuba_capacity_scratch_bytes(ctypes.byref(params)))


def cuba_suggest_cell_capacity(params: cuba_params, n: int, x: int, y: int, z: int,
                               scratch: int, scratch_bytes: int, stream: int | None) -> int:
    cap = ctypes.c_int32()
    _check(_lib.cuba_suggest_cell_capacity(ctypes.byref(params), int(n), x, y, z, scratch,
                                           int(scratch_bytes), stream, ctypes.byref(cap)),
           "cuba_suggest_cell_capacity")
    return int(cap.value)


def cuba_init(params: cuba_params, n: int, x: int, y: int, z: int, px: int, py: int,
              pz: int, workspace: int, ws_bytes: int, stream: int | None) -> int:
    ctx = ctypes.c_void_p()
    rc = _lib.cuba_init(ctypes.byref(ctx), ctypes.byref(params), int(n), x, y, z, px, py,
                        pz, workspace, int(ws_bytes), stream)
    _check(rc, "cuba_init")
    return ctx.value


CUBA_STATIC_WORKSPACE_BYTES = 64 << 20


def cuba_init_static(params: cuba_params, n: int, x: int, y: int, z: int, px: int, py: int,
                     pz: int, stream: int | None) -> int:
    ctx = ctypes.c_void_p()
    rc = _lib.cuba_init_static(ctypes.byref(ctx), ctypes.byref(params), int(n), x, y, z,
                               px, py, pz, stream)
    _check(rc, "cuba_init_static")
    return ctx.value


def cuba_step(ctx: int, nsteps: int) -> None:
    _check(_lib.cuba_step(ctx, int(nsteps)), "cuba_step")


def cuba_observe(ctx: int, T00: int, T0x: int) -> None:
    _check(_lib.cuba_observe(ctx, T00, T0x), "cuba_observe")


def cuba_get_state(ctx: int, x: int, y: int, z: int, px: int, py: int, pz: int) -> None:
    _check(_lib.cuba_get_state(ctx, x, y, z, px, py, pz), "cuba_get_state")


def cuba_trace_step(ctx: int, trace: cuba_trace) -> None:
    _check(_lib.cuba_trace_step(ctx, ctypes.byref(trace)), "cuba_trace_step")


def cuba_sync(ctx: int) -> None:
    _check(_lib.cuba_sync(ctx), "cuba_sync")


CELL_LANES = (0, 8, 16, 32, 64)      # every context, batched or not
TWO_WAVES_PER_CELL = 128             # plain contexts only
PACKED_CELLS = 1                     # plain contexts only: whole cells packed into waves


def cuba_set_cell_lanes(ctx: int, lanes: int) -> None:
    _check(_lib.cuba_set_cell_lanes(ctx, int(lanes)), "cuba_set_cell_lanes")


def cuba_get_cell_lanes(ctx: int) -> int:
    v = ctypes.c_int32()
    _check(_lib.cuba_get_cell_lanes(ctx, ctypes.byref(v)), "cuba_get_cell_lanes")
    return int(v.value)


def cuba_set_dt(ctx: int, dt: float) -> None:
    _check(_lib.cuba_set_dt(ctx, float(dt)), "cuba_set_dt")


def cuba_get_dt(ctx: int) -> float:
    v = ctypes.c_double()
    _check(_lib.cuba_get_dt(ctx, ctypes.byref(v)), "cuba_get_dt")
    return float(v.value)


def cuba_info(ctx: int):
    t = ctypes.c_uint32()
    n = ctypes.c_int64()
    c = ctypes.c_int64()
    _check(_lib.cuba_info(ctx, ctypes.byref(t), ctypes.byref(n), ctypes.byref(c)),
           "cuba_info")
    return t.value, n.value, c.value


CUBA_NUM_STAGES = 5
STAGES = ("bin", "step", "collide", "observe", "offsets")


def cuba_counters(ctx: int):
    out = (ctypes.c_uint64 * 3)()
    _check(_lib.cuba_counters(ctx, out), "cuba_counters")
    return {"pair_tests": int(out[0]), "candidates": int(out[1]), "claims": int(out[2])}


def cuba_timing_begin(ctx: int, max_launches: int) -> None:
    _check(_lib.cuba_timing_begin(ctx, int(max_launches)), "cuba_timing_begin")


def cuba_timing_begin_sampled(ctx: int, max_launches: int, step_every: int) -> None:
    _check(_lib.cuba_timing_begin_sampled(ctx, int(max_launches), int(step_every)),
           "cuba_timing_begin_sampled")


def cuba_timing_end(ctx: int):
    ms = (ctypes.c_double * CUBA_NUM_STAGES)()
    nl = (ctypes.c_int64 * CUBA_NUM_STAGES)()
    _check(_lib.cuba_timing_end(ctx, ms, nl), "cuba_timing_end")
    return {STAGES[k]: (float(ms[k]), int(nl[k])) for k in range(CUBA_NUM_STAGES)}


def cuba_destroy(ctx: int) -> None:
    _lib.cuba_destroy(ctx)


# -- batches ------------------------------------------------------------------
def cuba_batch_workspace_bytes(max_slots: int) -> int:
    return int(_lib.cuba_batch_workspace_bytes(int(max_slots)))


def cuba_batch_create(max_slots: int, workspace: int, ws_bytes: int,
                      stream: int | None) -> int:
    b = ctypes.c_void_p()
    _check(_lib.cuba_batch_create(ctypes.byref(b), int(max_slots), workspace,
                                  int(ws_bytes), stream), "cuba_batch_create")
    return b.value


def cuba_batch_admit(b: int, slot: int, params: cuba_params, n: int, x: int, y: int,
                     z: int, px: int, py: int, pz: int, workspace: int,
                     ws_bytes: int) -> None:
    _check(_lib.cuba_batch_admit(b, int(slot), ctypes.byref(params), int(n), x, y, z, px,
                                 py, pz, workspace, int(ws_bytes)), "cuba_batch_admit")


def cuba_batch_admit_async(b: int, slot: int, params: cuba_params, n: int, x: int, y: int,
                           z: int, px: int, py: int, pz: int, workspace: int,
                           ws_bytes: int, lanes: int) -> None:
    _check(_lib.cuba_batch_admit_async(b, int(slot), ctypes.byref(params), int(n), x, y, z,
                                       px, py, pz, workspace, int(ws_bytes), int(lanes)),
           "cuba_batch_admit_async")


def cuba_batch_retire(b: int, slot: int) -> None:
    _check(_lib.cuba_batch_retire(b, int(slot)), "cuba_batch_retire")


def cuba_batch_slot(b: int, slot: int):
    return _lib.cuba_batch_slot(b, int(slot))


def cuba_batch_set_cells_per_item(b: int, slot: int, cells: int) -> None:
    _check(_lib.cuba_batch_set_cells_per_item(b, int(slot), int(cells)),
           "cuba_batch_set_cells_per_item")


MOMENTS = ("T00", "T0x", "Txx", "n", "e", "v")


def cuba_observe_moments(ctx: int, out: int) -> None:
    _check(_lib.cuba_observe_moments(ctx, out), "cuba_observe_moments")


def cuba_batch_observe_moments(b: int, slot: int, out: int) -> None:
    _check(_lib.cuba_batch_observe_moments(b, int(slot), out), "cuba_batch_observe_moments")


def cuba_batch_observe(b: int, slot: int, T00: int, T0x: int) -> None:
    _check(_lib.cuba_batch_observe(b, int(slot), T00, T0x), "cuba_batch_observe")


def cuba_batch_set_observe(b: int, slot: int, every: int, out: int | None, rows: int) -> None:
    _check(_lib.cuba_batch_set_observe(b, int(slot), int(every), out, int(rows)),
           "cuba_batch_set_observe")


def cuba_batch_set_cell_lanes(b: int, slot: int, lanes: int) -> None:
    _check(_lib.cuba_batch_set_cell_lanes(b, int(slot), int(lanes)),
           "cuba_batch_set_cell_lanes")


def cuba_batch_set_active(b: int, slot: int, active: bool) -> None:
    _check(_lib.cuba_batch_set_active(b, int(slot), 1 if active else 0),
           "cuba_batch_set_active")


def cuba_batch_set_dt(b: int, slot: int, dt: float) -> None:
    _check(_lib.cuba_batch_set_dt(b, int(slot), float(dt)), "cuba_batch_set_dt")


def cuba_batch_set_launch(b: int, persistent_waves: int, use_graphs: bool) -> None:
    _check(_lib.cuba_batch_set_launch(b, int(persistent_waves), 1 if use_graphs else 0),
           "cuba_batch_set_launch")


def cuba_batch_step(b: int, nsteps: int) -> None:
    _check(_lib.cuba_batch_step(b, int(nsteps)), "cuba_batch_step")


def cuba_batch_sync(b: int) -> None:
    bad = ctypes.c_int32(-1)
    rc = _lib.cuba_batch_sync(b, ctypes.byref(bad))
    if rc != CUBA_OK:
        err = CubaError(rc, "cuba_batch_sync", cuba_last_error())
        err.slot = bad.value
        raise err


def cuba_batch_timing_begin(b: int, max_launches: int) -> None:
    _check(_lib.cuba_batch_timing_begin(b, int(max_launches)), "cuba_batch_timing_begin")


def cuba_batch_timing_end(b: int):
    ms = (ctypes.c_double * CUBA_NUM_STAGES)()
    nl = (ctypes.c_int64 * CUBA_NUM_STAGES)()
    _check(_lib.cuba_batch_timing_end(b, ms, nl), "cuba_batch_timing_end")
    return {STAGES[k]: (float(ms[k]), int(nl[k])) for k in range(CUBA_NUM_STAGES)}


def cuba_batch_destroy(b: int) -> None:
    _lib.cuba_batch_destroy(b)
