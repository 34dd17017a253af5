"""ctypes wrapper around the C oracle (cuba_oracle.c).

TEST INFRASTRUCTURE ONLY: the plain sequential FP64 CPU implementation of
the PIC Boltzmann step of arXiv:1208.0961 (Sec. 2, Eqs. (2)-(3)) that the
HIP library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It imports nothing
from the GPU package and the GPU package imports nothing from here.

Every array argument is a contiguous numpy array indexed by particle id.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cuba_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE, ENOMEM = 0, -1, -2, -3


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (IEEE FP64, no contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC,
           "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    """Problem definition: box [fm], cells, sigma [fm^2], r_test, dt [fm/c],
    Philox seed."""
    _fields_ = [("box", ctypes.c_double * 3),
                ("cells", ctypes.c_int32 * 3),
                ("sigma", ctypes.c_double),
                ("r_test", ctypes.c_double),
                ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class Trace(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_void_p),
                ("perm", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p),
                ("cand", ctypes.c_void_p),
                ("cand_cap", ctypes.c_int64),
                ("n_cand", ctypes.c_int64),
                ("claim", ctypes.c_void_p),
                ("claim_cap", ctypes.c_int64),
                ("n_claim", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        dp, u32p, i32p = (ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_uint32),
                          ctypes.POINTER(ctypes.c_int32))
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_u53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_u53.restype = ctypes.c_double
        L.orc_constants.argtypes = [ctypes.POINTER(Params), dp, dp, dp]
        L.orc_constants.restype = None
        L.orc_check.argtypes = [ctypes.POINTER(Params), ctypes.c_int64] + [dp] * 6
        L.orc_check.restype = ctypes.c_int
        L.orc_step.argtypes = ([ctypes.POINTER(Params), ctypes.c_int64] + [dp] * 6
                               + [ctypes.c_uint32, ctypes.c_int,
                                  ctypes.POINTER(Trace)])
        L.orc_step.restype = ctypes.c_int
        L.orc_run.argtypes = ([ctypes.POINTER(Params), ctypes.c_int64] + [dp] * 6
                              + [ctypes.c_uint32, ctypes.c_int32, ctypes.c_int])
        L.orc_run.restype = ctypes.c_int
        L.orc_observe.argtypes = ([ctypes.POINTER(Params), ctypes.c_int64]
                                  + [dp] * 4 + [dp, dp])
        L.orc_observe.restype = None
        L.orc_observe_moments.argtypes = ([ctypes.POINTER(Params), ctypes.c_int64]
                                          + [dp] * 4 + [dp] * 4)
        L.orc_observe_moments.restype = None
        L.orc_landau.argtypes = [ctypes.c_int32] + [dp] * 5
        L.orc_landau.restype = None
        L.orc_collide_cell_with_uniforms.argtypes = [
            ctypes.c_int32, dp, dp, dp, ctypes.c_double, dp, dp, i32p, i32p]
        L.orc_collide_cell_with_uniforms.restype = ctypes.c_int
        L.orc_scatter_pair.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double]
        L.orc_scatter_pair.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def make_params(box, cells, sigma, r_test, dt, seed) -> Params:
    p = Params()
    for d in range(3):
        p.box[d] = float(box[d])
        p.cells[d] = int(cells[d])
    p.sigma, p.r_test, p.dt = float(sigma), float(r_test), float(dt)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return p


class State:
    """Six FP64 arrays indexed by particle id (x, y, z, px, py, pz)."""

    def __init__(self, x, y, z, px, py, pz):
        self.arrs = [np.ascontiguousarray(a, dtype=np.float64).copy()
                     for a in (x, y, z, px, py, pz)]

    @property
    def n(self):
        return self.arrs[0].shape[0]

    def ptrs(self):
        return [_dp(a) for a in self.arrs]

    def copy(self):
        return State(*self.arrs)

    def __getitem__(self, i):
        return self.arrs[i]


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: ctr = 4 words, key = 2 words -> 4 words."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_u32p(c), _u32p(k), _u32p(o))
    return o


def u53(lo, hi):
    return lib().orc_u53(int(lo), int(hi))


def constants(p: Params):
    dx = np.zeros(3)
    v = ctypes.c_double()
    k = ctypes.c_double()
    lib().orc_constants(ctypes.byref(p), _dp(dx), ctypes.byref(v), ctypes.byref(k))
    return dx, v.value, k.value


def check(p: Params, st: State) -> int:
    return lib().orc_check(ctypes.byref(p), st.n, *st.ptrs())


def step(p: Params, st: State, t: int, nthreads: int = 1, trace: bool = False,
         cand_cap: int | None = None):
    """One step with index t, in place.  With trace=True returns a dict with
    cell [n], perm [n], offsets [C+1], cand [m,3], claim [m,3]."""
    n = st.n
    if not trace:
        rc = lib().orc_step(ctypes.byref(p), n, *st.ptrs(), t, nthreads, None)
        if rc != OK:
            raise RuntimeError(f"orc_step failed: {rc}")
        return None
    C = int(p.cells[0]) * int(p.cells[1]) * int(p.cells[2])
    cap = cand_cap if cand_cap is not None else max(64, n)
    saved = [a.copy() for a in st.arrs]
    while True:
        out = _traced_step(p, st, t, n, C, cap)
        if out is not None:
            return out
        # more candidates than room: redo the step from the saved state
        for a, b in zip(st.arrs, saved):
            a[:] = b
        cap = _traced_step.last_count + 64


def _traced_step(p, st, t, n, C, cap):
    cell = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.uint32)
    offs = np.zeros(C + 1, np.uint32)
    cand = np.zeros((cap, 3), np.uint32)
    claim = np.zeros((max(1, n // 2), 3), np.uint32)
    tr = Trace(cell.ctypes.data, perm.ctypes.data, offs.ctypes.data,
               cand.ctypes.data, cap, 0, claim.ctypes.data, claim.shape[0], 0)
    rc = lib().orc_step(ctypes.byref(p), n, *st.ptrs(), t, 1, ctypes.byref(tr))
    if rc != OK:
        raise RuntimeError(f"orc_step failed: {rc}")
    if tr.n_cand > cap:
        _traced_step.last_count = tr.n_cand
        return None
    return {"cell": cell, "perm": perm, "offsets": offs,
            "cand": cand[:tr.n_cand].copy(), "claim": claim[:tr.n_claim].copy()}


def run(p: Params, st: State, t0: int, nsteps: int, nthreads: int = 1):
    rc = lib().orc_run(ctypes.byref(p), st.n, *st.ptrs(), t0, nsteps, nthreads)
    if rc != OK:
        raise RuntimeError(f"orc_run failed: {rc}")


def observe(p: Params, st: State):
    nx = int(p.cells[0])
    T00 = np.zeros(nx)
    T0x = np.zeros(nx)
    lib().orc_observe(ctypes.byref(p), st.n, _dp(st[0]), _dp(st[3]), _dp(st[4]),
                      _dp(st[5]), _dp(T00), _dp(T0x))
    return T00, T0x


def observe_moments(p: Params, st: State):
    """Per-slab T00, T0x, Txx [GeV/fm^3] and density n [fm^-3]."""
    nx = int(p.cells[0])
    out = [np.zeros(nx) for _ in range(4)]
    lib().orc_observe_moments(ctypes.byref(p), st.n, _dp(st[0]), _dp(st[3]), _dp(st[4]),
                              _dp(st[5]), *[_dp(a) for a in out])
    return tuple(out)


def landau(T00, T0x, Txx):
    """Rest-frame energy density and velocity of each slab."""
    T00, T0x, Txx = (np.ascontiguousarray(a, dtype=np.float64) for a in (T00, T0x, Txx))
    e = np.zeros(len(T00))
    v = np.zeros(len(T00))
    lib().orc_landau(len(T00), _dp(T00), _dp(T0x), _dp(Txx), _dp(e), _dp(v))
    return e, v


def collide_cell_with_uniforms(p_cell, kfac, u_acc, u_kin):
    """Collide one cell whose members (canonical order) have momenta p_cell
    [nc,3]; u_acc[k], u_kin[2k], u_kin[2k+1] are the injected uniforms of
    pair k.  Returns (new momenta [nc,3], accepted pairs list)."""
    pc = np.ascontiguousarray(p_cell, dtype=np.float64)
    nc = pc.shape[0]
    px, py, pz = (pc[:, 0].copy(), pc[:, 1].copy(), pc[:, 2].copy())
    ua = np.ascontiguousarray(u_acc, dtype=np.float64)
    uk = np.ascontiguousarray(u_kin, dtype=np.float64)
    aa = np.zeros(max(1, nc), np.int32)
    bb = np.zeros(max(1, nc), np.int32)
    m = lib().orc_collide_cell_with_uniforms(
        nc, _dp(px), _dp(py), _dp(pz), float(kfac), _dp(ua), _dp(uk),
        aa.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        bb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if m < 0:
        raise RuntimeError(f"orc_collide_cell_with_uniforms failed: {m}")
    return np.stack([px, py, pz], axis=1), [(int(aa[i]), int(bb[i])) for i in range(m)]


def scatter_pair(pa, pb, uc, uphi):
    a = np.ascontiguousarray(pa, dtype=np.float64).copy()
    b = np.ascontiguousarray(pb, dtype=np.float64).copy()
    lib().orc_scatter_pair(_dp(a), _dp(b), float(uc), float(uphi))
    return a, b
