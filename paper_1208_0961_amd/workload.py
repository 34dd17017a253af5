"""Seeded synthetic inputs: thermal massless gluon gases in a box.

This module draws initial states only; it holds none of the per-step
arithmetic of the method and is the one module that both the GPU path's
callers and the oracle's tests use to make inputs.

The Riemann set-up follows the paper's benchmark (Sec. 5): two halves of a
box at different temperatures.  The paper's own parameter set (32^3 fm^3,
T = 0.4 / 0.2 GeV, sigma = 10 GeV^-2, dt = 0.1 fm/c) states no test-particle
count or cell size; the workloads below are the tube geometries used for
parity and measurement.  Densities are those of a Boltzmann gas with gluon
degeneracy 16, n = 16 T^3 / pi^2 / (hbar c)^3, and each half holds
N = round(r_test n V_half) test particles placed uniformly in that half.
|p| follows p^2 exp(-p/T), i.e. Gamma(3, T), drawn as -T ln(u1 u2 u3) with
u in (0, 1]; directions are isotropic (cos theta = 2u - 1, phi = 2 pi u).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

HBARC = 0.1973269804  # GeV fm (CODATA); the paper states no value
FIXTURE_SEED = 0x12080961
DYNAMICS_SEED = 1


def gluon_density(T: float) -> float:
    """Test-particle-free number density of a Boltzmann gluon gas [fm^-3]."""
    return 16.0 * T ** 3 / math.pi ** 2 / HBARC ** 3


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    box: tuple
    cells: tuple
    r_test: float
    sigma: float
    dt: float
    T_left: float
    T_right: float
    steps: int = 200
    observe_every: int = 50
    seed: int = DYNAMICS_SEED

    @property
    def n_cells(self) -> int:
        return int(self.cells[0]) * int(self.cells[1]) * int(self.cells[2])

    def side_counts(self):
        vh = 0.5 * self.box[0] * self.box[1] * self.box[2]
        nl = int(round(self.r_test * gluon_density(self.T_left) * vh))
        nr = int(round(self.r_test * gluon_density(self.T_right) * vh))
        return nl, nr

    @property
    def n(self) -> int:
        return sum(self.side_counts())

    def params(self) -> dict:
        return dict(box=tuple(float(b) for b in self.box),
                    cells=tuple(int(c) for c in self.cells),
                    sigma=float(self.sigma), r_test=float(self.r_test),
                    dt=float(self.dt), seed=int(self.seed))


# The three plain-method tubes: 1-D binned (parity scale), 3-D binned
# (measurement scale) and full-GPU scale; sigma = 0.4 fm^2 is the paper's
# 10 GeV^-2 rounded, dt = 0.02 fm/c keeps dt below every cell edge.
TUBE_1D = Workload("riemann-tube-10x1x1-c100x1x1-rt100", (10.0, 1.0, 1.0),
                   (100, 1, 1), 100.0, 0.4, 0.02, 0.40, 0.32)
TUBE_3D = Workload("riemann-tube-10x2x2-c100x10x10-rt2500", (10.0, 2.0, 2.0),
                   (100, 10, 10), 2500.0, 0.4, 0.02, 0.40, 0.32)
TUBE_FULL = Workload("riemann-tube-10x8x8-c100x40x40-rt2500", (10.0, 8.0, 8.0),
                     (100, 40, 40), 2500.0, 0.4, 0.02, 0.40, 0.32)
# The paper's own Riemann set-up (Sec. 5, Fig. 2): a 32^3 fm^3 box split at
# x = 16 fm, T = 0.4 / 0.2 GeV, sigma = 10 GeV^-2 = 0.3894 fm^2, dt = 0.1
# fm/c.  The paper states no test-particle ratio or cell size: r_test = 100
# and 0.25 fm cells (dt below every cell edge, ~21 / ~2.6 test particles
# per cell on the two sides).  50 steps reach t = 5 fm/c.
SIGMA_PAPER = 10.0 * HBARC ** 2       # 10 GeV^-2 in fm^2
PAPER_32 = Workload("riemann-box-32x32x32-c128x128x128-rt100", (32.0, 32.0, 32.0),
                    (128, 128, 128), 100.0, SIGMA_PAPER, 0.1, 0.40, 0.20, steps=50,
                    observe_every=10)
WORKLOADS = {w.name: w for w in (TUBE_1D, TUBE_3D, TUBE_FULL, PAPER_32)}
ALIASES = {"tube1d": TUBE_1D, "tube3d": TUBE_3D, "full": TUBE_FULL, "paper32": PAPER_32}


def sample_gas(rng, n, T, lo, hi):
    """n particles uniform in the box [lo, hi) with Gamma(3,T) |p| and
    isotropic directions.  Returns six float64 arrays."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    r = lo + (hi - lo) * rng.random((n, 3))
    u = 1.0 - rng.random((n, 3))            # (0, 1]
    pm = -T * np.log(u[:, 0] * u[:, 1] * u[:, 2])
    bad = ~(pm > 0.0)
    while bad.any():                        # |p| = 0 has probability ~2^-159
        u2 = 1.0 - rng.random((int(bad.sum()), 3))
        pm[bad] = -T * np.log(u2[:, 0] * u2[:, 1] * u2[:, 2])
        bad = ~(pm > 0.0)
    cth = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * math.pi * rng.random(n)
    sth = np.sqrt((1.0 - cth) * (1.0 + cth))
    p = np.stack([pm * sth * np.cos(phi), pm * sth * np.sin(phi), pm * cth], 1)
    return r[:, 0], r[:, 1], r[:, 2], p[:, 0], p[:, 1], p[:, 2]


def riemann_state(w: Workload, seed: int = FIXTURE_SEED, shuffle: bool = True):
    """Initial Riemann state of workload w: left half at T_left, right half
    at T_right.  Particle ids (array order) are shuffled so that id order
    carries no spatial order.  Returns six float64 arrays."""
    rng = np.random.default_rng(seed)
    nl, nr = w.side_counts()
    L = w.box
    left = sample_gas(rng, nl, w.T_left, (0.0, 0.0, 0.0), (0.5 * L[0], L[1], L[2]))
    right = sample_gas(rng, nr, w.T_right, (0.5 * L[0], 0.0, 0.0), (L[0], L[1], L[2]))
    arrs = [np.concatenate([a, b]) for a, b in zip(left, right)]
    if shuffle:
        perm = rng.permutation(nl + nr)
        arrs = [a[perm] for a in arrs]
    return [np.ascontiguousarray(a) for a in arrs]


def thermal_box(box, n, T, seed=FIXTURE_SEED):
    """n particles of one temperature filling the whole box."""
    rng = np.random.default_rng(seed)
    return [np.ascontiguousarray(a) for a in
            sample_gas(rng, n, T, (0.0, 0.0, 0.0), tuple(box))]


# ---------------------------------------------------------------------------
# Ensembles of independent Riemann events (batched and served workloads)
# ---------------------------------------------------------------------------
def ensemble_events(n_events=256, seed=4, dt=0.02, steps=200):
    """Events with r_test log-uniform in [50, 2500], sigma uniform in
    [0.05, 1] fm^2, T_L uniform in [0.30, 0.50] GeV, T_R = 0.8 T_L, box
    10 x L x L fm with L in {1, 2, 4}, cells 0.1 x 0.2 x 0.2 fm, event seed
    1000 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_events):
        r_test = float(math.exp(rng.uniform(math.log(50.0), math.log(2500.0))))
        sigma = float(rng.uniform(0.05, 1.0))
        TL = float(rng.uniform(0.30, 0.50))
        L = float(rng.choice([1.0, 2.0, 4.0]))
        nt = int(round(5 * L))
        out.append(Workload(f"event{i}", (10.0, L, L), (100, nt, nt), r_test,
                            sigma, dt, TL, 0.8 * TL, steps=steps, seed=1000 + i))
    return out


# ---------------------------------------------------------------------------
# The same recipe drawn on the GPU (large ensembles: ~1e8 particles)
# ---------------------------------------------------------------------------
def sample_gas_torch(gen, n, T, lo, hi, device):
    """As sample_gas, drawn with a seeded torch generator on `device`;
    returns six float64 tensors."""
    import torch
    kw = dict(generator=gen, device=device, dtype=torch.float64)
    lo_t = torch.tensor(lo, dtype=torch.float64, device=device)
    hi_t = torch.tensor(hi, dtype=torch.float64, device=device)
    r = lo_t + (hi_t - lo_t) * torch.rand((n, 3), **kw)
    u = 1.0 - torch.rand((n, 3), **kw)                      # (0, 1]
    pm = -T * torch.log(u[:, 0] * u[:, 1] * u[:, 2])
    pm = torch.where(pm > 0.0, pm, torch.full_like(pm, T))  # |p| = 0: probability ~2^-159
    cth = 2.0 * torch.rand(n, **kw) - 1.0
    phi = 2.0 * math.pi * torch.rand(n, **kw)
    sth = torch.sqrt((1.0 - cth) * (1.0 + cth))
    return (r[:, 0].contiguous(), r[:, 1].contiguous(), r[:, 2].contiguous(),
            (pm * sth * torch.cos(phi)).contiguous(), (pm * sth * torch.sin(phi)).contiguous(),
            (pm * cth).contiguous())


def riemann_state_torch(w: Workload, seed: int, device="cuda"):
    """Riemann state of workload w drawn on the GPU (ids not shuffled: the
    canonical order depends on ids only within a cell)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    nl, nr = w.side_counts()
    L = w.box
    left = sample_gas_torch(gen, nl, w.T_left, (0.0, 0.0, 0.0), (0.5 * L[0], L[1], L[2]), device)
    right = sample_gas_torch(gen, nr, w.T_right, (0.5 * L[0], 0.0, 0.0), (L[0], L[1], L[2]), device)
    return [torch.cat([a, b]) for a, b in zip(left, right)]


def max_mean_occupancy(w: Workload) -> float:
    """Mean test particles per cell on the denser (left) side."""
    vcell = w.box[0] * w.box[1] * w.box[2] / w.n_cells
    return w.r_test * gluon_density(w.T_left) * vcell


def capacity_for(w: Workload, sigmas: float = 4.0) -> int:
    """Cell capacity from the expected occupancy on the denser side: its
    mean plus `sigmas` Poisson standard deviations (and 2), rounded up to
    32.  A cell that holds more keeps its surplus in spill slots and is
    stepped inside the same kernels, so a tight block costs little: on the
    256-event ensemble, 4 sigmas measured as fast as 1.5 x (mean + 5 sigma)
    + 32 over 360 steps of the evolution, at 64 instead of 94 GB."""
    m = max_mean_occupancy(w)
    cap = int(math.ceil((m + sigmas * math.sqrt(m) + 2.0) / 32.0)) * 32
    return max(64, min(1024, cap))
