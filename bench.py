"""Benchmark of the PIC Boltzmann step (arXiv:1208.0961) on one MI355X.

A step is the whole per-time-step update: streaming, wall reflection,
binning (slot atomics into fixed-capacity cells), the pair tests with
claims and kinematics,
and the T00/T0x profiles every 50 steps.  The default workload is the 3-D
binned Riemann tube: 10 x 2 x 2 fm, 100 x 10 x 10 cells, r_test = 2500,
1 020 851 test particles, sigma = 0.4 fm^2, dt = 0.02 fm/c, FP64.  Inputs
are synthetic (seeded thermal gases) and resident in HBM before timing.

Prints one JSON line: particle-steps/s (whole job) plus pair tests/s; the
roofline of the dominant kernel (the fused pair-test kernel) as FP64 FLOP/s
of the pair stage against the FP64 vector peak, with its integer issue rate
(Philox4x32-10 bounds it) and VALU busy beside; the streaming/binning rate
against the HBM peak; per-stage times; the CPU oracle timed on a bounded
sample of the same workload on all usable host cores; and, unless
--no-extras, the two ensemble legs of the metric: the 256-event batched
ensemble against the same events one at a time, and a short served request
stream against a one-at-a-time FIFO (p50/p99 time-to-result).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks.
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# 32-bit VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
INT32_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic work of one pair test: the integer operations that the Philox
# word w1 deciding acceptance depends on, when the counter's cell and step
# words are shared by the cell's pairs: 16 products (32x32 -> 64, hi or lo),
# 15 three-input XORs, and the compare.
PHILOX_OPS_PER_PAIR = 16 + 15 + 1
# Algorithmic FP64 work of one pair test, Eq. (3): the dot product (5),
# E1 E2, s = 2 (E1 E2 - dot) (2), s / (2 E1 E2) (2), x K, and the compare.
FP64_FLOPS_PER_PAIR = 12
# HBM bytes per particle that the streaming + binning kernels move (read
# and write x y z px py pz id), done by the fused step kernel for all but
# the first step of a run and by the stream-bin kernel for that one.
BYTES_BIN = 52 + 52
# Algorithmic HBM bytes per particle-step of streaming + binning as a
# three-pass counting sort: stream + count (read r, p: 48 B; write r, cell,
# rank: 32 B) and scatter (read cell, rank, state, id: 60 B; write state and
# id: 52 B).
BYTES_BIN_ALGO = 80 + 112
# Of the fused-step launches of the timed run, every STEP_EVERY-th is timed
# with HIP events (the other stages at every launch).
STEP_EVERY = 10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tube3d",
                    choices=["tube1d", "tube3d", "full", "paper32", "batch", "serve",
                             "sigma-scan"])
    ap.add_argument("--events", type=int, default=256,
                    help="batch: number of ensemble events")
    ap.add_argument("--requests", type=int, default=2000,
                    help="serve: number of requests")
    ap.add_argument("--retune", action="store_true",
                    help="batch: ignore a stored tuning table")
    ap.add_argument("--serve-policy", choices=["classes", "fifo", "srpt", "all"],
                    default="classes",
                    help="serve: short requests in a batch of their own, stepped to "
                         "their end concurrently with the others on a second stream, the "
                         "others as under fifo (classes); the oldest requests in arrival "
                         "order within a particle budget per run (fifo); the oldest then "
                         "least remaining work first within the budget (srpt); or every "
                         "live request in every run (all); the other policies run on the "
                         "same trace for comparison")
    ap.add_argument("--serve-run-steps", type=int, default=25,
                    help="serve: at most this many steps per run; a run ends early where "
                         "one of its requests ends or is due for an observation")
    ap.add_argument("--serve-run-particles", type=int, default=4_000_000,
                    help="serve, fifo and srpt: particles per run (the oldest request "
                         "always runs)")
    ap.add_argument("--serve-fill-particles", type=int, default=1_000_000,
                    help="serve, fifo: particles of further requests, least remaining "
                         "work first, beside those taken in arrival order")
    ap.add_argument("--serve-short-particles", type=int, default=150_000,
                    help="serve, classes: requests of at most this many particles go "
                         "to the short batch")
    ap.add_argument("--serve-observe", choices=["final", "50"], default="final",
                    help="serve: observe each request's profile at its end only (its "
                         "result) or also every 50 steps, in the server and in the "
                         "one-at-a-time replay")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch: skip the one-at-a-time comparison")
    ap.add_argument("--lanes", type=int, default=None, choices=[0, 1, 8, 16, 32, 64, 128],
                    help="plain workloads: lanes per cell of the cell kernels, 1 for "
                         "packed cells, 128 for "
                         "two waves per cell (default: the library's choice from the "
                         "initial occupancy)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=None,
                    help="oracle threads (default: every usable host core)")
    ap.add_argument("--cpu-seconds", type=float, default=25.0,
                    help="wall-clock budget of the CPU baseline's threaded run")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the ensemble and serving legs")
    ap.add_argument("--extra-steps", type=int, default=50,
                    help="ensemble leg: timed steps of the batched ensemble")
    ap.add_argument("--extra-requests", type=int, default=2000,
                    help="serving leg: requests in the served stream")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the run, copy a 1 GiB device buffer 3 times (a plain "
                         "copy kernel of known size for scaling HBM counters)")
    ap.add_argument("--pmc-csv", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="rocprofv3 counter_collection.csv files of a --calibrate-copy run "
                         "(FETCH_SIZE, WRITE_SIZE): write the measured HBM traffic of "
                         "the dominant kernel to profiles/ and exit")
    ap.add_argument("--pmc-fp64", metavar="FP64_CSV",
                    help="with --pmc-csv: a counter pass with SQ_INSTS_VALU_ADD_F64, "
                         "_MUL_F64, _FMA_F64 and _TRANS_F64; adds the FP64 operations the "
                         "dominant kernel executes per launch")
    ap.add_argument("--pmc-sq", nargs=2, metavar=("SQ_CSV", "KERNEL_STATS_CSV"),
                    help="with --pmc-csv: a counter pass with SQ_ACTIVE_INST_VALU and the "
                         "kernel_stats.csv of a --kernel-trace --stats run of the same "
                         "command; adds the dominant kernel's VALU busy")
    return ap.parse_args()


KERNEL_SOURCES = ("paper_1208_0961_amd/csrc/kernels.hip", "paper_1208_0961_amd/csrc/device.hpp")
DOMINANT_KERNEL = "k_step<true, false,"   # the fused step, any cell capacity


def device_copy_gbs(stream, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Read + write GB/s of torch's device-to-device copy of nbytes."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        src.fill_(1.0)
        for _ in range(2):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def code_text(text: str) -> str:
    """Source text without comments and blank lines: what the compiler
    sees, so that an edit of a comment keeps the measured traffic valid."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    return "\n".join(ln for ln in lines if ln.strip())


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_step_{workload}.json")


def write_traffic(a):
    """HBM bytes per launch of the dominant kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the 1 GiB device copy of --calibrate-copy."""
    import csv

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        kern = [float(r["Counter_Value"]) for r in rows
                if DOMINANT_KERNEL.replace(" ", "") in r["Kernel_Name"].replace(" ", "")]
        # the profiled run uses the benchmark's workload, whose capacity
        # selects one instantiation
        copy = [float(r["Counter_Value"]) for r in rows
                if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 65536]
        if not kern or not copy:
            raise SystemExit(f"{path}: no {DOMINANT_KERNEL} or 1 GiB copy dispatches")
        scale = (1 << 30) / (sorted(copy)[len(copy) // 2] * 1024.0)
        return sum(kern) / len(kern) * 1024.0 * scale, scale

    fetch, fscale = per_kernel(a.pmc_csv[0], "FETCH_SIZE")
    write, wscale = per_kernel(a.pmc_csv[1], "WRITE_SIZE")
    out = {"kernel": DOMINANT_KERNEL.rstrip(",") + " ...>", "workload": a.workload,
           "kernel_source_hash": kernel_source_hash(),
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write,
           "fetch_scale": fscale, "write_scale": wscale}
    if a.pmc_sq:
        out.update(valu_busy(*a.pmc_sq))
    if a.pmc_fp64:
        out.update(fp64_executed(a.pmc_fp64))
    with open(traffic_path(a.workload), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def usable_cores() -> dict:
    """Host cores this process may run on: the CPU affinity set, capped by
    the cgroup CPU quota where one is set (a container's share of a larger
    host); os.cpu_count() beside it for the record."""
    affinity = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
        if q != "max":
            quota = float(q) / float(period)
    except (OSError, ValueError):
        pass
    usable = affinity if quota is None else max(1, min(affinity, int(quota + 0.5)))
    return {"usable": usable, "affinity": affinity, "cpu_quota": quota,
            "cpu_count": os.cpu_count()}


def cpu_baseline(w, state, max_steps, threads, budget_s):
    """The oracle as it stands, on the benchmark's initial state: up to
    max_steps steps with `threads` threads over cells, stopping at the
    first 10-step boundary past budget_s seconds; then, for boxes of at most
    4 M particles, one or two steps on a single thread."""
    from oracle import oracle as O
    st = O.State(*state)
    p = O.make_params(**w.params())
    done = 0
    t0 = time.perf_counter()
    while done < max_steps:
        k = min(10, max_steps - done)
        O.run(p, st, done, k, threads)
        done += k
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cores = usable_cores()
    out = {"value": w.n * done / dt, "unit": "particle-steps/s", "cores": threads,
           "kind": "oracle", "host": cores,
           "sample": f"{w.name}: steps 0..{done - 1} of all {w.n} particles from the "
                     f"benchmark's initial state, {threads} threads over cells "
                     f"({cores['usable']} usable host cores, os.cpu_count() "
                     f"{cores['cpu_count']}), {dt:.1f} s wall"}
    if w.n <= 4_000_000:
        steps1 = 2 if w.n < 2_000_000 else 1
        st1 = O.State(*state)
        t0 = time.perf_counter()
        O.run(p, st1, 0, steps1, 1)
        dt1 = time.perf_counter() - t0
        out["single_thread_value"] = w.n * steps1 / dt1
        out["sample"] += f"; single thread: {steps1} step(s), {dt1:.1f} s"
    return out


SIMDS = 256 * 4
CLOCK_HZ = 2.4e9


def valu_busy(sq_csv: str, stats_csv: str) -> dict:
    """VALU busy of the dominant kernel: 4 SQ_ACTIVE_INST_VALU (quad-cycles,
    summed over the chip) / (SIMDs x cycles of its average trace duration)."""
    import csv
    rows = [r for r in csv.DictReader(open(sq_csv))
            if r["Counter_Name"] == "SQ_ACTIVE_INST_VALU"
            and DOMINANT_KERNEL.replace(" ", "") in r["Kernel_Name"].replace(" ", "")]
    stats = [r for r in csv.DictReader(open(stats_csv))
             if DOMINANT_KERNEL.replace(" ", "") in r["Name"].replace(" ", "")]
    if not rows or not stats:
        raise SystemExit(f"{sq_csv} / {stats_csv}: no {DOMINANT_KERNEL} entries")
    active = sum(float(r["Counter_Value"]) for r in rows) / len(rows)
    ns = float(stats[0]["AverageNs"])
    return {"valu_busy": 4.0 * active / (SIMDS * ns * 1e-9 * CLOCK_HZ),
            "sq_active_inst_valu_per_launch": active, "trace_avg_ns": ns}


def fp64_executed(csv_path: str) -> dict:
    """FP64 operations the dominant kernel executes per launch: 64 lanes x
    (add + mul + transcendental + 2 x fma) wave-instructions, from the SQ
    FP64 instruction counters (executed work, against the algorithmic count
    of 12 flops per pair test: the kernel evaluates Eq. (3) only for the
    pairs that pass the Philox w1 filter)."""
    import csv
    weight = {"SQ_INSTS_VALU_ADD_F64": 1, "SQ_INSTS_VALU_MUL_F64": 1,
              "SQ_INSTS_VALU_TRANS_F64": 1, "SQ_INSTS_VALU_FMA_F64": 2}
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if (r["Counter_Name"] in weight
                and DOMINANT_KERNEL.replace(" ", "") in r["Kernel_Name"].replace(" ", "")):
            per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not per:
        raise SystemExit(f"{csv_path}: no FP64 counters of {DOMINANT_KERNEL}")
    flops = sum(64.0 * weight[k] * sum(v) / len(v) for k, v in per.items())
    return {"fp64_executed_flops_per_launch": flops,
            "fp64_wave_instructions_per_launch": {k: sum(v) / len(v) for k, v in per.items()}}


def measured_profile(workload: str):
    """Measured traffic and VALU busy of the dominant kernel, if taken on the
    current kernel source (None otherwise)."""
    try:
        with open(traffic_path(workload)) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t


def ensemble_leg(steps: int, warmup: int = 5, n_events: int = 256) -> dict:
    """The batched half of the metric: the 256-event ensemble through the
    batch API (tuned, graph-captured runs of up to 50 steps, every profile
    observed after each run) against the same events one at a time through
    cuba_step (the same runs and observations)."""
    import torch
    from paper_1208_0961_amd import autotune as AT
    from paper_1208_0961_amd import batch as BT
    from paper_1208_0961_amd import sim as S
    from paper_1208_0961_amd import workload as W
    events = W.ensemble_events(n_events)
    total_n = sum(w.n for w in events)
    table = AT.load()
    if table is None:
        print("# ensemble: tuning", file=sys.stderr, flush=True)
        table = AT.tune(events)
    oe = events[0].observe_every
    runs = [oe] * (steps // oe) + ([steps % oe] if steps % oe else [])
    print(f"# ensemble: {len(events)} events, {total_n} particles, {steps} steps",
          file=sys.stderr, flush=True)
    B = BT.Batch(len(events))
    for i, w in enumerate(events):
        st = W.riemann_state_torch(w, 100000 + i)
        B.admit(i, {**w.params(), "cell_capacity": W.capacity_for(w)}, st)
        del st
    AT.apply(B, table, dict(enumerate(events)), use_graphs=True)
    footprint = sum(int(B.slots[i]["workspace"].numel()) for i in range(len(events)))
    B.step(warmup)
    B.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in runs:
        B.step(k)
        for i in range(len(events)):
            B.observe_async(i)
    B.sync()
    batched_s = time.perf_counter() - t0
    B.close()
    del B
    torch.cuda.empty_cache()
    print("# ensemble: one event at a time", file=sys.stderr, flush=True)
    busy = 0.0
    for i, w in enumerate(events):
        st = W.riemann_state_torch(w, 100000 + i)
        sim = S.Sim({**w.params(), "cell_capacity": W.capacity_for(w)}, st)
        del st
        sim.step(warmup)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for k in runs:
            sim.step(k)
            sim.observe_async()
        torch.cuda.synchronize()
        busy += time.perf_counter() - s0
        sim.close()
    torch.cuda.empty_cache()
    batched = total_n * steps / batched_s
    seq = total_n * steps / busy
    return {"workload": f"ensemble-{len(events)}-events (r_test 50..2500 log-uniform, "
                        "sigma 0.05..1 fm^2, T_L 0.30..0.50 GeV, T_R = 0.8 T_L, "
                        "box 10 x L x L fm, L in 1, 2, 4)",
            "n_particles": total_n, "steps": steps, "warmup": warmup,
            "batched_particle_steps_per_s": batched,
            "sequential_particle_steps_per_s": seq,
            "speedup_vs_sequential": batched / seq,
            "batched_ms_per_step": 1e3 * batched_s / steps,
            "workspace_bytes": footprint,
            "compact_state_bytes": 2 * 52 * total_n,
            "tuning": {k: table.get(k) for k in ("cell_lanes", "cells_per_item",
                                                 "persistent_waves")}}


def serve_leg(n_requests: int) -> dict:
    """The served half of the metric on a request stream (sizes 1e4 to 4e6
    test particles, 200 steps each, Poisson arrivals at 0.8 of the server's
    measured capacity), served with runs of at most 25 steps: p50/p99
    time-to-result and particle-steps/s of the default policy and of fifo
    (the others: --workload serve) against a one-at-a-time FIFO of plain
    runs on the same trace."""
    from paper_1208_0961_amd import serve
    return serve.measure(n_requests, other_policies=("fifo",))


def bench_sigma_scan(a):
    """Cross-section scan (Sec. 5, Fig. 3): 16 events per sigma, batched, to
    t = 4 fm/c; the ensemble-mean slab moments against the ideal-fluid
    Riemann solution (L1 distance of T00 over 0.5 fm bins; rest-frame e and
    v on the plateau at the largest sigma)."""
    import numpy as np
    from paper_1208_0961_amd import sigma_scan as SS
    from paper_1208_0961_amd import workload as W
    from paper_1208_0961_amd import hydro
    eL = 3 * W.gluon_density(SS.T_LEFT) * SS.T_LEFT
    eR = 3 * W.gluon_density(SS.T_RIGHT) * SS.T_RIGHT
    R = hydro.Riemann(eL, eR)
    tend = 4.0
    sub = (np.arange(20)[:, None] + (np.arange(50)[None, :] + 0.5) / 50) * 0.5
    want = np.array([[R.profiles((x - 5.0) / tend)[0] for x in row] for row in sub]).mean(1)
    xs = (np.arange(100) + 0.5) * 0.1
    plateau = (xs > 3.6) & (xs < 7.0)
    seeds = range(1, 17)
    SS.run(0.4, 0.01, seeds=range(1, 3), t_end=0.5)       # untimed warm-up
    rows, total_ps, total_s = [], 0.0, 0.0
    for sigma, dt in SS.SCAN:
        print(f"# sigma-scan: sigma {sigma} fm^2, dt {dt} fm/c, {len(seeds)} events",
              file=sys.stderr, flush=True)
        r = SS.run(sigma, dt, seeds=seeds, t_end=tend)
        m = r["mean"]
        total_ps += r["particles"] * r["steps"]
        total_s += r["seconds"]
        rows.append({"sigma_fm2": sigma, "dt_fm": dt, "steps": r["steps"],
                     "particles": r["particles"], "seconds": r["seconds"],
                     "l1_T00_vs_ideal_GeV_fm3": float(np.abs(m["T00"].reshape(20, 5).mean(1)
                                                             - want).mean()),
                     "plateau_e": float(m["e"][plateau].mean()),
                     "plateau_v": float(m["v"][plateau].mean()),
                     "plateau_T00": float(m["T00"][plateau].mean()),
                     "plateau_T0x": float(m["T0x"][plateau].mean())})
    out = {"metric": "sigma scan: approach to ideal hydro (Sec. 5, Fig. 3)",
           "value": total_ps / total_s, "unit": "particle-steps/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64",
           "data": "synthetic: seeded thermal Riemann events",
           "config": {"workload": "riemann-tube-10x1x1-c100x4x4-rt400", "events_per_sigma":
                      len(seeds), "t_end_fm": tend},
           "ideal": {"e_star": R.es, "v_star": R.vs, "shock_speed": R.shock},
           "scan": rows}
    print(json.dumps(out), flush=True)


def bench_batch(a):
    """Ensemble of independent Riemann events (r_test log-uniform in
    [50, 2500], sigma in [0.05, 1] fm^2, T_L in [0.30, 0.50] GeV, T_R = 0.8 T_L,
    10 x L x L fm boxes with L in {1, 2, 4}) advanced together by the batch
    API in graph-captured runs of 50 steps with all profiles observed after
    each run, against the same events run one at a time through cuba_step."""
    import torch
    from paper_1208_0961_amd import autotune as AT
    from paper_1208_0961_amd import batch as BT
    from paper_1208_0961_amd import cuba as C
    from paper_1208_0961_amd import sim as S
    from paper_1208_0961_amd import workload as W

    events = W.ensemble_events(a.events)
    total_n = sum(w.n for w in events)
    table = None if a.retune else AT.load()
    if table is None:
        print("# tuning", file=sys.stderr, flush=True)
        table = AT.tune(events)
        AT.save(table)
    print(f"# batch: {len(events)} events, {total_n} particles; tuning {table}",
          file=sys.stderr, flush=True)
    B = BT.Batch(len(events))
    for i, w in enumerate(events):
        st = W.riemann_state_torch(w, 100000 + i)
        B.admit(i, {**w.params(), "cell_capacity": W.capacity_for(w)}, st)
        del st
    AT.apply(B, table, dict(enumerate(events)), use_graphs=True)
    B.step(a.warmup)
    B.sync()
    oe = events[0].observe_every
    runs = [oe] * (a.steps // oe) + ([a.steps % oe] if a.steps % oe else [])
    pairs0 = sum(B.counters(i)["pair_tests"] for i in range(len(events)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in runs:
        B.step(k)
        for i in range(len(events)):
            B.observe_async(i)
    B.sync()
    t1 = time.perf_counter()
    batched = total_n * a.steps / (t1 - t0)
    pairs = sum(B.counters(i)["pair_tests"] for i in range(len(events))) - pairs0
    # per-stage kernel times of one more run, without graphs (diagnostic)
    B.set_launch(int(table.get("persistent_waves", 0)), False)
    C.cuba_batch_timing_begin(B.b, 4 * oe + 8)
    B.step(oe)
    stage_times = C.cuba_batch_timing_end(B.b)
    B.close()
    del B
    torch.cuda.empty_cache()

    seq = None
    if not a.no_sequential:
        print("# one event at a time", file=sys.stderr, flush=True)
        busy = 0.0
        for i, w in enumerate(events):
            st = W.riemann_state_torch(w, 100000 + i)
            sim = S.Sim({**w.params(), "cell_capacity": W.capacity_for(w)}, st)
            del st
            sim.step(a.warmup)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for k in runs:
                sim.step(k)
                sim.observe_async()
            torch.cuda.synchronize()
            busy += time.perf_counter() - s0
            sim.close()
        seq = total_n * a.steps / busy
    out = {"metric": "batched ensemble particle-steps/s vs one event at a time",
           "value": batched, "unit": "particle-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": 1e3 * (t1 - t0) / a.steps, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic: seeded thermal Riemann events",
           "config": {"workload": f"ensemble-{len(events)}-events", "n_particles": total_n,
                      "observe_every": events[0].observe_every},
           "pair_tests_per_s": pairs / (t1 - t0),
           "sequential_value": seq,
           "speedup_vs_sequential": (batched / seq) if seq else None,
           "stage_ms_per_launch": {k: (v[0] / v[1] if v[1] else None)
                                   for k, v in stage_times.items()},
           "tuning": table}
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.pmc_csv:
        return write_traffic(a)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); a multi-GPU "
              "slab decomposition of the box is not implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    from paper_1208_0961_amd import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()
    from paper_1208_0961_amd import cuba as C
    from paper_1208_0961_amd import sim as S
    from paper_1208_0961_amd import workload as W

    if a.workload == "batch":
        return bench_batch(a)
    if a.workload == "sigma-scan":
        return bench_sigma_scan(a)
    if a.workload == "serve":
        from paper_1208_0961_amd import serve
        return serve.bench(a)
    w = W.ALIASES[a.workload]
    state = W.riemann_state(w)
    sim = S.Sim(w.params(), state, cell_lanes=a.lanes)
    lanes = sim.cell_lanes
    print(f"# {w.name}: {w.n} particles, {w.n_cells} cells, {lanes} lanes per "
          f"cell; warmup {a.warmup}", file=sys.stderr, flush=True)
    sim.step(a.warmup)
    sim.sync()
    c0 = C.cuba_counters(sim.ctx)
    # runs of steps between observations (every observe_every steps)
    runs = []
    done = 0
    while done < a.steps:
        t_abs = a.warmup + done
        k = min(a.steps - done, w.observe_every - t_abs % w.observe_every)
        runs.append((k, (t_abs + k) % w.observe_every == 0))
        done += k
    # HIP events around every launch of the rare stages and around every
    # STEP_EVERY-th fused step: a bracketed launch delays the next one by a
    # few microseconds, which would otherwise slow the timed run itself
    C.cuba_timing_begin_sampled(sim.ctx, 2 * a.steps + 6 * len(runs) + 16, STEP_EVERY)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, obs in runs:
        C.cuba_step(sim.ctx, k)
        if obs:
            sim.observe_async()
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    stages = C.cuba_timing_end(sim.ctx)
    c1 = C.cuba_counters(sim.ctx)
    sim.sync()
    elapsed = t1 - t0
    pairs = c1["pair_tests"] - c0["pair_tests"]
    cand = c1["candidates"] - c0["candidates"]
    claims = c1["claims"] - c0["claims"]
    value = w.n * a.steps / elapsed

    def avg_ms(name):
        ms, k = stages[name]
        return ms / k if k else float("nan")

    # the dominant kernel: the fused step (collisions of step t, streaming and
    # binning of step t+1)
    step_ms = avg_ms("step") if stages["step"][1] else avg_ms("collide")
    pairs_per_step = pairs / a.steps
    fp64_tflops = FP64_FLOPS_PER_PAIR * pairs_per_step / (step_ms * 1e-3) / 1e12
    int32_tops = PHILOX_OPS_PER_PAIR * pairs_per_step / (step_ms * 1e-3) / 1e12
    prof = measured_profile(a.workload)
    fp64_exec = None
    if prof and prof.get("fp64_executed_flops_per_launch") is not None:
        ex = prof["fp64_executed_flops_per_launch"] / (step_ms * 1e-3) / 1e12
        fp64_exec = {"achieved": ex, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": ex / FP64_PEAK_TFLOPS,
                     "flops_per_launch": prof["fp64_executed_flops_per_launch"]}

    def gbs(nbytes, ms):
        return nbytes / (ms * 1e-3) / 1e9

    stage_out = {}
    for name in C.STAGES:
        ms, k = stages[name]
        stage_out[name] = {"ms_per_launch": ms / k if k else None, "launches_timed": k}
    stage_out["step"]["timed_every"] = STEP_EVERY
    stage_out["bin"]["gbs_moved"] = gbs(BYTES_BIN * w.n, avg_ms("bin"))
    stage_out["step"]["pair_tests_per_launch"] = pairs_per_step
    stage_out["step"]["binning_gbs_moved"] = gbs(BYTES_BIN * w.n, step_ms)

    # a plain device copy of 1 GiB, timed after the run, as the practical
    # HBM ceiling beside the 8 TB/s peak (read + write bytes per second)
    copy_gbs = device_copy_gbs(sim.stream)
    bin_ms = avg_ms("bin")
    hbm = {"kernel": "k_stream_bin (streaming, reflection, binning)",
           "bytes_per_particle_step": BYTES_BIN_ALGO,
           "achieved": gbs(BYTES_BIN_ALGO * w.n, bin_ms), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": gbs(BYTES_BIN_ALGO * w.n, bin_ms) / HBM_PEAK_GBS,
           "ms_per_launch": bin_ms, "moved_bytes_per_particle": BYTES_BIN,
           "moved_gbs": gbs(BYTES_BIN * w.n, bin_ms), "copy_gbs": copy_gbs,
           "moved_frac_of_copy": gbs(BYTES_BIN * w.n, bin_ms) / copy_gbs}

    cpu = None
    cpu_steps = a.cpu_steps if a.cpu_steps is not None else {"tube1d": 200, "tube3d": 200,
                                                              "full": 2,
                                                              "paper32": 2}[a.workload]
    if cpu_steps > 0:
        threads = a.cpu_threads or usable_cores()["usable"]
        print(f"# cpu baseline: up to {cpu_steps} oracle steps, {threads} threads",
              file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, state, cpu_steps, threads, a.cpu_seconds)

    out = {
        "metric": "particle-steps/s + FP64 pair-tests/s; ensemble p50/p99 latency vs plain",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": f"synthetic: seeded thermal Riemann gas (T {w.T_left:.2f} / "
                f"{w.T_right:.2f} GeV), no dataset",
        "config": {"workload": w.name, "n_particles": w.n, "cells": list(w.cells),
                   "box_fm": list(w.box), "r_test": w.r_test, "sigma_fm2": w.sigma,
                   "dt_fm": w.dt, "observe_every": w.observe_every,
                   "cell_lanes": lanes},
        "pair_tests_per_s": pairs / elapsed,
        "fp64_pair_test_flops_per_s": FP64_FLOPS_PER_PAIR * pairs / elapsed,
        "candidates_per_step": cand / a.steps,
        "scatterings_per_step": claims / a.steps,
        "roofline": {"bound": "alu", "kernel": "k_step (fused): pair stage, FP64 vector",
                     "achieved": fp64_tflops, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": fp64_tflops / FP64_PEAK_TFLOPS,
                     "traffic": prof["bytes_per_launch"] if prof else None,
                     "flops_per_pair_test": FP64_FLOPS_PER_PAIR,
                     "algorithmic_bytes_per_launch": BYTES_BIN * w.n,
                     "ms_per_launch": step_ms,
                     "int32_issue": {"achieved": int32_tops, "peak": INT32_PEAK_TOPS,
                                     "unit": "Tops/s", "frac": int32_tops / INT32_PEAK_TOPS,
                                     "ops_per_pair_test": PHILOX_OPS_PER_PAIR},
                     "valu_busy": prof.get("valu_busy") if prof else None,
                     "basis": "algorithmic: 12 FP64 flops per pair test of Eq. (3) over all "
                              "pair tests; the kernel runs Eq. (3) only for pairs that pass "
                              "the Philox w1 filter (fp64_executed: the counters' count)",
                     "fp64_executed": fp64_exec},
        "hbm": hbm,
        "stages": stage_out,
        "cpu_baseline": cpu,
        "library": {"build_info": C.cuba_build_info(),
                    "matches_sources": C.build_hash() == hip_build.source_hash()},
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if a.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 1 << 30
    if a.workload == "tube3d" and not a.no_extras:
        for key, leg in (("ensemble", lambda: ensemble_leg(a.extra_steps)),
                         ("serve", lambda: serve_leg(a.extra_requests))):
            try:
                out[key] = leg()
            except Exception as e:    # the headline line is printed regardless
                out[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
