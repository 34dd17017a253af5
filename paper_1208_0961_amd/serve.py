"""Serving: continuous batching of simulation requests.

Each request is one Riemann event (parameters from the ensemble
distribution, an initial state drawn from its seed) to be advanced a fixed
number of steps, with T00/T0x observed every 50 steps (or, with final_only,
at the end only); the result is the final profile.  The server admits
arrived requests in FIFO order as a batch slot and enough HBM (the event's
workspace footprint) free up, advances live events together in runs of at
most `run_steps` steps (one launch per step for all of them), each ending
where an event in it ends or is due for an observation, and retires events
that are done.  Admission, retirement and result copies do not wait for the
GPU: runs are queued back to back and requests that arrive while others are
on the GPU join the next queued run, so their work overlaps on the device.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import numpy as np
import torch

from . import workload as W
from .batch import Batch, event_workspace_bytes
from .sim import Sim


@dataclasses.dataclass
class Request:
    rid: int
    work: W.Workload
    arrival: float      # seconds from the start of the trace
    state_seed: int


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    T00: np.ndarray
    T0x: np.ndarray
    state: list | None = None
    admitted_run: int = 0     # runs queued before admission
    finished_run: int = 0     # runs queued up to its last

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def request_stream(n_requests: int, rate: float, seed: int = 5, nmin: float = 1e4,
                   nmax: float = 4e6, steps: int = 200) -> list[Request]:
    """Requests from the ensemble distribution truncated to nmin <= N <= nmax,
    with Poisson arrivals at `rate` requests per second."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    i = 0
    while len(out) < n_requests:
        r_test = float(math.exp(rng.uniform(math.log(50.0), math.log(2500.0))))
        sigma = float(rng.uniform(0.05, 1.0))
        TL = float(rng.uniform(0.30, 0.50))
        L = float(rng.choice([1.0, 2.0, 4.0]))
        nt = int(round(5 * L))
        w = W.Workload(f"req{i}", (10.0, L, L), (100, nt, nt), r_test, sigma, 0.02, TL,
                       0.8 * TL, steps=steps, seed=5000 + i)
        i += 1
        if not (nmin <= w.n <= nmax):
            continue
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        out.append(Request(len(out), w, t, 700000 + i))
    return out


def footprint(req: Request) -> int:
    return event_workspace_bytes({**req.work.params(),
                                  "cell_capacity": W.capacity_for(req.work)}, req.work.n)


def collect_ready(pending: deque, results: list, now, block: bool = False):
    """Moves every queued result whose copy to the host has completed from
    `pending` (entries (done event, result fields, host T00, host T0x)) to
    `results`, stamped with now().  The lanes' results complete out of
    order, so a short run's result does not wait behind a long run queued
    before it; block=True first waits for the oldest one."""
    if block and pending:
        pending[0][0].synchronize()
    for _ in range(len(pending)):
        item = pending.popleft()
        if not item[0].query():
            pending.append(item)      # those left keep their order
            continue
        _, fields, h00, h0x = item
        results.append(Result(**fields, finished=now(), T00=h00.numpy().copy(),
                              T0x=h0x.numpy().copy()))


class _Lane:
    """One batch of live events on its own stream, with the runs queued on
    it that have not completed yet."""

    def __init__(self, max_slots: int, device: str, use_graphs: bool, run_steps: int):
        self.B = Batch(max_slots, device=device, use_graphs=use_graphs)
        self.live: dict[int, dict] = {}
        self.inflight: deque = deque()   # an event after each queued run
        self.run_steps = run_steps


class Server:
    """Continuous batching of Riemann-event requests on one GPU.

    Requests are admitted in arrival order as a slot (at most max_slots
    live events) and HBM (the event's workspace footprint) free up, without
    waiting for the GPU
    (cuba_batch_admit_async); live events advance in runs of at most
    `run_steps` steps, one launch per step for every event in the run; an
    event that finishes is observed, its profile copied to pinned host
    memory, and its slot retired, again without waiting.  The host queues a
    run as soon as the previous one is queued, keeping at most `depth` runs
    in flight, and collects each result when its copy has completed (the
    time-to-result).  Requests that arrive while others are on the GPU join
    the next queued run.

    Which live events take part in a run:
      "all"     every live event (processor sharing);
      "srpt"    the oldest, then the others by least remaining work
                (particles x steps left) while they fit `run_particles`;
      "fifo"    the oldest events in arrival order while they fit
                `run_particles` (at least one), then others by least
                remaining work while they fit `fill_particles` more (small
                requests slip in beside the large ones at the head of the
                queue);
      "classes" two batches on two streams whose runs execute concurrently:
                requests of at most `short_particles` particles go to the
                short batch, whose runs take every live event there to its
                end (or next observation) in one run, so a short request
                waits only for the short run before it; the others go to
                the long batch, stepped as under "fifo".  A step of a few
                short events is bound by launch latency, not by the GPU's
                throughput, so it fills the gaps of the long batch's steps
                instead of queueing behind them.
    the others are held (cuba_batch_set_active) until chosen."""

    POLICIES = ("all", "srpt", "fifo", "classes")

    def __init__(self, max_slots: int = 256, hbm_budget: int | None = None,
                 run_steps: int = 25, device: str = "cuda", use_graphs: bool = False,
                 tuning: dict | None = None, keep_states: bool = False,
                 policy: str = "classes", run_particles: int = 4_000_000,
                 final_only: bool = False, depth: int = 2,
                 fill_particles: int = 1_000_000, short_particles: int = 150_000,
                 observe_in_runs: bool = True, short_run_steps: int = 1 << 30):
        if policy not in self.POLICIES:
            raise ValueError(f"policy must be one of {self.POLICIES}")
        if run_steps < 1:
            raise ValueError("run_steps must be at least 1")
        self.device = device
        self.policy = policy
        self.run_particles = int(run_particles)
        self.fill_particles = int(fill_particles)
        self.short_particles = int(short_particles) if policy == "classes" else 0
        self.final_only = final_only
        # observations every observe_every steps are written by the runs'
        # own launches (cuba_batch_set_observe), so runs need not stop at
        # them; False stops each run at the next observation and observes
        # from the host between runs
        self.observe_in_runs = bool(observe_in_runs) and not final_only
        self.run_steps = run_steps
        self.keep_states = keep_states
        self.depth = max(1, int(depth))
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget = int(0.7 * free)
        self.budget = hbm_budget
        self.max_slots = int(max_slots)
        self.lanes = [_Lane(max_slots, device, use_graphs, run_steps)]
        if policy == "classes":
            # short runs: at most short_run_steps (default: to the events' end)
            self.lanes.append(_Lane(max_slots, device, use_graphs, int(short_run_steps)))
        self.B = self.lanes[0].B
        self.tuning = tuning
        self.use_graphs = use_graphs
        self.peak_live = 0
        self.peak_bytes = 0
        self.peak_held = 0
        self.lane_runs = [0] * len(self.lanes)   # runs queued per lane

    def _lane_for(self, req: Request) -> _Lane:
        if len(self.lanes) > 1 and req.work.n <= self.short_particles:
            return self.lanes[1]
        return self.lanes[0]

    def _admit(self, lane: _Lane, slot: int, req: Request):
        from . import autotune as AT
        with torch.cuda.stream(lane.B.stream):
            state = W.riemann_state_torch(req.work, req.state_seed, device=self.device)
        lane.B.admit_async(slot, {**req.work.params(),
                                  "cell_capacity": W.capacity_for(req.work)}, state)
        if self.observe_in_runs:
            w = req.work
            lane.B.set_observe(slot, w.observe_every, rows=max(1, w.steps // w.observe_every))
        if self.tuning:
            AT.settings_for(lane.B, slot, req.work, self.tuning)

    def run(self, requests: list[Request], realtime=True) -> list[Result]:
        """Serves the requests.  realtime=True admits a request once its
        arrival time has passed on the wall clock; False treats every request
        as present at the start; "runs" reads arrival times as a count of
        queued runs (a logical clock: admission mid-stream at a reproducible
        point)."""
        if self.tuning:
            for lane in self.lanes:
                lane.B.set_launch(int(self.tuning.get("persistent_waves", 0)), self.use_graphs)
        queue = deque(sorted(requests, key=lambda r: r.arrival))
        used = 0
        results: list[Result] = []
        pending: deque = deque()   # (done event, result fields, host T00, host T0x)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        runs_done = [0]
        logical = realtime == "runs"
        clock = (lambda: runs_done[0]) if logical else now
        lanes = self.lanes
        n_live = lambda: sum(len(lane.live) for lane in lanes)

        def collect(block: bool = False):
            collect_ready(pending, results, now, block)

        while queue or n_live() or pending:
            collect()
            # admission: FIFO, by free slot and HBM footprint
            while queue and (not realtime or queue[0].arrival <= clock()):
                req = queue[0]
                need = footprint(req)
                lane = self._lane_for(req)
                slot = lane.B.free_slot() if n_live() < self.max_slots else None
                if slot is None or (used + need > self.budget and n_live()):
                    break
                queue.popleft()
                self._admit(lane, slot, req)
                used += need
                lane.live[slot] = {"req": req, "need": need, "done": 0, "admitted": now(),
                                   "admitted_run": runs_done[0], "active": True}
                self.peak_live = max(self.peak_live, n_live())
                self.peak_bytes = max(self.peak_bytes, used)
            if not n_live():
                if pending:
                    collect(block=not queue or (realtime and queue[0].arrival > clock()))
                elif queue and logical:
                    runs_done[0] = max(runs_done[0], int(math.ceil(queue[0].arrival)))
                elif queue and realtime:
                    time.sleep(max(0.0, min(queue[0].arrival - now(), 0.002)))
                continue
            queued = False
            for lane in lanes:
                while lane.inflight and lane.inflight[0].query():
                    lane.inflight.popleft()
                if lane.live and len(lane.inflight) < self.depth:
                    used -= self._queue_run(lane, pending, runs_done, now)
                    queued = True
            if not queued:
                # every lane with live events has `depth` runs in flight
                busy = [lane for lane in lanes if lane.live]
                if len(busy) == 1 and not (realtime and queue and not logical):
                    busy[0].inflight.popleft().synchronize()
                else:
                    time.sleep(0.0002)
                collect()
        for lane in lanes:
            lane.B.sync()
        return sorted(results, key=lambda r: r.finished)

    def _queue_run(self, lane: _Lane, pending: deque, runs_done: list, now) -> int:
        """Queues one run of the lane's chosen events, observes and retires
        those that finish in it; returns the HBM footprint released."""
        live = lane.live
        B = lane.B
        active = self._choose(lane)
        k = min(self.steps_to_stop(live[slot]["req"].work, live[slot]["done"], lane.run_steps)
                for slot in active)
        B.step(k)
        runs_done[0] += 1
        self.lane_runs[self.lanes.index(lane)] += 1
        finished = []
        for slot in sorted(active):
            ev = live[slot]
            ev["done"] += k
            w = ev["req"].work
            if self.observe_in_runs:
                # written by the run itself; the end, if it is no observation
                # step, from the host
                if ev["done"] >= w.steps and w.steps % w.observe_every != 0:
                    B.observe_async(slot)
            elif ((not self.final_only and ev["done"] % w.observe_every == 0)
                    or ev["done"] >= w.steps):
                B.observe_async(slot)
            if ev["done"] >= w.steps:
                finished.append(slot)
        freed = 0
        for slot in finished:
            ev = live.pop(slot)
            s = B.slots[slot]
            w = ev["req"].work
            t00, t0x = s["T00"], s["T0x"]
            if self.observe_in_runs and w.steps % w.observe_every == 0:
                obs = s["obs"]
                row = (w.steps // w.observe_every) % obs.shape[0]
                t00, t0x = obs[row, 0], obs[row, 1]
            with torch.cuda.stream(B.stream):
                h00 = torch.empty(t00.shape, dtype=torch.float64, pin_memory=True)
                h0x = torch.empty(t0x.shape, dtype=torch.float64, pin_memory=True)
                h00.copy_(t00, non_blocking=True)
                h0x.copy_(t0x, non_blocking=True)
                done_ev = torch.cuda.Event()
                done_ev.record(B.stream)
            fields = dict(rid=ev["req"].rid, n=ev["req"].work.n,
                          arrival=ev["req"].arrival, admitted=ev["admitted"],
                          admitted_run=ev["admitted_run"], finished_run=runs_done[0])
            if self.keep_states:
                fields["state"] = B.get_state(slot)
            pending.append((done_ev, fields, h00, h0x))
            B.retire(slot)
            freed += ev["need"]
        run_ev = torch.cuda.Event()
        run_ev.record(B.stream)
        lane.inflight.append(run_ev)
        return freed

    def steps_to_stop(self, work: W.Workload, done: int, run_steps: int | None = None) -> int:
        """Steps an event that has done `done` of its steps may take in the
        next run: at most run_steps, and never past its end or (unless only
        its final profile is wanted, or the runs write the observations) past
        its next observation."""
        k = min(self.run_steps if run_steps is None else run_steps, work.steps - done)
        if not self.final_only and not getattr(self, "observe_in_runs", False):
            k = min(k, work.observe_every - done % work.observe_every)
        return k

    def _choose(self, lane: _Lane) -> set:
        """The slots of the lane that take part in its next run (holding
        the others)."""
        live = lane.live
        policy = self.policy
        if policy == "classes":
            policy = "all" if lane is not self.lanes[0] else "fifo"
        if policy == "all":
            active = set(live)
        else:
            age = lambda s: (live[s]["req"].arrival, live[s]["req"].rid)
            size = lambda s: live[s]["req"].work.n
            left = lambda s: size(s) * (live[s]["req"].work.steps - live[s]["done"])
            if policy == "fifo":
                order = sorted(live, key=age)
                active, total = {order[0]}, size(order[0])
                for slot in order[1:]:
                    if total + size(slot) > self.run_particles:
                        break
                    active.add(slot)
                    total += size(slot)
                extra = 0
                for slot in sorted(live, key=left):
                    if slot in active or extra + size(slot) > self.fill_particles:
                        continue
                    active.add(slot)
                    extra += size(slot)
            else:
                oldest = min(live, key=age)
                active, total = {oldest}, size(oldest)
                for slot in sorted(live, key=left):
                    if slot == oldest or total + size(slot) > self.run_particles:
                        continue
                    active.add(slot)
                    total += size(slot)
        for slot, ev in live.items():
            want = slot in active
            if ev["active"] != want:
                lane.B.set_active(slot, want)
                ev["active"] = want
        self.peak_held = max(self.peak_held, len(live) - len(active))
        return active

    def close(self):
        for lane in self.lanes:
            lane.B.close()


def run_alone(req: Request, device: str = "cuda", keep_state: bool = False,
              final_only: bool = False):
    """The same request through the plain path: (service seconds, T00, T0x, state)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state = W.riemann_state_torch(req.work, req.state_seed, device=device)
    sim = Sim({**req.work.params(), "cell_capacity": W.capacity_for(req.work)}, state,
              device=device)
    del state
    w = req.work
    done = 0
    every = w.steps if final_only else w.observe_every
    while done < w.steps:
        k = min(every, w.steps - done)
        sim.step(k)
        done += k
        sim.observe_async()
    T00, T0x = sim.observe()
    st = sim.get_state() if keep_state else None
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.close()
    return dt, T00, T0x, st


def fifo_replay(requests: list[Request], service: dict) -> dict:
    """Completion times of a one-at-a-time FIFO server with the given
    service times and the requests' arrival times."""
    finish, t = {}, 0.0
    for r in sorted(requests, key=lambda r: r.arrival):
        t = max(t, r.arrival) + service[r.rid]
        finish[r.rid] = t
    return finish


def percentiles(lat):
    lat = np.asarray(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def measure(n_req: int, policy: str = "classes", run_steps: int = 25,
            final_only: bool = True, run_particles: int = 4_000_000,
            other_policies: tuple = (), sequential: bool = True, seed: int = 5,
            load: float = 0.8, fill_particles: int = 1_000_000,
            short_particles: int = 150_000) -> dict:
    """n_req requests (sizes 1e4 .. 4e6 test particles), Poisson arrivals at
    `load` of the server's batched capacity (measured on a closed batch of 64
    requests); p50/p99 time-to-result and aggregate particle-steps/s of the
    served stream against a one-at-a-time FIFO of plain runs on the same
    trace (each request's service time measured alone, the FIFO recurrence
    giving completion times).  other_policies: further policies served on
    the same trace, reported beside."""
    import sys
    from . import autotune as AT
    tuning = AT.load()

    def server(pol):
        return Server(tuning=tuning, use_graphs=False, policy=pol, run_steps=run_steps,
                      run_particles=run_particles, final_only=final_only,
                      fill_particles=fill_particles, short_particles=short_particles)

    # untimed warm-up of both paths (first launches load code objects and
    # grow the allocator's pools)
    warm = request_stream(16, 0.0, seed=56)
    srv = server(policy)
    srv.run(warm, realtime=False)
    srv.close()
    run_alone(warm[0], final_only=final_only)
    # capacity: a closed batch of 64 requests all present at t = 0
    probe = request_stream(64, 0.0, seed=55)
    srv = server("all")
    t0 = time.perf_counter()
    srv.run(probe, realtime=False)
    cap_dt = time.perf_counter() - t0
    srv.close()
    throughput = sum(r.work.n * r.work.steps for r in probe) / cap_dt
    reqs0 = request_stream(n_req, 1.0, seed=seed)
    mean_ps = float(np.mean([r.work.n * r.work.steps for r in reqs0]))
    rate = load * throughput / mean_ps
    reqs = request_stream(n_req, rate, seed=seed)
    print(f"# serve: {n_req} requests at {rate:.1f}/s (capacity {throughput:.3e} "
          f"particle-steps/s)", file=sys.stderr, flush=True)
    total_ps = sum(r.work.n * r.work.steps for r in reqs)
    out = {"metric": "served request stream: p50/p99 time-to-result and particle-steps/s",
           "unit": "particle-steps/s", "policy": policy, "run_steps": run_steps,
           "observed": "final profile" if final_only else "every 50 steps",
           "run_particles": run_particles, "fill_particles": fill_particles,
           "short_particles": short_particles if policy == "classes" else None,
           "requests": n_req, "load": load,
           "request_sizes": "1e4 .. 4e6 test particles, 200 steps",
           "arrival_rate_per_s": rate, "capacity_particle_steps_per_s": throughput}
    for pol in (policy,) + tuple(p for p in other_policies if p != policy):
        print(f"# serve policy {pol}", file=sys.stderr, flush=True)
        srv = server(pol)
        t0 = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        makespan = time.perf_counter() - t0
        peak = {"peak_live": srv.peak_live, "peak_bytes": srv.peak_bytes,
                "lane_runs": list(srv.lane_runs)}
        srv.close()
        assert len(res) == n_req
        p50, p99 = percentiles([r.latency for r in res])
        row = {"value": total_ps / makespan, "p50_s": p50, "p99_s": p99,
               "makespan_s": makespan, **peak}
        if pol == policy:
            out.update(row)
        else:
            out[pol] = row
    if sequential:
        print("# sequential FIFO replay", file=sys.stderr, flush=True)
        service = {}
        for r in reqs:
            service[r.rid] = run_alone(r, final_only=final_only)[0]
        fin = fifo_replay(reqs, service)
        lat = [fin[r.rid] - r.arrival for r in reqs]
        sp50, sp99 = percentiles(lat)
        out.update({"sequential_p50_s": sp50, "sequential_p99_s": sp99,
                    "sequential_value": total_ps / max(fin.values()),
                    "sequential_busy_particle_steps_per_s": total_ps / sum(service.values())})
        out["beats_fifo_p50"] = out["p50_s"] < sp50
        out["beats_fifo_p99"] = out["p99_s"] < sp99
    return out


def bench(a):
    """2000 requests (sizes 1e4 .. 4e6 test particles), Poisson arrivals at 0.8
    of the measured batched capacity; p50/p99 time-to-result and aggregate
    particle-steps/s of the served stream against a one-at-a-time FIFO of
    plain runs on the same trace."""
    import json
    out = measure(int(a.requests), policy=getattr(a, "serve_policy", "classes"),
                  run_steps=int(getattr(a, "serve_run_steps", 25)),
                  final_only=getattr(a, "serve_observe", "final") == "final",
                  run_particles=int(getattr(a, "serve_run_particles", 4_000_000)),
                  fill_particles=int(getattr(a, "serve_fill_particles", 1_000_000)),
                  short_particles=int(getattr(a, "serve_short_particles", 150_000)),
                  other_policies=Server.POLICIES,
                  sequential=not getattr(a, "no_sequential", False))
    print(json.dumps(out), flush=True)
