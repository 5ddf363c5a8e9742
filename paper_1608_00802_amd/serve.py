"""Continuous-batching request loop for independent particle-mesh runs.

Requests (mesh size, box size, boson mass, IC seed, number of steps) arrive
over time.  The loop admits them as device memory and slots free up, keeps
every admitted run resident on the GPU, and advances all of them together:

* mesh sizes up to ``batch_max_n`` run as slots of a ``PMBatch`` pool: one
  launch per kernel advances every active slot of the pool;
* larger meshes get a ``PMContext`` and a stream of their own, so their
  steps overlap with each other and with the pools' work.

Work is issued in chunks of steps.  A pool or run has at most ``inflight``
chunks queued on its stream; completion is found by polling events.  The
state of a finished run is checked for non-finite values and copied to the
host on a separate stream before its slot or memory is released.  A run
whose state went non-finite is reported as failed; a request that could
never fit the memory budget is refused, one that does not fit now waits.
Time to result runs from the request's arrival to the moment its state is
on the host.

Each run takes its own time steps: a Zel'dovich start at a = 0.01, uniform
steps in ln a towards a = 1, each shortened where needed so that no particle
moves more than c_x cells and the fastest linear quantum-pressure mode stays
stable (omega_max dt <= c_q), and at most the requested number of steps --
so a run in a small box or with a light boson stops short of a = 1 and
reports where it stopped.  The displacement bound needs the run's largest
velocity: it is reduced on the device after every chunk of steps, and chunk
j is planned with the value after chunk j - 2 (the newest one that has
always arrived when chunk j is issued), so a run's steps depend on its own
state only, never on what else is being served.

The scheduling logic is independent of the executor: ``FakeExecutor`` runs
it on a virtual clock without a GPU.

Command line: ``python -m paper_1608_00802_amd.serve --help``.
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import math
import time
from collections import deque

import numpy as np

A_START = 0.01
A_END = 1.0
# omega_max a^2 dx^2 / (hbar/m): the largest linear quantum-pressure
# frequency of the 7-point Laplacian with CIC interpolation on the mesh.
OMEGA_MAX_COEF = 1.1155
OMEGA_M = 0.3
LITTLE_H = 0.7


@dataclasses.dataclass
class Request:
    rid: int
    n: int              # mesh cells per side, n^3 particles
    box: float          # side length in Mpc/h
    m_ev: float         # boson mass in eV
    seed: int           # seed of the initial conditions
    nsteps: int         # most steps the run may take
    arrival: float      # seconds from the start of the trace


@dataclasses.dataclass
class Result:
    rid: int
    status: str         # "ok", "failed" or "refused"
    steps: int          # steps taken
    a_final: float      # scale factor reached
    arrival: float      # seconds on the loop's clock (after time compression)
    admitted: float
    finished: float
    pos: object = None  # host arrays [3, Np] when the executor keeps results
    vel: object = None
    times: list = None  # the scale factors of the run's steps

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_trace(n_requests: int = 200, rate: float = 4.0, seed: int = 2026,
               sizes=(32, 64, 128, 256), steps=(50, 200), box=(1.0, 10.0),
               log10_m=(-23.0, -21.0)) -> list:
    """Poisson arrivals at ``rate`` per second; per request a uniformly drawn
    mesh size, box and step count and a log-uniform boson mass.  The IC seed
    is the request id."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    out = []
    for i in range(n_requests):
        out.append(Request(rid=i, n=int(rng.choice(np.asarray(sizes))),
                           box=float(rng.uniform(*box)),
                           m_ev=float(10.0 ** rng.uniform(*log10_m)), seed=i,
                           nsteps=int(rng.integers(steps[0], steps[1] + 1)),
                           arrival=float(t[i])))
    return out


def hbar_over_m(m_ev: float, h: float = LITTLE_H) -> float:
    """hbar/m in (Mpc/h)^2 H0 for a boson mass in eV (one (Mpc/h)^2 H0 is
    100/h Mpc km/s)."""
    hbar_ev_s, c_kms, mpc_km = 6.582119569e-16, 299792.458, 3.0856775814913673e19
    return hbar_ev_s * c_kms ** 2 / m_ev / mpc_km * h / 100.0


def dlna_step(req: Request, a: float, vmax: float = 0.0, omega_m: float = OMEGA_M,
              c_q: float = 0.5, c_x: float = 1.0) -> float:
    """d ln a of the step starting at scale factor a (Sec. II A time-step
    condition: no particle moves more than a cell): ln(100)/nsteps,
    shortened so that a particle of canonical momentum vmax (cells H0) moves
    at most c_x cells (dx/dt = p/a^2, dt = d ln a / H) and so that
    omega_max dt <= c_q.  Both bounds are taken at the start of the step,
    where they are tightest within it in the matter era."""
    dx = req.box / req.n
    hm = hbar_over_m(req.m_ev) / (dx * dx)          # cells^2 H0
    hub = math.sqrt(omega_m / a ** 3 + 1.0 - omega_m)
    d = math.log(A_END / A_START) / req.nsteps
    if hm > 0:
        d = min(d, c_q * hub * a * a / (OMEGA_MAX_COEF * hm))
    if vmax > 0:
        d = min(d, c_x * a * a * hub / vmax)
    return d


def extend_times(req: Request, times: list, count: int, vmax: float = 0.0) -> int:
    """Append up to count scale factors to the run's schedule `times`
    (starting [0.01]), stopping at a = 1 or after nsteps steps; returns how
    many were added."""
    added = 0
    while added < count and len(times) <= req.nsteps and times[-1] < A_END:
        a = times[-1]
        nxt = a * math.exp(dlna_step(req, a, vmax))
        if nxt >= A_END * (1.0 - 1e-12):
            nxt = A_END
        times.append(nxt)
        added += 1
    return added


def schedule(req: Request, vmax: float = 0.0) -> list:
    """The whole schedule for a fixed velocity bound vmax (0: the quantum
    pressure and step-count bounds only)."""
    times = [A_START]
    extend_times(req, times, req.nsteps, vmax)
    return times


def footprint_bytes(n: int, precision: int | None = None) -> int:
    """Device bytes of one standalone run: workspace plus particles."""
    from ._lib import PM_FIXED32, make_params, pm_workspace_bytes
    p = make_params(n, n ** 3, 1.0, precision=PM_FIXED32 if precision is None else precision)
    return pm_workspace_bytes(p) + 24 * n ** 3


# ------------------------------------------------------------------ scheduler

class Scheduler:
    """First-come-first-served admission, chunked advancement, completion.

    The executor interface: ``fits(req)`` (could it ever run),
    ``can_admit(req)`` (can it start now), ``admit(req, state, arrival,
    now)``, ``advance(chunk) -> bool`` (whether new work was queued),
    ``poll(now) -> [Result]`` and ``busy()``.
    """

    def __init__(self, executor, chunk: int = 10):
        self.ex = executor
        self.chunk = chunk
        self.results = {}
        self.events = []            # (time, what, rid)

    def run(self, trace, ics, clock=time.perf_counter, sleep=time.sleep,
            time_scale: float = 1.0, idle: float = 2e-4) -> list:
        """Serve ``trace``; ``ics(req)`` returns the request's initial state.
        Arrival times are divided by ``time_scale`` (a compressed replay).
        Returns one Result per request, in trace order."""
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        queue = deque()
        t0 = clock()

        def now():
            return clock() - t0

        while pending or queue or self.ex.busy():
            t = now()
            while pending and pending[0].arrival / time_scale <= t:
                req = pending.popleft()
                if self.ex.fits(req):
                    queue.append(req)
                else:
                    self.results[req.rid] = Result(req.rid, "refused", 0, A_START,
                                                   req.arrival / time_scale, t, t)
                    self.events.append((t, "refuse", req.rid))
            # arrival order; a request that does not fit now holds back the
            # later requests of its own size only
            blocked = set()
            for req in list(queue):
                if req.n in blocked:
                    continue
                if not self.ex.can_admit(req):
                    blocked.add(req.n)
                    continue
                queue.remove(req)
                ta = now()
                try:
                    self.ex.admit(req, ics(req), req.arrival / time_scale, ta)
                    self.events.append((ta, "admit", req.rid))
                except MemoryError:
                    self.results[req.rid] = Result(req.rid, "failed", 0, A_START,
                                                   req.arrival / time_scale, ta, now())
                    self.events.append((ta, "admit-failed", req.rid))
            progressed = self.ex.advance(self.chunk)
            for res in self.ex.poll(now):
                self.results[res.rid] = res
                self.events.append((res.finished, "finish", res.rid))
            if not progressed:
                if pending and not queue and not self.ex.busy():
                    wait = pending[0].arrival / time_scale - now()
                    if wait > 0:
                        sleep(min(wait, 0.01))
                else:
                    sleep(idle)
        return [self.results[r.rid] for r in trace]


def summarize(results, trace) -> dict:
    """Latency percentiles and throughput of a served trace."""
    by_id = {r.rid: r for r in trace}
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.array([float("nan")])
    work = sum(by_id[r.rid].n ** 3 * r.steps for r in ok)
    span = (max(r.finished for r in results) - min(r.arrival for r in results)) if results else 0.0
    per_size = {}
    for n in sorted({q.n for q in trace}):
        ln = [r.latency for r in ok if by_id[r.rid].n == n]
        if ln:
            per_size[str(n)] = {"count": len(ln), "p50_s": float(np.percentile(ln, 50)),
                                "p99_s": float(np.percentile(ln, 99))}
    return {"requests": len(trace), "ok": len(ok),
            "failed": sum(r.status == "failed" for r in results),
            "refused": sum(r.status == "refused" for r in results),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": float(span),
            "particle_updates": int(work),
            "particle_updates_per_s": float(work / span) if span > 0 else float("nan"),
            "stopped_short_of_a1": int(sum(r.a_final < A_END for r in ok)),
            "per_size": per_size}


# ------------------------------------------------------------------ GPU executor

class _Chunk:
    __slots__ = ("event", "finishing")

    def __init__(self, event, finishing):
        self.event = event
        self.finishing = finishing


class GpuExecutor:
    """Runs admitted requests on one GPU through libfdmpm."""

    def __init__(self, device="cuda:0", batch_max_n: int = 64, pool_slots=None,
                 budget_bytes: int | None = None, max_large: int = 4, inflight: int = 2,
                 sort_every: int = 10, precision: int | None = None, keep_results: bool = False,
                 vmax_safety: float = 2.0, graphs: bool = True):
        import torch

        from . import _lib as pm
        self.torch = torch
        self.pm = pm
        self.device = torch.device(device)
        self.precision = pm.PM_FIXED32 if precision is None else precision
        self.fixed = self.precision == pm.PM_FIXED32
        self.batch_max_n = batch_max_n
        self.pool_slots = dict(pool_slots or {32: 64, 64: 32})
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.max_large = max_large
        self.inflight = inflight
        self.sort_every = sort_every
        self.keep_results = keep_results
        self.vmax_safety = vmax_safety
        # pool calls are captured in HIP graphs and replayed (PM_BATCH_GRAPH)
        self.graphs = graphs
        self.upload_stream = torch.cuda.Stream(self.device)
        self.copy_stream = torch.cuda.Stream(self.device)
        self.free_streams = []
        self.pools = {}             # n -> pool dict
        self.large = []             # active standalone runs
        self.copies = []            # result copies in flight
        self.used = 0

    # -- memory accounting
    def _run_bytes(self, n):
        return footprint_bytes(n, self.precision)

    def _pool_bytes(self, n, slots):
        pm = self.pm
        p = pm.make_params(n, n ** 3, 1.0, precision=self.precision, comoving=True)
        return pm.pm_batch_workspace_bytes(p, slots) + slots * 24 * n ** 3

    def _pooled(self, n):
        return n <= self.batch_max_n

    def fits(self, req):
        if self._pooled(req.n):
            return self._pool_bytes(req.n, 1) <= self.budget
        return self._run_bytes(req.n) <= self.budget

    def _reclaim_idle_pools(self):
        for n in [n for n, p in self.pools.items() if not p["runs"] and not p["chunks"]]:
            pool = self.pools.pop(n)
            pool["batch"].close()
            self.used -= pool["bytes"]

    def can_admit(self, req):
        if self._pooled(req.n):
            pool = self.pools.get(req.n)
            if pool is not None:
                return bool(pool["free"])
            need = self._pool_bytes(req.n, 1)
        else:
            if len(self.large) >= self.max_large:
                return False
            need = self._run_bytes(req.n)
        if self.used + need > self.budget:
            self._reclaim_idle_pools()
        return self.used + need <= self.budget

    # -- admission
    def _new_pool(self, n):
        pm, torch = self.pm, self.torch
        slots = self.pool_slots.get(n, 16)
        while slots > 1 and self.used + self._pool_bytes(n, slots) > self.budget:
            slots //= 2
        p = pm.make_params(n, n ** 3, 1.0, precision=self.precision, comoving=True,
                           omega_m=OMEGA_M, omega_l=1.0 - OMEGA_M, h0=1.0)
        stream = torch.cuda.Stream(self.device)
        with torch.cuda.stream(stream):
            batch = pm.PMBatch(p, slots, device=self.device, stream=stream)
        nbytes = self._pool_bytes(n, slots)
        self.used += nbytes
        pool = {"batch": batch, "free": list(range(slots)), "runs": {}, "chunks": deque(),
                "stream": stream, "bytes": nbytes}
        self.pools[n] = pool
        return pool

    def _upload(self, arrays, stream):
        """Host arrays -> device tensors usable on ``stream`` (copied on the
        idle upload stream, so the host never waits for queued steps)."""
        torch = self.torch
        with torch.cuda.stream(self.upload_stream):
            out = [torch.from_numpy(np.ascontiguousarray(a)).to(self.device) for a in arrays]
            ev = torch.cuda.Event()
            ev.record(self.upload_stream)
        stream.wait_event(ev)
        for t in out:
            t.record_stream(stream)
        return out

    def admit(self, req, state, arrival, now):
        torch, pm = self.torch, self.pm
        pos_np, vel_np = state[0], state[1]
        vm_ic = float(state[2]) if len(state) > 2 else float(np.abs(vel_np).max())
        run = {"req": req, "times": [A_START], "k": 0, "arrival": arrival, "admitted": now,
               "started": False, "issued_all": False, "vm_ic": vm_ic, "vm_after": []}
        hm = hbar_over_m(req.m_ev)
        if self._pooled(req.n):
            pool = self.pools.get(req.n) or self._new_pool(req.n)
            pos, vel = self._upload((pos_np, vel_np), pool["stream"])
            slot = pool["free"].pop(0)
            pool["batch"].load(slot, pos, vel, req.box, hm)
            run["slot"] = slot
            pool["runs"][slot] = run
            return
        stream = self.free_streams.pop() if self.free_streams else torch.cuda.Stream(self.device)
        p = pm.make_params(req.n, req.n ** 3, req.box, precision=self.precision, comoving=True,
                           omega_m=OMEGA_M, omega_l=1.0 - OMEGA_M, h0=1.0, hbar_over_m=hm)
        with torch.cuda.stream(stream):
            ctx = pm.PMContext(p, device=self.device, stream=stream)
        pos, vel = self._upload((pos_np, vel_np), stream)
        run.update(ctx=ctx, pos=pos, vel=vel, stream=stream, chunks=deque(),
                   bytes=self._run_bytes(req.n))
        self.used += run["bytes"]
        self.large.append(run)

    def _plan(self, run, chunk):
        """Extend the run's schedule by its next chunk; returns the steps.
        Chunk j is planned with the run's largest velocity after chunk j - 2
        (its reduction has always completed by the time chunk j is issued:
        at most two chunks are queued), times a safety factor for the
        growth since."""
        j = len(run["vm_after"])
        if j < 2:
            v = run["vm_ic"]
        else:
            ev, host, idx = run["vm_after"][j - 2]
            ev.synchronize()
            v = float(host[idx])
        kk = extend_times(run["req"], run["times"], chunk, self.vmax_safety * v)
        run["issued_all"] = (run["times"][-1] >= A_END or
                             len(run["times"]) - 1 >= run["req"].nsteps)
        return kk

    def busy(self):
        return bool(self.large or self.copies or
                    any(p["runs"] or p["chunks"] for p in self.pools.values()))

    # -- work
    def _flags(self, started, pooled=True):
        """Pools sort every sort_every steps; a standalone run in fixed point
        lets its context adapt the interval."""
        pm = self.pm
        if not self.sort_every:
            sort = 0
        elif not pooled and self.fixed:
            sort = pm.PM_SORT_AUTO
        else:
            sort = pm.PM_SORT_EVERY(self.sort_every)
        return sort | (pm.PM_CONTINUE if started else 0)

    def advance(self, chunk):
        torch = self.torch
        progressed = False
        for pool in self.pools.values():
            while len(pool["chunks"]) < self.inflight:
                ready = [r for r in pool["runs"].values() if not r["issued_all"]]
                if not ready:
                    break
                # one call per (first call or not, step count) group
                groups = {}
                for r in ready:
                    kk = self._plan(r, chunk)
                    groups.setdefault((r["started"], kk), []).append(r)
                finishing = []
                for (started, kk), runs in groups.items():
                    pool["batch"].step([r["slot"] for r in runs],
                                       [r["times"][r["k"]: r["k"] + kk + 1] for r in runs],
                                       self._flags(started) |
                                       (self.pm.PM_BATCH_GRAPH if self.graphs else 0))
                    for r in runs:
                        r["k"] += kk
                        r["started"] = True
                        if r["issued_all"]:
                            finishing.append(r)
                # every slot's largest velocity, for planning later chunks
                b = pool["batch"]
                with torch.cuda.stream(pool["stream"]):
                    vm = b.vel.abs().amax(dim=2).amax(dim=1)
                    host = torch.empty(vm.shape, dtype=vm.dtype, pin_memory=True)
                    host.copy_(vm, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(pool["stream"])
                for r in ready:
                    r["vm_after"].append((ev, host, r["slot"]))
                pool["chunks"].append(_Chunk(ev, finishing))
                progressed = True
        for run in self.large:
            while len(run["chunks"]) < self.inflight and not run["issued_all"]:
                kk = self._plan(run, chunk)
                run["ctx"].step(run["pos"], run["vel"], run["times"][run["k"]: run["k"] + kk + 1],
                                self._flags(run["started"], pooled=False))
                run["k"] += kk
                run["started"] = True
                with torch.cuda.stream(run["stream"]):
                    vm = run["vel"].abs().amax().reshape(1)
                    host = torch.empty(1, dtype=vm.dtype, pin_memory=True)
                    host.copy_(vm, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(run["stream"])
                run["vm_after"].append((ev, host, 0))
                run["chunks"].append(_Chunk(ev, [run] if run["issued_all"] else []))
                progressed = True
        return progressed

    def _start_copy(self, run, pos, vel, after, release):
        """Check a finished run's state for non-finite values and copy it to
        the host on the copy stream once ``after`` has completed; ``release``
        frees its slot or memory when the copy is done."""
        torch = self.torch
        cs = self.copy_stream
        with torch.cuda.stream(cs):
            cs.wait_event(after)
            ok = torch.isfinite(vel).all().reshape(1)
            h_ok = torch.empty(1, dtype=torch.bool, pin_memory=True)
            hp = torch.empty(pos.shape, dtype=pos.dtype, pin_memory=True)
            hv = torch.empty(vel.shape, dtype=vel.dtype, pin_memory=True)
            h_ok.copy_(ok, non_blocking=True)
            hp.copy_(pos, non_blocking=True)
            hv.copy_(vel, non_blocking=True)
            done = torch.cuda.Event()
            done.record(cs)
        self.copies.append((done, run, h_ok, hp, hv, release))

    def poll(self, now):
        for pool in self.pools.values():
            while pool["chunks"] and pool["chunks"][0].event.query():
                ch = pool["chunks"].popleft()
                for r in ch.finishing:
                    def release(pool=pool, slot=r["slot"]):
                        del pool["runs"][slot]
                        pool["free"].append(slot)
                    b = pool["batch"]
                    self._start_copy(r, b.pos[r["slot"]], b.vel[r["slot"]], ch.event, release)
        for run in list(self.large):
            while run["chunks"] and run["chunks"][0].event.query():
                ch = run["chunks"].popleft()
                if ch.finishing:
                    self.large.remove(run)

                    def release(run=run):
                        run["ctx"].close()
                        run["ctx"] = run["pos"] = run["vel"] = None
                        self.used -= run["bytes"]
                        self.free_streams.append(run["stream"])
                    self._start_copy(run, run["pos"], run["vel"], ch.event, release)
        out, still = [], []
        for item in self.copies:
            done, run, h_ok, hp, hv, release = item
            if not done.query():
                still.append(item)
                continue
            ok = bool(h_ok[0])
            req = run["req"]
            keep = ok and self.keep_results
            out.append(Result(req.rid, "ok" if ok else "failed", len(run["times"]) - 1,
                              run["times"][-1], run["arrival"], run["admitted"], now(),
                              hp.numpy() if keep else None, hv.numpy() if keep else None,
                              list(run["times"])))
            run["vm_after"] = []
            release()
        self.copies = still
        return out

    def close(self):
        self.torch.cuda.synchronize(self.device)
        for pool in self.pools.values():
            pool["batch"].close()
        self.pools.clear()
        for run in self.large:
            run["ctx"].close()
        self.large.clear()
        self.copies.clear()
        self.used = 0


class SerialExecutor(GpuExecutor):
    """Run-at-a-time baseline: one request on the GPU at a time, each with a
    context of its own (no batching, no overlap between runs)."""

    def __init__(self, device="cuda:0", **kw):
        kw["batch_max_n"] = 0
        kw["max_large"] = 1
        super().__init__(device, **kw)


# ------------------------------------------------------------------ virtual-clock executor

class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    """Stand-in for GpuExecutor on a virtual clock, for testing the loop.

    A chunk of k steps costs k (base + per_particle * particles in the
    chunk) virtual seconds on its pool or run; memory and slots are
    accounted like on the GPU (``run_bytes(n)`` per run and per pool slot,
    pools of ``pool_slots[n]`` slots, halved until they fit).
    ``compute(req, state, times)``, if given, produces the final state;
    requests in ``fail`` finish non-finite, those in ``oom`` raise
    MemoryError at admission.
    """

    def __init__(self, clock, batch_max_n=64, pool_slots=None, budget_bytes=1 << 30,
                 run_bytes=None, base=1e-4, per_particle=1e-9, max_large=4,
                 compute=None, fail=(), oom=()):
        self.clock = clock
        self.batch_max_n = batch_max_n
        self.pool_slots = dict(pool_slots or {32: 4, 64: 2})
        self.budget = budget_bytes
        self.run_bytes = run_bytes or (lambda n: 50 * n ** 3)
        self.base = base
        self.per_particle = per_particle
        self.max_large = max_large
        self.compute = compute
        self.fail = set(fail)
        self.oom = set(oom)
        self.pools = {}
        self.large = []
        self.used = 0
        self.peak_used = 0
        self.peak_active = 0

    def _pooled(self, n):
        return n <= self.batch_max_n

    def fits(self, req):
        return self.run_bytes(req.n) <= self.budget

    def can_admit(self, req):
        if self._pooled(req.n):
            pool = self.pools.get(req.n)
            if pool is not None:
                return bool(pool["free"])
        elif len(self.large) >= self.max_large:
            return False
        if self.used + self.run_bytes(req.n) > self.budget:
            for n in [n for n, p in self.pools.items() if not p["runs"]]:
                self.used -= self.pools.pop(n)["bytes"]
        return self.used + self.run_bytes(req.n) <= self.budget

    def admit(self, req, state, arrival, now):
        times = schedule(req)
        if req.rid in self.oom:
            raise MemoryError(f"request {req.rid}: injected allocation failure")
        run = {"req": req, "times": times, "k": 0, "arrival": arrival, "admitted": now,
               "state": state}
        if self._pooled(req.n):
            if req.n not in self.pools:
                slots = self.pool_slots.get(req.n, 2)
                while slots > 1 and self.used + slots * self.run_bytes(req.n) > self.budget:
                    slots //= 2
                nbytes = slots * self.run_bytes(req.n)
                self.used += nbytes
                self.pools[req.n] = {"free": list(range(slots)), "runs": {}, "busy_until": 0.0,
                                     "bytes": nbytes, "finishing": []}
            pool = self.pools[req.n]
            run["slot"] = pool["free"].pop(0)
            pool["runs"][run["slot"]] = run
        else:
            self.used += self.run_bytes(req.n)
            run["busy_until"] = 0.0
            run["finishing"] = False
            self.large.append(run)
        self.peak_used = max(self.peak_used, self.used)
        self.peak_active = max(self.peak_active, len(self.large) +
                               sum(len(p["runs"]) for p in self.pools.values()))

    def busy(self):
        return bool(self.large or any(p["runs"] for p in self.pools.values()))

    def advance(self, chunk):
        t = self.clock()
        progressed = False
        for n, pool in self.pools.items():
            ready = [r for r in pool["runs"].values() if r["k"] < len(r["times"]) - 1]
            if ready and pool["busy_until"] <= t and not pool["finishing"]:
                most = 0
                for r in ready:
                    kk = min(chunk, len(r["times"]) - 1 - r["k"])
                    r["k"] += kk
                    most = max(most, kk)
                    if r["k"] == len(r["times"]) - 1:
                        pool["finishing"].append(r)
                pool["busy_until"] = t + most * (self.base + n ** 3 * len(ready) *
                                                 self.per_particle)
                progressed = True
        for r in self.large:
            if r["k"] < len(r["times"]) - 1 and r["busy_until"] <= t:
                kk = min(chunk, len(r["times"]) - 1 - r["k"])
                r["k"] += kk
                r["busy_until"] = t + kk * (self.base + r["req"].n ** 3 * self.per_particle)
                r["finishing"] = r["k"] == len(r["times"]) - 1
                progressed = True
        return progressed

    def _result(self, r, now):
        req = r["req"]
        ok = req.rid not in self.fail
        pos = vel = None
        if ok and self.compute is not None:
            pos, vel = self.compute(req, r["state"], r["times"])
        return Result(req.rid, "ok" if ok else "failed", len(r["times"]) - 1, r["times"][-1],
                      r["arrival"], r["admitted"], now(), pos, vel, list(r["times"]))

    def poll(self, now):
        t = self.clock()
        out = []
        for pool in self.pools.values():
            if pool["busy_until"] <= t and pool["finishing"]:
                for r in pool["finishing"]:
                    out.append(self._result(r, now))
                    del pool["runs"][r["slot"]]
                    pool["free"].append(r["slot"])
                pool["finishing"] = []
        for r in list(self.large):
            if r["finishing"] and r["busy_until"] <= t:
                out.append(self._result(r, now))
                self.large.remove(r)
                self.used -= self.run_bytes(r["req"].n)
        return out


# ------------------------------------------------------------------ client side

def make_ic(n, box, m_ev, seed, fp32=False):
    """Zel'dovich initial state of one request: (positions, velocities,
    largest velocity component), arrays [3, Np]; positions fixed point
    (int32 bit patterns) or float32 cells."""
    from synth import zeldovich_state
    st = zeldovich_state(n, box, A_START, seed, m_ev=m_ev, om=OMEGA_M, h=LITTLE_H)
    pos = st.pos_f32 if fp32 else np.ascontiguousarray(st.pos_fixed.view(np.int32))
    vel = np.ascontiguousarray(st.vel32)
    return pos, vel, float(np.abs(vel).max())


def _make_ic_job(job):
    return make_ic(*job)


def generate_ics(trace, workers: int = 8, fp32: bool = False) -> dict:
    """Initial states of every request, built before the clock starts (the
    client's side of the exchange), keyed by request id."""
    jobs = [(r.n, r.box, r.m_ev, r.seed, fp32) for r in trace]
    if workers <= 1:
        states = [_make_ic_job(j) for j in jobs]
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            states = list(ex.map(_make_ic_job, jobs, chunksize=1))
    return {r.rid: s for r, s in zip(trace, states)}


def fp32_ics(ics: dict, trace) -> dict:
    """The same initial states with float32 cell positions (the input of
    the plain FP32 form)."""
    from synth import State
    by_id = {r.rid: r for r in trace}
    return {rid: (State(by_id[rid].n, pos.view(np.uint32), vel, {}).pos_f32, vel, vm)
            for rid, (pos, vel, vm) in ics.items()}


def serve_trace(trace, ics, executor, time_scale=1.0, chunk=10):
    """Serve ``trace`` on ``executor`` (initial states from the dict
    ``ics``); returns (results, summary)."""
    sched = Scheduler(executor, chunk=chunk)
    results = sched.run(trace, lambda r: ics[r.rid], time_scale=time_scale)
    return results, summarize(results, trace)


def run_modes(trace, ics, scales=(1.0, 10.0, 100.0), serial=True, chunk=10, emit=print,
              eager=False):
    """Serve the trace batched at each time compression (pool calls replayed
    from HIP graphs; with ``eager`` also launched call by call), then
    (optionally) one request at a time in fixed point and in plain FP32 with
    all requests queued at once; ``emit`` receives one summary dict per mode."""
    out = []
    for scale in scales:
        for mode, graphs in (("batched", True), ("batched_eager", False))[:2 if eager else 1]:
            ex = GpuExecutor(graphs=graphs)
            _, summ = serve_trace(trace, ics, ex, scale, chunk)
            ex.close()
            out.append({"mode": mode, "time_scale": scale, **summ})
            emit(out[-1])
    if serial:
        from ._lib import PM_FP32
        for name, states, prec in (("serial_fixed", ics, None),
                                   ("serial_fp32", fp32_ics(ics, trace), PM_FP32)):
            ex = SerialExecutor(precision=prec)
            _, summ = serve_trace(trace, states, ex, 1e9, chunk)
            ex.close()
            out.append({"mode": name, "time_scale": None, **summ})
            emit(out[-1])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="Serve a synthetic request trace on the GPU.")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=4.0, help="arrivals per second")
    ap.add_argument("--seed", type=int, default=2026)
    ap.add_argument("--sizes", default="32,64,128,256")
    ap.add_argument("--scales", default="1,10,100", help="time compressions to replay")
    ap.add_argument("--no-serial", action="store_true",
                    help="skip the one-request-at-a-time baselines")
    ap.add_argument("--workers", type=int, default=16, help="IC generation processes")
    ap.add_argument("--chunk", type=int, default=10)
    a = ap.parse_args(argv)
    trace = make_trace(a.requests, a.rate, a.seed, tuple(int(s) for s in a.sizes.split(",")))
    # initial states first, before this process touches the GPU
    t0 = time.perf_counter()
    ics = generate_ics(trace, a.workers)
    print(json.dumps({"ics_s": round(time.perf_counter() - t0, 2), "requests": len(trace)}),
          flush=True)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("serve: needs a GPU")
    run_modes(trace, ics, [float(s) for s in a.scales.split(",")], not a.no_serial, a.chunk,
              emit=lambda d: print(json.dumps(d), flush=True))


if __name__ == "__main__":
    main()
