"""Serving form: independent channel-flow solves arriving over time, continuously batched.

Requests of different meshes, velocity grids and Knudsen numbers arrive (Poisson).  The
server admits them in arrival order while its HBM budget and slot count allow, keeps their
f/W state resident on the GPU, and advances every resident request together: one
``ugks_step_batch`` call packs all of them into one launch per phase.  A request that arrives
while a batch is running is admitted (its solver created on a separate stream) before the
server waits for that batch, so admission overlaps the device work.  A request leaves after
its step count, with its moments copied to the host; its latency is arrival -> result on the
host.  A request whose state turns invalid fails alone.  A request can be cancelled at any
time (``Server.cancel``, or ``Request.cancel_at``): a queued one is dropped, a running one
leaves at the end of the batch in flight, its solver released and its memory returned.

``Server`` is independent of the GPU: it drives any executor with ``footprint``, ``create``,
``step``, ``wait``, ``finish`` and ``release``.  ``GpuExecutor`` is the one that runs here.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import workloads as WL


@dataclass
class Request:
    rid: int
    case: dict          # workload fields (mesh, velocity grid, kn, boundary, seed, ...)
    steps: int
    arrival: float      # seconds after the start of the run
    precision: str = "fp32_store"
    status: str = "queued"   # queued, running, done, failed, rejected, cancelled
    cancel_at: float = None  # the client cancels the request at this time (run clock), if set
    admitted: float = None
    finished: float = None
    result: np.ndarray = field(default=None, repr=False)
    error: str = None

    @property
    def updates(self):
        return WL.updates(self.case) * self.steps

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


MESHES = [(50, 12), (100, 25), (200, 50), (400, 100)]
VGRIDS = [24, 32, 48]


def serving_requests(n, rate, seed=4, steps=500, precision="fp32_store", meshes=MESHES,
                     vgrids=VGRIDS):
    """Seeded request stream shaped like the serving workload: mesh uniform over `meshes`
    (4 x 1 channel), square velocity grid over `vgrids` on [-6, 6]^2, Kn log-uniform in
    [0.01, 1], pressure ratio uniform in [1.5, 3], 1% density noise, Poisson arrivals at
    `rate` per second (rate = inf: all at t = 0)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        if math.isfinite(rate):
            t += rng.exponential(1.0 / rate)
        nx, ny = meshes[rng.integers(len(meshes))]
        nv = vgrids[rng.integers(len(vgrids))]
        kn = float(10.0 ** rng.uniform(-2.0, 0.0))
        ratio = float(rng.uniform(1.5, 3.0))
        case = dict(WL.CHANNEL_DEFAULTS, nx=nx, ny=ny, lx=4.0, ly=1.0, nu=nv, nv=nv, umax=6.0,
                    vmax=6.0, kn=kn, p_ratio=ratio, noise=0.01, seed=1000 + rid)
        out.append(Request(rid, case, steps, 0.0 if not math.isfinite(rate) else t,
                           precision))
    return out


class GpuExecutor:
    """Runs requests as UGKS solvers on the current GPU, stepped together: one batch per
    storage precision and collision model (BGK or Shakhov) present, all on one stream, so a
    step of the resident requests is one launch per phase and group.
    ``velocity_chunks`` caps every solver's moment-kernel velocity chunks (0: automatic).  A
    batch of resident requests fills the GPU by itself, so the default 1 saves the per-chunk
    setup and the chunk-sum pass: on the 256-request serving workload it saturated 2.5% higher
    than a cap of 4 and halved the p50 latency at 0.8 of that rate, for 10% more p50 latency
    at half of it."""

    def __init__(self, max_slots, velocity_chunks=1):
        import torch

        from . import ugks

        self.torch = torch
        self.ugks = ugks
        self.run_stream = torch.cuda.Stream()
        self.admit_stream = torch.cuda.Stream()
        self.max_slots = max_slots
        self.batches = {}   # (precision, Shakhov model) -> Batch
        self.velocity_chunks = int(velocity_chunks)
        self.done_event = None

    def footprint(self, req):
        kn, kw = WL.solver_kwargs(req.case, req.precision)
        mesh, vgrid, bc, opts = self.ugks.make_structs(velocity_chunks=self.velocity_chunks, **kw)
        return self.ugks.ugks_required_bytes(mesh, vgrid, opts)

    @staticmethod
    def group_of(req):
        pr = req.case.get("prandtl", 1.0)
        return (req.precision, 0.0 < pr < 1.0)

    def create(self, req):
        kn, kw = WL.solver_kwargs(req.case, req.precision)
        with self.torch.cuda.stream(self.admit_stream):
            s = self.ugks.Solver(kn, stream=self.admit_stream,
                                 velocity_chunks=self.velocity_chunks, **kw)
        s.serving_group = self.group_of(req)
        return s

    def step(self, solvers, n):
        groups = {}
        for s in solvers:
            groups.setdefault(s.serving_group, []).append(s)
        for key in sorted(groups):
            if key not in self.batches:
                self.batches[key] = self.ugks.Batch(self.max_slots, stream=self.run_stream)
            self.batches[key].step(groups[key], n)
        ev = self.torch.cuda.Event()
        ev.record(self.run_stream)
        self.done_event = ev

    def wait(self):
        if self.done_event is not None:
            self.done_event.synchronize()

    def finish(self, solver):
        return solver.moments()

    def release(self, solver):
        solver.close()

    def close(self):
        for b in self.batches.values():
            b.close()
        self.batches = {}


class Server:
    """Continuous batching with FIFO admission by memory footprint.

    ``quantum`` caps the steps of one batch: a request that arrives while a batch runs joins
    the next one.  ``admit_per_round`` caps the solvers created between two batches, so that a
    burst of arrivals is created while the first of them already run (creation overlaps the
    device work instead of delaying it)."""

    def __init__(self, executor, budget_bytes, max_slots=256, quantum=50, admit_per_round=16,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.quantum = int(quantum)
        self.admit_per_round = max(1, int(admit_per_round))
        self.clock = clock
        self.sleep = sleep
        self.batches = 0
        self.max_resident = 0
        self.host_s = {}
        self._cancel = set()   # request ids cancelled through cancel()

    def cancel(self, rid):
        """Cancel request `rid` (safe to call from another thread while run() executes): a
        queued request is dropped at the next admission round, a running one after the batch
        in flight."""
        self._cancel.add(rid)

    def run(self, requests):
        pending = sorted(requests, key=lambda r: r.arrival)
        queue, active = [], []   # active entries: [request, solver, steps done, bytes]
        used = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0
        host = {"create": 0.0, "step": 0.0, "wait": 0.0, "finish": 0.0}
        self.host_s = host

        def timed(part, fn, *a):
            s0 = self.clock()
            try:
                return fn(*a)
            finally:
                host[part] += self.clock() - s0

        def cancelled(r):
            return r.rid in self._cancel or (r.cancel_at is not None and now() >= r.cancel_at)

        def drop_cancelled():
            # requests not yet admitted leave at once; running ones leave between batches
            for lst in (pending, queue):
                for r in [r for r in lst if cancelled(r)]:
                    lst.remove(r)
                    r.status, r.finished = "cancelled", now()

        def admit():
            nonlocal used
            drop_cancelled()
            while pending and pending[0].arrival <= now():
                queue.append(pending.pop(0))
            created = 0
            while queue and len(active) < self.max_slots and created < self.admit_per_round:
                r = queue[0]
                need = self.ex.footprint(r)
                if need > self.budget:
                    r.status, r.error = "rejected", "footprint exceeds the HBM budget"
                    queue.pop(0)
                    continue
                if used + need > self.budget:
                    break
                queue.pop(0)
                try:
                    s = timed("create", self.ex.create, r)
                except Exception as e:  # a request that cannot start fails alone
                    r.status, r.error = "failed", str(e)
                    continue
                used += need
                created += 1
                r.status, r.admitted = "running", now()
                active.append([r, s, 0, need])
            self.max_resident = max(self.max_resident, len(active))

        while pending or queue or active:
            admit()
            # resident requests cancelled since the last batch (no batch is in flight here)
            for entry in [e for e in active if cancelled(e[0])]:
                r, s, _, need = entry
                r.status, r.finished = "cancelled", now()
                self.ex.release(s)
                used -= need
                active.remove(entry)
            if not active:
                if pending:
                    self.sleep(max(0.0, min(pending[0].arrival - now(), 0.05)))
                    continue
                break
            q = min(self.quantum, min(r.steps - d for r, _, d, _ in active))
            members = list(active)
            timed("step", self.ex.step, [s for _, s, _, _ in members], q)
            self.batches += 1
            admit()            # requests arriving meanwhile start while the batch runs
            timed("wait", self.ex.wait)
            stepped = {id(e) for e in members}
            still = []
            for entry in active:
                if id(entry) not in stepped:   # admitted during the batch: not stepped yet
                    still.append(entry)
                    continue
                r, s, d, need = entry
                entry[2] = d = d + q
                if d < r.steps and cancelled(r):   # cancelled while the batch ran
                    r.status, r.finished = "cancelled", now()
                    self.ex.release(s)
                    used -= need
                elif d >= r.steps:
                    try:
                        r.result = timed("finish", self.ex.finish, s)
                        r.status = "done"
                    except Exception as e:      # an invalid state fails this request alone
                        r.status, r.error = "failed", str(e)
                    r.finished = now()
                    self.ex.release(s)
                    used -= need
                else:
                    still.append(entry)
            active = still
        return summarize(requests, now())


def summarize(requests, makespan):
    done = [r for r in requests if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(0)
    upd = float(sum(r.updates for r in done))
    return {
        "requests": len(requests),
        "done": len(done),
        "failed": sum(r.status == "failed" for r in requests),
        "rejected": sum(r.status == "rejected" for r in requests),
        "cancelled": sum(r.status == "cancelled" for r in requests),
        "makespan_s": makespan,
        "p50_latency_s": float(np.percentile(lat, 50)) if done else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if done else None,
        "mean_latency_s": float(lat.mean()) if done else None,
        "updates": upd,
        "updates_per_s": upd / makespan if makespan > 0 else None,
    }
