"""Serving loop: a seeded stream of solver requests run by continuous batching.

Requests (cubic boxes of different sizes, droplet or jet set-ups, different
Re and We) arrive as a Poisson process.  The loop admits arrived requests in
FIFO order while the HBM budget (by default the device's free memory when the
stream starts, less a reserve) and the domain slots allow, and every poll of
the group launches one step of all admitted requests together (one
multi-domain kernel launch), so requests that arrive while others run share
the device from their first step on.  A request's latency is the time from its
arrival to its retirement; throughput is the total node updates over the
makespan.

The loop talks to a backend with a few calls (``required_bytes``, ``create``,
``admit``, ``poll``, ``finish``, and ``admission_budget`` when no budget is
given); :class:`GpuBackend` drives the C-ABI group (``tslb_group_*``).
Nothing here computes any part of the method.
"""
from __future__ import annotations

import collections
import math
import time
import concurrent.futures
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import inputs

SIZES = (32, 48, 64, 96, 128)
U = 0.05


@dataclass
class Request:
    id: int
    arrival: float  # seconds after the start of the stream
    L: int          # box side
    setup: str      # "droplet" or "jet"
    re: float
    we: float
    steps: int
    seed: int


def _uniform(seed, comp, n=1):
    """n uniform draws in [0, 1) from the counter hash (stream 3, node 0)."""
    xi = inputs.noise(seed, 3, 0, np.arange(n, dtype=np.uint64), comp)
    return (np.asarray(xi, np.float64) + 1.0) * 0.5


def make_requests(n=256, rate=20.0, master_seed=5, sizes=SIZES, re=(500.0, 5000.0), we=(10.0, 2000.0),
                  steps=(500, 5000)):
    """The seeded request stream: Poisson arrivals at ``rate`` per second, side
    uniform over ``sizes``, set-up droplet/jet 50/50, Re and We log-uniform,
    steps uniform over the integer range.  Request i draws from the counter
    hash keyed by mix(master_seed, i); the arrival gaps from master_seed."""
    gaps = -np.log1p(-_uniform(master_seed, 0, n)) / rate
    t = np.cumsum(gaps) - gaps[0]  # the first request arrives at t = 0
    reqs = []
    for i in range(n):
        seed = int(inputs.splitmix64_next(np.uint64(master_seed) ^ np.uint64(i)))
        u = _uniform(seed, 1, 5)
        L = sizes[min(int(u[0] * len(sizes)), len(sizes) - 1)]
        setup = "droplet" if u[1] < 0.5 else "jet"
        r = math.exp(math.log(re[0]) + u[2] * (math.log(re[1]) - math.log(re[0])))
        w = math.exp(math.log(we[0]) + u[3] * (math.log(we[1]) - math.log(we[0])))
        nst = steps[0] + min(int(u[4] * (steps[1] - steps[0] + 1)), steps[1] - steps[0])
        reqs.append(Request(i, float(t[i]), L, setup, r, w, nst, seed))
    return reqs


def request_setup(req: Request):
    """(lattice parameters, initial physical fields as float32) of a request.
    Jet: D = L/8, inlet on z = 0, outflow on z = L-1, free-slip sides,
    nu = U D / Re, sigma = U^2 D / We, 1 % inlet noise.  Droplet: periodic,
    R = L/4, W = 3, nu = U 2R / Re, sigma = U^2 2R / We, velocity noise 1e-3."""
    L = req.L
    if req.setup == "jet":
        d = L / 8.0
        p = inputs.jet_params(L, L, L, d=d, u=U, re=req.re, we=req.we, width=3.0, noise=0.01, seed=req.seed)
        st = inputs.quiescent(L, L, L)
    else:
        R = L / 4.0
        p = inputs.droplet_params(L, nu=U * 2 * R / req.re, sigma=U * U * 2 * R / req.we, width=3.0)
        st = inputs.droplet(L, R, 3.0, noise_amp=1e-3, seed=req.seed)
    fields = {"rho_dev": np.asarray(st["rho"] - 1.0, np.float32), "u": np.asarray(st["u"], np.float32),
              "P": np.asarray(st["P"], np.float32), "phi": np.asarray(st["phi"], np.float32)}
    return p, fields


@dataclass
class Record:
    req: Request
    admitted: float = math.nan
    done: float = math.nan
    finite: bool = True
    extra: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.done - self.req.arrival


def _create(backend, req, prepared):
    return backend.create(req, prepared.result())


def serve(requests, backend, budget_bytes=None, max_domains=64, clock=time.perf_counter, sleep=time.sleep,
          prepare_workers=4, on_done=None):
    """Run the stream; return one Record per request (in request order).

    Arrived requests wait in a FIFO queue; the head is admitted when its state
    bytes fit the budget next to the running ones and a slot is free (a head
    that does not fit blocks the queue: no overtaking).  budget_bytes None
    takes ``backend.admission_budget()`` (the device's free memory less a
    reserve).  Host-side initial fields are prepared by a thread pool as
    requests arrive.  Creating a request's lattice (device allocation, upload
    of its fields) and finishing a retired one (diagnostics, release) run on
    one worker thread, so the loop that keeps the device's launch queue filled
    never waits for them.  Lattices are admitted in the order their creation
    started: one the device refuses stays first in line and is offered again
    after the next poll, and no later lattice is admitted before it."""
    if budget_bytes is None:
        budget_bytes = backend.admission_budget()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue = collections.deque()
    recs = {r.id: Record(r) for r in requests}
    active = {}          # handle key -> (Record, bytes)
    creating = collections.deque()  # (request, bytes, future of the handle), FIFO
    finishing = []       # (Record, future of the finish info)
    in_use = 0
    idle_refusals = 0
    pool = ThreadPoolExecutor(max_workers=max(1, prepare_workers))
    worker = ThreadPoolExecutor(max_workers=1)
    futures = {}
    t0 = clock()

    def collect(block):
        for item in list(finishing):
            rec, fut = item
            if block or fut.done():
                info = fut.result()
                rec.finite = bool(info.get("finite", True))
                rec.extra = info
                finishing.remove(item)
                if on_done:
                    on_done(rec)

    try:
        while pending or queue or active or creating:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                queue.append(r)
                futures[r.id] = pool.submit(backend.prepare, r)
            while queue and len(active) + len(creating) < max_domains:
                r = queue[0]
                need = backend.required_bytes(r)
                if in_use + need > budget_bytes:
                    if not active and not creating:
                        raise ValueError("request %d needs %d bytes, more than the budget of %d"
                                         % (r.id, need, budget_bytes))
                    break
                queue.popleft()
                in_use += need
                creating.append((r, need, worker.submit(_create, backend, r, futures.pop(r.id))))
            while creating and creating[0][2].done():
                r, need, fut = creating[0]
                h = fut.result()
                if not backend.admit(h, r.steps):
                    # the device refused (its own budget or slots): the lattice keeps
                    # its place and is offered again after members retire; an idle
                    # device that refuses it twice never will take it
                    idle_refusals = idle_refusals + 1 if not active else 0
                    if idle_refusals >= 2:
                        raise RuntimeError("request %d was refused by an idle device" % r.id)
                    break
                idle_refusals = 0
                creating.popleft()
                recs[r.id].admitted = clock() - t0
                active[backend.key(h)] = (recs[r.id], need)
            if active:
                for h in backend.poll():
                    rec, need = active.pop(backend.key(h))
                    rec.done = clock() - t0
                    in_use -= need
                    finishing.append((rec, worker.submit(backend.finish, h)))
            elif creating:
                concurrent.futures.wait([creating[0][2]], timeout=0.002)
            elif pending and not queue:
                sleep(max(0.0, min(0.05, pending[0].arrival - (clock() - t0))))
            collect(False)
        collect(True)
    finally:
        pool.shutdown(wait=True)
        worker.shutdown(wait=True)
    return [recs[r.id] for r in requests]


def summarise(records, busy_s=None):
    """p50/p99 latency (s), makespan, aggregate GLUPS, the offered load (node
    updates requested per second of arrivals), counts and, given the device's
    busy seconds, the fraction of the makespan the device was busy."""
    lat = np.array([r.latency for r in records], np.float64)
    start = min(r.req.arrival for r in records)
    end = max(r.done for r in records)
    last_arrival = max(r.req.arrival for r in records)
    updates = float(sum(r.req.L ** 3 * r.req.steps for r in records))
    span = end - start
    return {
        "requests": len(records),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "makespan_s": float(span),
        "node_updates": updates,
        "aggregate_glups": updates / span / 1e9 if span > 0 else math.nan,
        "offered_glups": updates / (last_arrival - start) / 1e9 if last_arrival > start else math.nan,
        "device_busy_frac": busy_s / span if (busy_s is not None and span > 0) else None,
        "unstable": int(sum(1 for r in records if not r.finite)),
    }


class GpuBackend:
    """Backend over the C-ABI serving group (``tslb_group_*``)."""

    def __init__(self, group, device=0, check_finite=True):
        from . import tslb
        self.tslb = tslb
        self.group = group
        self.device = device
        self.check_finite = check_finite

    def prepare(self, req):
        return request_setup(req)

    def admission_budget(self, reserve_frac=1.0 / 16):
        """The device's free memory now, less reserve_frac of its total."""
        free, total = self.tslb.device_memory(self.device)
        return max(0, free - int(total * reserve_frac))

    def busy_seconds(self):
        """Summed device time of the group's completed launches."""
        ms, _ = self.group.busy()
        return ms * 1e-3

    def required_bytes(self, req):
        p, _ = request_setup_params_only(req)
        return self.tslb.required_bytes(self.tslb.make_params(**p, device=self.device))

    def create(self, req, prepared):
        p, f = prepared
        sim = self.tslb.Simulation(**p, device=self.device)
        sim.set_state(**f)
        sim.request_id = req.id
        return sim

    def admit(self, sim, nsteps):
        return self.group.admit(sim, nsteps)

    def key(self, sim):
        return sim.h.value

    def poll(self):
        return self.group.poll()

    def finish(self, sim):
        info = {"step": sim.step_index}
        if self.check_finite:
            d = sim.diagnostics()
            info.update(finite=d["finite"], mass=d["mass"], phase=d["phase"])
        sim.close()
        return info


def request_setup_params_only(req: Request):
    """Lattice parameters of a request without building its fields."""
    L = req.L
    if req.setup == "jet":
        d = L / 8.0
        return inputs.jet_params(L, L, L, d=d, u=U, re=req.re, we=req.we, width=3.0, noise=0.01,
                                 seed=req.seed), None
    R = L / 4.0
    return inputs.droplet_params(L, nu=U * 2 * R / req.re, sigma=U * U * 2 * R / req.we, width=3.0), None
