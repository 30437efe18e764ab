"""Serving loop for shear-rate sweep requests (continuous batching on one GPU).

Requests (independent Lees-Edwards simulations of different size and shear
rate) arrive over time.  The server admits a request when its device
footprint (workspace + sample ring) fits the HBM budget and a slot is free,
gives it its own HIP stream, and advances every admitted simulation in
chunks of steps, so the work of several requests overlaps on the device.  A
request finishes when its steps are done; its result is the sampled shear
stress series and the viscosity estimate.  Time-to-result is completion
minus arrival.

Each simulation is deterministic and independent of the others (own
workspace, own stream, own Philox key), so its result is the same alone and
in the mix.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import inputs
from .sim import Params, Sim


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    n: int
    shear_rate: float
    steps: int
    seed: int
    precision: str = "fp64"
    skin: float = 0.4
    sample_every: int = 10


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    n: int
    steps: int
    shear_rate: float
    eta: float
    stress: np.ndarray      # [samples][6]
    state_x: np.ndarray | None = None
    state_u: np.ndarray | None = None
    eta_se: float | None = None  # standard error of eta from 10 blocks of the window

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def sweep_trace(count=64, rate=4.0, n_lo=2000, n_hi=64000, sr_lo=1e-3, sr_hi=1.0, steps=5000,
                seed=41, precision="fp64", burst=False):
    """Requests with N ~ U{n_lo..n_hi}, shear rate log-uniform, Poisson arrivals
    (mean gap 1/rate; all at t = 0 when burst)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        if not burst:
            t += float(rng.exponential(1.0 / rate))
        n = int(rng.integers(n_lo, n_hi + 1))
        sr = float(math.exp(rng.uniform(math.log(sr_lo), math.log(sr_hi))))
        out.append(Request(k, 0.0 if burst else t, n, sr, steps, 100 * seed + k, precision))
    return out


def request_params(r: Request) -> tuple:
    w = inputs.lj_workload(n=r.n, shear_rate=r.shear_rate, seed=r.seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=r.shear_rate, seed=r.seed, skin=r.skin,
               precision=r.precision, rc=2.5, dt=0.005, kT=1.0, gamma=1.0)
    return w, p


def footprint(p: Params, r: Request) -> int:
    from .sim import workspace_bytes
    return workspace_bytes(p) + (r.steps // r.sample_every + 1) * 6 * 8 + 6 * p.n * 8


class _Active:
    def __init__(self, req: Request, sim: Sim, ring: torch.Tensor, admitted: float, nbytes: int):
        self.req = req
        self.sim = sim
        self.ring = ring
        self.admitted = admitted
        self.nbytes = nbytes
        self.issued = 0         # steps enqueued
        self.events = []        # (steps covered, event) per enqueued chunk
        self.graph = None       # captured chunk (HIP graph) and its sample rows
        self.graph_ring = None


class Server:
    """Continuous-batching server.  hbm_budget: bytes the admitted requests may
    hold; max_active: concurrent simulations (streams); chunk: steps per
    enqueue; keep_state: copy the final state of each request (tests)."""

    def __init__(self, hbm_budget=16 << 30, max_active=16, chunk=500, ahead=2, keep_state=False,
                 graphs=True):
        self.hbm_budget = hbm_budget
        self.max_active = max_active
        self.chunk = chunk
        self.ahead = ahead
        self.keep_state = keep_state
        self.graphs = graphs

    def _enqueue(self, a: _Active):
        r = a.req
        k = min(self.chunk, r.steps - a.issued)
        if k <= 0:
            return
        # samples of this chunk land at ring rows [issued/sample_every, ...)
        row0 = a.issued // r.sample_every
        if (self.graphs and k == self.chunk and k % 2 == 0 and k % r.sample_every == 0
                and r.steps - a.issued > k):
            # full chunks (not the last) replay one captured graph: one host launch per chunk
            if a.graph is None:
                with torch.cuda.stream(a.sim.stream):
                    a.graph_ring = torch.zeros((k // r.sample_every, 6), dtype=torch.float64,
                                               device="cuda")
                a.graph = a.sim.graph(k, sample_every=r.sample_every, ring=a.graph_ring)
            a.graph.launch()
            with torch.cuda.stream(a.sim.stream):
                a.ring[row0:row0 + a.graph_ring.shape[0]].copy_(a.graph_ring)
        else:
            a.sim.step(k, sample_every=r.sample_every, ring=a.ring[row0:])
        ev = torch.cuda.Event()
        ev.record(a.sim.stream)
        a.issued += k
        a.events.append((a.issued, ev))

    def _finish(self, a: _Active, now: float) -> Result:
        r = a.req
        a.sim.stream.synchronize()
        a.sim.sync()
        sig = a.ring.cpu().numpy()
        half = sig[len(sig) // 2:]
        eta = float(half[:, 3].mean() / r.shear_rate)
        eta_se = None
        if len(half) >= 20:
            blocks = half[: len(half) // 10 * 10, 3].reshape(10, -1).mean(axis=1) / r.shear_rate
            eta_se = float(blocks.std(ddof=1) / np.sqrt(10))
        xs = us = None
        if self.keep_state:
            xs, us, _, _ = a.sim.state()
        if a.graph is not None:
            a.graph.close()
        a.sim.close()
        return Result(r.rid, r.arrival, a.admitted, now, r.n, r.steps, r.shear_rate, eta, sig, xs, us,
                      eta_se=eta_se)

    def run(self, trace, realtime=True):
        """Serve the trace; returns the results in request order and a summary."""
        pending = sorted(trace, key=lambda q: (q.arrival, q.rid))
        active: list[_Active] = []
        results = []
        used = 0
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admit arrived requests in arrival order while slots and HBM allow
            while pending and (pending[0].arrival <= now or not realtime) and len(active) < self.max_active:
                req = pending[0]
                w, p = request_params(req)
                nb = footprint(p, req)
                if active and used + nb > self.hbm_budget:
                    break
                pending.pop(0)
                stream = torch.cuda.Stream()
                sim = Sim(p, w.x, w.u, step0=0, stream=stream)
                with torch.cuda.stream(stream):
                    ring = torch.zeros((req.steps // req.sample_every, 6), dtype=torch.float64,
                                       device="cuda")
                a = _Active(req, sim, ring, time.perf_counter() - t0, nb)
                used += nb
                active.append(a)
                for _ in range(self.ahead):
                    self._enqueue(a)
            # progress: retire finished chunks, keep `ahead` chunks in flight
            progressed = False
            for a in list(active):
                while a.events and a.events[0][1].query():
                    a.events.pop(0)
                    progressed = True
                if not a.events and a.issued >= a.req.steps:
                    results.append(self._finish(a, time.perf_counter() - t0))
                    used -= a.nbytes
                    active.remove(a)
                    continue
                while len(a.events) < self.ahead and a.issued < a.req.steps:
                    self._enqueue(a)
            if not progressed:
                if active:
                    time.sleep(50e-6)
                elif pending and realtime:
                    time.sleep(min(1e-3, max(0.0, pending[0].arrival - (time.perf_counter() - t0))))
        results.sort(key=lambda q: q.rid)
        return results, summarize(results)


def summarize(results) -> dict:
    lat = np.array([r.latency for r in results])
    first = min(r.arrival for r in results)
    last = max(r.done for r in results)
    work = sum(r.n * r.steps for r in results)
    return dict(requests=len(results), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                throughput=work / (last - first), makespan_s=last - first, particle_steps=work)
