"""Serving loop for shear-rate sweep requests (continuous batching on one GPU).

Requests (independent Lees-Edwards simulations of different size and shear
rate) arrive over time.  The server admits a request when its device
footprint (workspace + sample ring) fits the HBM budget and a slot is free;
a request finishes when its steps are done, and its result is the sampled
shear-stress series and the viscosity estimate (Eq. viscosity).
Time-to-result is completion minus arrival.

Two ways to advance the admitted simulations:

* ``mode="batched"`` (continuous batching): every admitted simulation lives
  on the server's one stream, and each chunk of steps advances all of them
  together with le_step_batch (one launch per kernel for the whole batch,
  or one replay of a captured batch graph while the batch is unchanged).
  Requests that arrive while others run join at the next chunk boundary;
  finished ones leave at theirs.
* ``mode="streams"``: each simulation gets its own stream and its own
  le_step (or single-simulation graph) per chunk; with ``max_active=1`` this
  is the plain one-simulation-at-a-time (FIFO) baseline.

Every simulation is deterministic and independent of the others (own
workspace, own Philox key, its own descriptor in a batch), so its result is
bitwise the same alone and in the mix, in either mode.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import binding as B
from . import inputs
from .sim import BatchGraph, Params, Sim, step_batch


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
    tune: int = 0


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
                seed=41, precision="fp64", burst=False, skin=0.4, tune=0):
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
        out.append(Request(k, 0.0 if burst else t, n, sr, steps, 100 * seed + k, precision, skin=skin,
                           tune=tune))
    return out


def request_params(r: Request) -> tuple:
    """LJ fluid of the request (density 0.8442, r_c 2.5, kT 1, Langevin gamma 1, dt 0.005).
    The skin is the request's, widened to fill the cells of its box (same cells, rarer
    rebuilds)."""
    from .tune import filling_skin
    w = inputs.lj_workload(n=r.n, shear_rate=r.shear_rate, seed=r.seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=r.shear_rate, seed=r.seed, skin=r.skin,
               precision=r.precision, rc=2.5, dt=0.005, kT=1.0, gamma=1.0, tune=r.tune)
    f = filling_skin(p, r.skin)
    if f is not None:
        p = dataclasses.replace(p, skin=f)
    return w, p


def footprint(p: Params, r: Request) -> int:
    from .sim import workspace_bytes
    return workspace_bytes(p) + (r.steps // r.sample_every + 1) * 6 * 8 + 6 * p.n * 8


def eta_of_series(sig: np.ndarray, shear_rate: float):
    """Viscosity over the second half of the samples and its 10-block standard error."""
    half = sig[len(sig) // 2:]
    eta = float(half[:, 3].mean() / shear_rate)
    eta_se = None
    if len(half) >= 20:
        blocks = half[: len(half) // 10 * 10, 3].reshape(10, -1).mean(axis=1) / shear_rate
        eta_se = float(blocks.std(ddof=1) / np.sqrt(10))
    return eta, eta_se


class _Active:
    def __init__(self, req: Request, sim: Sim, ring: torch.Tensor, admitted: float, nbytes: int):
        self.req = req
        self.sim = sim
        self.ring = ring
        self.admitted = admitted
        self.nbytes = nbytes
        self.issued = 0         # steps enqueued
        self.events = []        # (steps covered, event) per enqueued chunk (streams mode)
        self.graph = None       # captured chunk (HIP graph) and its sample rows (streams mode)
        self.graph_ring = None
        self.status = None      # device int32: latched status after the last chunk (batched mode)


@dataclasses.dataclass
class _Chunk:
    event: torch.cuda.Event
    finishing: list          # members whose last step is in this chunk
    keep: object = None      # graph used by the chunk (destroyed once it has run)


class Server:
    """Continuous-batching server.  hbm_budget: bytes the admitted requests may
    hold; max_active: concurrent simulations; chunk: steps per enqueue; ahead:
    chunks in flight; keep_state: copy the final state of each request (tests);
    graphs: replay captured chunks; mode: "batched" or "streams" (see module)."""

    def __init__(self, hbm_budget=16 << 30, max_active=64, chunk=500, ahead=2, keep_state=False,
                 graphs=True, mode="batched", graph_steps=100):
        assert mode in ("batched", "streams")
        self.hbm_budget = hbm_budget
        self.max_active = max_active
        self.chunk = chunk
        self.ahead = ahead
        self.keep_state = keep_state
        self.graphs = graphs
        self.mode = mode
        self.graph_steps = graph_steps  # steps per captured batch graph (replayed chunk/graph_steps times)

    # ------------------------------------------------------------ shared
    def _finish(self, a: _Active, now: float) -> Result:
        r = a.req
        if a.status is not None and not self.keep_state:
            # batched: the chunk holding the last step has completed, and the
            # status copy enqueued after it is final; no wait on the shared stream
            st = int(a.status.cpu()[0])
            if st != 0:
                raise B.LeError(st, f"request {r.rid}")
        else:
            a.sim.stream.synchronize()
            a.sim.sync()
        sig = a.ring.cpu().numpy()
        eta, eta_se = eta_of_series(sig, r.shear_rate)
        xs = us = None
        if self.keep_state:
            xs, us, _, _ = a.sim.state()
        if a.graph is not None:
            a.graph.close()
        a.sim.close()
        return Result(r.rid, r.arrival, a.admitted, now, r.n, r.steps, r.shear_rate, eta, sig, xs, us,
                      eta_se=eta_se)

    def _admit(self, pending, active, used, t0, realtime, stream):
        """Admit arrived requests in arrival order while slots and HBM allow."""
        now = time.perf_counter() - t0
        while pending and (pending[0].arrival <= now or not realtime) and len(active) < self.max_active:
            req = pending[0]
            w, p = request_params(req)
            nb = footprint(p, req)
            if active and used + nb > self.hbm_budget:
                break
            pending.pop(0)
            st = stream if stream is not None else torch.cuda.Stream()
            sim = Sim(p, w.x, w.u, step0=0, stream=st, sync=stream is None)
            with torch.cuda.stream(st):
                ring = torch.zeros((req.steps // req.sample_every, 6), dtype=torch.float64,
                                   device="cuda")
            active.append(_Active(req, sim, ring, time.perf_counter() - t0, nb))
            used += nb
        return used

    def run(self, trace, realtime=True):
        """Serve the trace; returns the results in request order and a summary."""
        if self.mode == "batched":
            results = self._run_batched(trace, realtime)
        else:
            results = self._run_streams(trace, realtime)
        results.sort(key=lambda q: q.rid)
        return results, summarize(results)

    # ------------------------------------------------------------ batched
    def _enqueue_batch(self, members, k, se, stream, state):
        """One chunk of k steps for every member: replays of the cached batch graph
        (graph_steps steps each) when the batch is the one it was captured for, else a
        capture for this batch first; le_step_batch when k is not a whole number of
        graph chunks.  A short graph keeps the capture cost small, since the batch
        changes with every arrival and departure."""
        g_steps = min(self.graph_steps, k)
        key = (tuple(id(a) for a in members), g_steps)
        rows = [a.issued // se for a in members]
        keep = None
        if self.graphs and g_steps % 2 == 0 and g_steps % se == 0 and k % g_steps == 0:
            if state.get("key") != key:
                old = state.pop("graph", None)
                if old is not None:
                    state.setdefault("retired", []).append(old)
                with torch.cuda.stream(stream):
                    grings = [torch.zeros((g_steps // se, 6), dtype=torch.float64, device="cuda")
                              for _ in members]
                state["graph"] = BatchGraph([a.sim for a in members], g_steps, sample_every=se, rings=grings)
                state["key"] = key
            g = state["graph"]
            for rep in range(k // g_steps):
                g.launch()
                with torch.cuda.stream(stream):
                    for a, r0, gr in zip(members, rows, g.rings):
                        r1 = r0 + rep * gr.shape[0]
                        a.ring[r1:r1 + gr.shape[0]].copy_(gr)
            keep = g
        else:
            rings = [a.ring[r0:] for a, r0 in zip(members, rows)]
            cap = min(r.shape[0] for r in rings)
            B.le_step_batch([a.sim.handle for a in members], k, se, [r.data_ptr() for r in rings], cap)
        return keep

    def _run_batched(self, trace, realtime):
        pending = sorted(trace, key=lambda q: (q.arrival, q.rid))
        se = pending[0].sample_every if pending else 10
        assert all(q.sample_every == se for q in pending), "one sampling interval per server"
        stream = torch.cuda.Stream()
        active: list[_Active] = []
        inflight: list[_Chunk] = []
        results = []
        used = 0
        state = {}
        t0 = time.perf_counter()
        while pending or active:
            progressed = False
            while inflight and inflight[0].event.query():
                ch = inflight.pop(0)
                now = time.perf_counter() - t0
                for a in ch.finishing:
                    results.append(self._finish(a, now))
                    used -= a.nbytes
                    active.remove(a)
                progressed = True
            if not inflight:
                for g in state.pop("retired", []):
                    g.close()
            used = self._admit(pending, active, used, t0, realtime, stream)
            while len(inflight) < self.ahead:
                members = [a for a in active if a.issued < a.req.steps]
                if not members:
                    break
                k = min(self.chunk, min(a.req.steps - a.issued for a in members))
                keep = self._enqueue_batch(members, k, se, stream, state)
                for a in members:
                    a.issued += k
                    if a.issued >= a.req.steps:
                        with torch.cuda.stream(stream):
                            a.status = torch.full((1,), -99, dtype=torch.int32, device="cuda")
                        B.le_status_out(a.sim.handle, a.status.data_ptr())
                ev = torch.cuda.Event()
                ev.record(stream)
                inflight.append(_Chunk(ev, [a for a in members if a.issued >= a.req.steps], keep))
                progressed = True
            if not progressed:
                if inflight:
                    time.sleep(50e-6)
                elif pending and realtime:
                    time.sleep(min(1e-3, max(0.0, pending[0].arrival - (time.perf_counter() - t0))))
        stream.synchronize()
        for g in state.pop("retired", []) + ([state["graph"]] if "graph" in state else []):
            g.close()
        return results

    # ------------------------------------------------------------ streams
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

    def _run_streams(self, trace, realtime):
        pending = sorted(trace, key=lambda q: (q.arrival, q.rid))
        active: list[_Active] = []
        results = []
        used = 0
        t0 = time.perf_counter()
        while pending or active:
            n_before = len(active)
            used = self._admit(pending, active, used, t0, realtime, None)
            for a in active[n_before:]:
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
        return results


def summarize(results) -> dict:
    lat = np.array([r.latency for r in results])
    first = min(r.arrival for r in results)
    last = max(r.done for r in results)
    work = sum(r.n * r.steps for r in results)
    return dict(requests=len(results), p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                throughput=work / (last - first), makespan_s=last - first, particle_steps=work)
