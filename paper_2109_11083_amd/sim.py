"""Python handle over one simulation of the C library (torch for device memory).

Torch only allocates the workspace and the input/output buffers and supplies
the HIP stream; every step of the method runs in libleshear.so.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B

PAIRS = {"lj": B.LE_PAIR_LJ, "wca": B.LE_PAIR_WCA}
PRECISIONS = {"fp64": B.LE_FP64, "mixed": B.LE_MIXED}
THERMOSTATS = {"langevin": B.LE_THERMO_LANGEVIN, "dpd": B.LE_THERMO_DPD,
               "langevin_abs": B.LE_THERMO_LANGEVIN_LAB}
VELOCITIES = {"lab": B.LE_VEL_LAB, "peculiar": B.LE_VEL_PECULIAR}


@dataclass
class Params:
    """Python mirror of le_params with the paper's defaults (reduced units)."""
    n: int
    box: tuple
    shear_rate: float = 0.0
    dt: float = 0.005
    kT: float = 1.0
    gamma: float = 1.0
    mass: float = 1.0
    eps: float = 1.0
    sigma: float = 1.0
    rc: float = 2.5
    skin: float = 0.3
    fene_k: float = 30.0
    fene_r0: float = 1.5
    n_chains: int = 0
    chain_len: int = 0
    seed: int = 1
    pair: str = "lj"
    precision: str = "fp64"
    cells: tuple = (0, 0, 0)
    max_neighbors: int = 0
    tune: int = 0
    thermostat: str = "langevin"
    dpd_rc: float = 0.0
    velocity: str = "lab"
    angle_k: float = 0.0
    force_cap: float = 0.0

    def to_c(self) -> B.le_params:
        p = B.le_params()
        p.n = int(self.n)
        for a in range(3):
            p.box[a] = float(self.box[a])
            p.cells[a] = int(self.cells[a])
        p.shear_rate = float(self.shear_rate)
        p.dt, p.kT, p.gamma, p.mass = float(self.dt), float(self.kT), float(self.gamma), float(self.mass)
        p.eps, p.sigma, p.rc, p.skin = float(self.eps), float(self.sigma), float(self.rc), float(self.skin)
        p.fene_k, p.fene_r0 = float(self.fene_k), float(self.fene_r0)
        p.n_chains, p.chain_len = int(self.n_chains), int(self.chain_len)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.pair = PAIRS[self.pair]
        p.precision = PRECISIONS[self.precision]
        p.max_neighbors = int(self.max_neighbors)
        p.tune = int(self.tune)
        p.thermostat = THERMOSTATS[self.thermostat]
        p.dpd_rc = float(self.dpd_rc)
        p.velocity = VELOCITIES[self.velocity]
        p.angle_k = float(self.angle_k)
        p.force_cap = float(self.force_cap)
        return p

    @property
    def rlist(self) -> float:
        return self.rc + self.skin


def workspace_bytes(params: Params) -> int:
    return B.le_workspace_bytes(params.to_c())


def _dev(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
    return t.contiguous()


class Sim:
    """One Lees-Edwards simulation living in a torch-allocated workspace."""

    def __init__(self, params: Params, x0, u0, step0: int = 0, f0=None, device="cuda",
                 stream: torch.cuda.Stream | None = None, workspace: torch.Tensor | None = None,
                 sync: bool = True):
        self.params = params
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._c = params.to_c()
        self.ws_bytes = B.le_workspace_bytes(self._c)
        if workspace is None:
            with torch.cuda.stream(self.stream):
                workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        assert workspace.numel() >= self.ws_bytes
        self.workspace = workspace
        with torch.cuda.stream(self.stream):
            # the uploads are ordered before le_init on the simulation's stream
            x0 = _dev(x0, self.device)
            u0 = _dev(u0, self.device)
            f0 = _dev(f0, self.device) if f0 is not None else None
            assert x0.shape == (3, params.n) and u0.shape == (3, params.n)
            self.handle = B.le_init(self._c, x0.data_ptr(), u0.data_ptr(),
                                    f0.data_ptr() if f0 is not None else None,
                                    workspace.data_ptr(), workspace.numel(), self.stream.cuda_stream,
                                    int(step0))
        # inputs must outlive the asynchronous copy in le_init: wait for it, or
        # (sync=False, e.g. a server whose stream is busy) keep them until close
        self._keep = (x0, u0, f0)
        if sync:
            self.stream.synchronize()
            self._keep = None

    # ---------------------------------------------------------------- calls
    def build_cells(self, want_pairs: bool = True):
        n = self.params.n
        cell_of = torch.empty(n, dtype=torch.int32, device=self.device)
        order = torch.empty(n, dtype=torch.int32, device=self.device)
        cap = 0
        pairs = None
        if want_pairs:
            cap = max(1024, int(n * 4.0 / 3.0 * math.pi * self.params.rlist ** 3 * n
                                / (self.params.box[0] * self.params.box[1] * self.params.box[2])))
            pairs = torch.empty((cap, 2), dtype=torch.int64, device=self.device)
        while True:
            cnt = B.le_build_cells(self.handle, cell_of.data_ptr(), order.data_ptr(),
                                   pairs.data_ptr() if pairs is not None else None, cap)
            if pairs is None or cnt <= cap:
                break
            cap = cnt
            pairs = torch.empty((cap, 2), dtype=torch.int64, device=self.device)
        out = dict(cell_of=cell_of.cpu().numpy(), order=order.cpu().numpy())
        if pairs is not None:
            out["pairs"] = pairs[:cnt].cpu().numpy()
        return out

    def forces(self):
        f = torch.empty((3, self.params.n), dtype=torch.float64, device=self.device)
        w = torch.empty(6, dtype=torch.float64, device=self.device)
        B.le_forces(self.handle, f.data_ptr(), w.data_ptr())
        self.sync()
        return f.cpu().numpy(), w.cpu().numpy()

    def step(self, nsteps: int, sample_every: int = 0, ring: torch.Tensor | None = None):
        """Advance nsteps; returns the ring of sampled stresses (device tensor) if sampling."""
        if sample_every > 0:
            ns = nsteps // sample_every
            if ring is None:
                ring = torch.zeros((max(ns, 1), 6), dtype=torch.float64, device=self.device)
            B.le_step(self.handle, nsteps, sample_every, ring.data_ptr(), ring.shape[0])
            return ring
        B.le_step(self.handle, nsteps, 0, None, 0)
        return None

    def graph(self, nsteps: int, sample_every: int = 0, ring: torch.Tensor | None = None) -> "StepGraph":
        """Capture le_step(nsteps, sample_every, ring) as a HIP graph (nsteps even)."""
        return StepGraph(self, nsteps, sample_every, ring)

    def stress(self):
        s = torch.empty(6, dtype=torch.float64, device=self.device)
        B.le_stress(self.handle, s.data_ptr())
        self.sync()
        return s.cpu().numpy()

    def observables(self, nbins: int = 50, out: torch.Tensor | None = None, host: bool = True):
        """y-profiles of count, summed u_x and summed m c^2, kinetic kT and CoM
        velocity of the current state."""
        if out is None:
            out = torch.empty(3 * nbins + 4, dtype=torch.float64, device=self.device)
        B.le_observables(self.handle, nbins, out.data_ptr())
        if not host:
            return out
        self.sync()
        o = out.cpu().numpy()
        return dict(count=o[:nbins], sum_ux=o[nbins:2 * nbins], sum_mc2=o[2 * nbins:3 * nbins],
                    kT=float(o[3 * nbins]), com=o[3 * nbins + 1:3 * nbins + 4])

    def unwrapped(self, host: bool = True):
        """Unwrapped y and z of every particle ([2][n] by tag)."""
        out = torch.empty((2, self.params.n), dtype=torch.float64, device=self.device)
        B.le_unwrapped(self.handle, out.data_ptr())
        if not host:
            return out
        self.sync()
        return out.cpu().numpy()

    def msd(self, ref: torch.Tensor):
        """Mean squared y and z displacement against ref (a device tensor from
        unwrapped(host=False))."""
        assert ref.is_cuda and ref.dtype == torch.float64 and ref.shape == (2, self.params.n)
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        B.le_msd(self.handle, ref.data_ptr(), out.data_ptr())
        self.sync()
        return out.cpu().numpy()

    def state(self):
        n = self.params.n
        x = torch.empty((3, n), dtype=torch.float64, device=self.device)
        u = torch.empty_like(x)
        f = torch.empty_like(x)
        step = B.le_get_state(self.handle, x.data_ptr(), u.data_ptr(), f.data_ptr())
        return x.cpu().numpy(), u.cpu().numpy(), f.cpu().numpy(), step

    def sync(self):
        st = B.le_sync(self.handle)
        B.check(st, "le_sync")

    def stats(self):
        st, rebuilds, max_nb = B.le_stats(self.handle)
        return dict(status=st, rebuilds=rebuilds, max_neighbors=max_nb)

    def close(self):
        if getattr(self, "handle", None):
            B.le_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params_from_workload(w, **over) -> Params:
    """Params for an inputs.Workload (LJ or KG), overridable by keyword."""
    kw = dict(w.params)
    kw.update(over)
    allowed = set(Params.__dataclass_fields__)
    return Params(**{k: v for k, v in kw.items() if k in allowed})


class StepGraph:
    """A captured chunk of steps of one simulation (le_graph_*); replay with launch()."""

    def __init__(self, sim: Sim, nsteps: int, sample_every: int = 0, ring: torch.Tensor | None = None):
        self.sim = sim
        self.ring = ring
        self.handle = B.le_graph_create(sim.handle, nsteps, sample_every,
                                        ring.data_ptr() if ring is not None else None,
                                        ring.shape[0] if ring is not None else 0)

    def launch(self):
        B.le_graph_launch(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            B.le_graph_destroy(self.handle)
            self.handle = None


def _rings_for(sims, nsteps: int, sample_every: int, rings):
    if sample_every <= 0:
        return None, 0
    ns = max(nsteps // sample_every, 1)
    if rings is None:
        rings = []
        for s in sims:
            with torch.cuda.stream(s.stream):
                rings.append(torch.zeros((ns, 6), dtype=torch.float64, device=s.device))
    cap = min(r.shape[0] for r in rings)
    return rings, cap


def step_batch(sims, nsteps: int, sample_every: int = 0, rings=None):
    """Advance several simulations together with le_step_batch (one launch per
    kernel and kernel configuration for all of them).  They must share one
    stream.  Returns the per-simulation stress rings (device tensors) when
    sampling."""
    rings, cap = _rings_for(sims, nsteps, sample_every, rings)
    B.le_step_batch([s.handle for s in sims], nsteps, sample_every,
                    [r.data_ptr() for r in rings] if rings is not None else None, cap)
    return rings


class BatchGraph:
    """A captured chunk of batched steps (le_batch_graph_create); replay with launch()."""

    def __init__(self, sims, nsteps: int, sample_every: int = 0, rings=None):
        self.sims = list(sims)
        self.rings, cap = _rings_for(self.sims, nsteps, sample_every, rings)
        self.handle = B.le_batch_graph_create([s.handle for s in self.sims], nsteps, sample_every,
                                              [r.data_ptr() for r in self.rings]
                                              if self.rings is not None else None, cap)

    def launch(self):
        B.le_graph_launch(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            B.le_graph_destroy(self.handle)
            self.handle = None
