"""Warm-up of overlapping starts (random-walk Kremer-Grest melts) on the GPU.

The paper heats and equilibrates every system without shear before the shear
runs (Section 2.4).  A melt built from random walks of bond 0.97 has beads of
different chains almost on top of each other, where the WCA force (Eq.
lj-shift) is astronomically large, so the run starts with the pair force
capped in magnitude (le_params.force_cap) and the cap raised stage by stage
while the overlaps open; FENE bonds (Eq. fene) stay uncapped and hold the
chains.  The warm-up ends with an uncapped run at a small time step, after
which the largest force on any bead must be below `max_force`.

Every stage runs in the HIP library (le_step / le_step_batch with the capped
force law); this module only sequences the stages and reads the result back.
Several melts are warmed up together, each stage one batched run.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import binding as B
from .sim import Params, Sim, step_batch

# (cap, steps, dt) of the capped stages; the cap opens the overlaps gradually
DEFAULT_STAGES = ((10.0, 300, 0.002), (30.0, 300, 0.002), (100.0, 300, 0.002),
                  (300.0, 300, 0.002), (500.0, 300, 0.002))


@dataclasses.dataclass
class WarmupInfo:
    stages: list            # per stage: dict(cap, steps, dt, kT)
    max_force: float        # largest uncapped force on a bead at the end
    steps: int              # steps taken in total


def _max_force(p: Params, x, u, device) -> float:
    sim = Sim(dataclasses.replace(p, force_cap=0.0, tune=0), x, u, device=device)
    f = torch.empty((3, p.n), dtype=torch.float64, device=sim.device)
    B.le_forces(sim.handle, f.data_ptr(), None)
    sim.sync()
    m = float(torch.sqrt((f * f).sum(dim=0)).max().item())
    sim.close()
    return m


def warm_up_many(members, stages=DEFAULT_STAGES, final_steps=500, final_dt=0.005, gamma=1.0,
                 max_force=1e3, extra_rounds=4, device="cuda"):
    """Warm up several states together.  members: list of (params, x, u).
    Returns a list of (x, u, WarmupInfo): positions wrapped into the box and
    thermal velocities (peculiar: the caller adds its streaming profile).
    Raises RuntimeError if a member's largest uncapped force stays above
    max_force."""
    base = [dataclasses.replace(p, shear_rate=0.0, gamma=gamma, precision="fp64", thermostat="langevin",
                                velocity="lab", tune=2) for p, _, _ in members]
    xs = [np.ascontiguousarray(x, dtype=np.float64) for _, x, _ in members]
    us = [np.ascontiguousarray(u, dtype=np.float64) for _, _, u in members]
    infos = [[] for _ in members]
    total = 0

    def run(idx, cap, steps, dt):
        nonlocal total
        stream = torch.cuda.Stream(device=device)
        sims = [Sim(dataclasses.replace(base[k], force_cap=float(cap), dt=float(dt)), xs[k], us[k],
                    device=device, stream=stream) for k in idx]
        step_batch(sims, int(steps))
        for k, s in zip(idx, sims):
            kt = s.observables(1)["kT"]
            xs[k], us[k], _, _ = s.state()
            s.close()
            infos[k].append(dict(cap=cap, steps=int(steps), dt=dt, kT=kt))
        total += int(steps)

    everyone = list(range(len(members)))
    for cap, steps, dt in stages:
        run(everyone, cap, steps, dt)
    run(everyone, 0.0, final_steps, final_dt)
    forces = [_max_force(base[k], xs[k], us[k], device) for k in everyone]
    for _ in range(extra_rounds):
        hot = [k for k in everyone if not forces[k] < max_force]
        if not hot:
            break
        run(hot, stages[-1][0], stages[-1][1], stages[-1][2])
        run(hot, 0.0, final_steps, final_dt)
        for k in hot:
            forces[k] = _max_force(base[k], xs[k], us[k], device)
    out = []
    for k in everyone:
        m = forces[k]
        if not (m < max_force) or not math.isfinite(m):
            raise RuntimeError(f"warm-up of member {k} left a force of {m:.3g} >= {max_force:.3g}")
        infos[k][-1]["max_force"] = m
        out.append((xs[k], us[k], WarmupInfo(infos[k], m, sum(s["steps"] for s in infos[k]))))
    return out


def warm_up(params: Params, x, u, **kw):
    """Warm up one state; returns (x, u, WarmupInfo) (see warm_up_many)."""
    return warm_up_many([(params, x, u)], **kw)[0]
