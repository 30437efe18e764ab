"""Warm-up of overlapping starts (random-walk Kremer-Grest melts) on the GPU.

The paper heats and equilibrates every system without shear before the shear
runs (Section 2.4).  A melt built from random walks of bond 0.97 has beads of
different chains almost on top of each other, where the WCA force (Eq.
lj-shift) is astronomically large, so the run starts with the pair force
capped in magnitude (le_params.force_cap) and the cap raised stage by stage
while the overlaps open; FENE bonds (Eq. fene) stay uncapped and hold the
chains.  The warm-up ends with an uncapped run at a small time step, after
which the largest force on any bead must be below `max_force`.

Every stage runs in the HIP library (le_step with the capped force law); this
module only sequences the stages and reads the result back.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from .sim import Params, Sim

# (cap, steps, dt) of the capped stages; the cap opens the overlaps gradually
DEFAULT_STAGES = ((10.0, 300, 0.002), (30.0, 300, 0.002), (100.0, 300, 0.002),
                  (300.0, 300, 0.002), (500.0, 300, 0.002))


@dataclasses.dataclass
class WarmupInfo:
    stages: list            # per stage: dict(cap, steps, dt, max_force, kT)
    max_force: float        # largest uncapped force on a bead at the end
    steps: int              # steps taken in total


def _max_force(p: Params, x, u, device) -> float:
    sim = Sim(dataclasses.replace(p, force_cap=0.0, tune=0), x, u, device=device)
    f = torch.empty((3, p.n), dtype=torch.float64, device=sim.device)
    from . import binding as B
    B.le_forces(sim.handle, f.data_ptr(), None)
    sim.sync()
    m = float(torch.sqrt((f * f).sum(dim=0)).max().item())
    sim.close()
    return m


def warm_up(params: Params, x, u, stages=DEFAULT_STAGES, final_steps=500, final_dt=0.005,
            gamma=1.0, max_force=1e3, extra_rounds=4, device="cuda"):
    """Warm up the state (x, u) of `params` (no shear during the warm-up).

    Returns (x, u, WarmupInfo): positions wrapped into the box and thermal
    velocities (peculiar: the caller adds its streaming profile).  Raises
    RuntimeError if the largest uncapped force stays above max_force."""
    base = dataclasses.replace(params, shear_rate=0.0, gamma=gamma, precision="fp64",
                               thermostat="langevin", velocity="lab", tune=2)
    info = []
    total = 0
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)

    def run(cap, steps, dt):
        nonlocal x, u, total
        q = dataclasses.replace(base, force_cap=float(cap), dt=float(dt))
        sim = Sim(q, x, u, device=device)
        sim.step(int(steps))
        kt = sim.observables(1)["kT"]
        x, u, _, _ = sim.state()
        sim.close()
        total += int(steps)
        info.append(dict(cap=cap, steps=int(steps), dt=dt, kT=kt))

    for cap, steps, dt in stages:
        run(cap, steps, dt)
    run(0.0, final_steps, final_dt)
    m = _max_force(base, x, u, device)
    rounds = 0
    while m >= max_force and rounds < extra_rounds:
        run(stages[-1][0], stages[-1][1], stages[-1][2])
        run(0.0, final_steps, final_dt)
        m = _max_force(base, x, u, device)
        rounds += 1
    info[-1]["max_force"] = m
    if not (m < max_force) or not math.isfinite(m):
        raise RuntimeError(f"warm-up left a force of {m:.3g} >= {max_force:.3g}")
    return x, u, WarmupInfo(info, m, total)
