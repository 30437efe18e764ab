"""Throughput autotuner for the neighbour-list skin and the pair-kernel layout.

The physics does not depend on either choice (the lists always hold every
pair within r_c + skin, and the rebuild criterion keeps them complete); only
the split of time between list builds and pair work does.  Each candidate is
run for a short burst from the same start on the caller's device and the
fastest is returned.
"""
from __future__ import annotations

import dataclasses
import math
import time

import torch

from .sim import Params, Sim


def filling_skin(p: Params, skin: float):
    """Largest skin whose cell grid equals that of `skin`: the grid has
    floor(L_a / (r_c + skin)) cells per axis, so every skin up to
    min_a L_a / n_a - r_c searches the same cells and rebuilds less often.
    None if the grid would be too coarse."""
    r = p.rc + skin
    nc = [int(math.floor(L / (r * (1.0 + 1e-9)))) for L in p.box]
    if min(nc) < 3:
        return None
    return min(L / c for L, c in zip(p.box, nc)) / (1.0 + 1e-6) - p.rc


def autotune(p: Params, x0, u0, skins=(0.2, 0.3, 0.4, 0.5, 0.6, 0.8), tunes=(0,), steps=1500,
             warmup=200, step0=0, fill=True):
    """Return (best Params, table of (skin, tune, particle-steps/s)).  With
    `fill`, every candidate is replaced by its cell-filling skin (same cells,
    fewer rebuilds)."""
    if fill:
        filled = [filling_skin(p, s) for s in skins]
        skins = sorted({round(e, 6) for e in filled if e is not None and e > 0.0})
    table = []
    best = None
    for tune in tunes:
        for skin in skins:
            q = dataclasses.replace(p, skin=float(skin), tune=int(tune))
            try:
                sim = Sim(q, x0, u0, step0=step0)
            except Exception:  # geometry not valid for this skin (too few cells)
                continue
            try:
                sim.step(warmup)
                sim.sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.step(steps)
                sim.sync()
                t1 = time.perf_counter()
            finally:
                sim.close()
            rate = q.n * steps / (t1 - t0)
            table.append((float(skin), int(tune), rate))
            if best is None or rate > best[2]:
                best = (float(skin), int(tune), rate)
    if best is None:
        raise RuntimeError("no candidate layout is valid for this system")
    return dataclasses.replace(p, skin=best[0], tune=best[1]), table


def autotune_batch(members, skins=(0.2, 0.3, 0.4, 0.5, 0.6), tunes=(1, 2), steps=300, warmup=60):
    """Cell size and tile schedule for a batch.  members: list of (x0, u0, Params).
    Each candidate (skin, tune) gives every member the cell-filling skin of `skin`
    in its own box (its cell size) and the pair layout `tune` (1: partners staged
    per tile in LDS, 2: partners from global memory); the batch then runs one burst
    through le_step_batch on a fresh stream.  Returns ((skin, tune), table of
    (skin, tune, particle-steps/s))."""
    from .sim import step_batch
    table = []
    best = None
    work = sum(p.n for _, _, p in members) * steps
    for tune in tunes:
        for skin in skins:
            stream = torch.cuda.Stream()
            sims = []
            try:
                for x0, u0, p in members:
                    f = filling_skin(p, skin)
                    q = dataclasses.replace(p, skin=float(f if f is not None else skin), tune=int(tune))
                    sims.append(Sim(q, x0, u0, stream=stream))
            except Exception:  # a geometry this skin does not allow
                for s in sims:
                    s.close()
                continue
            try:
                step_batch(sims, warmup)
                stream.synchronize()
                t0 = time.perf_counter()
                step_batch(sims, steps)
                stream.synchronize()
                t1 = time.perf_counter()
                for s in sims:
                    s.sync()
            finally:
                for s in sims:
                    s.close()
            rate = work / (t1 - t0)
            table.append((float(skin), int(tune), rate))
            if best is None or rate > best[2]:
                best = (float(skin), int(tune), rate)
    if best is None:
        raise RuntimeError("no candidate is valid for every member")
    return (best[0], best[1]), table
