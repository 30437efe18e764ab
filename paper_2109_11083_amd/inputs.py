"""Seeded synthetic inputs for Lees-Edwards shear-flow workloads.

This module only draws initial states (positions, velocities, chain
topology); it holds no force, integration or boundary arithmetic.  Every
generator is a pure function of its arguments and seed, so the CPU oracle and
the GPU library can be fed bit-identical inputs.

Arrays are float64 SoA of shape (3, n), indexed by particle tag.  Axes: x flow,
y gradient, z vorticity.  Workload recipes follow the model systems of the
paper's Section 2.4 (LJ fluid at density ~0.844, Kremer-Grest melts at ~0.85).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "LJ_DENSITY", "KG_DENSITY", "box_for", "lj_lattice", "lj_lattice_subset",
    "maxwell", "streaming_initial_velocity", "kg_random_walk", "kg_lattice_snake",
    "Workload", "lj_workload", "kg_workload",
]

LJ_DENSITY = 0.8442
KG_DENSITY = 0.85


def box_for(n: int, density: float) -> float:
    """Edge of the cubic box holding n particles at the given number density."""
    return (n / density) ** (1.0 / 3.0)


def lj_lattice(n_side: int, L: float, jitter: float, seed: int) -> np.ndarray:
    """Simple-cubic lattice of n_side^3 sites in a cube of edge L.

    Site (i, j, k) sits at ((i+1/2) a, (j+1/2) a, (k+1/2) a), a = L / n_side,
    and every coordinate gets an independent U(-jitter, jitter) displacement.
    Tags run x fastest, then y, then z.
    """
    rng = np.random.default_rng(seed)
    a = L / n_side
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    return np.ascontiguousarray(pos)


def lj_lattice_subset(n: int, density: float, jitter: float, seed: int):
    """n particles on ceil(n^(1/3))^3 lattice sites chosen by a seeded permutation.

    Returns (positions, L) with L = (n / density)^(1/3).
    """
    L = box_for(n, density)
    m = int(math.ceil(round(n ** (1.0 / 3.0), 9)))
    while m ** 3 < n:
        m += 1
    full = lj_lattice(m, L, jitter, seed)
    rng = np.random.default_rng(seed + 7919)
    pick = np.sort(rng.permutation(m ** 3)[:n])
    return np.ascontiguousarray(full[:, pick]), L


def maxwell(n: int, kT: float, mass: float, seed: int) -> np.ndarray:
    """Maxwell-Boltzmann velocities (std sqrt(kT/m) per component), CoM removed."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, math.sqrt(kT / mass), size=(3, n))
    if n > 1:
        v -= v.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(v)


def streaming_initial_velocity(pos: np.ndarray, peculiar: np.ndarray, shear_rate: float,
                               Ly: float) -> np.ndarray:
    """Initial lab velocity: the thermal draw plus a linear flow profile.

    Starts the run on the steady linear profile of the paper's Eq. shear-rate
    (zero at mid-height) so that the shear need not build up from rest.
    """
    u = peculiar.copy()
    u[0] += shear_rate * (pos[1] - 0.5 * Ly)
    return u


def _unit_vectors(rng, k):
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def kg_random_walk(n_chains: int, chain_len: int, density: float, bond: float, seed: int,
                   min_second: float = 1.02):
    """Linear chains as random walks with fixed bond length.

    Chain starts are uniform in the box; each new bead sits at distance `bond`
    from the previous one in a uniform direction, redrawn while it lies closer
    than `min_second` to the bead two back (non-reversal).  Coordinates are
    left unwrapped.  Tag = chain * chain_len + k.  Returns (positions, L).
    """
    rng = np.random.default_rng(seed)
    n = n_chains * chain_len
    L = box_for(n, density)
    pos = np.empty((n_chains, chain_len, 3))
    pos[:, 0, :] = rng.uniform(0.0, L, size=(n_chains, 3))
    for k in range(1, chain_len):
        step = _unit_vectors(rng, n_chains) * bond
        cand = pos[:, k - 1, :] + step
        if k >= 2:
            bad = np.linalg.norm(cand - pos[:, k - 2, :], axis=1) < min_second
            while bad.any():
                redo = _unit_vectors(rng, int(bad.sum())) * bond
                cand[bad] = pos[bad, k - 1, :] + redo
                bad = np.linalg.norm(cand - pos[:, k - 2, :], axis=1) < min_second
        pos[:, k, :] = cand
    out = np.ascontiguousarray(pos.reshape(n, 3).T)
    return out, L


def kg_lattice_snake(n_chains: int, chain_len: int, density: float, jitter: float, seed: int):
    """Overlap-free melt: one boustrophedon path through a cubic lattice cut into chains.

    The lattice has m^3 >= n sites with spacing a = L / m; the path visits x
    rows back and forth, layer by layer, so consecutive sites are always one
    lattice spacing apart.  The first n sites of the path are taken, chain k
    owning sites [k*chain_len, (k+1)*chain_len).  Each coordinate then gets a
    U(-jitter, jitter) displacement.  Returns (positions, L).
    """
    rng = np.random.default_rng(seed)
    n = n_chains * chain_len
    L = box_for(n, density)
    m = 1
    while m ** 3 < n:
        m += 1
    a = L / m
    sites = []
    for iz in range(m):
        ys = range(m) if iz % 2 == 0 else range(m - 1, -1, -1)
        for row, iy in enumerate(ys):
            xs = range(m) if (row + iz * m) % 2 == 0 else range(m - 1, -1, -1)
            for ix in xs:
                sites.append((ix, iy, iz))
                if len(sites) == n:
                    break
            if len(sites) == n:
                break
        if len(sites) == n:
            break
    s = np.asarray(sites, dtype=np.float64)
    pos = ((s + 0.5) * a).T
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    return np.ascontiguousarray(pos), L


@dataclass
class Workload:
    """A complete synthetic initial state plus the physical parameters it was drawn for."""
    name: str
    x: np.ndarray
    u: np.ndarray
    box: tuple
    params: dict = field(default_factory=dict)


def lj_workload(n_side: int = 10, density: float = LJ_DENSITY, kT: float = 1.0,
                shear_rate: float = 0.1, jitter: float = 0.05, seed: int = 11,
                n: int | None = None, **extra) -> Workload:
    """LJ fluid: lattice (n_side^3 sites, or n of them when n is given), Maxwell + profile."""
    if n is None:
        n = n_side ** 3
        L = box_for(n, density)
        x = lj_lattice(n_side, L, jitter, seed)
    else:
        x, L = lj_lattice_subset(n, density, jitter, seed)
    c = maxwell(n, kT, 1.0, seed + 1)
    u = streaming_initial_velocity(x, c, shear_rate, L)
    params = dict(n=n, box=(L, L, L), shear_rate=shear_rate, kT=kT, pair="lj", rc=2.5)
    params.update(extra)
    return Workload(f"lj_n{n}", x, u, (L, L, L), params)


def kg_workload(n_chains: int, chain_len: int, density: float = KG_DENSITY, kT: float = 1.0,
                shear_rate: float = 0.01, seed: int = 31, layout: str = "snake",
                **extra) -> Workload:
    """Kremer-Grest melt of linear chains; layout 'snake' (overlap-free) or 'walk'."""
    if layout == "snake":
        x, L = kg_lattice_snake(n_chains, chain_len, density, 0.02, seed)
    else:
        x, L = kg_random_walk(n_chains, chain_len, density, 0.97, seed)
    n = n_chains * chain_len
    c = maxwell(n, kT, 1.0, seed + 1)
    u = streaming_initial_velocity(x, c, shear_rate, L)
    params = dict(n=n, box=(L, L, L), shear_rate=shear_rate, kT=kT, pair="wca",
                  rc=2.0 ** (1.0 / 6.0), chain_len=chain_len, n_chains=n_chains)
    params.update(extra)
    return Workload(f"kg_{n_chains}x{chain_len}", x, u, (L, L, L), params)
