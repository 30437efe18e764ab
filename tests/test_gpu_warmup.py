"""The capped force law of the warm-up (le_params.force_cap) against the
oracle's, and the warm-up of a random-walk Kremer-Grest melt (Section 2.4:
systems are equilibrated before shear) checked by the oracle."""
import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2109_11083_amd import inputs
from paper_2109_11083_amd.sim import Params, Sim
from paper_2109_11083_amd.warmup import warm_up

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _op(p: Params, **over):
    kw = dict(shear_rate=p.shear_rate, dt=p.dt, kT=p.kT, gamma=p.gamma, mass=p.mass, eps=p.eps,
              sigma=p.sigma, rc=p.rc, fene_k=p.fene_k, fene_r0=p.fene_r0, seed=p.seed,
              chain_len=p.chain_len, n_chains=p.n_chains, thermostat=p.thermostat,
              velocity=p.velocity, angle_k=p.angle_k, force_cap=p.force_cap)
    kw.update(over)
    return O.make_params(p.n, p.box, **kw)


def _walk(n_chains, chain_len, seed=31, **kw):
    w = inputs.kg_workload(n_chains, chain_len, shear_rate=0.0, seed=seed, layout="walk")
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=0.0, seed=seed, rc=2 ** (1 / 6), pair="wca",
               n_chains=n_chains, chain_len=chain_len, gamma=1.0, dt=0.002, **kw)
    return w, p


def e_F(F, Fref):
    rms = math.sqrt(float((Fref ** 2).sum(axis=0).mean()))
    return float(np.sqrt(((F - Fref) ** 2).sum(axis=0)).max()) / rms


@pytest.mark.parametrize("cap", [5.0, 50.0, 1e4])
def test_capped_forces_match_oracle(cap):
    w, p = _walk(30, 20, force_cap=cap)
    sim = Sim(p, w.x, w.u, step0=0)
    F, W = sim.forces()
    op = _op(p)
    xw, _ = O.le_wrap(w.x, w.u, 0.0, op)
    Fr, Wr, _ = O.forces(xw, 0.0, op, 0)
    ef = e_F(F, Fr)
    ew = np.abs(W - Wr).max() / np.abs(Wr).max()
    _log(f"cap {cap}: e_F={ef:.3e} e_W={ew:.3e} max|F|={np.sqrt((Fr ** 2).sum(axis=0)).max():.3e}")
    assert ef <= 1e-12 and ew <= 1e-12
    sim.close()


def test_capped_trajectory_matches_oracle():
    w, p = _walk(30, 20, force_cap=20.0, skin=0.3)
    p = dataclasses.replace(p, shear_rate=0.05)
    sim = Sim(p, w.x, w.u, step0=0)
    ref = O.Sim(w.x, w.u, _op(p))
    sim.step(20)
    ref.run(20)
    gx, gu, gf, st = sim.state()
    L = np.array(p.box)[:, None]
    dx = gx - ref.x
    dx = dx - L * np.round(dx / L)
    _log(f"capped trajectory: max|dx|={np.abs(dx).max():.3e} e_F={e_F(gf, ref.F):.3e}")
    assert np.abs(dx).max() < 1e-9
    assert e_F(gf, ref.F) < 1e-8
    sim.close()


def test_warm_up_of_a_random_walk_melt():
    """100 chains x 100 beads as random walks (overlapping): after the warm-up
    the oracle finds every bond shorter than R0 and the largest force below
    10^3, and the kinetic temperature near kT."""
    w, p = _walk(100, 100)
    op0 = _op(p)
    xw, _ = O.le_wrap(w.x, w.u, 0.0, op0)
    F0, _, _ = O.forces(xw, 0.0, op0, 1)
    m0 = float(np.sqrt((F0 ** 2).sum(axis=0)).max())
    x, u, info = warm_up(p, w.x, w.u)
    for s in info.stages:
        _log(f"stage {s}")
    F, _, _ = O.forces(x, 0.0, op0, 1)  # raises on a bond at or beyond R0
    m = float(np.sqrt((F ** 2).sum(axis=0)).max())
    kt = float((u ** 2).sum() / (3 * p.n - 3))
    _log(f"warm-up: start max|F|={m0:.3e} end max|F|={m:.3e} (library {info.max_force:.3e}) kT={kt:.3f} "
         f"steps={info.steps}")
    assert m0 > 1e6
    assert m < 1e3 and abs(m - info.max_force) <= 1e-9 * m
    assert 0.8 < kt < 1.2
