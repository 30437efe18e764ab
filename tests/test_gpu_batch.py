"""Batched stepping (le_step_batch, le_batch_graph_create): uneven simulations
advanced together give, member by member, bitwise the results of each one run
alone with le_step (which the other GPU tests pin to the oracle); a member
that latches an error stops alone."""
import sys

import numpy as np
import pytest
import torch

from paper_2109_11083_amd import binding as B
from paper_2109_11083_amd import inputs
from paper_2109_11083_amd.sim import BatchGraph, Params, Sim, step_batch

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lj(n, sr, seed, **kw):
    w = inputs.lj_workload(n=n, shear_rate=sr, seed=seed)
    return w.x, w.u, Params(n=w.x.shape[1], box=w.box, shear_rate=sr, seed=seed, **kw)


def _kg(nc, cl, sr, seed, **kw):
    w = inputs.kg_workload(nc, cl, shear_rate=sr, seed=seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=sr, seed=seed, rc=2 ** (1 / 6), pair="wca",
               n_chains=nc, chain_len=cl, gamma=0.5, dt=0.01, **kw)
    return w.x, w.u, p


def _members():
    """Uneven members: sizes, shear rates, skins, precisions, thermostats,
    bonds, velocity storage and list layouts all differ."""
    return [
        _lj(1000, 0.1, 11, skin=0.3),
        _lj(2744, 0.5, 12, skin=0.45),
        _lj(4100, 1.0, 13, skin=0.0),                       # rebuild every step
        _lj(1500, 0.2, 14, skin=0.3, precision="mixed"),
        _lj(1331, 0.3, 15, skin=0.3, tune=2),               # global pair layout
        _lj(1800, 0.4, 16, skin=0.3, thermostat="dpd", gamma=5.0),
        _lj(1200, 0.25, 17, skin=0.3, velocity="peculiar"),
        _kg(20, 20, 0.05, 18, skin=0.4, angle_k=1.5),
        _kg(30, 10, 0.02, 19, skin=0.3),
    ]


def _state(sim):
    x, u, f, st = sim.state()
    return x, u, f, st


def _alone(members, chunks, sample_every):
    out = []
    for x, u, p in members:
        sim = Sim(p, x, u)
        rings = []
        for c in chunks:
            r = sim.step(c, sample_every=sample_every) if sample_every else None
            if r is None and sample_every == 0:
                sim.step(c)
            rings.append(r.cpu().numpy() if r is not None else None)
        out.append((_state(sim), rings))
        sim.close()
    return out


def _batched(members, chunks, sample_every):
    stream = torch.cuda.Stream()
    sims = [Sim(p, x, u, stream=stream) for x, u, p in members]
    rings_all = [[] for _ in sims]
    for c in chunks:
        rings = step_batch(sims, c, sample_every=sample_every)
        stream.synchronize()  # the rings are read on another stream
        for k in range(len(sims)):
            rings_all[k].append(rings[k].cpu().numpy() if rings is not None else None)
    out = [(_state(s), rings_all[k]) for k, s in enumerate(sims)]
    for s in sims:
        s.close()
    return out


def _same(a, b, tag):
    (xa, ua, fa, sa), ra = a
    (xb, ub, fb, sb), rb = b
    assert sa == sb, tag
    assert np.array_equal(xa, xb), tag
    assert np.array_equal(ua, ub), tag
    assert np.array_equal(fa, fb), tag
    for p, q in zip(ra, rb):
        if p is not None:
            assert np.array_equal(p, q), tag


def test_batch_members_equal_alone_bitwise():
    members = _members()
    chunks = [60]
    alone = _alone(members, chunks, 10)
    batch = _batched(members, chunks, 10)
    for k, (a, b) in enumerate(zip(alone, batch)):
        _same(a, b, k)
    _log(f"{len(members)} members, 60 steps: bitwise equal alone and batched")


def test_batch_odd_chunks_and_state_reads():
    """Odd step counts flip the members' control copies; state reads between
    calls force rebuilds; the batch follows each member exactly."""
    members = _members()[:5]
    chunks = [7, 13, 1, 30]
    alone = _alone(members, chunks, 0)
    batch = _batched(members, chunks, 0)
    for k, (a, b) in enumerate(zip(alone, batch)):
        _same(a, b, k)


def test_batch_graph_replays_match_eager():
    members = _members()[:4]
    stream = torch.cuda.Stream()
    sims = [Sim(p, x, u, stream=stream) for x, u, p in members]
    refs = [Sim(p, x, u) for x, u, p in members]
    g = BatchGraph(sims, 40, sample_every=10)
    for rep in range(3):
        g.launch()
        ref_rings = [r.step(40, sample_every=10) for r in refs]
        stream.synchronize()
        for k in range(len(sims)):
            _same((_state(sims[k]), [g.rings[k].cpu().numpy()]),
                  (_state(refs[k]), [ref_rings[k].cpu().numpy()]), (rep, k))
        if rep == 1:  # an odd eager step count on one member and its reference
            sims[2].step(3)
            refs[2].step(3)
    g.close()
    for s in sims + refs:
        s.close()


def test_batch_more_members_than_one_launch_holds():
    """More members than one launch's descriptor table (64): split into
    several launches, still equal to alone."""
    members = [_lj(216 + 7 * k, 0.1 + 0.01 * k, 100 + k, skin=0.3, rc=1.5) for k in range(70)]
    alone = _alone(members, [12], 0)
    batch = _batched(members, [12], 0)
    for k, (a, b) in enumerate(zip(alone, batch)):
        _same(a, b, k)


def _stretched_bond(seed=5):
    """A KG-like system whose one bond is pulled apart at once (r = 1.45 with the
    two beads flying apart at +-60), plus free WCA beads on a lattice of
    spacing 1.5 (no overlaps)."""
    rng = np.random.default_rng(seed)
    L = 9.0
    g = (np.arange(6) + 0.5) * 1.5
    z, y, xx = np.meshgrid(g, g, g, indexing="ij")
    free = np.stack([xx.ravel(), y.ravel(), z.ravel()])
    x = np.concatenate([np.array([[3.0, 4.45], [4.5, 4.5], [4.5, 4.5]]), free], axis=1)
    n = x.shape[1]
    u = rng.normal(size=(3, n))
    u[:, 0] = (-60.0, 0.0, 0.0)
    u[:, 1] = (60.0, 0.0, 0.0)
    p = Params(n=n, box=(L, L, L), shear_rate=0.05, seed=seed, rc=2 ** (1 / 6), pair="wca",
               n_chains=1, chain_len=2, gamma=0.5, dt=0.01, skin=0.3)
    return x, u, p


def _overfull_cell(seed=6):
    """200 non-interacting particles, all inside one cell of a 6x6x6 grid:
    more than the per-cell capacity (a latched capacity error at the first
    binning)."""
    rng = np.random.default_rng(seed)
    L = 9.0
    n = 200
    x = rng.uniform(0.2, 1.2, size=(3, n))
    u = rng.normal(size=(3, n))
    p = Params(n=n, box=(L, L, L), shear_rate=0.05, seed=seed, eps=0.0, rc=1.2, skin=0.2)
    return x, u, p


def test_one_failing_member_does_not_perturb_the_others():
    healthy = [_kg(20, 20, 0.05, 21, skin=0.4), _kg(25, 16, 0.02, 22, skin=0.3),
               _lj(1000, 0.3, 23, skin=0.3), _lj(1331, 0.1, 24, skin=0.3)]
    bad = [_stretched_bond(), _overfull_cell()]
    alone = _alone(healthy, [50], 10)
    stream = torch.cuda.Stream()
    mix = [healthy[0], bad[0], healthy[1], healthy[2], bad[1], healthy[3]]
    sims = [Sim(p, x, u, stream=stream) for x, u, p in mix]
    rings = step_batch(sims, 50, sample_every=10)
    with pytest.raises(B.LeError) as e:
        sims[1].sync()
    assert e.value.code == B.LE_E_BOND
    with pytest.raises(B.LeError) as e:
        sims[4].sync()
    assert e.value.code == B.LE_E_CAPACITY
    for k, j in ((0, 0), (2, 1), (3, 2), (5, 3)):
        _same((_state(sims[k]), [rings[k].cpu().numpy()]), alone[j], k)
    # a later call skips the members whose errors were seen and goes on with the rest
    step_batch(sims, 4)
    for k in (0, 2, 3, 5):
        sims[k].sync()
    for s in sims:
        s.close()


def test_batch_argument_errors():
    x, u, p = _lj(1000, 0.1, 11)
    a = Sim(p, x, u)
    b = Sim(p, x, u, stream=torch.cuda.Stream())
    with pytest.raises(B.LeError) as e:  # members on different streams
        B.le_step_batch([a.handle, b.handle], 2)
    assert e.value.code == B.LE_E_ARG
    with pytest.raises(B.LeError) as e:  # the same member twice
        B.le_step_batch([a.handle, a.handle], 2)
    assert e.value.code == B.LE_E_ARG
    with pytest.raises(B.LeError) as e:  # the default stream cannot be captured
        BatchGraph([a], 10)
    assert e.value.code == B.LE_E_STATE
    a.close()
    b.close()
