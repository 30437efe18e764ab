"""GPU parity of the HIP library (through the C ABI) against the FP64 oracle.

Bars: integer outputs (cells, order, pair sets, Philox words, offsets) are
bit-exact; FP64 forces and virial within 1e-12 relative (e_F = max_i |dF_i| /
F_rms); mixed precision within 1e-5 (forces) and 1e-4 (shear stress); short
trajectories within bounds set by the chaotic growth of rounding differences.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2109_11083_amd import binding as B
from paper_2109_11083_amd import inputs
from paper_2109_11083_amd.sim import Params, Sim

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def e_F(F, Fref):
    rms = math.sqrt(float((Fref ** 2).sum(axis=0).mean()))
    return float(np.sqrt(((F - Fref) ** 2).sum(axis=0)).max()) / rms


def _oracle_params(p: Params, **over):
    kw = dict(shear_rate=p.shear_rate, dt=p.dt, kT=p.kT, gamma=p.gamma, mass=p.mass, eps=p.eps,
              sigma=p.sigma, rc=p.rc, fene_k=p.fene_k, fene_r0=p.fene_r0, seed=p.seed,
              chain_len=p.chain_len, n_chains=p.n_chains, thermostat=p.thermostat, dpd_rc=p.dpd_rc,
              velocity=p.velocity, angle_k=p.angle_k)
    kw.update(over)
    return O.make_params(p.n, p.box, **kw)


def _lj_case(n_side=10, shear_rate=0.1, seed=11, **kw):
    w = inputs.lj_workload(n_side=n_side, shear_rate=shear_rate, seed=seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=shear_rate, seed=seed, **kw)
    return w, p


def _kg_case(n_chains=20, chain_len=20, shear_rate=0.01, seed=31, **kw):
    w = inputs.kg_workload(n_chains, chain_len, shear_rate=shear_rate, seed=seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=shear_rate, seed=seed, rc=2 ** (1 / 6),
               pair="wca", n_chains=n_chains, chain_len=chain_len, gamma=0.5, dt=0.01, **kw)
    return w, p


def _step0_for_fraction(p: Params, frac):
    """A step index whose offset is close to frac * L_x."""
    sv = p.shear_rate * p.box[1]
    return int(round(frac * p.box[0] / (sv * p.dt)))


# ------------------------------------------------------------------ offsets, Philox
def test_offsets_bitwise():
    for sr, Lx, Ly, dt in [(0.1, 10.5808, 10.5808, 0.005), (1.0, 67.18, 67.18, 0.005),
                           (-0.37, 9.0, 11.5, 0.01), (1e-4, 77.78, 77.78, 0.01)]:
        out = torch.empty(5000, dtype=torch.float64, device=DEV)
        for step0 in (0, 123456, 10 ** 9):
            B.le_offsets(sr, Lx, Ly, dt, step0, 5000, out.data_ptr(), None)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            ref = np.array([O.offset(step0 + k, dt, sr, Lx, Ly) for k in range(5000)])
            assert np.array_equal(got.view(np.int64), ref.view(np.int64)), (sr, step0)


def test_philox_bitwise():
    rng = np.random.default_rng(1)
    n = 4096
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0; key[0] = 0
    ctr[1] = 0xFFFFFFFF; key[1] = 0xFFFFFFFF
    tc = torch.from_numpy(ctr.view(np.int32)).to(DEV)
    tk = torch.from_numpy(key.view(np.int32)).to(DEV)
    to = torch.empty((n, 4), dtype=torch.int32, device=DEV)
    B.le_philox(tc.data_ptr(), tk.data_ptr(), to.data_ptr(), n, None)
    torch.cuda.synchronize()
    got = to.cpu().numpy().view(np.uint32)
    for k in range(0, n, 7):
        assert list(got[k]) == O.philox(ctr[k], key[k]), k


# ------------------------------------------------------------------ cells and pairs
def _check_cells_pairs(w_x, w_u, p: Params, step0):
    _log(f"cells/pairs n={p.n} box={p.box} step0={step0}")
    sim = Sim(p, w_x, w_u, step0=step0)
    out = sim.build_cells()
    op = _oracle_params(p)
    Delta = O.offset(step0, p.dt, p.shear_rate, p.box[0], p.box[1])
    xw, uw = O.le_wrap(w_x, w_u, Delta, op)
    nc = tuple(c if c > 0 else int(math.floor(p.box[a] / (p.rlist * (1 + 1e-9))))
               for a, c in enumerate(p.cells))
    cell_ref, order_ref = O.cells(xw, nc, p.box)
    assert np.array_equal(out["cell_of"], cell_ref)
    assert np.array_equal(out["order"], order_ref)
    got = out["pairs"]
    ref = O.pairs_cells(xw, Delta, p.box, p.rlist) if p.n > 3000 else O.pairs_brute(xw, Delta, p.box, p.rlist)
    key = lambda a: np.sort(np.minimum(a[:, 0], a[:, 1]).astype(np.int64) * p.n + np.maximum(a[:, 0], a[:, 1]))
    kg, kr = key(got), key(ref)
    assert len(kg) == len(np.unique(kg)), "pair listed twice"
    assert np.array_equal(kg, kr)
    # rebuild telemetry: the largest list (partners within r_list, all images)
    deg = np.bincount(np.concatenate([ref[:, 0], ref[:, 1]]).astype(np.int64), minlength=p.n)
    assert sim.stats()["max_neighbors"] == int(deg.max())
    x, u, f, step = sim.state()
    assert step == step0
    assert np.array_equal(x, xw) and np.array_equal(u, uw)
    sim.close()


@pytest.mark.parametrize("frac", [0.0, 0.25, 0.5, 0.75, 0.999999])
def test_cells_and_pairs_lj_c1(frac):
    w, p = _lj_case()
    _check_cells_pairs(w.x, w.u, p, _step0_for_fraction(p, frac))


def test_cells_and_pairs_ragged_noncubic():
    rng = np.random.default_rng(7)
    n = 777
    box = (11.3, 9.1, 12.7)
    x = np.stack([rng.uniform(-3, box[a] + 3, n) for a in range(3)])  # outside the box too
    u = rng.normal(size=(3, n))
    for cells in [(0, 0, 0), (4, 3, 4)]:
        p = Params(n=n, box=box, shear_rate=0.73, rc=2.2, skin=0.5, cells=cells, seed=3)
        for step0 in (0, 17, 4321):
            _check_cells_pairs(x, u, p, step0)


def test_cells_and_pairs_wca_small_cells():
    w, p = _kg_case()
    for step0 in (0, 5000, 123457):
        _check_cells_pairs(w.x, w.u, p, step0)


def test_sort_at_extreme_cell_occupancies():
    """The scan-and-permute pass at its two extremes: about 555 particles per
    cell (one cell per block of the pass) and one particle per 20 cells (256
    cells per block, a ragged last block).  The (cell, tag) order and the
    wrapped state must equal the oracle's bit for bit."""
    rng = np.random.default_rng(11)
    n = 15000
    box = (3.7, 3.7, 3.7)
    x = np.stack([rng.uniform(0.0, box[a], n) for a in range(3)])
    u = rng.normal(size=(3, n))
    p = Params(n=n, box=box, shear_rate=0.4, rc=1.0, skin=0.2, eps=0.0, cells=(3, 3, 3), seed=5,
               max_neighbors=6000)
    _log(f"dense sort n={n} cells=27")
    sim = Sim(p, x, u, step0=9)
    out = sim.build_cells(want_pairs=False)
    _log(f"dense sort: largest list {sim.stats()['max_neighbors']}")
    op = _oracle_params(p)
    Delta = O.offset(9, p.dt, p.shear_rate, p.box[0], p.box[1])
    xw, uw = O.le_wrap(x, u, Delta, op)
    cell_ref, order_ref = O.cells(xw, (3, 3, 3), p.box)
    assert np.array_equal(out["cell_of"], cell_ref)
    assert np.array_equal(out["order"], order_ref)
    xs, us, _, _ = sim.state()
    assert np.array_equal(xs, xw) and np.array_equal(us, uw)
    sim.close()
    # sparse: 500 particles over 21^3 cells
    m = 500
    sbox = (30.0, 30.0, 30.0)
    xs0 = np.stack([rng.uniform(0.0, sbox[a], m) for a in range(3)])
    us0 = rng.normal(size=(3, m))
    ps = Params(n=m, box=sbox, shear_rate=0.2, rc=2 ** (1 / 6), pair="wca", skin=0.3, seed=6)
    _check_cells_pairs(xs0, us0, ps, 31)


# ------------------------------------------------------------------ forces, stress
def _forces_case(w_x, w_u, p: Params, step0, tol_f, tol_w, method=0):
    sim = Sim(p, w_x, w_u, step0=step0)
    F, W = sim.forces()
    sig = sim.stress()
    op = _oracle_params(p)
    Delta = O.offset(step0, p.dt, p.shear_rate, p.box[0], p.box[1])
    xw, uw = O.le_wrap(w_x, w_u, Delta, op)
    Fr, Wr, _ = O.forces(xw, Delta, op, method)
    sr = O.stress(xw, uw, Wr, op)
    ef = e_F(F, Fr)
    ew = np.abs(W - Wr).max() / np.abs(Wr).max()
    # shear-stress error relative to the scale of the stress contributions
    es = abs(sig[3] - sr[3]) / max(abs(sr[3]), 1e-3 * np.abs(sr[:3]).max())
    _log(f"forces n={p.n} prec={p.precision} e_F={ef:.3e} e_W={ew:.3e} e_sxy={es:.3e}")
    assert ef <= tol_f
    assert ew <= tol_w
    assert es <= max(tol_w, 1e-10 if p.precision == "fp64" else 1e-4)
    sim.close()
    return ef, ew


# tune: 0 = layout chosen from density, 1 = LDS halo, 2 = partners from global memory
@pytest.mark.parametrize("tune", [0, 2])
@pytest.mark.parametrize("frac", [0.0, 0.3, 0.999])
def test_forces_fp64_lj(frac, tune):
    w, p = _lj_case(tune=tune)
    _forces_case(w.x, w.u, p, _step0_for_fraction(p, frac), 1e-12, 1e-12)


@pytest.mark.parametrize("tune", [0, 2])
@pytest.mark.parametrize("frac", [0.0, 0.6])
def test_forces_mixed_lj(frac, tune):
    w, p = _lj_case(precision="mixed", tune=tune)
    _forces_case(w.x, w.u, p, _step0_for_fraction(p, frac), 1e-5, 1e-4)


@pytest.mark.parametrize("tune", [0, 1, 2])
def test_forces_fp64_kg_fene(tune):
    w, p = _kg_case(tune=tune)
    _forces_case(w.x, w.u, p, 777, 1e-12, 1e-12)


@pytest.mark.parametrize("tune", [0, 1, 2])
def test_forces_fp64_kg_angles(tune):
    """KG chains with the cosine angle term: forces and virial (the angle's
    virial counted once, at its middle bead) against the oracle."""
    w, p = _kg_case(tune=tune, angle_k=1.5)
    _forces_case(w.x, w.u, p, 4321, 1e-12, 1e-12)


def test_kg_angles_trajectory():
    w, p = _kg_case(angle_k=1.5, skin=0.4, shear_rate=0.05)
    sim = Sim(p, w.x, w.u)
    ref = O.Sim(w.x, w.u, _oracle_params(p))
    ring = sim.step(60, sample_every=10)
    sref = ref.run(60, sample_every=10)
    gx, gu, gf, st = sim.state()
    L = np.array(p.box)[:, None]
    dx = gx - ref.x
    dx = dx - L * np.round(dx / L)
    _log(f"kg angles trajectory max|dx|={np.abs(dx).max():.3e}")
    assert np.abs(dx).max() < 1e-8
    assert e_F(gf, ref.F) < 1e-7
    assert np.abs(ring.cpu().numpy() - sref).max() / np.abs(sref[:, :3]).max() < 1e-9
    sim.close()


@pytest.mark.parametrize("tune", [0, 1])
def test_forces_mixed_kg(tune):
    w, p = _kg_case(precision="mixed", tune=tune)
    _forces_case(w.x, w.u, p, 777, 1e-5, 1e-4)


def test_forces_ragged():
    rng = np.random.default_rng(9)
    for n in (2, 3, 255, 257, 1000):
        L = max((n / 0.5) ** (1 / 3), 3 * 2.81)
        x = rng.uniform(0, L, size=(3, n))
        # avoid overlaps that make the energy scale meaningless
        u = rng.normal(size=(3, n))
        p = Params(n=n, box=(L, L, L), shear_rate=0.2, eps=1e-3, seed=2)
        sim = Sim(p, x, u, step0=91)
        F, W = sim.forces()
        op = _oracle_params(p)
        Delta = O.offset(91, p.dt, p.shear_rate, L, L)
        xw, _ = O.le_wrap(x, u, Delta, op)
        Fr, Wr, _ = O.forces(xw, Delta, op)
        if np.abs(Fr).max() > 0:
            assert np.abs(F - Fr).max() <= 1e-12 * max(1.0, np.abs(Fr).max()) * 10
        else:
            assert np.abs(F).max() == 0.0
        sim.close()


# ------------------------------------------------------------------ dynamics
def test_ideal_gas_trajectory_bitwise_skin0():
    """No pair force (eps = 0) and a rebuild every step: integrator, Lees-Edwards
    crossing, Langevin force and Philox noise reproduce the oracle bit for bit."""
    rng = np.random.default_rng(4)
    n, L = 500, 9.0
    x = rng.uniform(0, L, size=(3, n))
    c = inputs.maxwell(n, 1.0, 1.0, 5)
    u = inputs.streaming_initial_velocity(x, c, 0.9, L)
    p = Params(n=n, box=(L, L, L), shear_rate=0.9, eps=0.0, rc=1.0, skin=0.0, gamma=1.3, kT=1.1,
               dt=0.01, seed=77)
    sim = Sim(p, x, u, step0=3)
    ref = O.Sim(x, u, _oracle_params(p), step0=3)
    for _ in range(4):
        sim.step(50)
        ref.run(50)
        gx, gu, gf, st = sim.state()
        assert st == ref.step
        assert np.array_equal(gx, ref.x)
        assert np.array_equal(gu, ref.u)
        assert np.array_equal(gf, ref.F)
    sim.close()


@pytest.mark.parametrize("skin,tune", [(0.0, 0), (0.3, 0), (0.3, 2)])
def test_lj_trajectory_100_steps(skin, tune):
    w, p = _lj_case(shear_rate=0.5, skin=skin, tune=tune)
    sim = Sim(p, w.x, w.u, step0=0)
    ref = O.Sim(w.x, w.u, _oracle_params(p), step0=0)
    ring = sim.step(100, sample_every=10)
    sref = ref.run(100, sample_every=10)
    gx, gu, gf, st = sim.state()
    assert st == 100 == ref.step
    L = np.array(p.box)[:, None]
    dx = gx - ref.x
    dx = dx - L * np.round(dx / L)  # an x-wrap of either side is an L_x shift
    _log(f"traj skin={skin}: max|dx|={np.abs(dx).max():.3e} max|du|={np.abs(gu - ref.u).max():.3e}")
    assert np.abs(dx).max() < 1e-8
    # velocities of particles that sit at the faces may differ by one jump if the
    # two sides resolved a crossing on different sides of the face: compare peculiar
    cg = gu[0] - p.shear_rate * (gx[1] - p.box[1] / 2)
    cr = ref.u[0] - p.shear_rate * (ref.x[1] - p.box[1] / 2)
    assert np.abs(cg - cr).max() < 1e-7
    assert np.abs(gu[1:] - ref.u[1:]).max() < 1e-7
    sg = ring.cpu().numpy()
    scale = np.abs(sref[:, :3]).max()
    assert np.abs(sg - sref).max() / scale < 1e-9
    st_ = sim.stats()
    _log(f"rebuilds={st_['rebuilds']} max_nb={st_['max_neighbors']}")
    sim.close()


def test_determinism_and_exact_restart():
    w, p = _lj_case(shear_rate=0.3)
    a = Sim(p, w.x, w.u)
    a.step(40)
    xa, ua, fa, sa = a.state()
    a.step(40)
    xa2, ua2, fa2, sa2 = a.state()
    b = Sim(p, w.x, w.u)
    b.step(40)
    xb, ub, fb, sb = b.state()
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub) and np.array_equal(fa, fb)
    c = Sim(p, xb, ub, step0=sb, f0=fb)
    c.step(40)
    xc, uc, fc, sc = c.state()
    assert sc == sa2
    assert np.array_equal(xa2, xc) and np.array_equal(ua2, uc) and np.array_equal(fa2, fc)
    for s in (a, b, c):
        s.close()


def _check_observables(got, ref, tag):
    assert np.array_equal(got["count"], ref["count"]), tag
    scale = max(np.abs(ref["sum_ux"]).max(), 1.0)
    assert np.abs(got["sum_ux"] - ref["sum_ux"]).max() / scale < 1e-12, tag
    assert np.abs(got["sum_mc2"] - ref["sum_mc2"]).max() / ref["sum_mc2"].max() < 1e-12, tag
    assert abs(got["kT"] - ref["kT"]) / ref["kT"] < 1e-12, tag
    assert np.abs(got["com"] - ref["com"]).max() < 1e-12 * max(1.0, np.abs(ref["com"]).max() * 1e3), tag


@pytest.mark.parametrize("nbins", [1, 50, 256])
def test_observables_mid_run(nbins):
    """y-profiles, kinetic temperature and CoM velocity of a state whose
    pending boundary crossings are not yet applied (lazy wrap between
    rebuilds) against the oracle on the same state."""
    w, p = _lj_case(shear_rate=0.5, skin=0.3)
    sim = Sim(p, w.x, w.u, step0=0)
    sim.step(37)
    got = sim.observables(nbins)
    x, u, f, step = sim.state()
    ref = O.observables(x, u, 0.0, _oracle_params(p), nbins=nbins)
    assert got["count"].sum() == p.n
    _check_observables(got, ref, nbins)
    sim.close()


def test_observables_along_a_run_with_pending_crossings():
    """Observables every few steps of a sheared run with a skin, so that many
    particles have crossed a face without being wrapped yet, against the oracle
    run beside it (trajectories agree to ~1e-9, hence the looser bounds)."""
    w, p = _lj_case(shear_rate=0.8, skin=0.4)
    sim = Sim(p, w.x, w.u, step0=0)
    ref = O.Sim(w.x, w.u, _oracle_params(p), step0=0)
    for k in range(6):
        sim.step(7)
        ref.run(7)
        got = sim.observables(20)
        want = O.observables(ref.x, ref.u, ref.Delta, ref.p, nbins=20)
        assert np.array_equal(got["count"], want["count"]), k
        assert np.abs(got["sum_ux"] - want["sum_ux"]).max() < 1e-6, k
        assert np.abs(got["sum_mc2"] - want["sum_mc2"]).max() < 1e-6, k
        assert abs(got["kT"] - want["kT"]) < 1e-9, k
        assert np.abs(got["com"] - want["com"]).max() < 1e-9, k
    assert sim.stats()["rebuilds"] < 40
    sim.close()


def test_msd_matches_oracle():
    """Unwrapped y, z and their mean squared displacement over a sheared run
    in a small box (many face crossings) against the oracle's unwrapped
    coordinates, accumulated from per-step minimum-image increments."""
    w, p = _lj_case(n_side=8, shear_rate=1.0, skin=0.3, kT=2.0)
    p.dt = 0.01
    sim = Sim(p, w.x, w.u, step0=0)
    ref = O.Sim(w.x, w.u, _oracle_params(p), step0=0)
    r_gpu = sim.unwrapped(host=False)
    r0 = sim.unwrapped()
    # the origin of the wrap counts is the input
    assert np.abs(r0 - np.asarray(w.x)[1:]).max() < 1e-12
    unw = ref.x[1:].copy()
    r_ref = unw.copy()
    for k in range(4):
        sim.step(25)
        unw = ref.run_tracked(25, unw)
        m_gpu = sim.msd(r_gpu)
        m_ref = O.msd(unw, r_ref)
        g = sim.unwrapped()
        dg = g - r0
        dr = unw - r_ref
        assert np.abs(dg - dr).max() < 1e-8, k
        assert np.allclose(m_gpu, m_ref, rtol=1e-7), (k, m_gpu, m_ref)
    outside = (unw[0] < 0) | (unw[0] >= p.box[1])
    assert outside.sum() >= 5  # particles that crossed a sheared face
    sim.close()


def test_observables_rejects_bad_bins():
    w, p = _lj_case()
    sim = Sim(p, w.x, w.u)
    for nb in (0, B.LE_MAX_BINS + 1):
        with pytest.raises(B.LeError) as e:
            sim.observables(nb)
        assert e.value.code == B.LE_E_ARG
    sim.close()


# ------------------------------------------------------------------ errors
def test_bond_break_is_latched():
    x = np.array([[1.0, 2.6, 5.0, 7.0], [5.0, 5.0, 5.0, 5.0], [5.0, 5.0, 5.0, 5.0]])
    u = np.zeros((3, 4))
    p = Params(n=4, box=(9.0, 9.0, 9.0), rc=2 ** (1 / 6), pair="wca", n_chains=2, chain_len=2,
               gamma=0.0, kT=0.0, dt=0.001)
    sim = Sim(p, x, u)
    with pytest.raises(B.LeError) as e:
        sim.sync()
    assert e.value.code == B.LE_E_BOND
    with pytest.raises(B.LeError):
        sim.step(1)
    sim.close()


def test_nonfinite_is_latched():
    w, p = _lj_case()
    x = w.x.copy()
    x[1, 17] = np.nan
    sim = Sim(p, x, w.u)
    with pytest.raises(B.LeError) as e:
        sim.sync()
    assert e.value.code == B.LE_E_NONFINITE
    sim.close()


def test_neighbor_capacity_is_latched():
    w, p = _lj_case(max_neighbors=8)
    sim = Sim(p, w.x, w.u)
    with pytest.raises(B.LeError) as e:
        sim.sync()
    assert e.value.code == B.LE_E_CAPACITY
    sim.close()


# ------------------------------------------------------------------ full-size samples
def test_full_size_lj_256k_sampled():
    """The 256,000-particle LJ system at its real size (the benchmarked
    configuration): cells bit-exact, pair set at r_list bit-exact, forces at
    400 sampled particles within 1e-12, observables."""
    w = inputs.lj_workload(n=256000, shear_rate=0.1, seed=21)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=0.1, seed=21)
    step0 = 7777
    sim = Sim(p, w.x, w.u, step0=step0)
    out = sim.build_cells()
    op = _oracle_params(p)
    Delta = O.offset(step0, p.dt, p.shear_rate, p.box[0], p.box[1])
    xw, uw = O.le_wrap(w.x, w.u, Delta, op)
    nc = tuple(int(math.floor(p.box[a] / (p.rlist * (1 + 1e-9)))) for a in range(3))
    cref, oref = O.cells(xw, nc, p.box)
    assert np.array_equal(out["cell_of"], cref) and np.array_equal(out["order"], oref)
    ref = O.pairs_cells(xw, Delta, p.box, p.rlist)
    key = lambda a: np.sort(np.minimum(a[:, 0], a[:, 1]).astype(np.int64) * p.n + np.maximum(a[:, 0], a[:, 1]))
    assert np.array_equal(key(out["pairs"]), key(ref))
    F, W = sim.forces()
    rng = np.random.default_rng(0)
    ys = np.argsort(xw[1])
    idx = np.concatenate([ys[:100], ys[-100:], rng.choice(p.n, 200, replace=False)])
    Fs = O.forces_sample(xw, Delta, op, idx)
    rms = math.sqrt(float((Fs ** 2).sum(axis=1).mean()))
    err = float(np.sqrt(((F[:, idx].T - Fs) ** 2).sum(axis=1)).max()) / rms
    _log(f"256k sampled e_F={err:.3e}")
    assert err <= 1e-12
    _check_observables(sim.observables(50), O.observables(xw, uw, Delta, op, nbins=50), "256k")
    sim.close()


@pytest.mark.parametrize("angle_k", [0.0, 1.5])
def test_full_size_kg_400k_sampled(angle_k):
    """The Kremer-Grest melt at its benchmarked size (2000 chains x 200 beads,
    WCA + FENE, with and without the cosine angle term): cells bit-exact,
    pair set at r_list bit-exact, forces with bonds at 300 sampled beads
    within 1e-12."""
    w, p = _kg_case(n_chains=2000, chain_len=200, shear_rate=0.01, angle_k=angle_k)
    step0 = 4321
    sim = Sim(p, w.x, w.u, step0=step0)
    out = sim.build_cells()
    op = _oracle_params(p)
    Delta = O.offset(step0, p.dt, p.shear_rate, p.box[0], p.box[1])
    xw, uw = O.le_wrap(w.x, w.u, Delta, op)
    nc = tuple(int(math.floor(p.box[a] / (p.rlist * (1 + 1e-9)))) for a in range(3))
    cref, oref = O.cells(xw, nc, p.box)
    assert np.array_equal(out["cell_of"], cref) and np.array_equal(out["order"], oref)
    ref = O.pairs_cells(xw, Delta, p.box, p.rlist)
    key = lambda a: np.sort(np.minimum(a[:, 0], a[:, 1]).astype(np.int64) * p.n + np.maximum(a[:, 0], a[:, 1]))
    assert np.array_equal(key(out["pairs"]), key(ref))
    F, W = sim.forces()
    rng = np.random.default_rng(3)
    ys = np.argsort(xw[1])
    idx = np.concatenate([ys[:75], ys[-75:], rng.choice(p.n, 150, replace=False)])
    Fs = O.forces_sample(xw, Delta, op, idx)
    rms = math.sqrt(float((Fs ** 2).sum(axis=1).mean()))
    err = float(np.sqrt(((F[:, idx].T - Fs) ** 2).sum(axis=1)).max()) / rms
    _log(f"kg 400k sampled e_F={err:.3e}")
    assert err <= 1e-12
    sim.close()


def test_graph_replays_match_eager():
    """A captured chunk of steps replayed several times, with eager work and
    synchronisations between replays (state read-out, observables, an odd
    eager step count), equals the same chunks run eagerly, bit for bit."""
    w, p = _lj_case(shear_rate=0.4, skin=0.3)
    a = Sim(p, w.x, w.u)
    sb = torch.cuda.Stream()
    b = Sim(p, w.x, w.u, stream=sb)
    ring_a = torch.zeros((5, 6), dtype=torch.float64, device=DEV)
    with torch.cuda.stream(sb):
        ring_b = torch.zeros((5, 6), dtype=torch.float64, device=DEV)
    sb.synchronize()
    g = b.graph(50, sample_every=10, ring=ring_b)
    for rep in range(4):
        a.step(50, sample_every=10, ring=ring_a)
        g.launch()
        b.sync()
        xa, ua, fa, sta = a.state()
        xb, ub, fb, stb = b.state()
        assert sta == stb
        assert np.array_equal(xa, xb) and np.array_equal(ua, ub) and np.array_equal(fa, fb), rep
        torch.cuda.synchronize()
        assert torch.equal(ring_a, ring_b), rep
        oa, ob = a.observables(10), b.observables(10)
        assert np.array_equal(oa["sum_ux"], ob["sum_ux"])
        if rep == 1:  # an odd eager count in both
            a.step(3)
            b.step(3)
    g.close()
    a.close()
    b.close()


def test_graph_on_default_stream_is_refused():
    w, p = _lj_case()
    sim = Sim(p, w.x, w.u)  # torch's default stream
    with pytest.raises(B.LeError) as e:
        sim.graph(10)
    assert e.value.code == B.LE_E_STATE
    sim.close()
