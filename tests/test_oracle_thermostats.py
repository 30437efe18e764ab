"""Pins of the oracle's other two thermostats (Section 2.2):

* DPD (Eqs. dissipative, random, omega): pair-symmetric uniform noise, forces
  worked out by hand for two particles (also across the sheared face, where
  the image's streaming velocity enters), exact momentum conservation, the
  fluctuation-dissipation balance (kinetic temperature = kT) and a linear flow
  profile under shear;
* Langevin friction on the lab velocity (xi_abs): identical to the peculiar
  form without shear, and under shear it drags the flow profile flat, which
  is the failure the paper reports for it.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2109_11083_amd import inputs


def test_dpd_noise_pair_symmetric_uniform():
    th = np.array([O.dpd_theta(9, s, i, j) for s in range(40) for i in range(30) for j in range(i + 1, 30)])
    assert np.all(np.abs(th) < 0.5)
    assert abs(th.mean()) < 0.005
    assert th.var() == pytest.approx(1.0 / 12.0, rel=0.02)
    for s, i, j in [(0, 0, 1), (7, 3, 1000), (2 ** 33 + 5, 123456, 7)]:
        assert O.dpd_theta(4, s, i, j) == O.dpd_theta(4, s, j, i)
    # successive steps and neighbouring pairs are uncorrelated
    a = np.array([O.dpd_theta(3, s, 1, 2) for s in range(4000)])
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 0.05
    b = np.array([O.dpd_theta(3, s, 1, 3) for s in range(4000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.05
    # the pair stream is not the per-particle Langevin stream
    assert O.dpd_theta(3, 5, 0, 7) != O.noise(3, 5, 7)[0]


def _two(xi, xj, ui, uj, L=6.0, shear_rate=0.0, gamma=2.0, dpd_rc=1.0):
    x = np.array([xi, xj], dtype=float).T.copy()
    u = np.array([ui, uj], dtype=float).T.copy()
    # no conservative force, no noise (kT = 0): only the DPD dissipative term
    p = O.make_params(2, (L, L, L), shear_rate=shear_rate, gamma=gamma, kT=0.0, eps=0.0, rc=1.0,
                      thermostat="dpd", dpd_rc=dpd_rc)
    return O.Sim(x, u, p).F


def test_dpd_two_particles_by_hand():
    # i behind j on the x axis, moving towards it at speed 1: 0.5 apart, so
    # w = 1 - 0.5 = 0.5 and the drag on i is gamma w^2 = 0.5 backwards.
    F = _two([1.0, 1.0, 1.0], [1.5, 1.0, 1.0], [1.0, 0.3, -0.2], [0.0, 0.0, 0.0])
    assert F[:, 0] == pytest.approx([-0.5, 0.0, 0.0], abs=1e-15)
    assert F[:, 1] == pytest.approx([0.5, 0.0, 0.0], abs=1e-15)
    # motion perpendicular to the bond is not damped
    F = _two([1.0, 1.0, 1.0], [1.5, 1.0, 1.0], [0.0, 0.7, -0.4], [0.0, -0.1, 0.3])
    assert np.abs(F).max() == 0.0
    # outside dpd_rc nothing acts
    F = _two([1.0, 1.0, 1.0], [2.0, 1.0, 1.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0])
    assert np.abs(F).max() == 0.0


def test_dpd_across_the_sheared_face():
    """i sits just above y = 0, j just below y = L_y; the image of j that i
    sees lies one box down and streams slower by shear_rate L_y, so two
    particles at rest in the lab frame still separate along x."""
    L, sr, g = 6.0, 0.1, 2.0
    xi, xj = [1.3, 0.2, 1.0], [1.0, L - 0.3, 1.0]
    F = _two(xi, xj, [0, 0, 0], [0, 0, 0], L=L, shear_rate=sr, gamma=g)
    d = np.array([0.3, 0.5, 0.0])
    r = np.linalg.norm(d)
    e = d / r
    w = 1.0 - r
    ev = e[0] * sr * L     # relative velocity (+shear_rate L_y, 0, 0)
    expect = -g * w * w * ev * e
    assert F[:, 0] == pytest.approx(expect, rel=1e-13)
    assert F[:, 1] == pytest.approx(-expect, rel=1e-13)
    # separating along +x, so i is pulled back: both components negative
    assert F[0, 0] < 0 and F[1, 0] < 0


def _lj_dpd(shear_rate, gamma, kT=1.0, seed=11, dt=0.005):
    w = inputs.lj_workload(n_side=8, shear_rate=shear_rate, kT=kT, seed=seed)
    p = O.make_params(w.x.shape[1], w.box, shear_rate=shear_rate, gamma=gamma, kT=kT, seed=seed, dt=dt,
                      thermostat="dpd")
    return O.Sim(w.x, w.u, p), w


def test_dpd_conserves_momentum_without_shear():
    sim, _ = _lj_dpd(0.0, 5.0)
    P0 = sim.u.sum(axis=1)
    sim.run(60)
    assert np.abs(sim.u.sum(axis=1) - P0).max() < 1e-10
    # the thermostat did work on the system (it is not switched off)
    assert np.abs(sim.F).max() > 1.0


def test_dpd_momentum_only_through_velocity_jump():
    """Under shear the pair terms still cancel, so as without thermostat the lab
    momentum P_x changes only by -m shear_rate L_y per upward face crossing."""
    sr = 0.5
    sim, w = _lj_dpd(sr, 5.0)
    L = w.box[1]
    P0 = sim.u.sum(axis=1)
    ups = downs = 0
    for _ in range(250):
        y0 = sim.x[1].copy()
        sim.run(1)
        dy = sim.x[1] - y0
        ups += int((dy < -L / 2).sum())
        downs += int((dy > L / 2).sum())
    P = sim.u.sum(axis=1)
    assert ups + downs > 5
    assert abs(P[1] - P0[1]) < 1e-9 and abs(P[2] - P0[2]) < 1e-9
    assert P[0] - P0[0] == pytest.approx(-sr * L * (ups - downs), abs=1e-8)


def _dpd_gas(shear_rate, gamma, kT, n=500, L=8.0, seed=5, dt=0.005):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, L, size=(3, n))
    c = inputs.maxwell(n, kT, 1.0, seed + 1)
    u = inputs.streaming_initial_velocity(x, c, shear_rate, L)
    p = O.make_params(n, (L, L, L), shear_rate=shear_rate, gamma=gamma, kT=kT, eps=0.0, rc=1.0,
                      seed=seed, dt=dt, thermostat="dpd", dpd_rc=1.0)
    return O.Sim(x, u, p)


@pytest.mark.slow
@pytest.mark.parametrize("gamma,kT", [(5.0, 1.0), (25.0, 0.5)])
def test_dpd_gas_fluctuation_dissipation(gamma, kT):
    """Noise amplitude and friction balance: with only DPD forces acting, the
    stationary kinetic temperature (3N - 3 degrees of freedom, total momentum
    fixed) equals kT.  A wrong prefactor or weight power shifts it."""
    sim = _dpd_gas(0.0, gamma, kT)
    sim.u = sim.u - sim.u.mean(axis=1, keepdims=True)
    sim.run(200)
    ks = []
    for _ in range(60):
        sim.run(10)
        ks.append(O.observables(sim.x, sim.u, sim.Delta, sim.p)["kT"])
    assert np.mean(ks) == pytest.approx(kT, rel=0.03)


@pytest.mark.slow
def test_dpd_gas_linear_profile_under_shear():
    sr = 0.5
    sim = _dpd_gas(sr, 5.0, 1.0)
    L = sim.p.box[1]
    sim.run(200)
    nb = 8
    cnt, sux, ks = np.zeros(nb), np.zeros(nb), []
    for _ in range(80):
        sim.run(10)
        ob = O.observables(sim.x, sim.u, sim.Delta, sim.p, nbins=nb)
        cnt += ob["count"]; sux += ob["sum_ux"]; ks.append(ob["kT"])
    centres = (np.arange(nb) + 0.5) / nb * L
    slope, icpt = np.polyfit(centres, sux / cnt, 1)
    assert slope == pytest.approx(sr, rel=0.08)
    assert abs(icpt + sr * L / 2) < 0.25
    # viscous heating: DPD removes it only through relative motion, so the
    # gas runs warmer than kT (Section 3.1 reports the same at high shear)
    assert 1.0 < np.mean(ks) < 1.4


def _gas(shear_rate, thermostat, gamma=1.0, kT=1.0, n=600, L=9.0, seed=5):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, L, size=(3, n))
    c = inputs.maxwell(n, kT, 1.0, seed + 1)
    u = inputs.streaming_initial_velocity(x, c, shear_rate, L)
    p = O.make_params(n, (L, L, L), shear_rate=shear_rate, gamma=gamma, kT=kT, eps=0.0, rc=0.5,
                      seed=seed, dt=0.005, thermostat=thermostat)
    return O.Sim(x, u, p)


def test_lab_velocity_langevin_equals_peculiar_without_shear():
    a = _gas(0.0, "langevin")
    b = _gas(0.0, "langevin_abs")
    a.run(30); b.run(30)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.u, b.u)


@pytest.mark.slow
def test_lab_velocity_langevin_flattens_profile():
    """With the friction on the lab velocity every particle is pulled towards
    rest, so between the sheared faces the mean flow decays and the profile
    loses the imposed slope (Section 3.1); the peculiar form keeps it."""
    sr, gamma = 0.8, 1.0
    out = {}
    for th in ("langevin", "langevin_abs"):
        sim = _gas(sr, th, gamma=gamma)
        L = sim.p.box[1]
        sim.run(400)
        nb = 9
        cnt, sux = np.zeros(nb), np.zeros(nb)
        for _ in range(60):
            sim.run(20)
            ob = O.observables(sim.x, sim.u, sim.Delta, sim.p, nbins=nb)
            cnt += ob["count"]; sux += ob["sum_ux"]
        centres = (np.arange(nb) + 0.5) / nb * L
        out[th] = (np.polyfit(centres, sux / cnt, 1)[0], sux / cnt)
    assert out["langevin"][0] == pytest.approx(sr, rel=0.06)
    assert out["langevin_abs"][0] < 0.35 * sr
    # the middle of the box is (nearly) at rest
    prof = out["langevin_abs"][1]
    assert np.abs(prof[3:6]).max() < 0.25


def test_dpd_grid_and_brute_force_pairs_agree():
    """The DPD pair terms summed over the grid's pairs (method 1) equal the
    brute-force sum (method 0) to rounding, also across the sheared faces."""
    w = inputs.lj_workload(n_side=8, shear_rate=0.7, seed=5)
    p = O.make_params(w.x.shape[1], w.box, shear_rate=0.7, gamma=5.0, seed=5, thermostat="dpd")
    a = O.Sim(w.x, w.u, p, step0=123, method=0)
    b = O.Sim(w.x, w.u, p, step0=123, method=1)
    scale = np.abs(a.F).max()
    assert np.abs(a.F - b.F).max() < 1e-12 * scale


def test_dpd_sampled_sum_matches_full_sum():
    """The per-particle DPD sum used to check large systems equals the pair
    loop of the thermostat (total force minus the conservative force)."""
    w = inputs.lj_workload(n_side=8, shear_rate=0.6, seed=8)
    p = O.make_params(w.x.shape[1], w.box, shear_rate=0.6, gamma=5.0, seed=8, thermostat="dpd")
    step0 = 4242
    sim = O.Sim(w.x, w.u, p, step0=step0, method=0)
    Fc, _, _ = O.forces(sim.x, sim.Delta, p)
    idx = np.array([0, 3, 77, 200, 311, 511])
    G = O.dpd_sample(sim.x, sim.u, sim.Delta, p, step0, idx)
    assert np.allclose(G, (sim.F - Fc)[:, idx].T, rtol=0, atol=1e-11 * np.abs(sim.F).max())
    assert np.abs(G).max() > 1.0
