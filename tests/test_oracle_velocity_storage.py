"""Pins of the oracle's peculiar-velocity storage (Section 2.2: the stored
velocity is the peculiar part of Eq. vi and the streaming velocity enters
only the propagation of the coordinates):

* without shear it is the lab-velocity dynamics, bit for bit;
* free particles keep their stored velocity exactly, also across the
  sheared faces, and move along x with the streaming velocity of their
  height (closed form);
* a sheared ideal gas keeps the equilibrium moments (no -gamma_dot c_y
  coupling, so no heating and no kinetic shear stress) while the lab flow
  profile stays linear: the difference from the lab-velocity form.
"""
import numpy as np
import pytest

import oracle as O
from paper_2109_11083_amd import inputs


def _gas(shear_rate, gamma, velocity, kT=1.0, n=500, L=8.0, seed=9, dt=0.005):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, L, size=(3, n))
    c = inputs.maxwell(n, kT, 1.0, seed + 1)
    p = O.make_params(n, (L, L, L), shear_rate=shear_rate, gamma=gamma, kT=kT, eps=0.0, rc=0.5,
                      seed=seed, dt=dt, velocity=velocity)
    u = c if velocity == "peculiar" else inputs.streaming_initial_velocity(x, c, shear_rate, L)
    return O.Sim(x, u, p)


def test_equal_to_lab_storage_without_shear():
    w = inputs.lj_workload(n_side=8, shear_rate=0.0, seed=3)
    a = O.Sim(w.x, w.u, O.make_params(w.x.shape[1], w.box, seed=3, velocity="lab"))
    b = O.Sim(w.x, w.u, O.make_params(w.x.shape[1], w.box, seed=3, velocity="peculiar"))
    a.run(40); b.run(40)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.u, b.u)


def test_free_particles_closed_form():
    sr, L, dt = 0.6, 8.0, 0.01
    sim = _gas(sr, 0.0, "peculiar", L=L, dt=dt)
    x0, u0 = sim.x.copy(), sim.u.copy()
    nst = 400
    crossed = np.zeros(sim.n, bool)
    for _ in range(nst):
        y = sim.x[1].copy()
        sim.run(1)
        crossed |= np.abs(sim.x[1] - y) > L / 2
    assert crossed.sum() > 20
    # the stored velocity never changes (no jump at the faces)
    assert np.array_equal(sim.u, u0)
    # x_n = x_0 + n dt (u_x + gamma_dot (y_0 - L/2)) + gamma_dot dt^2 u_y n (n - 1) / 2 (mod L_x)
    k = ~crossed
    want = x0[0] + nst * dt * (u0[0] + sr * (x0[1] - L / 2)) + sr * dt * dt * u0[1] * nst * (nst - 1) / 2
    d = sim.x[0] - want
    d -= L * np.round(d / L)
    assert np.abs(d[k]).max() < 1e-9


@pytest.mark.slow
def test_sheared_gas_keeps_equilibrium_moments():
    sr, gamma, kT = 0.8, 1.0, 1.0
    out = {}
    for vel in ("peculiar", "lab"):
        sim = _gas(sr, gamma, vel)
        L = sim.p.box[1]
        sim.run(400)
        cxy, cxx, sxy, cnt, sux = [], [], [], np.zeros(8), np.zeros(8)
        for _ in range(100):
            s = sim.run(40, sample_every=40)
            sxy.append(s[0, 3])
            cx = sim.u[0] if vel == "peculiar" else sim.u[0] - sr * (sim.x[1] - L / 2)
            cxy.append((cx * sim.u[1]).mean())
            cxx.append((cx ** 2).mean())
            ob = O.observables(sim.x, sim.u, sim.Delta, sim.p, nbins=8)
            cnt += ob["count"]; sux += ob["sum_ux"]
        centres = (np.arange(8) + 0.5) / 8 * L
        out[vel] = dict(cxy=np.mean(cxy), cxx=np.mean(cxx), sxy=np.mean(sxy),
                        slope=np.polyfit(centres, sux / cnt, 1)[0], rho=sim.n / L ** 3)
    pe, lb = out["peculiar"], out["lab"]
    assert abs(pe["cxy"]) < 0.03
    assert pe["cxx"] == pytest.approx(kT, rel=0.04)
    assert abs(pe["sxy"]) < 0.03 * pe["rho"]
    assert pe["slope"] == pytest.approx(sr, rel=0.05)
    # the lab-velocity form couples c_x to c_y: <c_x c_y> = -gamma_dot kT / (2 gamma)
    assert lb["cxy"] == pytest.approx(-sr * kT / (2 * gamma), rel=0.12)
