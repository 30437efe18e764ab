"""Pins of the oracle's cosine angle term of the Kremer-Grest chains (Eq.
angle, read as V = k_a (1 + cos theta) with the minimum at theta_0 = 180 deg):
hand values for a right angle and a straight chain, forces as minus the
energy gradient, the virial as the affine-strain derivative of the energy
(angles that straddle the sheared faces included), and the per-particle
sampled sum equal to the full one.
"""
import numpy as np
import pytest

import oracle as O
from paper_2109_11083_amd import inputs


def _trimer(a, j, b, k=1.5, L=10.0):
    x = np.array([a, j, b], dtype=float).T.copy()
    # no pair force, FENE constant 0: only the angle term acts
    p = O.make_params(3, (L, L, L), eps=0.0, rc=1.0, chain_len=3, n_chains=1, angle_k=k, fene_k=0.0)
    F, W, e = O.forces(x, 0.0, p)
    return F, W, e


def test_right_angle_by_hand():
    k = 1.5
    F, W, e = _trimer([3.0, 2.0, 2.0], [2.0, 2.0, 2.0], [2.0, 3.0, 2.0], k=k)
    # cos = 0: V = k; the force opens the angle, a pushed away from b and back
    assert e == pytest.approx(k, abs=1e-15)
    assert F[:, 0] == pytest.approx([0.0, -k, 0.0], abs=1e-15)
    assert F[:, 2] == pytest.approx([-k, 0.0, 0.0], abs=1e-15)
    assert F[:, 1] == pytest.approx([k, k, 0.0], abs=1e-15)
    # virial b1 (x) F_a + b2 (x) F_b: xy = 1 * (-k) + 0, yx is W of (y, x) = 0 + 1 * (-k)
    assert W[3] == pytest.approx(-k, abs=1e-15)
    assert W[0] == pytest.approx(0.0, abs=1e-15) and W[1] == pytest.approx(0.0, abs=1e-15)


def test_straight_chain_has_no_bending_force():
    F, W, e = _trimer([1.0, 2.0, 2.0], [2.0, 2.0, 2.0], [3.0, 2.0, 2.0])
    assert np.abs(F).max() == 0.0
    assert e == 0.0
    # a slight bend is pushed back towards the straight line
    F, W, e = _trimer([1.0, 2.1, 2.0], [2.0, 2.0, 2.0], [3.0, 2.1, 2.0])
    assert F[1, 0] < 0 and F[1, 2] < 0 and F[1, 1] > 0 and e > 0


def _melt(shear_rate=0.0):
    w = inputs.kg_workload(6, 12, shear_rate=shear_rate, seed=7)
    p = O.make_params(w.x.shape[1], w.box, rc=2 ** (1 / 6), pair="wca", chain_len=12, n_chains=6,
                      angle_k=1.5, lj_shift=1.0)
    return w, p


def test_forces_are_minus_energy_gradient():
    w, p = _melt()
    Delta = 0.43 * w.box[0]
    xw, _ = O.le_wrap(w.x, None, Delta, p)
    F, _, _ = O.forces(xw, Delta, p)
    h = 1e-6
    ys = xw[1]
    cand = [0, 1, 5, 11, 12, 40] + list(np.argsort(ys)[:3]) + list(np.argsort(ys)[-3:])
    for i in cand:
        for a in range(3):
            xp = xw.copy(); xp[a, i] += h
            xm = xw.copy(); xm[a, i] -= h
            g = (O.energy(xp, Delta, p) - O.energy(xm, Delta, p)) / (2 * h)
            assert -g == pytest.approx(F[a, i], abs=2e-5 * max(1.0, abs(F[a, i]))), (i, a)


def test_virial_with_angles_is_affine_strain_derivative():
    w, p = _melt()
    L = w.box[1]
    Delta = 0.77 * w.box[0]
    xw, _ = O.le_wrap(w.x, None, Delta, p)
    _, W, _ = O.forces(xw, Delta, p)
    p0 = O.make_params(w.x.shape[1], w.box, rc=2 ** (1 / 6), pair="wca", chain_len=12, n_chains=6,
                       angle_k=0.0, lj_shift=1.0)
    _, W0, _ = O.forces(xw, Delta, p0)
    assert np.abs(W - W0).max() > 1e-3  # the angles contribute
    eps = 1e-6

    def e_at(s):
        xs = xw.copy()
        xs[0] = xs[0] + s * xs[1]
        return O.energy(xs, Delta + s * L, p)

    dE = (e_at(eps) - e_at(-eps)) / (2 * eps)
    assert dE == pytest.approx(-W[3], rel=1e-5, abs=1e-6)


def test_sampled_sum_matches_full_sum():
    w, p = _melt(shear_rate=0.2)
    Delta = 0.2 * w.box[0]
    xw, _ = O.le_wrap(w.x, None, Delta, p)
    F, _, _ = O.forces(xw, Delta, p)
    idx = np.array([0, 1, 2, 6, 10, 11, 12, 13, 50, 71])
    Fs = O.forces_sample(xw, Delta, p, idx)
    assert np.allclose(Fs, F[:, idx].T, rtol=0, atol=1e-11)
