"""Pins of the oracle's interactions and virial (Eqs. lj, lj-shift, fene, tensor).

Closed forms are evaluated independently (exact rational arithmetic where the
value is rational), forces are checked as derivatives of the energy, and the
Lees-Edwards virial is checked against the derivative of the energy under an
affine shear strain, which also moves the image offset.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _two(r, box=(20.0, 20.0, 20.0)):
    """Particle 0 at (r, 1, 1), particle 1 at (0, 1, 1): d = q_0 - q_1 = (r, 0, 0) exactly."""
    return np.array([[float(r), 0.0], [1.0, 1.0], [1.0, 1.0]])


def test_lj_force_zero_at_potential_minimum():
    r = 2.0 ** (1.0 / 6.0)
    p = O.make_params(2, (20.0, 20.0, 20.0))
    F, W, e = O.forces(_two(r), 0.0, p)
    assert abs(F[0, 0]) < 1e-13
    assert e == pytest.approx(-1.0, abs=1e-14)


def test_lj_force_at_cutoff_edge_rational():
    """At r = 5/2 - tiny the truncated LJ force magnitude is
    24 (2 (2/5)^13 - (2/5)^7) = -0.0389995...; at r just above 5/2 it is 0."""
    exact = 24 * (2 * Fraction(2, 5) ** 13 - Fraction(2, 5) ** 7)
    assert float(exact) == pytest.approx(-0.0389995, abs=5e-8)
    p = O.make_params(2, (20.0, 20.0, 20.0))
    r = np.nextafter(2.5, 0)
    F, _, _ = O.forces(_two(r), 0.0, p)
    assert F[0, 0] == pytest.approx(float(exact), rel=1e-12)
    F, _, _ = O.forces(_two(np.nextafter(2.5, 3)), 0.0, p)
    assert F[0, 0] == 0.0


def test_lj_two_body_rational_values():
    p = O.make_params(2, (20.0, 20.0, 20.0))
    for r in (Fraction(9, 10), Fraction(1), Fraction(5, 4), Fraction(2)):
        exact = 24 * (2 * r ** -13 - r ** -7)
        F, W, e = O.forces(_two(float(r)), 0.0, p)
        assert F[0, 0] == pytest.approx(float(exact), rel=1e-13)
        assert F[0, 1] == -F[0, 0]
        # virial of one pair: d_x F_x = r * F
        assert W[0] == pytest.approx(float(r * exact), rel=1e-13)
        assert e == pytest.approx(float(4 * (r ** -12 - r ** -6)), rel=1e-13)


def test_wca_shift_makes_energy_vanish_at_cutoff():
    rc = 2.0 ** (1.0 / 6.0)
    p = O.make_params(2, (20.0, 20.0, 20.0), rc=rc, lj_shift=1.0)
    F, W, e = O.forces(_two(rc * (1 - 1e-9)), 0.0, p)
    assert abs(e) < 1e-7
    assert abs(F[0, 0]) < 1e-6


def test_fene_closed_form_and_bond_break():
    p = O.make_params(2, (20.0, 20.0, 20.0), rc=0.5, chain_len=2, n_chains=1)
    for r in (Fraction(97, 100), Fraction(6, 5), Fraction(149, 100)):
        q = 1 - r * r / Fraction(9, 4)
        exact_f = -30 * r / q
        F, W, e = O.forces(_two(float(r)), 0.0, p)
        assert F[0, 0] == pytest.approx(float(exact_f), rel=1e-12)
        assert e == pytest.approx(-0.5 * 30 * 2.25 * math.log(float(q)), rel=1e-12)
    with pytest.raises(O.OracleError) as ei:
        O.forces(_two(1.5), 0.0, p)
    assert ei.value.code == O.E_BOND


def _liquid(n_side, density, seed, jitter=0.15):
    n = n_side ** 3
    L = (n / density) ** (1 / 3)
    a = L / n_side
    g = (np.arange(n_side) + 0.5) * a
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    rng = np.random.default_rng(seed)
    pos += rng.uniform(-jitter, jitter, pos.shape)
    return pos, L


def test_forces_are_minus_energy_gradient_with_offset():
    pos, L = _liquid(5, 0.8, 1)
    box = (L, L, L)
    Delta = 0.37 * L
    p = O.make_params(pos.shape[1], box, lj_shift=O.lj_energy_shift(2.5))
    xw, _ = O.le_wrap(pos, None, Delta, p)
    F, _, _ = O.forces(xw, Delta, p)
    h = 1e-6
    rng = np.random.default_rng(2)
    # include particles next to the gradient faces, where pairs use the offset image
    ys = xw[1]
    cand = list(np.argsort(ys)[:4]) + list(np.argsort(ys)[-4:]) + list(rng.choice(pos.shape[1], 4))
    for i in cand:
        for a in range(3):
            xp = xw.copy(); xp[a, i] += h
            xm = xw.copy(); xm[a, i] -= h
            g = (O.energy(xp, Delta, p) - O.energy(xm, Delta, p)) / (2 * h)
            assert -g == pytest.approx(F[a, i], abs=2e-5 * max(1.0, abs(F[a, i])))


def test_forces_sum_to_zero_and_methods_agree():
    pos, L = _liquid(6, 0.8442, 3)
    box = (L, L, L)
    Delta = 0.9 * L
    p = O.make_params(pos.shape[1], box)
    xw, _ = O.le_wrap(pos, None, Delta, p)
    Fb, Wb, eb = O.forces(xw, Delta, p, method=0)
    Fc, Wc, ec = O.forces(xw, Delta, p, method=1)
    assert np.allclose(Fb, Fc, rtol=0, atol=1e-11)
    assert np.allclose(Wb, Wc, rtol=1e-12)
    assert np.abs(Fb.sum(axis=1)).max() < 1e-10
    idx = np.array([0, 5, 100, 215])
    Fs = O.forces_sample(xw, Delta, p, idx)
    assert np.allclose(Fs, Fb[:, idx].T, rtol=0, atol=1e-11)


def test_virial_is_affine_strain_derivative_of_energy():
    """Shearing every coordinate x -> x + eps*y and the offset Delta -> Delta +
    eps*L_y maps every Lees-Edwards pair displacement d to d + eps d_y e_x, so
    dE/deps = -sum_{i<j} d_y F_ij,x = -W_xy, including pairs that meet across
    the gradient faces."""
    pos, L = _liquid(5, 0.8442, 4)
    box = (L, L, L)
    Delta = 0.61 * L
    p = O.make_params(pos.shape[1], box, lj_shift=O.lj_energy_shift(2.5))
    xw, _ = O.le_wrap(pos, None, Delta, p)
    _, W, _ = O.forces(xw, Delta, p)
    eps = 1e-6

    def e_at(s):
        xs = xw.copy()
        xs[0] = xs[0] + s * xs[1]
        return O.energy(xs, Delta + s * L, p)

    dE = (e_at(eps) - e_at(-eps)) / (2 * eps)
    assert dE == pytest.approx(-W[3], rel=1e-5, abs=1e-6)
    # the diagonal components follow from stretching one axis together with
    # its box length (and the offset when the axis is the flow axis)
    for a in range(3):
        def e_st(s):
            xs = xw.copy()
            xs[a] = xs[a] * (1 + s)
            b = list(box)
            b[a] = b[a] * (1 + s)
            ps = O.make_params(pos.shape[1], b, lj_shift=O.lj_energy_shift(2.5))
            return O.energy(xs, Delta * (1 + s) if a == 0 else Delta, ps)

        dEa = (e_st(eps) - e_st(-eps)) / (2 * eps)
        assert dEa == pytest.approx(-W[a], rel=1e-5, abs=1e-6)


def test_kinetic_stress_of_a_single_particle():
    box = (4.0, 5.0, 6.0)
    p = O.make_params(1, box, shear_rate=0.3, mass=2.0)
    x = np.array([[1.0], [4.0], [2.0]])
    c = np.array([0.5, -0.25, 0.125])
    u = c.copy()[:, None]
    u[0, 0] += 0.3 * (4.0 - 2.5)
    s = O.stress(x, u, np.zeros(6), p)
    V = 120.0
    expect = -2.0 / V * np.array([c[0] * c[0], c[1] * c[1], c[2] * c[2], c[0] * c[1], c[0] * c[2],
                                  c[1] * c[2]])
    assert np.allclose(s, expect, rtol=1e-14, atol=1e-16)


def test_force_cap_limits_the_magnitude_and_keeps_the_direction():
    """Warm-up cap: a pair closer than the point where 24 (2 r^-13 - r^-7)
    reaches the cap feels exactly the cap along d; a pair beyond it feels the
    plain force; an attractive pair is capped symmetrically."""
    cap = 100.0
    p = O.make_params(2, (20.0, 20.0, 20.0), force_cap=cap)
    p0 = O.make_params(2, (20.0, 20.0, 20.0))
    # r = 3/4: plain force 24 (2 (4/3)^13 - (4/3)^7) = 1996.9... > cap
    r = Fraction(3, 4)
    plain = 24 * (2 * r ** -13 - r ** -7)
    assert plain > cap
    F, W, _ = O.forces(_two(float(r)), 0.0, p)
    assert F[0, 0] == pytest.approx(cap, rel=1e-15) and F[0, 1] == -F[0, 0]
    assert F[1, 0] == 0.0 and F[2, 0] == 0.0
    assert W[0] == pytest.approx(float(r) * cap, rel=1e-15)
    # a skewed pair: magnitude cap, direction d / r
    x = np.array([[0.3, 0.0], [0.4, 0.0], [1.2, 1.0]])  # d = (0.3, 0.4, 0.2)
    d = np.array([0.3, 0.4, 0.2])
    F, _, _ = O.forces(x, 0.0, p)
    assert np.linalg.norm(F[:, 0]) == pytest.approx(cap, rel=1e-14)
    assert np.allclose(F[:, 0] / cap, d / np.linalg.norm(d), rtol=1e-14, atol=0)
    # below the cap the force is untouched, bit for bit
    for rr in (1.0, 1.12, 2.0):
        Fa, _, _ = O.forces(_two(rr), 0.0, p)
        Fb, _, _ = O.forces(_two(rr), 0.0, p0)
        assert np.array_equal(Fa, Fb)
    # an attractive force above a tiny cap: -cap along d
    pt = O.make_params(2, (20.0, 20.0, 20.0), force_cap=1e-3)
    F, _, _ = O.forces(_two(1.5), 0.0, pt)
    assert F[0, 0] == pytest.approx(-1e-3, rel=1e-15)
