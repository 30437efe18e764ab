"""Pins of the oracle's Lees-Edwards geometry (offset, wrap, cells, pair set).

Each test checks the oracle against something other than its own formula:
closed forms of the streaming motion, a hand-derived edge-case table, an
explicit replication of the sheared image lattice, and the textbook periodic
minimum image in the zero-offset special case.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- O1 offset
def test_offset_zero_at_start_and_in_range():
    for sr in (0.0, 0.1, -0.3, 1.0):
        assert O.offset(0, 0.005, sr, 10.0, 12.0) == 0.0
        for n in (1, 17, 1000, 123457):
            d = O.offset(n, 0.005, sr, 10.0, 12.0)
            assert 0.0 <= d < 10.0


def test_offset_tracks_relative_motion_of_the_upper_image():
    """The image above moves at shear_rate*L_y relative to the box (the two
    faces move at +/- shear_rate L_y / 2, Fig. lebc), so its offset grows by
    exactly that speed times t, folded back by whole box lengths."""
    Lx, Ly, dt, sr = 10.5, 7.25, 0.01, 0.37
    for n in (1, 3, 250, 4001, 99999):
        t = n * dt
        travelled = (sr * Ly / 2) * t - (-(sr * Ly / 2) * t)  # top face minus bottom face
        folds = math.floor(travelled / Lx)
        expect = travelled - folds * Lx
        assert O.offset(n, dt, sr, Lx, Ly) == pytest.approx(expect, abs=1e-9)


def test_offset_negative_shear_mirrors():
    Lx, Ly, dt = 9.0, 9.0, 0.005
    for n in (1, 50, 777):
        a = O.offset(n, dt, 0.2, Lx, Ly)
        b = O.offset(n, dt, -0.2, Lx, Ly)
        assert (a + b) % Lx == pytest.approx(0.0, abs=1e-9) or abs(a + b - Lx) < 1e-9


# ---------------------------------------------------------------- O2 wrap
def test_wrap_edge_table():
    with open(os.path.join(GOLDEN, "wrap_edges.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        x, L = float.fromhex(c["x"]), float.fromhex(c["L"])
        xo, k = O.wrap(x, L)
        assert xo == float.fromhex(c["x_out"]), c["note"]
        assert k == c["k"], c["note"]
        assert 0.0 <= xo < L


# ---------------------------------------------------------------- O3 crossing
def _params(box, sr=0.0, **kw):
    return O.make_params(1, box, shear_rate=sr, **kw)


def test_crossing_top_face_shifts_and_jumps():
    box = (10.0, 8.0, 6.0)
    sr = 0.25
    p = _params(box, sr)
    Delta = 3.5
    x = np.array([[4.0], [8.0 + 0.125], [1.0]])
    u = np.array([[sr * (8.125 - 4.0) + 0.3], [0.1], [-0.2]])
    xw, uw = O.le_wrap(x, u, Delta, p)
    assert xw[1, 0] == 0.125
    assert xw[0, 0] == (4.0 - Delta) % 10.0
    assert uw[0, 0] == pytest.approx(u[0, 0] - sr * 8.0, abs=1e-15)
    # peculiar velocity (Eq. vi) unchanged by the crossing
    c_before = u[0, 0] - sr * (x[1, 0] - 4.0)
    c_after = uw[0, 0] - sr * (xw[1, 0] - 4.0)
    assert c_after == pytest.approx(c_before, abs=1e-14)


def test_crossing_bottom_face_mirrors():
    box = (10.0, 8.0, 6.0)
    sr = 0.25
    p = _params(box, sr)
    Delta = 7.75
    x = np.array([[9.5], [-0.5], [5.9]])
    u = np.array([[-1.0], [-0.1], [0.0]])
    xw, uw = O.le_wrap(x, u, Delta, p)
    assert xw[1, 0] == 7.5
    assert xw[0, 0] == pytest.approx((9.5 + Delta) % 10.0, abs=1e-14)
    assert uw[0, 0] == pytest.approx(-1.0 + sr * 8.0, abs=1e-15)


# ------------------------------------------------ O5 against the streaming flow
def test_displacement_follows_affine_flow_across_the_faces():
    """Particles carried by the linear profile (Eq. shear-rate) with zero
    peculiar velocity keep their relative position in the sheared frame:
    d(t) = d(0) + shear_rate t d_y(0) e_x, also for pairs whose minimum image
    crosses the gradient faces.  A wrong sign of the offset breaks this at
    the faces by 2 shear_rate L_y t."""
    rng = np.random.default_rng(3)
    L = (9.0, 9.0, 9.0)
    sr = 0.2
    n = 60
    x0 = rng.uniform(0, 9.0, size=(3, n))
    x0[1, :20] = rng.uniform(8.0, 9.0, 20)  # near the top face
    x0[1, 20:40] = rng.uniform(0.0, 1.0, 20)  # near the bottom face
    p = _params(L, sr)
    for n_steps in (1, 40, 300):
        dt = 0.01
        t = n_steps * dt
        xt = x0.copy()
        xt[0] += sr * (x0[1] - L[1] / 2) * t
        Delta = O.offset(n_steps, dt, sr, L[0], L[1])
        xw, _ = O.le_wrap(xt, None, Delta, p)
        checked = 0
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                d0, r20, _ = O.disp(x0, i, j, 0.0, L)
                if r20 > 2.0 ** 2:
                    continue
                dt_, _, _ = O.disp(xw, i, j, Delta, L)
                expect = d0.copy()
                expect[0] += sr * t * d0[1]
                assert np.allclose(dt_, expect, atol=1e-9), (i, j, n_steps)
                checked += 1
        assert checked > 20


# ---------------------------------------------- O4/O6 cells, brute force, images
def _random_config(n, box, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0, box[a], n) for a in range(3)])


def _explicit_image_pairs(x, Delta, box, rcut):
    """Pairs within rcut by explicit replication of the sheared image lattice:
    the copy of particle j in image (sx, sy, sz) sits at
    x_j + sy*Delta + sx*L_x, y_j + sy*L_y, z_j + sz*L_z (the upper image box
    displaced by +Delta, Fig. lebc)."""
    n = x.shape[1]
    Lx, Ly, Lz = box
    out = set()
    near = []
    for sy in (-1, 0, 1):
        for sx in (-2, -1, 0, 1, 2):
            for sz in (-1, 0, 1):
                img = np.stack([x[0] + sy * Delta + sx * Lx, x[1] + sy * Ly, x[2] + sz * Lz])
                d = x[:, :, None] - img[:, None, :]
                r = np.sqrt((d ** 2).sum(axis=0))
                ii, jj = np.nonzero(r < rcut)
                for i, j in zip(ii, jj):
                    if i < j:
                        out.add((int(i), int(j)))
                ii, jj = np.nonzero(np.abs(r - rcut) < 1e-9)
                near += [(int(min(i, j)), int(max(i, j))) for i, j in zip(ii, jj) if i != j]
    return out, set(near)


@pytest.mark.parametrize("frac", [0.0, 0.25, 0.5, 0.75, 1.0 - 2.0 ** -40])
@pytest.mark.parametrize("ncell", [3, 4, 5])
def test_pair_set_brute_equals_cells_equals_images(frac, ncell):
    rcut = 1.3
    L = ncell * rcut * 1.05
    box = (L, L * 1.1, L * 0.97)
    lx = box[0] / int(box[0] // rcut)
    Delta = (frac * lx) % box[0]
    for seed in (1, 2):
        x = _random_config(90, box, seed + ncell * 10)
        p = _params(box)
        xw, _ = O.le_wrap(x, None, Delta, p)
        pb = {tuple(r) for r in O.pairs_brute(xw, Delta, box, rcut)}
        pc = O.pairs_cells(xw, Delta, box, rcut)
        pcs = {tuple(sorted(r)) for r in pc}
        assert len(pcs) == len(pc), "a pair was visited twice"
        assert pb == pcs
        pe, near = _explicit_image_pairs(xw, Delta, box, rcut)
        assert pb - near == pe - near
        assert len(pb) > 20


def test_pair_set_over_offset_sweep_and_wrap_around():
    rcut = 2.5
    L = 10.5808
    box = (L, L, L)
    x = _random_config(400, box, 5)
    p = _params(box)
    lx = L / 4
    for Delta in [0.0, lx * 0.999999, lx, 2.5 * lx, L - 1e-12, L * 0.5, 1e-13]:
        xw, _ = O.le_wrap(x, None, Delta, p)
        pb = {tuple(r) for r in O.pairs_brute(xw, Delta, box, rcut)}
        pc = {tuple(sorted(r)) for r in O.pairs_cells(xw, Delta, box, rcut)}
        assert pb == pc


def test_zero_offset_is_periodic_minimum_image():
    box = (7.0, 8.0, 9.0)
    x = _random_config(50, box, 8)
    for i in range(0, 50, 7):
        for j in range(50):
            if i == j:
                continue
            d, r2, img = O.disp(x, i, j, 0.0, box)
            raw = x[:, i] - x[:, j]
            L = np.array(box)
            ref = raw - L * np.round(raw / L)
            assert np.array_equal(d, ref)
            assert r2 == (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]


def test_cells_are_geometric_and_order_sorted():
    box = (10.0, 11.0, 12.0)
    nc = (4, 5, 3)
    x = _random_config(500, box, 9)
    x[:, 0] = [0.0, 0.0, 0.0]
    x[:, 1] = [np.nextafter(10.0, 0), np.nextafter(11.0, 0), np.nextafter(12.0, 0)]
    cell_of, order = O.cells(x, nc, box)
    ix = cell_of % nc[0]
    iy = (cell_of // nc[0]) % nc[1]
    iz = cell_of // (nc[0] * nc[1])
    for a, ia in enumerate((ix, iy, iz)):
        l = box[a] / nc[a]
        assert np.all(x[a] >= ia * l - 1e-12)
        assert np.all(x[a] < (ia + 1) * l + 1e-12)
    keys = cell_of[order].astype(np.int64) * 10 ** 6 + order
    assert np.all(np.diff(keys) > 0)
    assert sorted(order.tolist()) == list(range(500))
    assert cell_of[1] == nc[0] * nc[1] * nc[2] - 1


def test_cell_index_clamped_when_product_rounds_up():
    """x one ulp below L_x with x * (n/L_x) rounding up to n must land in the
    last cell, never in a cell n that does not exist."""
    L = float.fromhex("0x1.7db3795860d14p+5")
    x = float.fromhex("0x1.7db3795860d13p+5")
    nc = (12, 12, 12)
    assert int(x * (12 / L)) == 12  # the rounding this case is about
    pos = np.array([[x, 1.0], [x, 1.0], [x, 1.0]])
    cell_of, order = O.cells(pos, nc, (L, L, L))
    assert cell_of[0] == 12 ** 3 - 1
    assert cell_of[1] == 0
