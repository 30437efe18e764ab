"""The no-allocation entry point le_forces_static (forces and virial of one
configuration in the library's own device scratch) against the existing entry
points le_init + le_forces on the same inputs, called twice in a row with the
second input smaller (the scratch keeps the first call's contents)."""
import math

import numpy as np
import pytest
import torch

from paper_2109_11083_amd import binding as B
from paper_2109_11083_amd import inputs
from paper_2109_11083_amd.sim import Params, Sim

pytestmark = pytest.mark.gpu


def _static(p: Params, x, step):
    xt = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    f = torch.full((3, p.n), float("nan"), dtype=torch.float64, device="cuda")
    w = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    B.le_forces_static(p.to_c(), xt.data_ptr(), f.data_ptr(), w.data_ptr(), st.data_ptr(), step, stream)
    torch.cuda.synchronize()
    return f.cpu().numpy(), w.cpu().numpy(), int(st.cpu()[0])


def _workspace(p: Params, x, step):
    u = np.zeros_like(x)
    sim = Sim(p, x, u, step0=step)
    F, W = sim.forces()
    sim.close()
    return F, W


def test_forces_static_matches_le_forces_twice():
    w1 = inputs.lj_workload(n_side=12, shear_rate=0.3, seed=11)  # 1728 particles
    p1 = Params(n=w1.x.shape[1], box=w1.box, shear_rate=0.3, seed=11, skin=0.4)
    rng = np.random.default_rng(3)
    n2 = 700  # second call: fewer particles, a ragged non-cubic box, other skin
    box2 = (12.1, 10.3, 11.7)
    x2 = np.stack([rng.uniform(-2.0, box2[a] + 2.0, n2) for a in range(3)])
    p2 = Params(n=n2, box=box2, shear_rate=0.7, seed=2, skin=0.25, eps=1e-3)
    for p, x, step in ((p1, w1.x, 4321), (p2, x2, 97)):
        f, wv, st = _static(p, x, step)
        F, W = _workspace(p, x, step)
        assert st == 0
        rms = math.sqrt(float((F ** 2).sum(axis=0).mean()))
        ef = float(np.sqrt(((f - F) ** 2).sum(axis=0)).max()) / rms
        ew = np.abs(wv - W).max() / np.abs(W).max()
        print(f"n={p.n}: e_F={ef:.3e} e_W={ew:.3e} bitwise={np.array_equal(f, F) and np.array_equal(wv, W)}",
              flush=True)
        assert ef <= 1e-12 and ew <= 1e-12
        assert np.array_equal(f, F) and np.array_equal(wv, W)  # the same kernels in the same order


def test_forces_static_rejects_too_large_and_reports_latched_status():
    big = Params(n=256000, box=(67.1838,) * 3)
    x = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(B.LeError) as e:
        B.le_forces_static(big.to_c(), x.data_ptr(), x.data_ptr(), None, None, 0, None)
    assert e.value.code == B.LE_E_WORKSPACE
    # a latched device error (a non-finite coordinate) comes back through status_out
    w = inputs.lj_workload(n_side=8, shear_rate=0.1, seed=4)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=0.1, seed=4)
    xb = w.x.copy()
    xb[2, 5] = np.inf
    _, _, st = _static(p, xb, 0)
    assert st == B.LE_E_NONFINITE
    # and the next call on the same scratch starts clean
    f, wv, st = _static(p, w.x, 0)
    F, W = _workspace(p, w.x, 0)
    assert st == 0 and np.array_equal(f, F) and np.array_equal(wv, W)
