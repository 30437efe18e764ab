"""ctypes front end of the FP64 CPU oracle (oracle/le_oracle.c).

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the CPU-baseline leg of
the benchmark may use it; the library under paper_2109_11083_amd/ never does.
It shares no code with the HIP path.  Arrays are float64 SoA (3, n) by tag.

Build: ``python oracle/oracle.py --build`` (gcc -O2 -ffp-contract=off).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "le_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")
LIB_OMP = os.path.join(HERE, "_build", "liboracle_omp.so")  # timing build (CPU baseline only)

PAIR_LJ, PAIR_WCA = 0, 1
E_BOND, E_NONFINITE = -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/_build/liboracle.so, and its OpenMP timing
    build (the CPU baseline's all-cores run) into liboracle_omp.so."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            tmp = out + ".tmp"
            cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC",
                   *extra, "-shared", "-o", tmp, SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(tmp, out)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("box", C.c_double * 3),
        ("shear_rate", C.c_double),
        ("dt", C.c_double), ("kT", C.c_double), ("gamma", C.c_double), ("mass", C.c_double),
        ("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double),
        ("fene_k", C.c_double), ("fene_r0", C.c_double),
        ("lj_shift", C.c_double),
        ("dpd_rc", C.c_double),
        ("angle_k", C.c_double),
        ("force_cap", C.c_double),
        ("seed", C.c_uint64),
        ("n", C.c_int64),
        ("n_chains", C.c_int64),
        ("chain_len", C.c_int32),
        ("thermostat", C.c_int32),
        ("velocity", C.c_int32),
        ("pad_", C.c_int32),
    ]

THERMOSTATS = {"langevin": 0, "dpd": 1, "langevin_abs": 2}
VELOCITIES = {"lab": 0, "peculiar": 1}


_lib = None
_lib_omp = None


def lib(timing: bool = False):
    """The serial oracle, or with timing=True its OpenMP timing build (same
    functions; sums in another order; for the CPU baseline only)."""
    global _lib, _lib_omp
    if timing:
        if _lib_omp is None:
            lib()
            _lib_omp = _declare(C.CDLL(LIB_OMP))
            _lib_omp.orc_threads.argtypes = [C.c_int]
            _lib_omp.orc_threads.restype = C.c_int
        return _lib_omp
    if _lib is None:
        if not all(os.path.exists(f) and os.path.getmtime(f) >= os.path.getmtime(SRC) for f in (LIB, LIB_OMP)):
            build(force=True)
        _lib = _declare(C.CDLL(LIB))
    return _lib


def timing_threads(n: int = 0) -> int:
    """Set (n > 0) and return the thread count of the timing build."""
    return lib(timing=True).orc_threads(int(n))


def _declare(L):
    if True:
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        u32p = C.POINTER(C.c_uint32)
        pp = C.POINTER(Params)
        L.orc_offset.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_offset.restype = C.c_double
        L.orc_wrap.argtypes = [dp, C.c_double]
        L.orc_wrap.restype = C.c_double
        L.orc_le_wrap.argtypes = [C.c_int64, dp, dp, C.c_double, pp]
        L.orc_le_wrap.restype = None
        L.orc_cell_id.argtypes = [C.c_double, C.c_double, C.c_double, i32p, dp]
        L.orc_cell_id.restype = C.c_int32
        L.orc_cells.argtypes = [C.c_int64, dp, i32p, dp, i32p, i32p]
        L.orc_cells.restype = None
        L.orc_disp.argtypes = [dp, C.c_int64, C.c_int64, C.c_int64, C.c_double, dp, dp, i32p]
        L.orc_disp.restype = C.c_double
        L.orc_pairs_brute.argtypes = [C.c_int64, dp, C.c_double, dp, C.c_double, i64p, C.c_int64]
        L.orc_pairs_brute.restype = C.c_int64
        L.orc_pairs_cells.argtypes = [C.c_int64, dp, C.c_double, dp, C.c_double, i64p, C.c_int64]
        L.orc_pairs_cells.restype = C.c_int64
        L.orc_forces.argtypes = [C.c_int64, dp, C.c_double, pp, C.c_int, dp, dp, dp]
        L.orc_forces.restype = C.c_int
        L.orc_forces_sample.argtypes = [C.c_int64, dp, C.c_double, pp, C.c_int64, i64p, dp]
        L.orc_forces_sample.restype = C.c_int
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_philox.restype = None
        L.orc_noise.argtypes = [C.c_uint64, C.c_int64, C.c_int64, dp]
        L.orc_noise.restype = None
        L.orc_dpd_sample.argtypes = [C.c_int64, dp, dp, C.c_double, pp, C.c_int64, C.c_int64, i64p, dp]
        L.orc_dpd_sample.restype = None
        L.orc_dpd_theta.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64]
        L.orc_dpd_theta.restype = C.c_double
        L.orc_stress.argtypes = [C.c_int64, dp, dp, dp, pp, dp]
        L.orc_stress.restype = None
        L.orc_step.argtypes = [C.c_int64, dp, dp, dp, i64p, pp, C.c_int, dp, dp]
        L.orc_step.restype = C.c_int
        L.orc_init.argtypes = [C.c_int64, dp, dp, dp, C.c_int64, pp, C.c_int]
        L.orc_init.restype = C.c_int
        L.orc_run.argtypes = [C.c_int64, dp, dp, dp, i64p, pp, C.c_int, C.c_int64, C.c_int64, dp]
        L.orc_run.restype = C.c_int
        L.orc_observables.argtypes = [C.c_int64, dp, dp, C.c_double, pp, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_observables.restype = None
        L.orc_energy.argtypes = [C.c_int64, dp, C.c_double, pp, dp]
        L.orc_energy.restype = C.c_int
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def make_params(n, box, shear_rate=0.0, dt=0.005, kT=1.0, gamma=1.0, mass=1.0, pair="lj",
                eps=1.0, sigma=1.0, rc=2.5, fene_k=30.0, fene_r0=1.5, lj_shift=0.0,
                seed=1, chain_len=0, n_chains=0, thermostat="langevin", dpd_rc=0.0, velocity="lab",
                angle_k=0.0, force_cap=0.0,
                **_ignored) -> Params:
    p = Params()
    for a in range(3):
        p.box[a] = float(box[a])
    p.shear_rate = shear_rate
    p.dt, p.kT, p.gamma, p.mass = dt, kT, gamma, mass
    p.eps, p.sigma, p.rc = eps, sigma, rc
    p.fene_k, p.fene_r0 = fene_k, fene_r0
    p.lj_shift = lj_shift
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    p.n = n
    p.chain_len = chain_len
    p.n_chains = n_chains
    p.thermostat = THERMOSTATS[thermostat] if isinstance(thermostat, str) else int(thermostat)
    p.dpd_rc = dpd_rc if dpd_rc > 0 else rc
    p.angle_k = angle_k
    p.force_cap = force_cap
    p.velocity = VELOCITIES[velocity] if isinstance(velocity, str) else int(velocity)
    return p


def dpd_sample(x, u, Delta, p: Params, step, idx):
    """DPD pair terms on the particles idx (ns, 3), brute force in tag order."""
    x, u = _c64(x), _c64(u)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((len(idx), 3))
    lib().orc_dpd_sample(x.shape[1], _dp(x), _dp(u), Delta, C.byref(p), int(step), len(idx),
                         idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
    return out


def dpd_theta(seed, step, ti, tj):
    return lib().orc_dpd_theta(seed & 0xFFFFFFFFFFFFFFFF, int(step), int(ti), int(tj))


def lj_energy_shift(rc, eps=1.0, sigma=1.0):
    """-V_LJ(rc): added to every pair energy so that V(rc) = 0 (energy checks only)."""
    s6 = (sigma / rc) ** 6
    return -4.0 * eps * (s6 * s6 - s6)


def offset(n, dt, shear_rate, Lx, Ly):
    return lib().orc_offset(int(n), dt, shear_rate, Lx, Ly)


def wrap(x, L):
    v = C.c_double(x)
    k = lib().orc_wrap(C.byref(v), L)
    return v.value, k


def le_wrap(x, u, Delta, p: Params):
    x = _c64(x).copy()
    u = _c64(u).copy() if u is not None else None
    n = x.shape[1]
    lib().orc_le_wrap(n, _dp(x), _dp(u) if u is not None else None, Delta, C.byref(p))
    return x, u


def cells(x, nc, box):
    x = _c64(x)
    n = x.shape[1]
    nca = (C.c_int32 * 3)(*nc)
    boxa = (C.c_double * 3)(*box)
    cell_of = np.zeros(n, np.int32)
    order = np.zeros(n, np.int32)
    lib().orc_cells(n, _dp(x), nca, boxa, cell_of.ctypes.data_as(C.POINTER(C.c_int32)),
                    order.ctypes.data_as(C.POINTER(C.c_int32)))
    return cell_of, order


def disp(x, i, j, Delta, box):
    x = _c64(x)
    d = np.zeros(3)
    img = np.zeros(3, np.int32)
    boxa = (C.c_double * 3)(*box)
    r2 = lib().orc_disp(_dp(x), x.shape[1], i, j, Delta, boxa, _dp(d),
                        img.ctypes.data_as(C.POINTER(C.c_int32)))
    return d, r2, img


def _pairs(fn, x, Delta, box, rcut):
    x = _c64(x)
    n = x.shape[1]
    boxa = (C.c_double * 3)(*box)
    cap = max(16, n * 64)
    while True:
        buf = np.zeros(2 * cap, np.int64)
        m = fn(n, _dp(x), Delta, boxa, rcut, buf.ctypes.data_as(C.POINTER(C.c_int64)), cap)
        if m <= cap:
            return buf[: 2 * m].reshape(m, 2)
        cap = m


def pairs_brute(x, Delta, box, rcut):
    """All unordered pairs (i<j) within rcut, brute force O(N^2)."""
    return _pairs(lib().orc_pairs_brute, x, Delta, box, rcut)


def pairs_cells(x, Delta, box, rcut):
    """The same set through the oracle's own grid (x must already be wrapped)."""
    return _pairs(lib().orc_pairs_cells, x, Delta, box, rcut)


def forces(x, Delta, p: Params, method=0):
    """Conservative forces (3, n), pair virial W (6,), potential energy."""
    x = _c64(x)
    n = x.shape[1]
    F = np.zeros((3, n))
    W = np.zeros(6)
    e = C.c_double(0.0)
    rc = lib().orc_forces(n, _dp(x), Delta, C.byref(p), method, _dp(F), _dp(W), C.byref(e))
    if rc != 0:
        raise OracleError(rc)
    return F, W, e.value


def forces_sample(x, Delta, p: Params, idx):
    x = _c64(x)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((len(idx), 3))
    rc = lib().orc_forces_sample(x.shape[1], _dp(x), Delta, C.byref(p), len(idx),
                                 idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
    if rc != 0:
        raise OracleError(rc)
    return out


def energy(x, Delta, p: Params):
    x = _c64(x)
    e = C.c_double(0.0)
    rc = lib().orc_energy(x.shape[1], _dp(x), Delta, C.byref(p), C.byref(e))
    if rc != 0:
        raise OracleError(rc)
    return e.value


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return [o[0], o[1], o[2], o[3]]


def noise(seed, step, tag):
    th = np.zeros(3)
    lib().orc_noise(seed & 0xFFFFFFFFFFFFFFFF, int(step), int(tag), _dp(th))
    return th


def stress(x, u, W, p: Params):
    x, u, W = _c64(x), _c64(u), _c64(W)
    s = np.zeros(6)
    lib().orc_stress(x.shape[1], _dp(x), _dp(u), _dp(W), C.byref(p), _dp(s))
    return s


def observables(x, u, Delta, p: Params, nbins=50):
    x, u = _c64(x), _c64(u)
    cnt = np.zeros(nbins)
    sux = np.zeros(nbins)
    smc2 = np.zeros(nbins)
    kt = C.c_double(0.0)
    com = np.zeros(3)
    lib().orc_observables(x.shape[1], _dp(x), _dp(u), Delta, C.byref(p), nbins, _dp(cnt), _dp(sux),
                          _dp(smc2), C.byref(kt), _dp(com))
    return dict(count=cnt, sum_ux=sux, sum_mc2=smc2, kT=kt.value, com=com)


def msd(unw, ref):
    """Mean squared displacement along y and z of unwrapped coordinates
    [2][n] relative to ref [2][n]."""
    d = np.asarray(unw) - np.asarray(ref)
    return (d ** 2).mean(axis=1)


class Sim:
    """A running oracle simulation (state in tag order, wrapped every step)."""

    def __init__(self, x0, u0, p: Params, step0=0, method=1, timing=False):
        self.p = p
        self.method = method
        self.L = lib(timing)
        self.x = _c64(x0).copy()
        self.u = _c64(u0).copy()
        self.n = self.x.shape[1]
        self.F = np.zeros_like(self.x)
        self.step = int(step0)
        rc = self.L.orc_init(self.n, _dp(self.x), _dp(self.u), _dp(self.F), self.step, C.byref(p),
                            method)
        if rc != 0:
            raise OracleError(rc)

    @property
    def Delta(self):
        p = self.p
        return offset(self.step, p.dt, p.shear_rate, p.box[0], p.box[1])

    def run(self, nsteps, sample_every=0):
        ns = nsteps // sample_every if sample_every > 0 else 0
        out = np.zeros((max(ns, 1), 6))
        st = C.c_int64(self.step)
        rc = self.L.orc_run(self.n, _dp(self.x), _dp(self.u), _dp(self.F), C.byref(st), C.byref(self.p),
                           self.method, int(nsteps), int(sample_every), _dp(out))
        self.step = st.value
        if rc != 0:
            raise OracleError(rc)
        return out[:ns]

    def run_tracked(self, nsteps, unw):
        """Run nsteps one at a time and add each particle's per-step change of
        y and z, taken as the minimum image (a particle moves far less than half
        a box in one step), to unw [2][n]: the unwrapped gradient and vorticity
        coordinates.  Returns unw."""
        Ly, Lz = self.p.box[1], self.p.box[2]
        for _ in range(nsteps):
            y0, z0 = self.x[1].copy(), self.x[2].copy()
            self.run(1)
            dy, dz = self.x[1] - y0, self.x[2] - z0
            unw[0] += dy - Ly * np.round(dy / Ly)
            unw[1] += dz - Lz * np.round(dz / Lz)
        return unw

    def conservative(self):
        return forces(self.x, self.Delta, self.p, self.method)

    def stress(self):
        _, W, _ = self.conservative()
        return stress(self.x, self.u, W, self.p)


if __name__ == "__main__":
    if "--build" in sys.argv:
        print(build(force=True))
