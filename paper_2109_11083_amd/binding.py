"""ctypes binding of the C ABI in include/le.h (argument marshalling only).

Functions carry the C names (le_init, le_step, ...).  Device pointers are
passed as integers (e.g. ``tensor.data_ptr()``); every step of the path runs
in the HIP library.  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libleshear.so")

LE_OK = 0
LE_E_ARG = -1
LE_E_GEOMETRY = -2
LE_E_WORKSPACE = -3
LE_E_BOND = -4
LE_E_NONFINITE = -5
LE_E_CAPACITY = -6
LE_E_HIP = -7
LE_E_STATE = -8

LE_PAIR_LJ = 0
LE_PAIR_WCA = 1
LE_FP64 = 0
LE_MIXED = 1
LE_THERMO_LANGEVIN = 0
LE_THERMO_DPD = 1
LE_THERMO_LANGEVIN_LAB = 2
LE_VEL_LAB = 0
LE_VEL_PECULIAR = 1

EXPORTED = [
    "le_workspace_bytes", "le_init", "le_build_cells", "le_forces", "le_step", "le_stress",
    "le_get_state", "le_sync", "le_stats", "le_destroy", "le_strerror", "le_offsets", "le_philox",
    "le_timing_enable", "le_timing_read", "le_observables", "le_graph_create", "le_graph_launch",
    "le_graph_destroy", "le_unwrapped", "le_msd", "le_forces_static", "le_step_batch",
    "le_batch_graph_create", "le_status_out",
]
LE_MAX_BINS = 256


class le_params(C.Structure):
    """Mirror of struct le_params (8-byte fields first, no padding)."""
    _fields_ = [
        ("n", C.c_int64),
        ("box", C.c_double * 3),
        ("shear_rate", C.c_double),
        ("dt", C.c_double),
        ("kT", C.c_double),
        ("gamma", C.c_double),
        ("mass", C.c_double),
        ("eps", C.c_double),
        ("sigma", C.c_double),
        ("rc", C.c_double),
        ("skin", C.c_double),
        ("fene_k", C.c_double),
        ("fene_r0", C.c_double),
        ("dpd_rc", C.c_double),
        ("force_cap", C.c_double),
        ("angle_k", C.c_double),
        ("n_chains", C.c_int64),
        ("seed", C.c_uint64),
        ("chain_len", C.c_int32),
        ("pair", C.c_int32),
        ("precision", C.c_int32),
        ("cells", C.c_int32 * 3),
        ("max_neighbors", C.c_int32),
        ("tune", C.c_int32),
        ("thermostat", C.c_int32),
        ("velocity", C.c_int32),
    ]


class LeError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib() -> C.CDLL:
    """Load libleshear.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_2109_11083_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64
    P = C.POINTER(le_params)
    sim_pp = C.POINTER(C.c_void_p)
    L.le_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    L.le_init.argtypes = [P, vp, vp, vp, vp, C.c_size_t, vp, i64, sim_pp]
    L.le_build_cells.argtypes = [vp, vp, vp, vp, i64, C.POINTER(i64)]
    L.le_forces.argtypes = [vp, vp, vp]
    L.le_step.argtypes = [vp, i64, i32, vp, i64]
    L.le_stress.argtypes = [vp, vp]
    L.le_get_state.argtypes = [vp, vp, vp, vp, C.POINTER(i64)]
    L.le_sync.argtypes = [vp]
    L.le_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i32)]
    L.le_destroy.argtypes = [vp]
    L.le_strerror.argtypes = [i32]
    L.le_strerror.restype = C.c_char_p
    L.le_offsets.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, i64, i64, vp, vp]
    L.le_philox.argtypes = [vp, vp, vp, i64, vp]
    L.le_timing_enable.argtypes = [vp, i32]
    L.le_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
    L.le_observables.argtypes = [vp, i32, vp]
    L.le_graph_create.argtypes = [vp, i64, i32, vp, i64, sim_pp]
    L.le_graph_launch.argtypes = [vp]
    L.le_graph_destroy.argtypes = [vp]
    L.le_unwrapped.argtypes = [vp, vp]
    L.le_msd.argtypes = [vp, vp, vp]
    L.le_forces_static.argtypes = [P, vp, vp, vp, vp, i64, vp]
    L.le_status_out.argtypes = [vp, vp]
    L.le_step_batch.argtypes = [C.POINTER(vp), i32, i64, i32, C.POINTER(vp), i64]
    L.le_batch_graph_create.argtypes = [C.POINTER(vp), i32, i64, i32, C.POINTER(vp), i64, sim_pp]
    for name in EXPORTED:
        if name != "le_strerror":
            getattr(L, name).restype = i32
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().le_strerror(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def check(code: int, where: str = "") -> None:
    if code != LE_OK:
        raise LeError(code, where)


def le_workspace_bytes(p: le_params) -> int:
    n = C.c_size_t(0)
    check(lib().le_workspace_bytes(C.byref(p), C.byref(n)), "le_workspace_bytes")
    return n.value


def le_init(p: le_params, x0: int, u0: int, f0: int | None, workspace: int, ws_bytes: int,
            stream: int | None, step0: int) -> int:
    h = C.c_void_p(0)
    check(lib().le_init(C.byref(p), x0, u0, f0, workspace, ws_bytes, stream, step0, C.byref(h)),
          "le_init")
    return h.value


def le_build_cells(sim: int, cell_of: int | None, order: int | None, pairs: int | None,
                   pairs_cap: int, want_count: bool = True) -> int:
    cnt = C.c_int64(0)
    check(lib().le_build_cells(sim, cell_of, order, pairs, pairs_cap,
                               C.byref(cnt) if want_count else None), "le_build_cells")
    return cnt.value


def le_forces(sim: int, f_out: int | None, virial6: int | None) -> None:
    check(lib().le_forces(sim, f_out, virial6), "le_forces")


def le_step(sim: int, nsteps: int, sample_every: int = 0, stress_ring: int | None = None,
            ring_cap: int = 0) -> None:
    check(lib().le_step(sim, nsteps, sample_every, stress_ring, ring_cap), "le_step")


def _ptr_array(ptrs):
    arr = (C.c_void_p * max(len(ptrs), 1))()
    for k, v in enumerate(ptrs):
        arr[k] = v
    return arr


def le_step_batch(sims, nsteps: int, sample_every: int = 0, stress_rings=None, ring_cap: int = 0) -> None:
    """sims: handles; stress_rings: device pointers (one per simulation) or None."""
    hs = _ptr_array(list(sims))
    rings = _ptr_array(list(stress_rings)) if stress_rings is not None else None
    check(lib().le_step_batch(hs, len(sims), nsteps, sample_every, rings, ring_cap), "le_step_batch")


def le_batch_graph_create(sims, nsteps: int, sample_every: int = 0, stress_rings=None,
                          ring_cap: int = 0) -> int:
    hs = _ptr_array(list(sims))
    rings = _ptr_array(list(stress_rings)) if stress_rings is not None else None
    g = C.c_void_p(0)
    check(lib().le_batch_graph_create(hs, len(sims), nsteps, sample_every, rings, ring_cap, C.byref(g)),
          "le_batch_graph_create")
    return g.value


def le_stress(sim: int, sigma6: int) -> None:
    check(lib().le_stress(sim, sigma6), "le_stress")


def le_get_state(sim: int, x: int | None, u: int | None, f: int | None) -> int:
    step = C.c_int64(0)
    check(lib().le_get_state(sim, x, u, f, C.byref(step)), "le_get_state")
    return step.value


def le_status_out(sim: int, status_out: int) -> None:
    check(lib().le_status_out(sim, status_out), "le_status_out")


def le_sync(sim: int) -> int:
    return lib().le_sync(sim)


def le_stats(sim: int):
    r = C.c_int64(0)
    m = C.c_int32(0)
    st = lib().le_stats(sim, C.byref(r), C.byref(m))
    return st, r.value, m.value


def le_destroy(sim: int) -> None:
    check(lib().le_destroy(sim), "le_destroy")


def le_offsets(shear_rate: float, Lx: float, Ly: float, dt: float, step0: int, count: int, out: int,
               stream: int | None) -> None:
    check(lib().le_offsets(shear_rate, Lx, Ly, dt, step0, count, out, stream), "le_offsets")


def le_philox(ctr: int, key: int, out: int, count: int, stream: int | None) -> None:
    check(lib().le_philox(ctr, key, out, count, stream), "le_philox")


def le_observables(sim: int, nbins: int, out: int) -> None:
    check(lib().le_observables(sim, nbins, out), "le_observables")


def le_unwrapped(sim: int, yz_out: int) -> None:
    check(lib().le_unwrapped(sim, yz_out), "le_unwrapped")


def le_msd(sim: int, ref_yz: int, out2: int) -> None:
    check(lib().le_msd(sim, ref_yz, out2), "le_msd")


def le_graph_create(sim: int, nsteps: int, sample_every: int = 0, stress_ring: int | None = None,
                    ring_cap: int = 0) -> int:
    g = C.c_void_p(0)
    check(lib().le_graph_create(sim, nsteps, sample_every, stress_ring, ring_cap, C.byref(g)),
          "le_graph_create")
    return g.value


def le_graph_launch(graph: int) -> None:
    check(lib().le_graph_launch(graph), "le_graph_launch")


def le_graph_destroy(graph: int) -> None:
    check(lib().le_graph_destroy(graph), "le_graph_destroy")


def le_forces_static(p: le_params, x: int, f_out: int | None, virial6: int | None,
                     status_out: int | None, step: int, stream: int | None) -> None:
    """Forces and virial of one configuration in the library's own device
    scratch (no workspace, no handle, nothing allocated)."""
    check(lib().le_forces_static(C.byref(p), x, f_out, virial6, status_out, step, stream),
          "le_forces_static")


def le_timing_enable(sim: int, phases) -> None:
    """phases: bit mask over PHASES (True = all, False = off)."""
    if phases is True:
        phases = 0xF
    elif phases is False:
        phases = 0
    check(lib().le_timing_enable(sim, int(phases)), "le_timing_enable")


PHASES = ("force", "rebuild", "bookkeeping", "stress")


def le_timing_read(sim: int):
    """Per-phase device milliseconds and launch-group counts since enabling."""
    ms = (C.c_double * 4)()
    n = (C.c_int64 * 4)()
    check(lib().le_timing_read(sim, ms, n), "le_timing_read")
    return {PHASES[k]: (ms[k], n[k]) for k in range(4)}
