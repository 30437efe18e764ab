"""CPU checks of the C ABI: the library loads, exports every declared symbol,
agrees with the header on the parameter layout, and rejects bad arguments on
the host (no device work is issued by any call here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2109_11083_amd import binding as B
from paper_2109_11083_amd.sim import Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "le.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:le_status|const char\*)\s+(le_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 13
    lib = B.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == names


def test_params_layout_matches_header(tmp_path):
    fields = [f[0] for f in B.le_params._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "le.h"', "int main(void){",
            'printf("%zu\\n", sizeof(le_params));']
    for f in fields:
        prog.append(f'printf("%zu\\n", offsetof(le_params, {f}));')
    prog.append("return 0;}")
    c = tmp_path / "lay.c"
    c.write_text("\n".join(prog))
    exe = tmp_path / "lay"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == C.sizeof(B.le_params)
    for f, off in zip(fields, vals[1:]):
        assert getattr(B.le_params, f).offset == off, f


def _lj(n=1000, L=10.5808, **kw):
    return Params(n=n, box=(L, L, L), **kw)


def test_workspace_bytes_and_geometry_errors():
    assert B.le_workspace_bytes(_lj().to_c()) > 1000 * 100
    with pytest.raises(B.LeError) as e:
        B.le_workspace_bytes(_lj(L=8.0).to_c())  # 8 / 2.8 < 3 cells
    assert e.value.code == B.LE_E_GEOMETRY
    with pytest.raises(B.LeError) as e:
        B.le_workspace_bytes(_lj(n=1).to_c())
    assert e.value.code == B.LE_E_ARG
    with pytest.raises(B.LeError) as e:
        B.le_workspace_bytes(_lj(dt=0.0).to_c())
    assert e.value.code == B.LE_E_ARG
    with pytest.raises(B.LeError) as e:
        B.le_workspace_bytes(_lj(cells=(4, 3, 3)).to_c())  # 10.58/4 < 2.8
    assert e.value.code == B.LE_E_GEOMETRY
    with pytest.raises(B.LeError) as e:
        B.le_workspace_bytes(_lj(n_chains=100, chain_len=20).to_c())  # 2000 > n
    assert e.value.code == B.LE_E_ARG
    for t in (-1, 3):
        with pytest.raises(B.LeError) as e:
            B.le_workspace_bytes(_lj(tune=t).to_c())
        assert e.value.code == B.LE_E_ARG
    # thermostats: unknown code, DPD with the LDS halo layout or a weight
    # cutoff beyond the pair cutoff, an unknown velocity storage
    for bad in (dict(thermostat="dpd", tune=1), dict(thermostat="dpd", dpd_rc=2.6)):
        with pytest.raises(B.LeError) as e:
            B.le_workspace_bytes(_lj(**bad).to_c())
        assert e.value.code == B.LE_E_ARG, bad
    for code in (-1, 3):
        c = _lj().to_c()
        c.thermostat = code
        with pytest.raises(B.LeError) as e:
            B.le_workspace_bytes(c)
        assert e.value.code == B.LE_E_ARG
    c = _lj().to_c()
    c.velocity = 2
    with pytest.raises(B.LeError) as e:
        B.le_workspace_bytes(c)
    assert e.value.code == B.LE_E_ARG
    for th in ("dpd", "langevin_abs"):  # peculiar storage takes the Langevin force on c only
        with pytest.raises(B.LeError) as e:
            B.le_workspace_bytes(_lj(velocity="peculiar", thermostat=th).to_c())
        assert e.value.code == B.LE_E_ARG
    for ok in (dict(thermostat="dpd"), dict(thermostat="dpd", dpd_rc=1.0, tune=2),
               dict(thermostat="langevin_abs", tune=1), dict(velocity="peculiar")):
        assert B.le_workspace_bytes(_lj(**ok).to_c()) > 0


def test_init_rejects_small_workspace_before_any_device_work():
    p = _lj().to_c()
    need = B.le_workspace_bytes(p)
    with pytest.raises(B.LeError) as e:
        B.le_init(p, 1, 1, None, 1, need - 1, None, 0)
    assert e.value.code == B.LE_E_WORKSPACE
    with pytest.raises(B.LeError) as e:
        B.le_init(p, None, 1, None, 1, need, None, 0)
    assert e.value.code == B.LE_E_ARG


def test_strerror_is_static_text():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 99):
        assert isinstance(B.strerror(code), str) and B.strerror(code)


def test_force_cap_is_validated_on_the_host():
    ok = _lj(force_cap=100.0)
    assert B.le_workspace_bytes(ok.to_c()) > 0
    for bad in (_lj(force_cap=-1.0), _lj(force_cap=100.0, precision="mixed"),
                _lj(force_cap=100.0, thermostat="dpd"), _lj(force_cap=100.0, tune=1),
                _lj(force_cap=float("inf"))):
        with pytest.raises(B.LeError) as e:
            B.le_workspace_bytes(bad.to_c())
        assert e.value.code == B.LE_E_ARG


def test_particle_count_fits_the_list_entries():
    """A global-list entry holds a slot (0..n, n the sentinel) in 24 bits next
    to a 7-bit image code, so n is at most 2^24 - 2."""
    assert B.le_workspace_bytes(_lj(n=2**24 - 2, L=200.0).to_c()) > 0
    for n in (2**24 - 1, 2**24):
        with pytest.raises(B.LeError) as e:
            B.le_workspace_bytes(_lj(n=n, L=200.0).to_c())
        assert e.value.code == B.LE_E_ARG
