"""CPU checks of the autotuner's candidate rule against the library's own
geometry validation (host code only; no device work)."""
import math

import pytest

from paper_2109_11083_amd import binding as B
from paper_2109_11083_amd.sim import Params
from paper_2109_11083_amd.tune import filling_skin

CASES = [
    ((67.18380, 67.18380, 67.18380), 2.5),          # the 256k LJ fluid
    ((77.78218, 77.78218, 77.78218), 2 ** (1 / 6)),  # the 400k-bead KG melt
    ((30.1, 25.3, 41.7), 2.5),                       # non-cubic
]


def _ws(box, rc, skin, cells=(0, 0, 0)):
    return B.le_workspace_bytes(Params(n=20000, box=box, rc=rc, skin=skin, cells=cells).to_c())


@pytest.mark.parametrize("box,rc", CASES)
def test_filling_skin_keeps_the_grid_and_is_the_largest(box, rc):
    for s in (0.2, 0.3, 0.4, 0.5, 0.6, 0.8):
        p = Params(n=20000, box=box, rc=rc, skin=s)
        f = filling_skin(p, s)
        if f is None:
            continue
        assert f >= s - 1e-12
        nc = tuple(int(math.floor(L / ((rc + s) * (1 + 1e-9)))) for L in box)
        # the library's own grid for s and for the filling skin is nc: the
        # workspace with cells left to the library equals the one with nc given
        assert _ws(box, rc, s) == _ws(box, rc, s, nc)
        assert _ws(box, rc, f) == _ws(box, rc, f, nc)
        # a slightly larger skin no longer fits that grid
        with pytest.raises(B.LeError) as e:
            _ws(box, rc, f + 1e-4, nc)
        assert e.value.code == B.LE_E_GEOMETRY
