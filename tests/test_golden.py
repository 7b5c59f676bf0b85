"""The stored oracle values under tests/golden belong to the system they name
and are the oracle's own output: the digest of the regenerated inputs
matches, and a few molecules solved afresh by the oracle reproduce them."""
import hashlib
import os

import numpy as np
import pytest

import synth
from oracle import nolsm as o

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube4096_traces.npz")


@pytest.fixture(scope="module")
def cube():
    return synth.make_config(2)


def test_cube4096_traces_are_the_oracles(cube):
    g = np.load(GOLDEN)
    h = hashlib.sha256()
    for a in (cube.K.row_ptr, cube.K.col_idx, cube.K.val, cube.S.row_ptr, cube.S.col_idx, cube.S.val):
        h.update(np.ascontiguousarray(a).tobytes())
    assert str(g["digest"]) == h.hexdigest()
    assert g["N"].shape == (cube.nmol,) and np.all(g["status"] == 0)
    m = np.diff(cube.K.row_ptr)
    for J in (0, int(np.argmin(m)), int(np.argmax(m)), cube.nmol - 1):
        r = o.solve_molecule(cube, J)
        assert abs(r.N_J - g["N"][J]) <= 1e-12 and abs(r.E_J - g["E"][J]) <= 1e-11, J
    # N_J counts occupied orbitals per molecule up to the truncation: close
    # to 4, and 4 on average
    assert abs(g["N"].mean() - 4.0) < 1e-2
