"""The stored oracle expectations match a fresh oracle run on regenerated inputs.

tests/golden/*_oracle.npz were written by make_oracle_golden.py (oracle only);
re-solving one stored pair per file pins the generator, the oracle and the
files to each other (the 256-orbital 128^3 system takes about 30 s and 4.3 GB
to regenerate).
"""
import glob
import os

import numpy as np
import pytest

import oracle
from exx_inputs import batch_recipes, make_system, system

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILES = sorted(glob.glob(os.path.join(GOLDEN, "*_oracle.npz")))


def _system(name):
    if name.startswith("batch16_s"):
        return make_system(batch_recipes()[int(name.split("_s")[1])])
    return system(name)


@pytest.mark.parametrize("path", FILES, ids=lambda p: os.path.basename(p).replace("_oracle.npz", ""))
def test_one_pair_recomputes(path):
    name = os.path.basename(path).replace("_oracle.npz", "")
    g = dict(np.load(path))
    s = _system(name)
    assert int(g["n"]) == s.n and int(g["n_orb"]) == s.n_orb
    if "pairs" in g:
        i, j = (int(x) for x in g["pairs"][-1])
        want = float(g["pair_energies"][-1])
    else:
        i, j = 0, s.n_orb - 1
        want = float(g["pair_e"][i, j])
        E = -0.5 * float(s.occ @ g["pair_e"] @ s.occ)
        assert E == pytest.approx(float(g["E"]), rel=1e-13)
    got = oracle.pair_energies(s.psi, [(i, j)], s.h, s.bc, R=s.R)[0]
    assert got == pytest.approx(want, rel=1e-12, abs=1e-15)
