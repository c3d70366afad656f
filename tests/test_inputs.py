"""The seeded generator: reproducible, orthonormal on the grid, right shapes."""
import numpy as np
import pytest

from exx_inputs import (FREE, PERIODIC, OrbitalRecipe, batch_recipes, make_system, recipe,
                        scaled)


def test_reproducible_and_orthonormal():
    rec = scaled(recipe("periodic32_n8"), n=16)
    a = make_system(rec)
    b = make_system(rec)
    assert np.array_equal(a.psi, b.psi)
    flat = a.psi.reshape(a.n_orb, -1)
    S = a.h ** 3 * flat @ flat.T
    assert np.max(np.abs(S - np.eye(a.n_orb))) < 1e-12
    assert a.psi.flags.c_contiguous and a.psi.dtype == np.float64
    assert np.all(a.occ == 2.0)


def test_free_default_radius_and_fractional_occupations():
    rec = OrbitalRecipe(n=16, h=0.4, n_orb=6, n_gauss=2, sigma=(0.6, 1.0), centres="middle",
                        bc=FREE, frac_last=2, seed=9)
    s = make_system(rec)
    assert s.R == pytest.approx(16 * 0.4)
    assert np.all(s.occ[:4] == 2.0)
    assert np.all((s.occ[4:] >= 0.0) & (s.occ[4:] <= 2.0))


def test_ptype_orbitals_are_orthonormal():
    rec = scaled(recipe("periodic96_n128"), n=16, n_orb=5)
    s = make_system(rec)
    flat = s.psi.reshape(5, -1)
    assert np.max(np.abs(s.h ** 3 * flat @ flat.T - np.eye(5))) < 1e-12
    assert s.bc == PERIODIC


def test_batch_recipes():
    recs = batch_recipes()
    assert len(recs) == 16
    assert all(r.n in (48, 64, 80, 96, 112) and 16 <= r.n_orb <= 96 for r in recs)
    assert len({r.seed for r in recs}) == 16
