"""Pins of oracle.kpsi_rows, which writes the stored K psi expectations of the
largest workloads (periodic 96^3 with 128 orbitals, free 128^3 with 256).

* it equals the full operator's rows from oracle.exx's ordered-pair loop, with
  occupations that differ for every orbital, so an occupation taken from the
  wrong orbital of the pair (f_i instead of f_j) or a missing one fails;
* independently of oracle.exx's K psi loop, its rows are the gradient of E_x
  (computed from pair energies only) along random directions that move a
  single orbital: dE/d(eps) = -2 f_i h^3 <(K psi)_i, d> (Eq. 3 as the derivative
  of Eq. 2), by Richardson differences, which are exact for a quartic;
* complex orbitals: V_ij psi_j with rho_ij = conj(psi_j) psi_i (Eq. 2), against
  the complex gradient of E_x.
Each test also plants the occupation slip in a copy of the row sum and checks
that the comparison it makes would catch it.
"""
import numpy as np
import pytest

import oracle
from exx_inputs import OrbitalRecipe, make_system


def _system(bc, n, N, seed, kmax=0.0):
    rec = OrbitalRecipe(n=n, h=0.5, n_orb=N, n_gauss=3, sigma=(0.9, 1.4),
                        centres="box" if bc == "periodic" else "middle", bc=bc, seed=seed,
                        kmax=kmax)
    s = make_system(rec)
    occ = np.linspace(2.0, 0.35, N)  # a different occupation for every orbital
    return s, occ


def _rows_with_slip(psi, occ, rows, h, bc):
    """kpsi_rows with the occupation of the row orbital instead of its partner."""
    khat = oracle.kernel_hat(psi.shape[1], h, bc)
    out = np.zeros((len(rows),) + psi.shape[1:], dtype=psi.dtype)
    for r, i in enumerate(rows):
        for j in range(psi.shape[0]):
            V = oracle.solve_poisson(oracle.co_density(psi[i], psi[j]), h, bc, khat=khat)
            out[r] += occ[i] * V * psi[j]
    return out


@pytest.mark.parametrize("bc", ["free", "periodic"])
def test_rows_equal_full_operator(bc):
    s, occ = _system(bc, 12, 5, 41)
    rows = [0, 3, 4]
    full = oracle.exx(s.psi, occ, s.h, bc)["kpsi"]
    got = oracle.kpsi_rows(s.psi, occ, rows, s.h, bc)
    scale = np.max(np.abs(full[rows]))
    assert np.max(np.abs(got - full[rows])) <= 1e-13 * scale
    slip = _rows_with_slip(s.psi, occ, rows, s.h, bc)
    assert np.max(np.abs(slip - full[rows])) > 1e-3 * scale


@pytest.mark.parametrize("bc,kmax", [("free", 0.0), ("periodic", 0.0), ("free", 0.8)])
def test_rows_are_the_energy_gradient(bc, kmax):
    s, occ = _system(bc, 10, 4, 43, kmax=kmax)
    rows = [1, 3]
    got = oracle.kpsi_rows(s.psi, occ, rows, s.h, bc)
    slip = _rows_with_slip(s.psi, occ, rows, s.h, bc)
    rng = np.random.default_rng(7)
    for r, i in enumerate(rows):
        d = np.zeros_like(s.psi)
        d[i] = rng.normal(size=s.psi.shape[1:])
        if np.iscomplexobj(s.psi):
            d[i] = d[i] + 1j * rng.normal(size=s.psi.shape[1:])

        def E(eps):
            return oracle.exx(s.psi + eps * d, occ, s.h, bc, want_kpsi=False)["E"]

        def D(eps):
            return (E(eps) - E(-eps)) / (2 * eps)

        eps = 1e-3
        fd = (4.0 * D(eps / 2) - D(eps)) / 3.0
        # dE = Re sum conj(dE/dpsi) d with dE/dpsi_i = -2 f_i h^3 (K psi)_i
        want = float(np.real(np.sum(np.conj(-2.0 * occ[i] * s.h ** 3 * got[r]) * d[i])))
        assert fd == pytest.approx(want, rel=1e-8)
        wrong = float(np.real(np.sum(np.conj(-2.0 * occ[i] * s.h ** 3 * slip[r]) * d[i])))
        assert abs(wrong - fd) > 1e-4 * abs(fd)
