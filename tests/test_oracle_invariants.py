"""Invariants, brute force and finite differences that pin the FP64 oracle.

* tiny grids: the FFT route equals an explicit real-space convolution whose
  kernel is built by a dense inverse DFT sum (pins padding, crop, index
  wrap and normalisation of the FFT route);
* V_ij = V_ji, e_ij >= 0, E_x <= 0, E_x(a f) = a^2 E_x;
* E_x = -1/2 sum_i f_i h^3 <psi_i, (K psi)_i>, which ties the pair-energy
  route to the K psi route (a dropped occupation factor breaks it);
* orthogonal rotations inside an equal-occupation block leave E_x unchanged
  and rotate K psi the same way (Eq. 2 depends on the density matrix only);
* the gradient -2 f_k h^3 (K psi)_k against Richardson finite differences,
  and the Euler identity for a quartic, sum_k <psi_k, dE/dpsi_k> = 4 E_x;
* the pair counts N(N+1)/2 of Table 1.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from exx_inputs import OrbitalRecipe, make_system, pair_count

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("bc,n", [("free", 4), ("free", 5), ("periodic", 6), ("periodic", 5)])
def test_fft_route_equals_bruteforce_sum(bc, n):
    rng = np.random.default_rng(n)
    h = 0.7
    rho = rng.normal(size=(n, n, n))
    V = oracle.solve_poisson(rho, h, bc)
    Vb = oracle.brute_force_potential(rho, h, bc)
    assert np.max(np.abs(V - Vb)) < 1e-12 * np.max(np.abs(Vb))


def test_bruteforce_detects_transposed_axes():
    # the pin above would fail if the solver mixed up axes on anisotropic data
    n, h = 4, 0.7
    rho = np.zeros((n, n, n))
    rho[0, 1, 3] = 1.0
    V = oracle.solve_poisson(rho, h, "free")
    Vt = oracle.solve_poisson(rho.transpose(2, 1, 0).copy(), h, "free").transpose(2, 1, 0)
    assert np.max(np.abs(V - Vt)) < 1e-12  # the kernel is isotropic on a cubic grid
    assert abs(V[0, 1, 3] - V[3, 1, 0]) > 1e-3  # but the source position matters


def _small_system(bc, n=16, N=4, seed=3, frac=0):
    rec = OrbitalRecipe(n=n, h=0.5, n_orb=N, n_gauss=3, sigma=(0.9, 1.4),
                        centres="box" if bc == "periodic" else "middle", bc=bc,
                        frac_last=frac, seed=seed)
    return make_system(rec)


@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_symmetry_positivity_and_kpsi_energy_identity(bc):
    s = _small_system(bc, frac=1)
    res = oracle.exx(s.psi, s.occ, s.h, bc)
    e = res["pair_e"]
    assert np.max(np.abs(e - e.T)) < 1e-12 * np.max(np.abs(e))
    assert np.all(np.diag(e) > 0)
    # the kernel is positive semidefinite: each e_ij is a self-energy
    assert np.all(e > -1e-14 * np.max(np.abs(e)))
    assert res["E"] < 0
    h3 = s.h ** 3
    E2 = -0.5 * h3 * sum(s.occ[i] * float(np.sum(s.psi[i] * res["kpsi"][i]))
                         for i in range(s.n_orb))
    assert res["E"] == pytest.approx(E2, rel=1e-12)
    res2 = oracle.exx(s.psi, 3.0 * s.occ, s.h, bc)
    assert res2["E"] == pytest.approx(9.0 * res["E"], rel=1e-13)


def test_pair_potential_symmetry():
    s = _small_system("free")
    Vij = oracle.solve_poisson(s.psi[0] * s.psi[2], s.h, "free")
    Vji = oracle.solve_poisson(s.psi[2] * s.psi[0], s.h, "free")
    assert np.array_equal(Vij, Vji) or np.max(np.abs(Vij - Vji)) < 1e-15


@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_rotation_invariance(bc):
    s = _small_system(bc, N=4)
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    rot = np.einsum("ji,jzyx->izyx", U, s.psi)  # psi'_i = sum_j U_ji psi_j
    a = oracle.exx(s.psi, s.occ, s.h, bc)
    b = oracle.exx(rot, s.occ, s.h, bc)
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    kr = np.einsum("ji,jzyx->izyx", U, a["kpsi"])
    assert np.max(np.abs(b["kpsi"] - kr)) < 1e-11 * np.max(np.abs(kr))


def test_single_orbital_is_minus_hartree():
    # Eq. 2, i = j: the self term cancels the Hartree energy of rho = psi^2
    s = _small_system("free", N=1)
    occ = np.array([1.0])
    res = oracle.exx(s.psi, occ, s.h, "free")
    rho = s.psi[0] ** 2
    EH = 0.5 * s.h ** 3 * float(np.sum(rho * oracle.solve_poisson(rho, s.h, "free")))
    assert res["E"] == pytest.approx(-EH, rel=1e-13)


@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_gradient_against_richardson_differences(bc):
    s = _small_system(bc, n=12, N=3, frac=1)
    res = oracle.exx(s.psi, s.occ, s.h, bc)
    grad = oracle.exx_grad_psi(res["kpsi"], s.occ, s.h)
    rng = np.random.default_rng(5)
    d = rng.normal(size=s.psi.shape)

    def E(eps):
        return oracle.exx(s.psi + eps * d, s.occ, s.h, bc, want_kpsi=False)["E"]

    def D(eps):
        return (E(eps) - E(-eps)) / (2 * eps)

    eps = 1e-3
    fd = (4.0 * D(eps / 2) - D(eps)) / 3.0  # exact for a quartic up to rounding
    assert fd == pytest.approx(float(np.sum(grad * d)), rel=1e-8)
    euler = float(np.sum(grad * s.psi))
    assert euler == pytest.approx(4.0 * res["E"], rel=1e-12)


def test_occupation_gradient():
    s = _small_system("periodic", n=12, N=3)
    res = oracle.exx(s.psi, s.occ, s.h, "periodic")
    g = oracle.exx_grad_occ(res["pair_e"], s.occ)
    for k in range(3):
        df = np.zeros(3)
        df[k] = 1e-2
        Ep = oracle.exx(s.psi, s.occ + df, s.h, "periodic", want_kpsi=False)["E"]
        Em = oracle.exx(s.psi, s.occ - df, s.h, "periodic", want_kpsi=False)["E"]
        assert (Ep - Em) / 2e-2 == pytest.approx(g[k], rel=1e-10)  # E is quadratic in f


def test_table1_pair_counts():
    with open(os.path.join(GOLDEN, "table1_pair_counts.json")) as f:
        table = json.load(f)
    for row in table["water"]:
        assert pair_count(row["orbitals"]) == row["co_densities"]


def test_symmetric_loop_matches_ordered_loop():
    s = _small_system("free", N=3)
    a = oracle.exx(s.psi, s.occ, s.h, "free")
    b = oracle.exx(s.psi, s.occ, s.h, "free", symmetric=True)
    assert b["E"] == pytest.approx(a["E"], rel=1e-13)
    assert np.max(np.abs(a["kpsi"] - b["kpsi"])) < 1e-12 * np.max(np.abs(a["kpsi"]))
