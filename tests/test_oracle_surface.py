"""Pins of the oracle's surface geometry (periodic x, y; isolated z).

The kernel formula is checked against quantities computed without it:
Gaussian pair energies from a 2-D lattice sum of the in-plane Fourier
components with the exact z-integrals of exp(-G|z - z'|) and |z - z'|
(tests/closed_forms.py), a brute-force real-space sum on a tiny grid (padding
along z only, crop, axis order), and in-plane translation covariance.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
from exx_inputs import SURFACE, OrbitalRecipe, make_system

N_GRID, H = 32, 0.4
L = N_GRID * H


def _normalised_gaussian(P, c):
    return cf.normalised_gaussian(N_GRID, H, P, c)


def _periodic_xy_gaussian(P, c, Q=1.0):
    """Q N(P, c) summed over in-plane images (x, y periodic with period L)."""
    out = np.zeros((N_GRID,) * 3)
    for ix in (-1, 0, 1):
        for iy in (-1, 0, 1):
            out += _normalised_gaussian((P[0] + ix * L, P[1] + iy * L, P[2]), c)
    return Q * out


@pytest.mark.parametrize("R_over_L", [1.0, 0.8, 1.3])
def test_self_energy_of_a_gaussian_density(R_over_L):
    # the cut radius R is exact as long as R exceeds the density's extent in
    # z and 2L - R does too (no wrapped partner within R); at R = L the
    # sin(G_z R) terms of the kernel vanish on the grid, so other radii are
    # needed to pin them
    c = 0.8
    rho = _periodic_xy_gaussian((3.1, 9.7, 0.5 * L), c)
    V = oracle.solve_poisson(rho, H, "surface", R=R_over_L * L)
    e = oracle.pair_energy(rho, V, H)
    ref = cf.slab_gaussian_self_energy(1.0, c, L, 40)
    assert e == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("R_over_L", [1.0, 0.9])
def test_interaction_of_two_gaussians_offset_in_plane_and_height(R_over_L):
    # centres near opposite in-plane edges (the images matter) and at two heights
    P1, c1 = (1.0, 11.9, 5.3), 0.7
    P2, c2 = (11.0, 0.6, 7.4), 0.75
    r1 = _periodic_xy_gaussian(P1, c1)
    r2 = _periodic_xy_gaussian(P2, c2, Q=-0.6)
    V2 = oracle.solve_poisson(r2, H, "surface", R=R_over_L * L)
    e12 = (H ** 3) * math.fsum((r1 * V2).ravel().tolist())
    ref = cf.slab_gaussian_interaction(1.0, P1, c1, -0.6, P2, c2, L, 40)
    assert e12 == pytest.approx(ref, rel=1e-9)
    # and the reverse order (symmetric kernel, same value)
    V1 = oracle.solve_poisson(r1, H, "surface", R=R_over_L * L)
    e21 = (H ** 3) * math.fsum((r2 * V1).ravel().tolist())
    assert e21 == pytest.approx(e12, rel=1e-12)


def test_pair_energies_of_gaussian_orbitals_through_exx():
    # psi_a, psi_b periodic s-Gaussians; rho_ab = psi_a psi_b is Q_ab N(P, c)
    A, a = (2.0, 3.0, 6.0), 0.9
    B, b = (3.2, 2.1, 7.0), 1.1
    def periodic_gauss(P, w):
        out = np.zeros((N_GRID,) * 3)
        for ix in (-1, 0, 1):
            for iy in (-1, 0, 1):
                out += cf.gaussian(N_GRID, H, (P[0] + ix * L, P[1] + iy * L, P[2]), w)
        return out
    psi = np.stack([periodic_gauss(A, a), periodic_gauss(B, b)])
    occ = np.array([1.0, 0.5])
    r = oracle.exx(psi, occ, H, "surface")
    pe = r["pair_e"]
    for (i, j, (P1, w1), (P2, w2)) in [(0, 0, (A, a), (A, a)), (1, 1, (B, b), (B, b)),
                                       (0, 1, (A, a), (B, b))]:
        Q, P, c = cf.gaussian_product(P1, w1, P2, w2)
        assert pe[i, j] == pytest.approx(cf.slab_gaussian_self_energy(Q, c, L, 40), rel=1e-9)
    assert pe[0, 1] == pytest.approx(pe[1, 0], rel=1e-13)
    E = -0.5 * float(occ @ pe @ occ)
    assert r["E"] == pytest.approx(E, rel=1e-13)


def test_fft_route_equals_brute_force_on_a_tiny_grid():
    rng = np.random.default_rng(7)
    n, h = 4, 0.7
    rho = rng.standard_normal((n, n, n))
    V_fft = oracle.solve_poisson(rho, h, "surface")
    V_bf = oracle.brute_force_potential(rho, h, "surface")
    assert np.max(np.abs(V_fft - V_bf)) <= 1e-12 * np.max(np.abs(V_bf))
    # the padding is along z (array axis 0) only
    assert oracle.fft_shape(n, "surface") == (2 * n, n, n)


def test_in_plane_translation_covariance():
    rng = np.random.default_rng(8)
    n = 12
    rho = rng.standard_normal((n, n, n))
    V = oracle.solve_poisson(rho, 0.5, "surface")
    Vs = oracle.solve_poisson(np.roll(rho, (3, -5), axis=(2, 1)), 0.5, "surface")
    assert np.allclose(Vs, np.roll(V, (3, -5), axis=(2, 1)), rtol=0, atol=1e-12 * np.abs(V).max())
    # along z the geometry is not periodic: a cyclic shift changes the potential
    Vz = oracle.solve_poisson(np.roll(rho, 3, axis=0), 0.5, "surface")
    assert np.max(np.abs(Vz - np.roll(V, 3, axis=0))) > 1e-3 * np.abs(V).max()


def test_surface_invariants_on_drawn_orbitals():
    rec = OrbitalRecipe(n=16, h=0.5, n_orb=4, n_gauss=3, sigma=(0.7, 1.2), centres="slab",
                        bc=SURFACE, seed=31)
    s = make_system(rec)
    r = oracle.exx(s.psi, s.occ, s.h, "surface")
    pe = r["pair_e"]
    assert np.allclose(pe, pe.T, rtol=1e-12, atol=0)
    # E_x = -1/2 h^3 sum_i f_i <psi_i, (K psi)_i>
    dots = (s.psi.reshape(4, -1) * r["kpsi"].reshape(4, -1)).sum(axis=1)
    assert r["E"] == pytest.approx(-0.5 * s.h ** 3 * float(s.occ @ dots), rel=1e-12)
    # rotation among equally occupied orbitals leaves E_x unchanged
    th = 0.37
    U = np.eye(4)
    U[:2, :2] = [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]
    psi_r = np.einsum("ij,jzyx->izyx", U.T, s.psi)
    r2 = oracle.exx(psi_r, s.occ, s.h, "surface", symmetric=True)
    assert r2["E"] == pytest.approx(r["E"], rel=1e-12)
