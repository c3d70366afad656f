"""Pins of the oracle's wire geometry (isolated x, y; periodic z).

The cylindrically cut kernel is checked against quantities computed without
it: Gaussian energies from a 1-D lattice sum over the axial Fourier components
with the in-plane averages of 2 K0(|G_z| rho) and -2 ln(rho) done by
quadrature of the Rice law (tests/closed_forms.py), a brute-force real-space
sum on a tiny grid (padding along x and y only), and axial translation
covariance.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
from exx_inputs import WIRE, OrbitalRecipe, make_system

N_GRID, H = 32, 0.4
L = N_GRID * H


def _periodic_z_gaussian(P, c, Q=1.0):
    """Q N(P, c) summed over axial images (z periodic with period L)."""
    out = np.zeros((N_GRID,) * 3)
    for iz in (-1, 0, 1):
        out += cf.normalised_gaussian(N_GRID, H, (P[0], P[1], P[2] + iz * L), c)
    return Q * out


@pytest.mark.parametrize("R_over_L", [1.0, 0.8])
def test_self_energy_of_a_gaussian_density(R_over_L):
    c = 0.8
    P = (0.5 * L, 0.5 * L, 1.7)
    rho = _periodic_z_gaussian(P, c)
    V = oracle.solve_poisson(rho, H, "wire", R=R_over_L * L)
    e = oracle.pair_energy(rho, V, H)
    ref = cf.wire_gaussian_interaction(1.0, P, c, 1.0, P, c, L, 60)
    assert e == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("R_over_L", [1.0, 0.9])
def test_interaction_of_two_gaussians_offset_in_plane_and_along_the_axis(R_over_L):
    P1, c1 = (5.2, 6.1, 0.8), 0.7    # near the axial cell edge: the images matter
    P2, c2 = (7.4, 5.0, 12.0), 0.75
    r1 = _periodic_z_gaussian(P1, c1)
    r2 = _periodic_z_gaussian(P2, c2, Q=-0.6)
    V2 = oracle.solve_poisson(r2, H, "wire", R=R_over_L * L)
    e12 = (H ** 3) * math.fsum((r1 * V2).ravel().tolist())
    ref = cf.wire_gaussian_interaction(1.0, P1, c1, -0.6, P2, c2, L, 60)
    assert e12 == pytest.approx(ref, rel=1e-9)


def test_fft_route_equals_brute_force_on_a_tiny_grid():
    rng = np.random.default_rng(11)
    n, h = 4, 0.7
    rho = rng.standard_normal((n, n, n))
    V_fft = oracle.solve_poisson(rho, h, "wire")
    V_bf = oracle.brute_force_potential(rho, h, "wire")
    assert np.max(np.abs(V_fft - V_bf)) <= 1e-12 * np.max(np.abs(V_bf))
    assert oracle.fft_shape(n, "wire") == (n, 2 * n, 2 * n)


def test_axial_translation_covariance():
    rng = np.random.default_rng(12)
    n = 12
    rho = rng.standard_normal((n, n, n))
    V = oracle.solve_poisson(rho, 0.5, "wire")
    Vs = oracle.solve_poisson(np.roll(rho, 5, axis=0), 0.5, "wire")
    assert np.allclose(Vs, np.roll(V, 5, axis=0), rtol=0, atol=1e-12 * np.abs(V).max())
    # in the plane the geometry is isolated: a cyclic shift changes the potential
    Vx = oracle.solve_poisson(np.roll(rho, 3, axis=2), 0.5, "wire")
    assert np.max(np.abs(Vx - np.roll(V, 3, axis=2))) > 1e-3 * np.abs(V).max()


def test_wire_invariants_on_drawn_orbitals():
    rec = OrbitalRecipe(n=16, h=0.5, n_orb=4, n_gauss=3, sigma=(0.7, 1.2), centres="rod",
                        bc=WIRE, seed=41)
    s = make_system(rec)
    r = oracle.exx(s.psi, s.occ, s.h, "wire")
    pe = r["pair_e"]
    assert np.allclose(pe, pe.T, rtol=1e-12, atol=0)
    dots = (s.psi.reshape(4, -1) * r["kpsi"].reshape(4, -1)).sum(axis=1)
    assert r["E"] == pytest.approx(-0.5 * s.h ** 3 * float(s.occ @ dots), rel=1e-12)
    th = 0.61
    U = np.eye(4)
    U[1:3, 1:3] = [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]
    psi_r = np.einsum("ij,jzyx->izyx", U.T, s.psi)
    r2 = oracle.exx(psi_r, s.occ, s.h, "wire", symmetric=True)
    assert r2["E"] == pytest.approx(r["E"], rel=1e-12)
