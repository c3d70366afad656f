"""Pins of the FP64 oracle against closed forms (no GPU, no HIP code).

Each test targets a specific mistake the oracle could make:
* plane waves pin the periodic kernel 4 pi/|G|^2, the folding of negative
  frequencies and the FFT normalisation;
* a Gaussian charge pins the free-boundary kernel (its 8 pi sin^2 form, the
  G = 0 value 2 pi R^2, the zero padding and the crop);
* products of Gaussians pin the co-density (Eq. 8) and the pair energy;
* a linear combination of Gaussians pins the whole E_x of Eq. 5 including
  the -1/2 f_i f_j weights;
* periodised Gaussians pin the periodic pair energy through an independent
  reciprocal-space sum.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle


def test_periodic_plane_wave_potential():
    n, h = 16, 0.5
    L = n * h
    Z, Y, X = cf.grid_coords(n, h)
    for k in [(1, 0, 0), (3, -2, 5), (-7, 4, 1), (2, 2, -3)]:
        G = 2.0 * math.pi * np.array(k, float) / L
        phase = G[0] * X + G[1] * Y + G[2] * Z
        for rho in (np.cos(phase), np.sin(phase)):
            V = oracle.solve_poisson(rho, h, oracle.PERIODIC)
            expect = 4.0 * math.pi / float(G @ G) * rho
            assert np.max(np.abs(V - expect)) < 1e-12 * np.max(np.abs(expect))


def test_periodic_constant_density_has_zero_potential():
    # the G = 0 term is dropped: a uniform background produces no potential
    V = oracle.solve_poisson(np.ones((8, 8, 8)), 0.5, oracle.PERIODIC)
    assert np.max(np.abs(V)) < 1e-14


@pytest.mark.parametrize("sigma", [1.0, 1.3])
def test_free_gaussian_charge_potential_and_self_energy(sigma):
    n, h = 48, 0.4
    L = n * h
    c = np.array([0.5 * L, 0.47 * L, 0.52 * L])
    Q = 1.7
    rho = Q * cf.normalised_gaussian(n, h, c, sigma)
    V = oracle.solve_poisson(rho, h, oracle.FREE)  # R = L by default
    exact = cf.gaussian_potential(n, h, c, sigma, Q)
    Z, Y, X = cf.grid_coords(n, h)
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    inside = r < L - 7.0 * sigma  # every point of the charge lies within R = L
    assert inside.sum() > 1000
    assert np.max(np.abs(V[inside] - exact[inside])) < 1e-10 * Q
    e = oracle.pair_energy(rho, V, h)
    assert abs(e - Q * Q * cf.self_energy_normalised(sigma)) < 1e-11 * Q * Q


def test_free_kernel_g0_term_matters():
    # dropping 2 pi R^2 at G = 0 would shift V by a constant Q*2piR^2/(m^3 h^3)
    n, h = 24, 0.5
    rho = cf.normalised_gaussian(n, h, [6.0, 6.0, 6.0], 1.2)
    K = oracle.kernel_hat(n, h, oracle.FREE)
    R = n * h
    assert K[0, 0, 0] == pytest.approx(2.0 * math.pi * R * R, rel=1e-15)
    # the closed form is continuous at G -> 0: 8 pi sin^2(GR/2)/G^2 -> 2 pi R^2
    G = 1e-6
    assert 8.0 * math.pi * math.sin(0.5 * G * R) ** 2 / G ** 2 == pytest.approx(K[0, 0, 0], rel=1e-9)
    V = oracle.solve_poisson(rho, h, oracle.FREE)
    assert V.min() > 0.0  # a positive charge has a positive potential everywhere


def test_product_of_gaussians_pair_energies():
    n, h = 48, 0.4
    L = n * h
    A = np.array([0.42, 0.5, 0.55]) * L
    B = np.array([0.58, 0.47, 0.5]) * L
    a, b = 1.1, 1.4
    psi = np.stack([cf.gaussian(n, h, A, a), cf.gaussian(n, h, B, b)])
    occ = np.array([1.0, 0.7])
    res = oracle.exx(psi, occ, h, oracle.FREE)
    for (i, j), (P1, s1, P2, s2) in {
        (0, 0): (A, a, A, a), (0, 1): (A, a, B, b), (1, 1): (B, b, B, b)}.items():
        Q, P, c = cf.gaussian_product(P1, s1, P2, s2)
        expect = Q * Q * cf.self_energy_normalised(c)
        assert res["pair_e"][i, j] == pytest.approx(expect, rel=1e-10)
        assert res["pair_e"][j, i] == pytest.approx(expect, rel=1e-10)
    # E_x = -1/2 sum_ij f_i f_j e_ij, i.e. off-diagonal pairs counted twice
    e = res["pair_e"]
    E = -0.5 * (occ[0] ** 2 * e[0, 0] + 2 * occ[0] * occ[1] * e[0, 1] + occ[1] ** 2 * e[1, 1])
    assert res["E"] == pytest.approx(E, rel=1e-14)


def test_full_exchange_energy_of_gaussian_combinations():
    """E_x of Loewdin-orthonormalised combinations of s-Gaussians vs the 4-index sum."""
    n, h = 48, 0.4
    L = n * h
    rng = np.random.default_rng(7)
    gauss = [(rng.uniform(0.42, 0.58, 3) * L, rng.uniform(1.0, 1.4)) for _ in range(4)]
    phi = np.stack([cf.gaussian(n, h, A, a) for A, a in gauss])
    S = h ** 3 * phi.reshape(4, -1) @ phi.reshape(4, -1).T
    w, U = np.linalg.eigh(S)
    C = (U / np.sqrt(w)) @ U.T  # psi_i = sum_k C_ik g_k
    psi = np.einsum("ik,kzyx->izyx", C, phi)
    occ = np.array([2.0, 2.0, 1.5, 0.5])
    res = oracle.exx(psi, occ, h, oracle.FREE)
    T = cf.four_index(gauss)
    e = np.einsum("ik,jl,im,jn,klmn->ij", C, C, C, C, T)
    E = -0.5 * float(occ @ e @ occ)
    assert np.allclose(res["pair_e"], e, rtol=1e-9, atol=1e-12)
    assert res["E"] == pytest.approx(E, rel=1e-10)


def test_periodic_gaussian_pair_energy_reciprocal_sum():
    n, h = 32, 0.4
    L = n * h
    c = 1.1
    P = np.array([3.0, 7.1, 9.4])
    rho = np.zeros((n, n, n))
    for tx in (-1, 0, 1):  # periodised Gaussian (images beyond one shell are < 1e-40)
        for ty in (-1, 0, 1):
            for tz in (-1, 0, 1):
                rho += cf.normalised_gaussian(n, h, P + L * np.array([tx, ty, tz]), c)
    V = oracle.solve_poisson(rho, h, oracle.PERIODIC)
    e = oracle.pair_energy(rho, V, h)
    expect = cf.periodic_gaussian_pair_energy(1.0, c, L, kmax=40)
    assert e == pytest.approx(expect, rel=1e-11)
