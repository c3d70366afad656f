"""Pins of the oracle for complex orbitals (rho_ij = conj(psi_j) psi_i, Eq. 2).

Each test targets a mistake the complex path could make (a missing or
misplaced complex conjugate, the wrong one of V_ij and V_ji in the K psi
update, a real part taken too early):
* plane waves are eigenfunctions of the periodic exchange operator with a
  closed-form eigenvalue, and their pair energies are 4 pi / (|G_a - G_b|^2 Omega);
* a Gaussian pair density modulated by exp(i kappa.r) has a closed-form
  free-space energy (Dawson's integral, tests/closed_forms.py) that depends on
  kappa = k_a - k_b only, while an unconjugated product would give k_a + k_b;
* per-orbital phases reduce the complex case to the real one already pinned
  elsewhere, with K psi picking up the orbital's own phase;
* a complex unitary mixing of equally occupied orbitals leaves E_x unchanged
  and transforms K psi like the orbitals;
* Richardson differences of E_x along complex directions fix the gradient
  -2 f h^3 K psi (with respect to Re psi + i Im psi);
* the FFT route equals the explicit real-space sum for a complex density.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
from exx_inputs import FREE, PERIODIC, SURFACE, WIRE, OrbitalRecipe, make_system

CENTRES = {PERIODIC: "box", FREE: "middle", SURFACE: "slab", WIRE: "rod"}


def _complex_system(bc, n=16, N=4, seed=21, kmax=1.0, frac=0):
    rec = OrbitalRecipe(n=n, h=0.5, n_orb=N, n_gauss=3, sigma=(0.9, 1.4), centres=CENTRES[bc],
                        bc=bc, frac_last=frac, seed=seed, kmax=kmax)
    return make_system(rec)


def test_plane_waves_are_exchange_eigenfunctions():
    n, h = 12, 0.5
    L = n * h
    Omega = L ** 3
    Z, Y, X = cf.grid_coords(n, h)
    ks = [(0, 0, 0), (1, 0, 0), (0, -2, 1), (2, 1, -1)]
    Gs = [2.0 * math.pi / L * np.array(k, float) for k in ks]
    psi = np.stack([np.exp(1j * (G[0] * X + G[1] * Y + G[2] * Z)) / math.sqrt(Omega) for G in Gs])
    occ = np.array([2.0, 1.5, 1.0, 0.25])
    r = oracle.exx(psi, occ, h, PERIODIC)
    N = len(ks)
    e_ref = np.zeros((N, N))
    for a in range(N):
        for b in range(N):
            if a != b:
                d = Gs[a] - Gs[b]
                e_ref[a, b] = 4.0 * math.pi / (float(d @ d) * Omega)
    assert np.allclose(r["pair_e"], e_ref, rtol=1e-12, atol=1e-15)
    for a in range(N):
        lam = sum(occ[b] * e_ref[a, b] for b in range(N))  # (K psi)_a = lam_a psi_a
        assert np.max(np.abs(r["kpsi"][a] - lam * psi[a])) < 1e-12 * abs(lam) * np.abs(psi[a]).max()
    assert r["E"] == pytest.approx(-0.5 * float(occ @ e_ref @ occ), rel=1e-13)


@pytest.mark.parametrize("ka,kb", [((0.6, 0.0, 0.0), (-0.3, 0.2, 0.0)),
                                   ((0.2, -0.5, 0.4), (0.5, 0.1, -0.3))])
def test_modulated_gaussian_pair_energies(ka, kb):
    n, h = 48, 0.4
    L = n * h
    Z, Y, X = cf.grid_coords(n, h)
    A, a = np.array([0.5 * L, 0.48 * L, 0.51 * L]), 1.5
    B, b = np.array([0.53 * L, 0.5 * L, 0.47 * L]), 1.6
    ka, kb = np.array(ka), np.array(kb)
    phase = lambda k: np.exp(1j * (k[0] * X + k[1] * Y + k[2] * Z))
    psi = np.stack([phase(ka) * cf.gaussian(n, h, A, a), phase(kb) * cf.gaussian(n, h, B, b)])
    pe = oracle.exx(psi, np.ones(2), h, FREE)["pair_e"]
    # rho_ab = conj(psi_b) psi_a = exp(i (k_a - k_b).r) g_a g_b = exp(i kappa.r) Q N(P, c)
    Q, _, c = cf.gaussian_product(A, a, B, b)
    kappa = float(np.linalg.norm(ka - kb))
    ref = cf.modulated_gaussian_self_energy(Q, c, kappa)
    assert pe[0, 1] == pytest.approx(ref, rel=1e-9)
    assert pe[1, 0] == pytest.approx(ref, rel=1e-9)
    # the unconjugated product would carry k_a + k_b instead
    wrong = cf.modulated_gaussian_self_energy(Q, c, float(np.linalg.norm(ka + kb)))
    assert abs(wrong - ref) > 1e-3 * ref
    # diagonal pairs: |psi_a|^2 carries no phase
    for k, (P, w) in enumerate([(A, a), (B, b)]):
        Qd, _, cd = cf.gaussian_product(P, w, P, w)
        assert pe[k, k] == pytest.approx(cf.self_energy_normalised(cd) * Qd * Qd, rel=1e-9)


@pytest.mark.parametrize("bc", [PERIODIC, FREE, SURFACE, WIRE])
def test_orbital_phases_reduce_to_the_real_case(bc):
    rec = OrbitalRecipe(n=16, h=0.5, n_orb=3, n_gauss=3, sigma=(0.9, 1.4), centres=CENTRES[bc],
                        bc=bc, frac_last=1, seed=23)
    s = make_system(rec)
    theta = np.array([0.3, -1.9, 2.6])
    psi_c = np.exp(1j * theta)[:, None, None, None] * s.psi
    r = oracle.exx(s.psi, s.occ, s.h, bc)
    rc = oracle.exx(psi_c, s.occ, s.h, bc)
    assert rc["E"] == pytest.approx(r["E"], rel=1e-13)
    assert np.allclose(rc["pair_e"], r["pair_e"], rtol=1e-12, atol=0)
    expect = np.exp(1j * theta)[:, None, None, None] * r["kpsi"]
    assert np.max(np.abs(rc["kpsi"] - expect)) < 1e-12 * np.abs(r["kpsi"]).max()


@pytest.mark.parametrize("bc", [PERIODIC, FREE])
def test_unitary_invariance_and_covariance(bc):
    s = _complex_system(bc, N=4, seed=25)
    r = oracle.exx(s.psi, s.occ, s.h, bc)
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    psi_u = np.einsum("ik,kzyx->izyx", U, s.psi)
    ru = oracle.exx(psi_u, s.occ, s.h, bc)  # every occupation is 2: K is invariant
    assert ru["E"] == pytest.approx(r["E"], rel=1e-12)
    expect = np.einsum("ik,kzyx->izyx", U, r["kpsi"])
    assert np.max(np.abs(ru["kpsi"] - expect)) < 1e-11 * np.abs(r["kpsi"]).max()


@pytest.mark.parametrize("bc", [PERIODIC, FREE])
def test_hermitian_pair_symmetry_and_energy_identity(bc):
    s = _complex_system(bc, N=3, seed=27, frac=1)
    V01 = oracle.solve_poisson(oracle.co_density(s.psi[0], s.psi[1]), s.h, bc)
    V10 = oracle.solve_poisson(oracle.co_density(s.psi[1], s.psi[0]), s.h, bc)
    assert np.max(np.abs(V10 - np.conj(V01))) < 1e-13 * np.abs(V01).max()
    assert np.abs(V01.imag).max() > 1e-3 * np.abs(V01).max()  # genuinely complex
    r = oracle.exx(s.psi, s.occ, s.h, bc)
    rs = oracle.exx(s.psi, s.occ, s.h, bc, symmetric=True)
    assert np.allclose(r["pair_e"], r["pair_e"].T, rtol=1e-12, atol=0)
    assert np.all(np.diag(r["pair_e"]) > 0)
    assert rs["E"] == pytest.approx(r["E"], rel=1e-13)
    assert np.max(np.abs(rs["kpsi"] - r["kpsi"])) < 1e-12 * np.abs(r["kpsi"]).max()
    # E_x = -1/2 h^3 sum_i f_i Re <psi_i, (K psi)_i>
    dots = (np.conj(s.psi).reshape(3, -1) * r["kpsi"].reshape(3, -1)).sum(axis=1)
    assert np.abs(dots.imag).max() < 1e-12 * np.abs(dots).max()
    assert r["E"] == pytest.approx(-0.5 * s.h ** 3 * float(s.occ @ dots.real), rel=1e-12)


@pytest.mark.parametrize("bc", [PERIODIC, FREE])
def test_gradient_against_richardson_differences(bc):
    s = _complex_system(bc, n=12, N=3, seed=29, frac=1)
    r = oracle.exx(s.psi, s.occ, s.h, bc)
    grad = oracle.exx_grad_psi(r["kpsi"], s.occ, s.h)
    rng = np.random.default_rng(11)
    d = rng.normal(size=s.psi.shape) + 1j * rng.normal(size=s.psi.shape)

    def E(eps):
        return oracle.exx(s.psi + eps * d, s.occ, s.h, bc, want_kpsi=False)["E"]

    def D(eps):
        return (E(eps) - E(-eps)) / (2 * eps)

    eps = 1e-3
    fd = (4.0 * D(eps / 2) - D(eps)) / 3.0  # exact for a quartic up to rounding
    # dE = sum dE/dRe Re d + dE/dIm Im d = Re sum conj(grad) d
    assert fd == pytest.approx(float(np.sum(np.conj(grad) * d).real), rel=1e-8)
    euler = float(np.sum(np.conj(grad) * s.psi).real)
    assert euler == pytest.approx(4.0 * r["E"], rel=1e-12)


@pytest.mark.parametrize("bc", [PERIODIC, FREE])
def test_fft_route_equals_brute_force_for_a_complex_density(bc):
    rng = np.random.default_rng(13)
    n, h = 4, 0.7
    rho = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    V_fft = oracle.solve_poisson(rho, h, bc)
    V_bf = oracle.brute_force_potential(rho, h, bc)
    assert np.max(np.abs(V_fft - V_bf)) <= 1e-12 * np.max(np.abs(V_bf))


def test_complex_recipe_draws_orthonormal_periodic_orbitals():
    s = _complex_system(PERIODIC, N=4, seed=31)
    assert s.psi.dtype == np.complex128
    flat = s.psi.reshape(4, -1)
    S = s.h ** 3 * (np.conj(flat) @ flat.T)
    assert np.max(np.abs(S - np.eye(4))) < 1e-12
    assert np.abs(s.psi.imag).max() > 0.1 * np.abs(s.psi).max()
    # periodic exchange is invariant under a cyclic translation of every orbital
    r1 = oracle.exx(s.psi, s.occ, s.h, PERIODIC)
    r2 = oracle.exx(np.roll(s.psi, (3, -2, 5), axis=(1, 2, 3)), s.occ, s.h, PERIODIC)
    assert r2["E"] == pytest.approx(r1["E"], rel=1e-12)
