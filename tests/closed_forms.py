"""Analytic results used to pin the FP64 oracle (no code shared with it).

All Gaussians are unnormalised, g(r) = exp(-|r - A|^2 / (2 a^2)), unless a
function says "normalised"; N(r; P, c) = (2 pi c^2)^{-3/2} exp(-|r-P|^2/(2c^2)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def grid_coords(n: int, h: float):
    """(z, y, x) coordinate arrays of the grid r = h * (ix, iy, iz)."""
    x = h * np.arange(n, dtype=np.float64)
    return np.meshgrid(x, x, x, indexing="ij")  # Z, Y, X


def gaussian(n: int, h: float, A, a: float) -> np.ndarray:
    Z, Y, X = grid_coords(n, h)
    r2 = (X - A[0]) ** 2 + (Y - A[1]) ** 2 + (Z - A[2]) ** 2
    return np.exp(-r2 / (2.0 * a * a))


def normalised_gaussian(n: int, h: float, P, c: float) -> np.ndarray:
    return gaussian(n, h, P, c) / (2.0 * math.pi * c * c) ** 1.5


def gaussian_potential(n: int, h: float, P, c: float, Q: float = 1.0) -> np.ndarray:
    """Free-space potential of Q N(P, c): Q erf(r / (c sqrt 2)) / r (limit at r = 0)."""
    Z, Y, X = grid_coords(n, h)
    r = np.sqrt((X - P[0]) ** 2 + (Y - P[1]) ** 2 + (Z - P[2]) ** 2)
    out = np.empty_like(r)
    small = r < 1e-12
    out[~small] = Q * erf(r[~small] / (c * math.sqrt(2.0))) / r[~small]
    out[small] = Q * math.sqrt(2.0 / math.pi) / c
    return out


def gaussian_product(A, a, B, b):
    """g_A,a * g_B,b = Q N(P, c): returns (Q, P, c)."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    s = a * a + b * b
    c2 = a * a * b * b / s
    P = (b * b * A + a * a * B) / s
    d2 = float(np.sum((A - B) ** 2))
    Q = (2.0 * math.pi * c2) ** 1.5 * math.exp(-d2 / (2.0 * s))
    return Q, P, math.sqrt(c2)


def coulomb_two_gaussians(Q1, P1, c1, Q2, P2, c2) -> float:
    """Free-space  int int Q1 N(P1,c1)(r) Q2 N(P2,c2)(r') / |r - r'|."""
    d = float(np.linalg.norm(np.asarray(P1, float) - np.asarray(P2, float)))
    s = math.sqrt(2.0 * (c1 * c1 + c2 * c2))
    if d < 1e-14:
        return Q1 * Q2 * 2.0 / (math.sqrt(math.pi) * s)
    return Q1 * Q2 * math.erf(d / s) / d


def self_energy_normalised(c: float) -> float:
    """int int N(c) N(c) / |r - r'| = 1 / (c sqrt(pi))."""
    return 1.0 / (c * math.sqrt(math.pi))


def four_index(gauss):
    """(kl|mn) for s-Gaussians gauss = [(A, a), ...] via products of pairs."""
    M = len(gauss)
    prod = {}
    for k in range(M):
        for l in range(M):
            prod[k, l] = gaussian_product(gauss[k][0], gauss[k][1], gauss[l][0], gauss[l][1])
    T = np.zeros((M, M, M, M))
    for k in range(M):
        for l in range(M):
            Qa, Pa, ca = prod[k, l]
            for m_ in range(M):
                for n_ in range(M):
                    Qb, Pb, cb = prod[m_, n_]
                    T[k, l, m_, n_] = coulomb_two_gaussians(Qa, Pa, ca, Qb, Pb, cb)
    return T


def periodic_gaussian_pair_energy(Q: float, c: float, L: float, kmax: int) -> float:
    """Periodic (G = 0 dropped) self-energy of a periodised Q N(c) in a cube L.

    e = (4 pi / Omega) sum_{G != 0} |rho^(G)|^2 / G^2 with
    rho^(G) = Q exp(-G^2 c^2 / 2) (continuous transform of the periodised
    Gaussian); the centre drops out of |rho^|^2.
    """
    k = np.arange(-kmax, kmax + 1)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    G2 = (2.0 * math.pi / L) ** 2 * (KX ** 2 + KY ** 2 + KZ ** 2).astype(np.float64)
    nz = G2 > 0
    terms = (Q * Q) * np.exp(-G2[nz] * c * c) / G2[nz]
    return 4.0 * math.pi / L ** 3 * math.fsum(np.sort(terms).tolist())


def screened_self_energy_normalised(c: float, omega: float) -> float:
    """int int N(c) N(c) erfc(omega |r - r'|) / |r - r'| in free space.

    erf(omega r)/r is the Coulomb potential of a Gaussian of variance
    1/(2 omega^2), so the erf part is the Coulomb self energy of width
    sqrt(2 c^2 + 1/(2 omega^2)) per axis for the difference coordinate.
    """
    return 2.0 / math.sqrt(math.pi) * (1.0 / math.sqrt(4.0 * c * c)
                                       - 1.0 / math.sqrt(4.0 * c * c + 1.0 / (omega * omega)))


def periodic_screened_pair_energy(Q: float, c: float, L: float, omega: float, kmax: int) -> float:
    """(1/Omega) sum_G K_omega(G) |rho^(G)|^2 with K_omega = 4 pi (1 - e^{-G^2/4w^2}) / G^2, K(0) = pi/w^2."""
    k = np.arange(-kmax, kmax + 1)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    G2 = (2.0 * math.pi / L) ** 2 * (KX ** 2 + KY ** 2 + KZ ** 2).astype(np.float64)
    nz = G2 > 0
    terms = (Q * Q) * np.exp(-G2[nz] * c * c) * 4.0 * math.pi * (-np.expm1(-G2[nz] / (4 * omega ** 2))) / G2[nz]
    total = math.fsum(np.sort(terms).tolist()) + Q * Q * math.pi / omega ** 2
    return total / L ** 3


def _slab_mean_exp(G: np.ndarray, d: float, s: float) -> np.ndarray:
    """E[exp(-G |u|)] for u ~ N(d, s^2), G > 0 (two erfc terms, scaled to avoid overflow)."""
    from scipy.special import erfcx
    # 1/2 e^{G^2 s^2/2} [e^{-G d} erfc((G s^2 - d)/(s sqrt2)) + e^{G d} erfc((G s^2 + d)/(s sqrt2))]
    # with erfc(x) = erfcx(x) e^{-x^2}: each term becomes erfcx(.) e^{-d^2 / (2 s^2)}
    a = (G * s * s - d) / (s * math.sqrt(2.0))
    b = (G * s * s + d) / (s * math.sqrt(2.0))
    g = math.exp(-d * d / (2.0 * s * s))
    ta = np.where(a > 0, erfcx(np.maximum(a, 0)) * g,
                  np.exp(G * G * s * s / 2.0 - G * d) * (2.0 - erfcx(np.maximum(-a, 0)) * np.exp(-a * a)))
    tb = np.where(b > 0, erfcx(np.maximum(b, 0)) * g,
                  np.exp(G * G * s * s / 2.0 + G * d) * (2.0 - erfcx(np.maximum(-b, 0)) * np.exp(-b * b)))
    return 0.5 * (ta + tb)


def slab_gaussian_interaction(Q1, P1, c1, Q2, P2, c2, L: float, kmax: int) -> float:
    """int int Q1 N(P1,c1)(r) Q2 N(P2,c2)(r') v(r - r') for a square cell L x L
    periodic in x and y and no images along z, v = 1/|r| with the in-plane
    G = 0 term taken as the transform of -2 pi |z - z'| (charged-sheet
    convention).  Lattice sum over in-plane G = 2 pi (kx, ky) / L, |k| <= kmax:

      (2 pi Q1 Q2 / A) [ sum_{G != 0} e^{-G^2 s^2 / 2} cos(G . D) E[e^{-G|u|}] / G - E|u| ]

    with u = z - z' ~ N(d, s^2), s^2 = c1^2 + c2^2, d = P1z - P2z, D the
    in-plane offset of the centres.
    """
    P1 = np.asarray(P1, float)
    P2 = np.asarray(P2, float)
    s = math.sqrt(c1 * c1 + c2 * c2)
    d = float(P1[2] - P2[2])
    Dx, Dy = float(P1[0] - P2[0]), float(P1[1] - P2[1])
    k = np.arange(-kmax, kmax + 1)
    KX, KY = np.meshgrid(k, k, indexing="ij")
    gx = 2.0 * math.pi * KX / L
    gy = 2.0 * math.pi * KY / L
    G = np.sqrt(gx * gx + gy * gy)
    nz = G > 0
    Gn = G[nz]
    terms = (np.exp(-Gn * Gn * s * s / 2.0) * np.cos(gx[nz] * Dx + gy[nz] * Dy)
             * _slab_mean_exp(Gn, d, s) / Gn)
    mean_abs = s * math.sqrt(2.0 / math.pi) * math.exp(-d * d / (2.0 * s * s)) + d * math.erf(d / (s * math.sqrt(2.0)))
    total = math.fsum(np.sort(terms).tolist()) - mean_abs
    return 2.0 * math.pi * Q1 * Q2 / (L * L) * total


def slab_gaussian_self_energy(Q: float, c: float, L: float, kmax: int) -> float:
    """The d = 0, same-Gaussian case: (2 pi Q^2 / A)[sum_{G != 0} erfc(G c) / G - 2 c / sqrt(pi)]."""
    from scipy.special import erfc as _erfc
    k = np.arange(-kmax, kmax + 1)
    KX, KY = np.meshgrid(k, k, indexing="ij")
    G = 2.0 * math.pi * np.sqrt(KX * KX + KY * KY).astype(np.float64) / L
    Gn = G[G > 0]
    total = math.fsum(np.sort(_erfc(Gn * c) / Gn).tolist()) - 2.0 * c / math.sqrt(math.pi)
    return 2.0 * math.pi * Q * Q / (L * L) * total


def _rice_mean(g, D: float, s: float) -> float:
    """E[g(r)] for r = |D + u|, u a 2-D Gaussian of variance s^2 per axis (Rice law),
    by adaptive quadrature of the Rice density (i0e keeps it finite)."""
    from scipy import integrate
    from scipy.special import i0e

    def pdf(r):
        return (r / (s * s)) * math.exp(-(r - D) ** 2 / (2.0 * s * s)) * i0e(r * D / (s * s))

    hi = D + 12.0 * s
    pts = [D] if D > 0 else None
    val, _ = integrate.quad(lambda r: g(r) * pdf(r), 0.0, hi, points=pts, limit=400,
                            epsabs=1e-14, epsrel=1e-12)
    return val


def wire_gaussian_interaction(Q1, P1, c1, Q2, P2, c2, L: float, kmax: int) -> float:
    """int int Q1 N(P1,c1)(r) Q2 N(P2,c2)(r') v(r - r') for densities isolated in x, y
    and periodic along z with period L, v = 1/|r| with the axial G = 0 term taken
    as the 2-D potential -2 ln(rho) (rho in bohr).  Lattice sum over
    G_z = 2 pi k / L, |k| <= kmax, with the in-plane average over the Rice law of
    rho = |D + u| done by quadrature:

      (Q1 Q2 / L) sum_{G_z} e^{-G_z^2 s^2 / 2} cos(G_z dz) E[k_{G_z}(rho)],
      k_{G_z}(rho) = 2 K0(|G_z| rho) (G_z != 0),  -2 ln rho (G_z = 0),

    s^2 = c1^2 + c2^2, dz and D the axial and in-plane offsets of the centres.
    """
    from scipy.special import k0
    P1 = np.asarray(P1, float)
    P2 = np.asarray(P2, float)
    s = math.sqrt(c1 * c1 + c2 * c2)
    dz = float(P1[2] - P2[2])
    D = float(math.hypot(P1[0] - P2[0], P1[1] - P2[1]))
    terms = [-2.0 * _rice_mean(lambda r: math.log(r) if r > 0 else 0.0, D, s)]
    for k in range(1, kmax + 1):
        G = 2.0 * math.pi * k / L
        w = math.exp(-G * G * s * s / 2.0)
        if w < 1e-30:
            break
        terms.append(2.0 * w * math.cos(G * dz) * _rice_mean(lambda r, G=G: 2.0 * k0(G * r), D, s))
    return Q1 * Q2 / L * math.fsum(terms)


def modulated_gaussian_self_energy(Q: float, c: float, kappa: float) -> float:
    """Free-space  int int conj(rho(r)) rho(r') / |r - r'|  for the complex
    density rho = exp(i kappa.r) Q N(P, c).

    In Fourier space |rho^(q)|^2 = Q^2 exp(-c^2 |q - kappa|^2), so the energy
    is Q^2 / (2 pi^2) int exp(-c^2 |q - kappa|^2) / q^2 d^3q; the angular
    integral leaves (2 pi / (c^2 kappa)) int_0^inf exp(-c^2 (q^2 + kappa^2))
    sinh(2 c^2 q kappa) / q dq, which is sqrt(pi) D(c kappa) with D Dawson's
    integral.  Result: Q^2 D(c kappa) / (sqrt(pi) c^2 kappa), tending to
    Q^2 / (c sqrt(pi)) as kappa -> 0.
    """
    from scipy.special import dawsn

    if kappa < 1e-12:
        return Q * Q / (c * math.sqrt(math.pi))
    return Q * Q * float(dawsn(c * kappa)) / (math.sqrt(math.pi) * c * c * kappa)
