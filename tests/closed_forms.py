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
