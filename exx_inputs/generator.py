"""Seeded synthetic orbitals for the exact-exchange workloads.

This module only *draws inputs*: real or complex orbitals on a uniform cubic
grid built from random Gaussians (complex ones carry plane-wave phase
factors and complex coefficients) and then Loewdin-orthonormalised, plus
occupation numbers.  It contains none of the exchange arithmetic (no co-densities, no
Poisson kernel, no FFT) so that both the FP64 oracle and the HIP path can use
it without sharing any of the method's code.

Grid convention (shared by every consumer): point (ix, iy, iz) sits at
r = h * (ix, iy, iz) with 0 <= i < n, the box length is L = n*h, and arrays
are C-contiguous ``[N][nz][ny][nx]`` with x fastest.

The paper's own workloads (water boxes and UO2 crystals, Section 3, Table 1)
need a DFT code, pseudopotentials and structures; these Gaussian orbitals
stand in for them with the same data layout (orbitals on a uniform real-space
grid, Section 4's stand-alone interface) and a controllable extent.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PERIODIC = "periodic"
FREE = "free"
SURFACE = "surface"  # periodic in x and y, isolated along z
WIRE = "wire"  # isolated in x and y, periodic along z


@dataclass(frozen=True)
class OrbitalRecipe:
    """How to draw one system's orbitals.

    n: grid points per axis; h: spacing (bohr); n_orb: number of orbitals;
    n_gauss: Gaussians per orbital; sigma: (lo, hi) of the uniform width draw;
    centres: "box" (uniform in [0, L)^3, minimum image -- periodic systems),
    "middle" (uniform in [0.25 L, 0.75 L]^3 -- isolated systems), "slab"
    (x, y uniform in [0, L) with minimum image, z in [0.25 L, 0.75 L] --
    surface systems) or "rod" (x, y in [0.25 L, 0.75 L], z uniform in [0, L)
    with minimum image -- wire systems);
    ptype: multiply each Gaussian by a random p-type factor u.(r - A)/sigma;
    frac_last: number of trailing orbitals with occupation drawn U[0, 2];
    occ: occupation of the others;
    kmax: 0 for real orbitals; > 0 draws complex orbitals, each Gaussian term
    times a complex coefficient of unit modulus and a phase exp(i k.(r - A)),
    with k_a uniform in [-kmax, kmax] (bohr^-1) along an isolated axis and the
    nearest multiple of 2 pi / L along a periodic one (so the orbital stays
    periodic there).
    """

    n: int
    h: float
    n_orb: int
    n_gauss: int
    sigma: tuple
    centres: str
    bc: str
    ptype: bool = False
    frac_last: int = 0
    occ: float = 2.0
    seed: int = 0
    kmax: float = 0.0


def _axis_displacement(n: int, h: float, a: float, periodic: bool) -> np.ndarray:
    """Signed displacement x - a along one axis (minimum image if periodic)."""
    x = h * np.arange(n, dtype=np.float64)
    d = x - a
    if periodic:
        L = n * h
        d = d - L * np.round(d / L)
    return d


def raw_gaussian_orbitals(rec: OrbitalRecipe, rng: np.random.Generator) -> np.ndarray:
    """Non-orthogonal orbitals phi_i = sum_g c_g * [p-factor] * exp(-|r-A|^2 / 2 s^2).

    Every term is separable along x, y, z, so a term is an outer product of
    three 1-D profiles (a p-factor is a sum of three separable terms).
    """
    n, h, L = rec.n, rec.h, rec.n * rec.h
    # per axis (x, y, z): periodic placement with minimum image, or confined
    periodic = {"box": (True, True, True), "middle": (False, False, False),
                "slab": (True, True, False), "rod": (False, False, True)}[rec.centres]
    cplx = rec.kmax > 0.0
    phi = np.zeros((rec.n_orb, n, n, n), dtype=np.complex128 if cplx else np.float64)
    for i in range(rec.n_orb):
        for _ in range(rec.n_gauss):
            coef = rng.uniform(-1.0, 1.0)
            s = rng.uniform(*rec.sigma)
            A = np.array([rng.uniform(0.0, L) if periodic[k] else rng.uniform(0.25 * L, 0.75 * L)
                          for k in range(3)])
            dx, dy, dz = (_axis_displacement(n, h, A[k], periodic[k]) for k in range(3))
            gx, gy, gz = (np.exp(-d * d / (2.0 * s * s)) for d in (dx, dy, dz))
            if rec.ptype:
                u = rng.normal(size=3)
                u /= np.linalg.norm(u)
                # u.(r-A)/s * G = (ux dx gx) gy gz + gx (uy dy gy) gz + gx gy (uz dz gz)
                term = (
                    np.einsum("z,y,x->zyx", gz, gy, u[0] * dx * gx / s)
                    + np.einsum("z,y,x->zyx", gz, u[1] * dy * gy / s, gx)
                    + np.einsum("z,y,x->zyx", u[2] * dz * gz / s, gy, gx)
                )
            else:
                term = np.einsum("z,y,x->zyx", gz, gy, gx)
            if cplx:  # drawn after the real recipe's numbers, which stay unchanged
                k = rng.uniform(-rec.kmax, rec.kmax, size=3)
                for a in range(3):
                    if periodic[a]:
                        k[a] = 2.0 * np.pi / L * np.round(k[a] * L / (2.0 * np.pi))
                px, py, pz = (np.exp(1j * k[a] * d) for a, d in enumerate((dx, dy, dz)))
                term = term * np.einsum("z,y,x->zyx", pz, py, px)
                coef = coef * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi))
            phi[i] += coef * term
    return phi


def loewdin(phi: np.ndarray, h: float, min_ratio: float = 1e-6):
    """Symmetric (Loewdin) orthonormalisation on the grid: psi = S^{-1/2} phi.

    S_ij = h^3 sum_g conj(phi_i(g)) phi_j(g) (Hermitian; real for real phi), and
    psi_i = sum_k conj(S^{-1/2})_ik phi_k makes h^3 sum conj(psi_i) psi_j = delta_ij.
    Returns (psi, eigenvalue ratio of S); the ratio lets the caller redraw an
    ill-conditioned set.
    """
    N = phi.shape[0]
    flat = phi.reshape(N, -1)
    S = (h ** 3) * (np.conj(flat) @ flat.T)
    w, U = np.linalg.eigh(S)
    ratio = float(w.min() / w.max())
    if w.min() <= 0.0 or ratio < min_ratio:
        return None, ratio
    C = np.conj((U * (1.0 / np.sqrt(w))) @ np.conj(U).T)
    psi = (C @ flat).reshape(phi.shape)
    return np.ascontiguousarray(psi), ratio


def occupations(rec: OrbitalRecipe, rng: np.random.Generator) -> np.ndarray:
    f = np.full(rec.n_orb, rec.occ, dtype=np.float64)
    if rec.frac_last:
        f[rec.n_orb - rec.frac_last:] = rng.uniform(0.0, 2.0, size=rec.frac_last)
    return f


def draw_system(rec: OrbitalRecipe, max_tries: int = 20):
    """Draw (psi, occ) for one system; redraws while S is ill-conditioned."""
    rng = np.random.default_rng(rec.seed)
    for _ in range(max_tries):
        phi = raw_gaussian_orbitals(rec, rng)
        psi, _ratio = loewdin(phi, rec.h)
        if psi is not None:
            return psi, occupations(rec, rng)
    raise RuntimeError(f"could not draw a well-conditioned orbital set for seed {rec.seed}")


@dataclass
class System:
    """One drawn system: orbitals psi [N][n][n][n] (FP64, complex128 when the
    recipe's kmax > 0) and occupations [N]."""

    recipe: OrbitalRecipe
    psi: np.ndarray
    occ: np.ndarray
    R: float = field(default=0.0)

    @property
    def n(self) -> int:
        return self.recipe.n

    @property
    def h(self) -> float:
        return self.recipe.h

    @property
    def bc(self) -> str:
        return self.recipe.bc

    @property
    def n_orb(self) -> int:
        return self.recipe.n_orb


def make_system(rec: OrbitalRecipe, R: float | None = None) -> System:
    psi, occ = draw_system(rec)
    if R is None:
        R = rec.n * rec.h if rec.bc in (FREE, SURFACE, WIRE) else 0.0
    return System(rec, psi, occ, float(R))
