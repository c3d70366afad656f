"""Plain FP64 CPU oracle for the exact-exchange operator.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call
this module; it is used by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  It shares no code with the HIP library: it
works from the paper's definitions with NumPy/SciPy primitives, one pair at a
time, with no packing, pruning, tiling or batching.

What it computes (Ratcliff et al., arXiv:1712.07973, Section 2):

* co-density of a pair, rho_ij(r) = psi_j*(r) psi_i(r) (Eq. 2; Eq. 8 writes the
  real-orbital case psi_i psi_j); real and complex orbitals are accepted;
* pair potential V_ij, the solution of lap V = -4 pi rho_ij (Eq. 4),
  obtained by a discrete convolution with a Green's kernel evaluated through
  FFTs with zero padding for isolated systems (Section 2.1.2);
* E_x = -1/2 sum_{i,j} f_i f_j  integral rho_ij* V_ij  (Eqs. 2 and 5, one spin
  channel; real for any orbitals since V_ij = K * rho_ij with a real even K);
* the Fock action, (K psi)_i = sum_j f_j V_ij psi_j, which is minus the
  operator D_X of Eq. 3; V_ji = conj(V_ij).

Discrete readings (the paper gives none of these; each is listed in the
design notes):

* grid point g = (ix, iy, iz) at r = h*g, 0 <= i < n, box L = n h, the
  integral is h^3 times the grid sum;
* periodic: FFT grid m = n, kernel 4 pi / |G|^2 with the G = 0 term dropped;
* free: FFT grid m = 2n with the density in the first octant and zeros
  elsewhere, the truncated Coulomb kernel 4 pi (1 - cos |G| R) / |G|^2 written
  as 8 pi sin^2(|G| R / 2) / |G|^2, its G = 0 limit 2 pi R^2 kept, and the
  potential cropped back to [0, n)^3; R defaults to L (the largest radius
  that the doubled box keeps free of images);
* surface (periodic in x and y, isolated along z, one of the mixed boundary
  conditions of Section 2.1.2): FFT grid n x n x 2n, zero padding along z
  only, and the Coulomb interaction cut at |z - z'| = R (default L):
  for G_par > 0
      4 pi / G^2 [1 + exp(-G_par R) (G_z / G_par sin(G_z R) - cos(G_z R))],
  for G_par = 0 the finite part, the transform of -2 pi |z| on |z| < R,
      4 pi / G_z^2 [1 - cos(G_z R) - G_z R sin(G_z R)],   -2 pi R^2 at G = 0
  (the in-plane integral of 1/r diverges at G_par = 0; dropping its constant
  is the usual convention for a 2-D periodic array of charges);
* wire (isolated in x and y, periodic along z): FFT grid 2n x 2n x n, zero
  padding in x and y, the Coulomb interaction cut at the in-plane distance
  rho = R (default L): with G_perp the in-plane and G_z the axial wave vector,
      4 pi / G^2 [1 + R (G_perp J1(G_perp R) K0(|G_z| R) - |G_z| J0(G_perp R) K1(|G_z| R))]
  for G_z != 0; for G_z = 0 the transform of the 2-D potential -2 ln(rho) on
  rho < R (rho in bohr), 4 pi / G_perp^2 [1 - J0(G_perp R) - G_perp R J1(G_perp R) ln R],
  and pi R^2 (1 - 2 ln R) at G = 0;
* G = 2 pi k / (m h) with k folded to the symmetric range (k > m/2 -> k - m);
* kernel="isf" (free boundary): the Green's function of the paper's own
  Poisson solver, the exact Coulomb potential at the grid points of the
  density interpolated by order-16 scaling functions (oracle/isf.py), applied
  as a convolution on the same doubled grid (no radius: the doubled box holds
  every displacement).

Parity pins: see tests/test_oracle_*.py (closed forms for plane waves and
Gaussians, brute-force sums on tiny grids, invariants, finite differences).
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

PERIODIC = "periodic"
FREE = "free"
SURFACE = "surface"  # periodic x, y; isolated z
WIRE = "wire"  # isolated x, y; periodic z
SCREENED = "screened"  # periodic-style erfc(omega r)/r kernel (screened hybrids)

_WORKERS = int(os.environ.get("EXX_ORACLE_WORKERS", "0")) or (os.cpu_count() or 1)


def fft_size(n: int, bc: str) -> int:
    """FFT grid points per axis: n for periodic, 2n (zero padded) for free."""
    if bc in (SURFACE, WIRE):
        raise ValueError("the mixed-boundary grids are not cubic: use fft_shape")
    return 2 * n if bc == FREE else n


def fft_shape(n: int, bc: str) -> tuple:
    """FFT grid in array order (z, y, x): padded axes have 2n points."""
    if bc == FREE:
        return (2 * n, 2 * n, 2 * n)
    if bc == SURFACE:
        return (2 * n, n, n)
    if bc == WIRE:
        return (n, 2 * n, 2 * n)
    return (n, n, n)


def default_radius(n: int, h: float) -> float:
    """Truncation radius of the free-boundary kernel: the box length L = n h."""
    return n * h


def wavevector_components(shape: tuple, h: float):
    """G_z, G_y, G_x (broadcastable) on an FFT grid of the given (z, y, x) shape."""
    out = []
    for a, m in enumerate(shape):
        k = np.fft.fftfreq(m, d=1.0 / m)  # 0, 1, .., m/2-1, -m/2, .., -1  (integers)
        g = 2.0 * math.pi * k / (m * h)
        sh = [1, 1, 1]
        sh[a] = m
        out.append(g.reshape(sh))
    return out


def wavevector_sq(m: int, h: float) -> np.ndarray:
    """|G|^2 on the m^3 FFT grid, array index order [kz][ky][kx]."""
    gz, gy, gx = wavevector_components((m, m, m), h)
    return gz * gz + gy * gy + gx * gx


def surface_kernel(n: int, h: float, R: float | None = None) -> np.ndarray:
    """Coulomb kernel cut at |z - z'| = R, periodic in x and y (n x n x 2n grid)."""
    if R is None or R <= 0.0:
        R = default_radius(n, h)
    gz, gy, gx = wavevector_components(fft_shape(n, SURFACE), h)
    gp = np.sqrt(gx * gx + gy * gy) + 0.0 * gz  # in-plane |G|, full shape
    gzf = gz + 0.0 * gp
    G2 = gp * gp + gzf * gzf
    out = np.empty_like(G2)
    par = gp > 0.0
    cz, sz = np.cos(gzf * R), np.sin(gzf * R)
    out[par] = (4.0 * math.pi / G2[par]) * (
        1.0 + np.exp(-gp[par] * R) * (gzf[par] / gp[par] * sz[par] - cz[par]))
    line = (~par) & (gzf != 0.0)
    out[line] = (4.0 * math.pi / G2[line]) * (1.0 - cz[line] - gzf[line] * R * sz[line])
    out[(~par) & (gzf == 0.0)] = -2.0 * math.pi * R * R
    return out


def wire_kernel(n: int, h: float, R: float | None = None) -> np.ndarray:
    """Coulomb kernel cut at in-plane distance R, periodic along z (2n x 2n x n grid)."""
    from scipy import special
    if R is None or R <= 0.0:
        R = default_radius(n, h)
    gz, gy, gx = wavevector_components(fft_shape(n, WIRE), h)
    gp = np.sqrt(gx * gx + gy * gy) + 0.0 * gz  # in-plane |G|, full shape
    az = np.abs(gz) + 0.0 * gp
    G2 = gp * gp + az * az
    out = np.empty_like(G2)
    ax = az > 0.0
    out[ax] = (4.0 * math.pi / G2[ax]) * (
        1.0 + R * (gp[ax] * special.j1(gp[ax] * R) * special.k0(az[ax] * R)
                   - az[ax] * special.j0(gp[ax] * R) * special.k1(az[ax] * R)))
    plane = (~ax) & (gp > 0.0)
    x = gp[plane] * R
    out[plane] = (4.0 * math.pi / G2[plane]) * (1.0 - special.j0(x) - x * special.j1(x) * math.log(R))
    out[(~ax) & (gp == 0.0)] = math.pi * R * R * (1.0 - 2.0 * math.log(R))
    return out


def kernel_hat(n: int, h: float, bc: str, R: float | None = None,
               omega: float = 0.0, kernel: str = "coulomb") -> np.ndarray:
    """Fourier-space Green's kernel on the FFT grid (real, even in G)."""
    if kernel == "isf":
        if bc != FREE:
            raise ValueError("the ISF kernel is built for the free boundary")
        from .isf import isf_kernel_circulant
        khat = sfft.fftn(isf_kernel_circulant(n, h), workers=_WORKERS)
        return np.ascontiguousarray(khat.real)  # even in every axis: real up to rounding
    if kernel != "coulomb":
        raise ValueError(kernel)
    if bc == SURFACE:
        return surface_kernel(n, h, R)
    if bc == WIRE:
        return wire_kernel(n, h, R)
    m = fft_size(n, bc)
    G2 = wavevector_sq(m, h)
    out = np.zeros_like(G2)
    nz = G2 > 0.0
    if bc == PERIODIC:
        if omega > 0.0:
            # Fourier transform of erfc(omega r)/r: 4 pi (1 - exp(-G^2 / 4 omega^2)) / G^2
            out[nz] = 4.0 * math.pi * (-np.expm1(-G2[nz] / (4.0 * omega * omega))) / G2[nz]
            out[~nz] = math.pi / (omega * omega)
        else:
            out[nz] = 4.0 * math.pi / G2[nz]
            out[~nz] = 0.0
    elif bc == FREE:
        if R is None or R <= 0.0:
            R = default_radius(n, h)
        G = np.sqrt(G2[nz])
        s = np.sin(0.5 * G * R)
        out[nz] = 8.0 * math.pi * s * s / G2[nz]
        out[~nz] = 2.0 * math.pi * R * R
    else:
        raise ValueError(bc)
    return out


def embed(rho: np.ndarray, m) -> np.ndarray:
    """Place an n^3 array at the origin corner of a zero array of shape m
    (an int for a cube, or a (z, y, x) shape)."""
    n = rho.shape[0]
    shape = (m, m, m) if np.isscalar(m) else tuple(m)
    if shape == rho.shape:
        return rho
    out = np.zeros(shape, dtype=rho.dtype)
    out[:n, :n, :n] = rho
    return out


def solve_poisson(rho: np.ndarray, h: float, bc: str, R: float | None = None,
                  omega: float = 0.0, khat: np.ndarray | None = None,
                  kernel: str = "coulomb") -> np.ndarray:
    """V with lap V = -4 pi rho (Eq. 4) by FFT convolution with the kernel.

    V = crop( IFFT( K^ . FFT( embed(rho) ) ) ); V is real for a real rho.
    """
    n = rho.shape[0]
    shape = fft_shape(n, bc)
    if khat is None:
        khat = kernel_hat(n, h, bc, R, omega, kernel)
    F = sfft.fftn(embed(rho, shape), workers=_WORKERS)
    V = sfft.ifftn(khat * F, workers=_WORKERS)
    V = V[:n, :n, :n]
    return np.ascontiguousarray(V if np.iscomplexobj(rho) else V.real)


def co_density(psi_i: np.ndarray, psi_j: np.ndarray) -> np.ndarray:
    """rho_ij = conj(psi_j) psi_i (Eq. 2); psi_i psi_j (Eq. 8) for real orbitals."""
    return np.conj(psi_j) * psi_i if np.iscomplexobj(psi_j) else psi_i * psi_j


def pair_energy(rho: np.ndarray, V: np.ndarray, h: float) -> float:
    """integral conj(rho) V ~ h^3 sum_g Re(conj(rho(g)) V(g)), summed with math.fsum."""
    prod = (np.conj(rho) * V).real if np.iscomplexobj(rho) or np.iscomplexobj(V) else rho * V
    return (h ** 3) * math.fsum(prod.ravel().tolist())


def exx(psi: np.ndarray, occ: np.ndarray, h: float, bc: str, R: float | None = None,
        omega: float = 0.0, symmetric: bool = False, want_kpsi: bool = True,
        kernel: str = "coulomb"):
    """E_x, K psi and the pair-energy matrix e_ij = integral rho_ij V_ij.

    Default: a plain double loop over *ordered* pairs (i, j), one Poisson
    solve each (so the oracle does not rely on V_ij = V_ji).  With
    ``symmetric=True`` only i <= j is solved and mirrored, halving the work
    for large inputs; the symmetry itself is pinned separately.
    """
    N = psi.shape[0]
    khat = kernel_hat(psi.shape[1], h, bc, R, omega, kernel)
    e = np.zeros((N, N))
    kpsi = np.zeros_like(psi) if want_kpsi else None
    for i in range(N):
        for j in range(N):
            if symmetric and j < i:
                continue
            rho = co_density(psi[i], psi[j])
            V = solve_poisson(rho, h, bc, khat=khat)
            e[i, j] = pair_energy(rho, V, h)
            if symmetric:
                e[j, i] = e[i, j]
            if want_kpsi:
                kpsi[i] += occ[j] * V * psi[j]
                if symmetric and j != i:
                    kpsi[j] += occ[i] * np.conj(V) * psi[i]  # V_ji = conj(V_ij)
    E = -0.5 * math.fsum((occ[:, None] * occ[None, :] * e).ravel().tolist())
    return {"E": E, "kpsi": kpsi, "pair_e": e}


def exx_grad_psi(kpsi: np.ndarray, occ: np.ndarray, h: float) -> np.ndarray:
    """dE_x / dpsi_k(g) = -2 f_k h^3 (K psi)_k(g) for the grid function (for complex
    orbitals the gradient with respect to (Re psi, Im psi) read as one complex number)."""
    return -2.0 * (h ** 3) * occ[:, None, None, None] * kpsi


def exx_grad_occ(pair_e: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """dE_x / df_k = -sum_j f_j e_kj."""
    return -(pair_e @ occ)


def pair_energies(psi: np.ndarray, pairs, h: float, bc: str, R: float | None = None,
                  omega: float = 0.0, kernel: str = "coulomb") -> np.ndarray:
    """e_ij for a list of (i, j) pairs only (sampled checks on large inputs)."""
    khat = kernel_hat(psi.shape[1], h, bc, R, omega, kernel)
    out = []
    for i, j in pairs:
        rho = co_density(psi[i], psi[j])
        out.append(pair_energy(rho, solve_poisson(rho, h, bc, khat=khat), h))
    return np.asarray(out)


def kpsi_rows(psi: np.ndarray, occ: np.ndarray, rows, h: float, bc: str,
              R: float | None = None, omega: float = 0.0, kernel: str = "coulomb") -> np.ndarray:
    """(K psi)_i for the listed orbitals only (N solves per orbital)."""
    khat = kernel_hat(psi.shape[1], h, bc, R, omega, kernel)
    out = np.zeros((len(rows),) + psi.shape[1:], dtype=psi.dtype)
    for r, i in enumerate(rows):
        for j in range(psi.shape[0]):
            V = solve_poisson(co_density(psi[i], psi[j]), h, bc, khat=khat)
            out[r] += occ[j] * V * psi[j]
    return out


# ---------------------------------------------------------------------------
# Tiny-grid brute force: no FFT library at all.
# ---------------------------------------------------------------------------

def realspace_kernel(n: int, h: float, bc: str, R: float | None = None,
                     omega: float = 0.0, kernel: str = "coulomb") -> np.ndarray:
    """K(d) on the m^3 grid of displacements by an explicit inverse DFT sum.

    K(d) = (1/m^3) sum_k K^(k) exp(+2 pi i k.d / m), evaluated with dense
    exponential matrices (O(m^4)), so that only the kernel formula is shared
    with the FFT route.  The ISF kernel is defined in real space: its
    displacement table itself.
    """
    if kernel == "isf":
        from .isf import isf_kernel_circulant
        return isf_kernel_circulant(n, h)
    mz, my, mx = fft_shape(n, bc)
    khat = kernel_hat(n, h, bc, R, omega)
    E = [np.exp(2j * math.pi * np.outer(np.arange(m), np.arange(m)) / m) for m in (mz, my, mx)]
    K = np.einsum("ak,bl,cq,klq->abc", E[0], E[1], E[2], khat, optimize=True) / (mz * my * mx)
    return K.real


def brute_force_potential(rho: np.ndarray, h: float, bc: str, R: float | None = None,
                          omega: float = 0.0, kernel: str = "coulomb") -> np.ndarray:
    """V(g) = sum_{g'} rho(g') K((g - g') mod m), an explicit O(n^3 m^3) sum
    (m per axis)."""
    n = rho.shape[0]
    mz, my, mx = fft_shape(n, bc)
    K = realspace_kernel(n, h, bc, R, omega, kernel)
    V = np.zeros((n, n, n), dtype=np.result_type(rho.dtype, K.dtype))
    src = np.argwhere(np.ones((n, n, n), dtype=bool))
    for (a, b, c) in src:
        w = rho[a, b, c]
        if w == 0.0:
            continue
        za = (np.arange(n) - a) % mz
        yb = (np.arange(n) - b) % my
        xc = (np.arange(n) - c) % mx
        V += w * K[np.ix_(za, yb, xc)]
    return V
