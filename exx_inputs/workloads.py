"""The named workloads (sizes, boundary conditions, seeds).

Each preset freezes one reading of a workload description: grid, spacing,
orbital count and Gaussian recipe.  ``small`` variants keep the same recipe
on grids the FP64 oracle finishes in seconds (used by the parity tests).
"""
from __future__ import annotations

import numpy as np

from .generator import FREE, PERIODIC, SURFACE, WIRE, OrbitalRecipe, System, make_system

H = 0.4  # grid spacing in bohr for every workload


def recipe(name: str) -> OrbitalRecipe:
    """Recipe of a single-system workload by name."""
    if name == "periodic32_n8":
        # periodic box L = 12.8 bohr, 32^3 grid, 8 orbitals of 4 s-Gaussians each
        return OrbitalRecipe(n=32, h=H, n_orb=8, n_gauss=4, sigma=(0.8, 1.6),
                             centres="box", bc=PERIODIC, seed=1001)
    if name == "free64_n32":
        # isolated, 64^3 grid zero-padded to 128^3, 32 orbitals
        return OrbitalRecipe(n=64, h=H, n_orb=32, n_gauss=4, sigma=(0.6, 1.5),
                             centres="middle", bc=FREE, seed=1002)
    if name == "periodic96_n128":
        # periodic 96^3, 128 orbitals of 8 p-type Gaussians each
        return OrbitalRecipe(n=96, h=H, n_orb=128, n_gauss=8, sigma=(0.8, 1.6),
                             centres="box", bc=PERIODIC, ptype=True, seed=1003)
    if name == "surface64_n32":
        # surface: periodic in x, y (L = 25.6 bohr), isolated along z (64 -> 128
        # zero padded, interaction cut at |z - z'| = L); 32 orbitals
        return OrbitalRecipe(n=64, h=H, n_orb=32, n_gauss=4, sigma=(0.6, 1.5),
                             centres="slab", bc=SURFACE, seed=1006)
    if name == "wire64_n32":
        # wire: isolated in x, y (64 -> 128 zero padded each, interaction cut at
        # in-plane distance L), periodic along z (L = 25.6 bohr); 32 orbitals
        return OrbitalRecipe(n=64, h=H, n_orb=32, n_gauss=4, sigma=(0.6, 1.5),
                             centres="rod", bc=WIRE, seed=1007)
    if name == "free64_n32_complex":
        # free64_n32's grid and orbital count with complex orbitals: every Gaussian
        # term carries a phase exp(i k.(r - A)), |k_a| <= 1 bohr^-1, and a unit
        # complex coefficient
        return OrbitalRecipe(n=64, h=H, n_orb=32, n_gauss=4, sigma=(0.6, 1.5),
                             centres="middle", bc=FREE, seed=1008, kmax=1.0)
    if name == "free128_n256":
        # isolated, 128^3 grid zero-padded to 256^3, 256 orbitals, last 16 fractional
        return OrbitalRecipe(n=128, h=H, n_orb=256, n_gauss=4, sigma=(0.6, 1.5),
                             centres="middle", bc=FREE, frac_last=16, seed=1004)
    raise KeyError(name)


SINGLE = ("periodic32_n8", "free64_n32", "periodic96_n128", "free128_n256", "surface64_n32",
          "wire64_n32", "free64_n32_complex")
BATCH = "batch16_free"
BATCH_SMALL = "batch48_small"


def small_batch_recipes(n_systems: int = 48, seed: int = 1009):
    """Many small isolated systems: n in {32, 48}, N in [4, 16]."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_systems):
        n = int(rng.choice([32, 48]))
        N = int(rng.integers(4, 17))
        out.append(OrbitalRecipe(n=n, h=H, n_orb=N, n_gauss=4, sigma=(0.6, 1.5),
                                 centres="middle", bc=FREE, seed=1100 + s))
    return out


def batch_recipes(n_systems: int = 16, seed: int = 1005):
    """Sixteen isolated systems of uneven size: n in {48..112}, N in [16, 96]."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_systems):
        n = int(rng.choice([48, 64, 80, 96, 112]))
        N = int(rng.integers(16, 97))
        out.append(OrbitalRecipe(n=n, h=H, n_orb=N, n_gauss=4, sigma=(0.6, 1.5),
                                 centres="middle", bc=FREE, seed=1050 + s))
    return out


def scaled(rec: OrbitalRecipe, n: int | None = None, n_orb: int | None = None,
           seed: int | None = None) -> OrbitalRecipe:
    """Same recipe on another grid / orbital count (box shrinks with n at fixed h)."""
    d = dict(rec.__dict__)
    if n is not None:
        d["n"] = n
    if n_orb is not None:
        d["n_orb"] = n_orb
        d["frac_last"] = min(d["frac_last"], n_orb // 4)
    if seed is not None:
        d["seed"] = seed
    return OrbitalRecipe(**d)


def system(name: str) -> System:
    return make_system(recipe(name))


def pair_count(n_orb: int) -> int:
    """Unordered orbital pairs including i == j (Poisson solves per channel)."""
    return n_orb * (n_orb + 1) // 2
