"""Shared helpers of the GPU parity tests (inputs, oracle runs, tolerances)."""
from __future__ import annotations

import functools
import math
import sys

import numpy as np

import oracle
from exx_inputs import OrbitalRecipe, make_system

# FP64 paths must reproduce the oracle up to rounding order.
TOL_FP64_E = 1e-12   # |dE| / |E|
TOL_FP64_K = 1e-11   # max_i ||dKpsi_i|| / ||Kpsi_i||
# FP32 transforms with FP64 accumulation.
TOL_FP32_E_PER_ORB = 1e-6  # |dE| / N in Hartree
TOL_FP32_K = 1e-5          # max_i ||dKpsi_i|| / ||Kpsi_i||


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def small_system(bc: str, n: int, N: int, seed: int, frac: int = 0, ptype: bool = False,
                 h: float = 0.4, kmax: float = 0.0):
    rec = OrbitalRecipe(n=n, h=h, n_orb=N, n_gauss=3,
                        sigma=(0.8, 1.6) if bc == "periodic" else (0.6, 1.5),
                        centres={"periodic": "box", "free": "middle", "surface": "slab",
                                 "wire": "rod"}[bc],
                        bc=bc, ptype=ptype, frac_last=frac, seed=seed, kmax=kmax)
    return make_system(rec)


@functools.lru_cache(maxsize=None)
@functools.lru_cache(maxsize=4)
def oracle_result(bc: str, n: int, N: int, seed: int, frac: int = 0, ptype: bool = False,
                  kmax: float = 0.0):
    s = small_system(bc, n, N, seed, frac, ptype, kmax=kmax)
    r = oracle.exx(s.psi, s.occ, s.h, bc, symmetric=True)
    return s, r


def kpsi_rel_err(a: np.ndarray, b: np.ndarray) -> float:
    N = a.shape[0]
    num = np.sqrt((np.abs(a - b).reshape(N, -1) ** 2).sum(1))
    den = np.sqrt((np.abs(b).reshape(N, -1) ** 2).sum(1))
    return float(np.max(num / np.maximum(den, 1e-300)))


def grid_of(s):
    import paper_1712_07973_amd as exx
    return exx.Grid(n=s.n, h=s.h, bc=s.bc, R=s.R if s.bc != "periodic" else None)


def kpsi_max_err(a: np.ndarray, b: np.ndarray) -> float:
    """max_i max_r |a_i - b_i| / max_r |b_i|: element-wise, per orbital."""
    N = a.shape[0]
    num = np.abs(a - b).reshape(N, -1).max(1)
    den = np.abs(b).reshape(N, -1).max(1)
    return float(np.max(num / np.maximum(den, 1e-300)))
