"""Interpolating-scaling-function (ISF) Green's function of the free boundary.

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle; nothing on the product path
may import it).

The Poisson solver the paper uses (Section 2.1.2) represents a density given
on the grid by interpolating scaling functions, rho(r) = sum_j rho_j
phi(r/h - j) with phi the tensor product of a 1-D Deslauriers-Dubuc function
of order m (phi(k) = delta_k0 at integers, so rho_j are the grid values), and
returns the potential at the grid points,

    V_i = integral rho(r') / |r_i - r'| dr' = sum_j K(i - j) rho_j,
    K(d) = h^2 integral phi(u1) phi(u2) phi(u3) / |d - u| du      (d in Z^3).

The convolution with zero padding to 2n per axis is exact: the displacements
of an n^3 grid fit the doubled box without wrapping.  This module computes K
from its definition with three textbook ingredients, each pinned in
tests/test_oracle_isf.py:

* phi on the dyadic grid 2^-L Z, by interpolating subdivision: the value at
  each new midpoint is the degree m-1 Lagrange interpolant of the m nearest
  known values;
* 1/r as a sum of Gaussians, from 1/r = (2/sqrt(pi)) int exp(s - e^{2s} r^2) ds
  discretised by the trapezoid rule in s;
* the 1-D integrals I(a, x) = int phi(u) exp(-a (x - u)^2) du at integers x,
  by the trapezoid rule on phi's dyadic samples (exact up to terms in the
  m-th moment of phi once the Gaussian is wide on the sampling scale, since
  phi reproduces polynomials below degree m), and by the small-width expansion
  sqrt(pi/a) (phi(x) + phi''(x) / (4a)) for the narrowest Gaussians.

Then K(d) = h^2 sum_q w_q I(a_q, d1) I(a_q, d2) I(a_q, d3).
"""
from __future__ import annotations

import functools
import math

import numpy as np

ORDER = 16  # the order of the paper's solver family (degree-15 interpolation)


def lagrange_half_weights(order: int = ORDER) -> np.ndarray:
    """Weights L_t, t = -order/2+1 .. order/2, of the interpolant at 1/2
    through the integer nodes t (the midpoint rule of the subdivision)."""
    nodes = np.arange(-order // 2 + 1, order // 2 + 1, dtype=np.float64)
    w = np.empty(order)
    for k, t in enumerate(nodes):
        others = nodes[nodes != t]
        w[k] = np.prod((0.5 - others) / (t - others))
    return w


@functools.lru_cache(maxsize=None)
def isf_samples(levels: int, order: int = ORDER):
    """phi at x = i 2^-levels on its support [-(order-1), order-1].

    Returns (x, phi) with phi as a read-only array.
    """
    support = order - 1
    w = lagrange_half_weights(order)
    half = order // 2
    vals = np.zeros(2 * support + 1)
    vals[support] = 1.0  # phi(k) = delta_k0
    for _ in range(levels):
        npts = vals.size
        padded = np.concatenate([np.zeros(half), vals, np.zeros(half)])
        mids = np.zeros(npts - 1)
        # midpoint between vals[i] and vals[i+1]: nodes vals[i-half+1 .. i+half]
        for k in range(order):
            off = k - half + 1  # node index relative to i
            mids += w[k] * padded[half + off: half + off + npts - 1]
        out = np.empty(2 * npts - 1)
        out[0::2] = vals
        out[1::2] = mids
        vals = out
    step = 2.0 ** -levels
    x = -support + step * np.arange(vals.size)
    vals.setflags(write=False)
    return x, vals


def coulomb_gaussians(r_min: float, r_max: float, delta: float = 0.15, eps: float = 1e-16):
    """(w, a) with 1/r ~ sum_q w_q exp(-a_q r^2) for r_min <= r <= r_max.

    Trapezoid rule with step delta in s for (2/sqrt(pi)) int exp(s - e^{2s} r^2) ds;
    the range of s drops the parts of the integral below eps / r_max (wide end)
    and where e^{2s} r_min^2 > 40 (narrow end).
    """
    s_lo = math.log(eps / r_max)
    s_hi = math.log(math.sqrt(40.0) / r_min)
    s = np.arange(s_lo, s_hi + delta, delta)
    w = (2.0 / math.sqrt(math.pi)) * delta * np.exp(s)
    a = np.exp(2.0 * s)
    return w, a


def gauss_integrals(a: float, xs: np.ndarray, order: int = ORDER) -> np.ndarray:
    """I(a, x) = int phi(u) exp(-a (x - u)^2) du for the integers xs >= 0."""
    support = order - 1
    xs = np.asarray(xs, dtype=np.float64)
    # sampling level: Gaussian exponent a / 4^L <= 2.5e-4 on the sampling scale,
    # where the m-th moment term of the trapezoid error is below 1e-17
    L = max(6, math.ceil(math.log(max(a, 1e-300) / 2.5e-4, 4.0)))
    if L > 15:
        # narrow Gaussian: sqrt(pi/a) (phi(x) + phi''(x) / (4a)), phi'' from the finest samples
        xf, pf = isf_samples(15, order)
        step = xf[1] - xf[0]
        out = np.zeros(xs.size)
        for k, x in enumerate(xs):
            if x >= support:  # phi vanishes with its derivatives from the support's edge on
                continue
            i = int(round((x + support) / step))
            d2 = (pf[i + 1] - 2.0 * pf[i] + pf[i - 1]) / (step * step)
            phi_x = 1.0 if x == 0 else 0.0
            out[k] = math.sqrt(math.pi / a) * (phi_x + d2 / (4.0 * a))
        return out
    xf, pf = isf_samples(L, order)
    step = xf[1] - xf[0]
    out = np.zeros(xs.size)
    reach = math.sqrt(40.0 / a)  # exp(-a d^2) < e^-40 beyond
    for k, x in enumerate(xs):
        lo, hi = max(-support, x - reach), min(support, x + reach)
        if lo > hi:
            continue
        i0 = int(math.floor((lo + support) / step))
        i1 = int(math.ceil((hi + support) / step)) + 1
        u = xf[i0:i1]
        out[k] = step * math.fsum((pf[i0:i1] * np.exp(-a * (x - u) ** 2)).tolist())
    return out


@functools.lru_cache(maxsize=None)
def isf_kernel(n: int, h: float, order: int = ORDER) -> np.ndarray:
    """K(d) for 0 <= d1, d2, d3 <= n, shape (n+1, n+1, n+1) (even in each d)."""
    d = np.arange(n + 1, dtype=np.float64)
    # every |d - u| of the doubled box lies below sqrt(3) (n + order); r_min sets
    # the part of the 1/r singularity left out (~ 2 pi r_min^2)
    w, a = coulomb_gaussians(r_min=1e-7, r_max=math.sqrt(3.0) * (n + order))
    K = np.zeros((n + 1, n + 1, n + 1))
    for wq, aq in zip(w, a):
        g = gauss_integrals(aq, d, order)
        if not np.any(g):
            continue
        K += wq * g[:, None, None] * g[None, :, None] * g[None, None, :]
    K *= h * h
    K.setflags(write=False)
    return K


def isf_kernel_circulant(n: int, h: float, order: int = ORDER) -> np.ndarray:
    """K on the (2n)^3 padded grid: entry k holds K(d) for d = k (k <= n) or
    k - 2n (k > n), per axis; the k = n entries are never reached by data on
    [0, n)^3 and hold K(n)."""
    K = isf_kernel(n, h, order)
    idx = np.array([k if k <= n else 2 * n - k for k in range(2 * n)])
    return np.ascontiguousarray(K[np.ix_(idx, idx, idx)])
