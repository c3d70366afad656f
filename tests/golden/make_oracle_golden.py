"""Writes FP64-oracle expectations for the full-size workloads.

Calls only ``oracle`` and the seeded generator ``exx_inputs``; the stored
values are what the GPU parity tests compare against at full size, where the
oracle itself would take minutes to hours.

Per workload it stores, in ``<preset>_oracle.npz``:
  pairs       sampled (i, j) pairs and their energies e_ij = h^3 sum rho V
  kpsi_rows   orbitals whose full (K psi)_i is sampled, the sampled point
              indices (flat, x fastest) and the values there
  E           E_x when every pair is computed (small workloads only)
  pair_e      the full pair-energy matrix (small workloads only)

Usage: python tests/golden/make_oracle_golden.py [preset ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from exx_inputs import batch_recipes, make_system, recipe  # noqa: E402

PLANS = {
    # preset: (full E and pair matrix?, number of sampled pairs, K psi rows, points per row)
    "free64_n32": (True, 0, [0, 7, 31], 2048),
    "periodic96_n128": (True, 0, [3, 77], 2048),
    "free128_n256": (False, 12, [250], 2048),
    "surface64_n32": (True, 0, [0, 7, 31], 2048),
    "wire64_n32": (True, 0, [0, 7, 31], 2048),
    "free64_n32_complex": (True, 0, [0, 7, 31], 2048),
}


def sample_pairs(N: int, k: int, rng) -> list:
    pairs = {(0, 0), (0, N - 1), (N - 1, N - 1)}
    while len(pairs) < k:
        i, j = sorted(rng.integers(0, N, size=2).tolist())
        pairs.add((i, j))
    return sorted(pairs)


def run(preset: str) -> None:
    t0 = time.time()
    if preset.startswith("batch16"):
        s_idx = int(preset.split("_s")[1])
        sysm = make_system(batch_recipes()[s_idx])
        full, npairs, rows, npts = False, 4, [sysm.n_orb // 2], 1024
    else:
        sysm = make_system(recipe(preset))
        full, npairs, rows, npts = PLANS[preset]
    N, n = sysm.n_orb, sysm.n
    rng = np.random.default_rng(12345)
    out = {"n": n, "h": sysm.h, "bc": sysm.bc, "R": sysm.R, "n_orb": N}
    if full:
        r = oracle.exx(sysm.psi, sysm.occ, sysm.h, sysm.bc, R=sysm.R, symmetric=True)
        out["E"] = r["E"]
        out["pair_e"] = r["pair_e"]
        kpsi_full = r["kpsi"]
    else:
        pairs = sample_pairs(N, npairs, rng)
        out["pairs"] = np.array(pairs, dtype=np.int64)
        out["pair_energies"] = oracle.pair_energies(sysm.psi, pairs, sysm.h, sysm.bc, R=sysm.R)
        kpsi_full = None
    pts = rng.choice(n ** 3, size=npts, replace=False)
    out["kpsi_rows"] = np.array(rows, dtype=np.int64)
    out["kpsi_points"] = pts.astype(np.int64)
    if kpsi_full is not None:
        vals = kpsi_full[rows].reshape(len(rows), -1)
    else:
        vals = oracle.kpsi_rows(sysm.psi, sysm.occ, rows, sysm.h, sysm.bc, R=sysm.R).reshape(len(rows), -1)
    out["kpsi_values"] = vals[:, pts]
    out["kpsi_norms"] = np.sqrt((np.abs(vals) ** 2).sum(axis=1))
    path = os.path.join(HERE, f"{preset}_oracle.npz")
    np.savez_compressed(path, **out)
    print(f"{preset}: wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(PLANS)
    for name in names:
        run(name)
