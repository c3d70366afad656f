"""GPU parity of the y/z pass forms and of the degenerate cases, element by element.

* both forms of the y/z pass (workgroup-shared and wave-local) on every
  boundary, on grids up to n = 128 (radices 2, 3, 5, 7), against the oracle:
  E_x, the pair-energy matrix and every K psi value (max over the grid of
  |dK psi_i| against max |K psi_i|, so a wrong value on the box edge, where the
  orbitals are small, cannot hide in a norm), in both energy modes;
* one orbital: E_x = -1/2 f^2 e_11, i.e. minus the Hartree energy of rho = psi^2
  for f = 1 (the self-interaction the exchange cancels, Section 2), and a single
  diagonal slot in the schedule;
* an orbital with zero occupation (it still receives K psi, contributes none);
* batches of real-orbital systems against the oracle, not only against
  single-system calls;
* a negative occupation in the energy-only mode (signed weights kept);
* both thread splits of pass C from n = 96 on (tile 4: one thread per row
  segment; tile 8: two, unevenly at n = 112).
"""
import numpy as np
import pytest
import torch

from gpu_common import (TOL_FP32_E_PER_ORB, TOL_FP32_K, TOL_FP64_E, TOL_FP64_K, grid_of,
                        kpsi_max_err, kpsi_rel_err, oracle_result, say, small_system)

import oracle

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")

DEV = torch.device("cuda", 0)

FORM_CASES = [
    # (bc, n, N, seed)
    ("free", 16, 3, 51), ("free", 32, 4, 52), ("free", 48, 3, 53), ("free", 64, 2, 54),
    ("free", 80, 2, 55), ("free", 96, 2, 56), ("free", 112, 2, 57), ("free", 128, 2, 58),
    ("surface", 32, 3, 59), ("surface", 112, 2, 60), ("surface", 128, 2, 61),
    ("wire", 48, 3, 62), ("wire", 128, 2, 63),
    ("periodic", 32, 3, 64), ("periodic", 112, 2, 65), ("periodic", 128, 2, 66),
]


def _tensors(s):
    return torch.from_numpy(s.psi).to(DEV), torch.from_numpy(s.occ).to(DEV)


def _check(s, ref, E, K, P, precision, N):
    if precision == "fp32":
        assert abs(E - ref["E"]) / N < TOL_FP32_E_PER_ORB
        assert kpsi_rel_err(K, ref["kpsi"]) < TOL_FP32_K
        assert kpsi_max_err(K, ref["kpsi"]) < TOL_FP32_K
        if P is not None:
            assert np.max(np.abs(P - ref["pair_e"])) <= 1e-6 * np.max(np.abs(ref["pair_e"]))
    else:
        assert abs(E - ref["E"]) <= TOL_FP64_E * abs(ref["E"])
        assert kpsi_rel_err(K, ref["kpsi"]) <= TOL_FP64_K
        assert kpsi_max_err(K, ref["kpsi"]) <= TOL_FP64_K
        if P is not None:
            assert np.max(np.abs(P - ref["pair_e"])) <= 1e-12 * np.max(np.abs(ref["pair_e"]))


@pytest.mark.parametrize("form", ["shared", "wave"])
@pytest.mark.parametrize("case", FORM_CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_slab_forms_match_oracle(case, form):
    bc, n, N, seed = case
    say(f"[forms] fp32 {form} {bc} n={n} N={N} seed={seed}")
    s, ref = oracle_result(bc, n, N, seed, 0)
    psi, occ = _tensors(s)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=N)
    plan.set_tuning(slab_form=form)
    pe = torch.empty((N, N), dtype=torch.float64, device=DEV)
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    e2, _, _ = plan.compute(psi, occ, "energy")  # Parseval route: forward transforms only
    torch.cuda.synchronize()
    _check(s, ref, ex.item(), kpsi.cpu().numpy(), pe.cpu().numpy(), "fp32", N)
    assert abs(e2.item() - ref["E"]) / N < TOL_FP32_E_PER_ORB


@pytest.mark.parametrize("tile", [4, 8])
@pytest.mark.parametrize("bc,n,N,seed", [("free", 80, 6, 84), ("free", 96, 6, 81),
                                         ("free", 112, 5, 85), ("free", 128, 5, 82),
                                         ("periodic", 112, 5, 86), ("periodic", 128, 5, 83)])
def test_pass_c_thread_split_matches_oracle(bc, n, N, seed, tile):
    # from n = 96 on a tile of 4 runs pass C with one thread per row segment
    # (256 threads), a tile of 8 with two threads per segment (512 threads); at
    # n = 112 the segment's n / 16 points split unevenly between the two (n = 80
    # has the one-thread form only, at both tiles)
    say(f"[pass C split] fp32 tile={tile} {bc} n={n} N={N} seed={seed}")
    s, ref = oracle_result(bc, n, N, seed, 1)
    psi, occ = _tensors(s)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=N)
    plan.set_tuning(tile=tile)
    pe = torch.empty((N, N), dtype=torch.float64, device=DEV)
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    torch.cuda.synchronize()
    _check(s, ref, ex.item(), kpsi.cpu().numpy(), pe.cpu().numpy(), "fp32", N)


@pytest.mark.parametrize("case", [c for c in FORM_CASES if c[1] <= 80],
                         ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_fp64_wave_form_matches_oracle(case):
    bc, n, N, seed = case
    say(f"[forms] fp64_fused wave {bc} n={n} N={N} seed={seed}")
    s, ref = oracle_result(bc, n, N, seed, 0)
    psi, occ = _tensors(s)
    plan = exx.Plan(grid_of(s), "fp64_fused", n_orb_max=N)
    plan.set_tuning(slab_form="wave")
    pe = torch.empty((N, N), dtype=torch.float64, device=DEV)
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    e2, _, _ = plan.compute(psi, occ, "energy")
    torch.cuda.synchronize()
    _check(s, ref, ex.item(), kpsi.cpu().numpy(), pe.cpu().numpy(), "fp64_fused", N)
    assert abs(e2.item() - ref["E"]) <= TOL_FP64_E * abs(ref["E"])


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused", "fp64_plain"])
@pytest.mark.parametrize("bc,n", [("free", 32), ("periodic", 32), ("free", 128)])
def test_single_orbital_is_minus_hartree(bc, n, precision):
    if precision == "fp64_fused" and n > 96:
        pytest.skip("the FP64 fused path stops at n = 96")
    say(f"[N=1] {precision} {bc} n={n}")
    s = small_system(bc, n, 1, seed=70)
    occ1 = np.ones(1)
    ref = oracle.exx(s.psi, occ1, s.h, bc, symmetric=True)
    psi = torch.from_numpy(s.psi).to(DEV)
    occ = torch.from_numpy(occ1).to(DEV)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=1)
    pe = torch.empty((1, 1), dtype=torch.float64, device=DEV)
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    torch.cuda.synchronize()
    E, e11 = ex.item(), pe.item()
    # E_x = -E_H[psi^2]: -1/2 f^2 e_11 with f = 1
    assert E == pytest.approx(-0.5 * e11, rel=1e-12)
    _check(s, ref, E, kpsi.cpu().numpy(), pe.cpu().numpy(), precision, 1)


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused", "fp64_plain"])
def test_zero_occupation_orbital(precision):
    say(f"[f=0] {precision}")
    s = small_system("free", 32, 5, seed=71)
    occ_np = np.array([2.0, 0.0, 1.3, 2.0, 0.0])
    ref = oracle.exx(s.psi, occ_np, s.h, "free", symmetric=True)
    psi = torch.from_numpy(s.psi).to(DEV)
    occ = torch.from_numpy(occ_np).to(DEV)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=5)
    plan.set_tuning(tile=2)  # the empty orbitals fall in different tile pairs
    pe = torch.empty((5, 5), dtype=torch.float64, device=DEV)
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    e2, _, _ = plan.compute(psi, occ, "energy")
    torch.cuda.synchronize()
    K = kpsi.cpu().numpy()
    _check(s, ref, ex.item(), K, pe.cpu().numpy(), precision, 5)
    assert abs(e2.item() - ref["E"]) / 5 < TOL_FP32_E_PER_ORB
    # an empty orbital receives K psi (sum over occupied partners) ...
    assert np.max(np.abs(K[1])) > 1e-3 * np.max(np.abs(K[0]))


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_real_batch_matches_oracle(precision, use_graph):
    say(f"[batch-oracle] {precision} graph={use_graph}")
    cases = [("free", 16, 5, 72), ("free", 32, 3, 73), ("free", 48, 4, 74), ("surface", 32, 3, 75),
             ("periodic", 32, 2, 76)]
    systems, refs = [], []
    for bc, n, N, seed in cases:
        s, r = oracle_result(bc, n, N, seed, 1)
        systems.append(s)
        refs.append(r)
    psis = [torch.from_numpy(s.psi).to(DEV) for s in systems]
    occs = [torch.from_numpy(s.occ).to(DEV) for s in systems]
    b = exx.Batch([grid_of(s) for s in systems], [s.n_orb for s in systems], precision,
                  use_graph=use_graph)
    outs = None
    for _ in range(2):
        outs = b.compute(psis, occs, "energy_kpsi", outputs=outs)
        torch.cuda.synchronize()
        for s, r, (ex, kp) in zip(systems, refs, outs):
            _check(s, r, ex.item(), kp.cpu().numpy(), None, precision, s.n_orb)


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused"])
def test_negative_occupation_energy_only(precision):
    # the energy-only (Parseval) route needs f >= 0; the binding takes the
    # pair-energy route for signed occupations, so E_x keeps the signs
    say(f"[f<0] {precision}")
    s = small_system("free", 32, 4, seed=77)
    occ_np = np.array([2.0, -0.4, 1.1, 0.7])
    ref = oracle.exx(s.psi, occ_np, s.h, "free", symmetric=True, want_kpsi=False)
    psi = torch.from_numpy(s.psi).to(DEV)
    occ = torch.from_numpy(occ_np).to(DEV)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=4)
    ex, _, pe = plan.compute(psi, occ, "energy")
    torch.cuda.synchronize()
    assert pe is None
    tol = 1e-6 * 4 if precision == "fp32" else TOL_FP64_E * abs(ref["E"])
    assert abs(ex.item() - ref["E"]) <= tol
