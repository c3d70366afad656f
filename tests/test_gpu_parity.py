"""GPU parity: the HIP paths (through the C ABI) against the FP64 oracle.

Sizes span several pair tiles with a ragged last tile (N not a multiple of
the tile edge), an odd number of pairs (a half-filled packed slot), the three
boundary conditions (periodic, free, surface, wire) and the mixed radices 3, 5 and 7
of the supported grids.
"""
import numpy as np
import pytest
import torch

from gpu_common import (TOL_FP32_E_PER_ORB, TOL_FP32_K, TOL_FP64_E, TOL_FP64_K, grid_of,
                        kpsi_max_err, kpsi_rel_err, oracle_result, say)

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")

CASES = [
    # (bc, n, N, seed, frac)
    ("periodic", 16, 3, 21, 0),
    ("free", 16, 5, 22, 1),
    ("periodic", 32, 8, 1001, 0),
    ("free", 32, 6, 23, 0),
    ("periodic", 48, 5, 24, 0),
    ("free", 48, 3, 25, 0),
    ("periodic", 80, 3, 26, 0),
    ("free", 16, 9, 27, 2),
    ("surface", 16, 5, 28, 1),
    ("surface", 32, 9, 29, 0),
    ("surface", 48, 4, 30, 0),
    ("surface", 64, 3, 31, 0),
    ("free", 80, 3, 32, 0),
    ("surface", 96, 3, 33, 0),
    ("wire", 16, 4, 39, 1),
    ("wire", 32, 7, 40, 0),
    ("wire", 48, 3, 41, 0),
    ("wire", 64, 3, 42, 0),
    ("wire", 96, 3, 43, 0),
    ("periodic", 96, 2, 44, 0),
]


def run(s, precision, pair_e=True):
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=s.n_orb)
    pe = torch.empty((s.n_orb, s.n_orb), dtype=torch.float64, device=dev) if pair_e else None
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    torch.cuda.synchronize()
    return float(ex.item()), kpsi.cpu().numpy(), (pe.cpu().numpy() if pe is not None else None)


@pytest.mark.parametrize("precision", ["fp64_plain", "fp64_fused"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_fp64_paths_match_oracle(case, precision):
    bc, n, N, seed, frac = case
    say(f"[parity] {precision} {bc} n={n} N={N} seed={seed}")
    s, ref = oracle_result(bc, n, N, seed, frac)
    E, K, P = run(s, precision)
    assert abs(E - ref["E"]) <= TOL_FP64_E * abs(ref["E"])
    assert kpsi_rel_err(K, ref["kpsi"]) <= TOL_FP64_K
    assert np.max(np.abs(P - ref["pair_e"])) <= 1e-12 * np.max(np.abs(ref["pair_e"]))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_fp32_path_within_tolerance(case):
    bc, n, N, seed, frac = case
    say(f"[parity] fp32 {bc} n={n} N={N} seed={seed}")
    s, ref = oracle_result(bc, n, N, seed, frac)
    E, K, P = run(s, "fp32")
    assert abs(E - ref["E"]) / N < TOL_FP32_E_PER_ORB
    assert kpsi_rel_err(K, ref["kpsi"]) < TOL_FP32_K
    assert np.max(np.abs(P - ref["pair_e"])) <= 1e-6 * np.max(np.abs(ref["pair_e"]))


@pytest.mark.parametrize("bc", ["free", "surface", "wire"])
@pytest.mark.parametrize("precision", ["fp32", "fp64_fused", "fp64_plain"])
def test_energy_only_and_kpsi_only_modes(precision, bc):
    say(f"[modes] {precision} {bc}")
    s, ref = oracle_result(bc, 32, 6, 23, 0)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=8)
    ex, _, _ = plan.compute(psi, occ, "energy")  # Parseval route on the fused paths
    _, kpsi, _ = plan.compute(psi, occ, "kpsi")
    torch.cuda.synchronize()
    tolE = TOL_FP64_E if precision != "fp32" else 1e-6 * 6 / abs(ref["E"])
    assert abs(ex.item() - ref["E"]) <= tolE * abs(ref["E"])
    tolK = TOL_FP64_K if precision != "fp32" else TOL_FP32_K
    assert kpsi_rel_err(kpsi.cpu().numpy(), ref["kpsi"]) <= tolK


def test_accumulate_flag_adds_into_kpsi():
    say("[accumulate] fp32")
    s, ref = oracle_result("periodic", 16, 3, 21, 0)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=4)
    k0 = torch.ones_like(psi)
    plan.compute(psi, occ, "kpsi", kpsi=k0, accumulate=True)
    torch.cuda.synchronize()
    assert kpsi_rel_err(k0.cpu().numpy() - 1.0, ref["kpsi"]) < TOL_FP32_K


def test_workspace_too_small_is_rejected():
    say("[workspace] fp32")
    s, _ = oracle_result("periodic", 16, 3, 21, 0)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=4)
    small = torch.empty(1024, dtype=torch.uint8, device=dev)
    with pytest.raises(RuntimeError, match="WORKSPACE"):
        plan.compute(psi, occ, "energy_kpsi", workspace=small)
    with pytest.raises(RuntimeError, match="CAPACITY"):
        big = torch.zeros((5, 16, 16, 16), dtype=torch.float64, device=dev)
        plan.compute(big, torch.ones(5, dtype=torch.float64, device=dev), "energy_kpsi")


# Large slabs on the FP32 path take the three-launch pass B (y columns, z lines,
# inverse y columns) from n = 112 on; n = 96 runs the 768-thread shared-y block;
# the FP64 fused path stops at n = 96.
SPLIT_CASES = [("free", 96, 3, 34, 0), ("free", 112, 2, 35, 0), ("surface", 112, 3, 36, 0),
               ("free", 128, 2, 38, 0), ("wire", 112, 2, 37, 0), ("wire", 128, 2, 39, 0)]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_fp32_split_pass_b_within_tolerance(case):
    bc, n, N, seed, frac = case
    say(f"[parity split] fp32 {bc} n={n} N={N} seed={seed}")
    s, ref = oracle_result(bc, n, N, seed, frac)
    E, K, P = run(s, "fp32")
    assert abs(E - ref["E"]) / N < TOL_FP32_E_PER_ORB
    assert kpsi_rel_err(K, ref["kpsi"]) < TOL_FP32_K
    assert np.max(np.abs(P - ref["pair_e"])) <= 1e-6 * np.max(np.abs(ref["pair_e"]))
    # the energy-only (Parseval) route through the split pass B
    dev = torch.device("cuda", 0)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=N)
    ex, _, _ = plan.compute(torch.from_numpy(s.psi).to(dev), torch.from_numpy(s.occ).to(dev), "energy")
    torch.cuda.synchronize()
    assert abs(ex.item() - ref["E"]) / N < TOL_FP32_E_PER_ORB


@pytest.mark.parametrize("bc,precision,kmax", [("free", "fp32", 0.0), ("periodic", "fp64_fused", 0.0),
                                                ("wire", "fp32", 0.0), ("free", "fp32", 1.0)])
def test_kpsi_output_is_overwritten(bc, precision, kmax):
    # K psi is not cleared beforehand: the first round of pass C stores every
    # orbital row, so stale contents (NaN here) must not survive
    say(f"[overwrite] {precision} {bc} kmax={kmax}")
    s, ref = oracle_result(bc, 32, 10, 47, 0, kmax=kmax)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=s.n_orb, complex_orbitals=kmax > 0)
    kpsi = torch.full_like(psi, float("nan"))
    for _ in range(2):  # and again over the previous result
        plan.compute(psi, occ, "kpsi", kpsi=kpsi)
        torch.cuda.synchronize()
        K = kpsi.cpu().numpy()
        assert np.all(np.isfinite(K))
        tol = TOL_FP32_K if precision == "fp32" else TOL_FP64_K
        assert kpsi_rel_err(K, ref["kpsi"]) < tol


def test_fp32_odd_slot_chunks_above_n64():
    # Above n = 64 a pass A block takes two consecutive slots.  Five orbitals in
    # tiles of 3 (sizes 3 and 2) give two launch chunks of 5 slots each (the
    # schedule is checked on the CPU in test_schedule_cpu.py): the first holds the
    # large diagonal tile pair, the second the small diagonal one and the
    # off-diagonal pair with its ragged 2-orbital edge, so both launches end in a
    # one-slot pass A block, one of them on an off-diagonal tile pair.
    bc, n, N, seed = "free", 80, 5, 45
    say(f"[parity chunks] fp32 {bc} n={n} N={N} seed={seed} tile=3 batch_slots=5")
    s, ref = oracle_result(bc, n, N, seed, 0)
    dev = torch.device("cuda", 0)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=N)
    plan.set_tuning(tile=3, batch_slots=5)
    assert plan.tuning["tile"] == 3
    assert plan.schedule_info(N) == (15, 10)
    plan.enable_profiling(True)
    plan.read_profile()
    pe = torch.empty((N, N), dtype=torch.float64, device=dev)
    ex, kp, pe = plan.compute(torch.from_numpy(s.psi).to(dev), torch.from_numpy(s.occ).to(dev),
                              "energy_kpsi", pair_e=pe)
    torch.cuda.synchronize()
    assert plan.read_profile()["pass_a"][1] == 2  # one launch per chunk
    assert abs(ex.item() - ref["E"]) / N < TOL_FP32_E_PER_ORB
    assert kpsi_rel_err(kp.cpu().numpy(), ref["kpsi"]) < TOL_FP32_K
    assert kpsi_max_err(kp.cpu().numpy(), ref["kpsi"]) < TOL_FP32_K
    P = pe.cpu().numpy()
    assert np.max(np.abs(P - ref["pair_e"])) <= 1e-6 * np.max(np.abs(ref["pair_e"]))
