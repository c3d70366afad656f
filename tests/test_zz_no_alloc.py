"""exx_compute_noalloc (the library's static per-GPU workspace) against
exx_compute (a caller's workspace) through the C ABI: two calls in a row on one
plan, the second with fewer orbitals, each bit for bit equal to exx_compute's
result (same kernels, same schedule, no atomics) and within the FP32 bar of the
oracle; plus the refusals (schedule not prepared, workspace above the static
maximum).
"""
import pytest
import torch

from gpu_common import (TOL_FP32_E_PER_ORB, TOL_FP32_K, grid_of, kpsi_max_err, oracle_result,
                        say)

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")
from paper_1712_07973_amd import _lib as L  # noqa: E402

DEV = torch.device("cuda", 0)


def _outputs(N, n):
    return (torch.full((), 7.0, dtype=torch.float64, device=DEV),
            torch.full((N, n, n, n), float("nan"), dtype=torch.float64, device=DEV),
            torch.full((N, N), float("nan"), dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("bc,n,N1,N2", [("free", 32, 9, 5), ("periodic", 48, 6, 3)])
def test_noalloc_matches_exx_compute(bc, n, N1, N2):
    say(f"[noalloc] {bc} n={n} N={N1} then {N2}")
    plan = exx.Plan(grid_of(oracle_result(bc, n, N1, 81)[0]), "fp32", n_orb_max=N1)
    plan.set_tuning(tile=4)
    for N in (N1, N2):
        plan.prepare(N)
    for N in (N1, N2):  # second call: a smaller input on the same static workspace
        s, ref = oracle_result(bc, n, N, 81)
        psi = torch.from_numpy(s.psi).to(DEV)
        occ = torch.from_numpy(s.occ).to(DEV)
        e0, k0, p0 = _outputs(N, n)
        plan.compute(psi, occ, "energy_kpsi", kpsi=k0, pair_e=p0, ex_out=e0)
        e1, k1, p1 = _outputs(N, n)
        plan.compute_noalloc(psi, occ, "energy_kpsi", kpsi=k1, pair_e=p1, ex_out=e1)
        e2, _, _ = _outputs(N, n)
        plan.compute_noalloc(psi, occ, "energy", ex_out=e2)  # Parseval route
        e3, _, _ = _outputs(N, n)
        plan.compute(psi, occ, "energy", ex_out=e3)
        torch.cuda.synchronize()
        assert e1.item() == e0.item() and e2.item() == e3.item()
        assert torch.equal(k1, k0) and torch.equal(p1, p0)
        assert abs(e1.item() - ref["E"]) / N < TOL_FP32_E_PER_ORB
        assert kpsi_max_err(k1.cpu().numpy(), ref["kpsi"]) < TOL_FP32_K


def test_noalloc_refusals():
    say("[noalloc] refusals")
    s, _ = oracle_result("free", 32, 9, 81)
    psi = torch.from_numpy(s.psi).to(DEV)
    occ = torch.from_numpy(s.occ).to(DEV)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=9)
    e, k, _ = _outputs(9, 32)
    # no schedule for this orbital count yet: nothing may be built here
    with pytest.raises(RuntimeError, match="NOT_PREPARED"):
        plan.compute_noalloc(psi, occ, "energy_kpsi", kpsi=k, ex_out=e)
    # a workspace above the static maximum is refused with the sizes
    big = exx.Plan(exx.Grid(n=128, h=0.4, bc="free"), "fp32", n_orb_max=64)
    need = big.workspace_bytes(64)
    psi_big = torch.zeros((64, 128, 128, 128), dtype=torch.float64, device=DEV)
    occ_big = torch.ones(64, dtype=torch.float64, device=DEV)
    kb = torch.empty_like(psi_big)
    eb = torch.empty((), dtype=torch.float64, device=DEV)
    assert need > (64 << 20)
    with pytest.raises(RuntimeError, match="WORKSPACE"):
        big.compute_noalloc(psi_big, occ_big, "energy_kpsi", kpsi=kb, ex_out=eb)
    assert b"static maximum" in L.lib().exx_last_error()
