"""Screened kernel (erfc(omega r)/r, Section 3.2.3: only the Poisson filter
changes) against the oracle on all three paths, and the autotuner."""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_common import TOL_FP32_K, kpsi_rel_err, say, small_system

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused", "fp64_plain"])
def test_screened_kernel_matches_oracle(precision):
    say(f"[screened] {precision}")
    s = small_system("periodic", 32, 5, seed=51)
    omega = 0.4
    ref = oracle.exx(s.psi, s.occ, s.h, "periodic", omega=omega, symmetric=True)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    g = exx.Grid(n=s.n, h=s.h, bc="periodic", kernel="screened", omega=omega)
    plan = exx.Plan(g, precision, n_orb_max=5)
    ex, kpsi, _ = plan.compute(psi, occ, "energy_kpsi")
    torch.cuda.synchronize()
    if precision == "fp32":
        assert abs(ex.item() - ref["E"]) / 5 < 1e-6
        assert kpsi_rel_err(kpsi.cpu().numpy(), ref["kpsi"]) < TOL_FP32_K
    else:
        assert ex.item() == pytest.approx(ref["E"], rel=1e-12)
        assert kpsi_rel_err(kpsi.cpu().numpy(), ref["kpsi"]) < 1e-11
    # the screened exchange is weaker than the full one
    full = oracle.exx(s.psi, s.occ, s.h, "periodic", symmetric=True, want_kpsi=False)["E"]
    assert abs(ref["E"]) < abs(full)


def test_autotune_picks_a_valid_tuning_and_caches(tmp_path):
    say("[autotune] free48 N=12")
    s = small_system("free", 48, 12, seed=52)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    g = exx.Grid(n=s.n, h=s.h, bc="free")
    plan = exx.Plan(g, "fp32", n_orb_max=12)
    ref_ex, ref_k, _ = plan.compute(psi, occ, "energy_kpsi")
    ref_ex, ref_k = ref_ex.item(), ref_k.cpu().numpy()
    cache = str(tmp_path / "tune.txt")
    t = plan.autotune(psi, occ, cache_path=cache)
    assert t["tile"] >= 1 and t["batch_slots"] >= 1
    assert os.path.exists(cache) and open(cache).read().count("|") == 1
    ex, k, _ = plan.compute(psi, occ, "energy_kpsi")
    assert ex.item() == pytest.approx(ref_ex, rel=1e-9)
    assert kpsi_rel_err(k.cpu().numpy(), ref_k) < 1e-6
    plan2 = exx.Plan(g, "fp32", n_orb_max=12)
    assert plan2.autotune(psi, occ, cache_path=cache) == t  # served from the cache
