"""Batches of uneven systems and HIP-graph replay.

The batched result of every system must equal its single-system evaluation,
and a captured graph must reproduce the eager result on every replay, with
other eager work and synchronisations between replays.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import grid_of, say, small_system

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")

SYSTEMS = [("free", 16, 5, 41), ("free", 32, 3, 42), ("free", 48, 4, 43), ("free", 16, 2, 44)]


def _load(precision):
    dev = torch.device("cuda", 0)
    systems = [small_system(bc, n, N, seed) for bc, n, N, seed in SYSTEMS]
    psis = [torch.from_numpy(s.psi).to(dev) for s in systems]
    occs = [torch.from_numpy(s.occ).to(dev) for s in systems]
    single = []
    for s, p, o in zip(systems, psis, occs):
        plan = exx.Plan(grid_of(s), precision, n_orb_max=s.n_orb)
        ex, kp, _ = plan.compute(p, o, "energy_kpsi")
        single.append((ex.item(), kp.cpu().numpy()))
    return systems, psis, occs, single


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_single_system_calls(precision, use_graph):
    say(f"[batch] {precision} graph={use_graph}")
    systems, psis, occs, single = _load(precision)
    b = exx.Batch([grid_of(s) for s in systems], [s.n_orb for s in systems], precision,
                  use_graph=use_graph)
    outs = None
    for rep in range(3):
        outs = b.compute(psis, occs, "energy_kpsi", outputs=outs)
        torch.cuda.synchronize()
        for (ex, kp), (E1, K1) in zip(outs, single):
            # same kernels, same schedule, no atomics: bitwise equal
            assert ex.item() == E1
            assert np.array_equal(kp.cpu().numpy(), K1)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device=psis[0].device)
        (x * 2).sum().item()
        for kp in outs:
            kp[1].fill_(123.0)
            kp[0].fill_(7.0)


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused"])
def test_repeated_evaluations_are_bitwise_identical(precision):
    say(f"[determinism] {precision}")
    s = small_system("free", 32, 9, seed=45)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=9)
    plan.set_tuning(tile=4)  # several rounds and tile pairs
    res = []
    for _ in range(3):
        pe = torch.empty((9, 9), dtype=torch.float64, device=dev)
        ex, kp, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
        e2, _, _ = plan.compute(psi, occ, "energy")
        res.append((ex.item(), kp.cpu().numpy(), pe.cpu().numpy(), e2.item()))
    for r in res[1:]:
        assert r[0] == res[0][0] and r[3] == res[0][3]
        assert np.array_equal(r[1], res[0][1]) and np.array_equal(r[2], res[0][2])


@pytest.mark.parametrize("complex_orbitals", [False, True])
def test_single_plan_captured_in_a_torch_graph(complex_orbitals):
    # one evaluation captured with torch.cuda.graph on the caller's stream and
    # replayed: every replay equals the eager result bit for bit, with eager work,
    # synchronisations and clobbered outputs between replays
    say(f"[graph] single plan complex={complex_orbitals}")
    s = small_system("free", 32, 9, seed=46, kmax=1.0 if complex_orbitals else 0.0)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=s.n_orb, complex_orbitals=complex_orbitals)
    kpsi = torch.empty_like(psi)
    ex = torch.empty((), dtype=torch.float64, device=dev)
    plan.workspace(s.n_orb)
    plan.compute(psi, occ, "energy_kpsi", kpsi=kpsi, ex_out=ex)  # builds the schedule
    torch.cuda.synchronize()
    E0, K0 = ex.item(), kpsi.cpu().numpy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.compute(psi, occ, "energy_kpsi", kpsi=kpsi, ex_out=ex)
    for rep in range(3):
        kpsi.fill_(float("nan"))
        ex.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        assert ex.item() == E0
        assert np.array_equal(kpsi.cpu().numpy(), K0)
        x = torch.randn(1 << 20, device=dev)
        (x * 2).sum().item()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_autotune_per_grid_class(use_graph):
    # exx_batch_autotune tunes one member per grid class and gives every member of
    # the class the same tuning; each member then equals a single-system plan
    # with that tuning, bit for bit, on every replay
    say(f"[batch autotune] graph={use_graph}")
    dev = torch.device("cuda", 0)
    cases = [("free", 32, 9, 46), ("free", 48, 6, 47), ("free", 32, 5, 48), ("periodic", 32, 4, 49)]
    systems = [small_system(bc, n, N, seed) for bc, n, N, seed in cases]
    psis = [torch.from_numpy(s.psi).to(dev) for s in systems]
    occs = [torch.from_numpy(s.occ).to(dev) for s in systems]
    b = exx.Batch([grid_of(s) for s in systems], [s.n_orb for s in systems], "fp32",
                  use_graph=use_graph)
    outs = b.compute(psis, occs, "energy_kpsi")
    torch.cuda.synchronize()
    tunings = b.autotune(psis, occs, budget_ms=3000)
    assert tunings[0] == tunings[2]  # the two free 32^3 systems share one class
    outs = b.compute(psis, occs, "energy_kpsi", outputs=outs)
    torch.cuda.synchronize()
    for rep in range(2):
        outs = b.compute(psis, occs, "energy_kpsi", outputs=outs)
        torch.cuda.synchronize()
        for s, p, o, t, (ex, kp) in zip(systems, psis, occs, tunings, outs):
            plan = exx.Plan(grid_of(s), "fp32", n_orb_max=s.n_orb)
            plan.set_tuning(**t)
            e1, k1, _ = plan.compute(p, o, "energy_kpsi")
            torch.cuda.synchronize()
            assert ex.item() == e1.item()
            assert torch.equal(kp, k1)


MERGE_CASES = [("free", 32, 5, 91), ("free", 32, 9, 92), ("free", 48, 4, 93), ("free", 32, 2, 94),
               ("periodic", 32, 3, 95), ("free", 48, 7, 96), ("free", 32, 1, 97)]


def _merge_inputs(cases, complex_orbitals=False):
    dev = torch.device("cuda", 0)
    kmax = 0.4 if complex_orbitals else 0.0
    systems = [small_system(bc, n, N, seed, kmax=kmax) for bc, n, N, seed in cases]
    psis = [torch.from_numpy(s.psi).to(dev) for s in systems]
    occs = [torch.from_numpy(s.occ).to(dev) for s in systems]
    return systems, psis, occs


@pytest.mark.parametrize("complex_orbitals", [False, True])
@pytest.mark.parametrize("use_graph", [False, True])
def test_merged_batch_equals_unmerged(use_graph, complex_orbitals):
    # systems on one grid share their pass launches (merged round-robin rounds);
    # every system's E_x and K psi equal the unmerged batch's bit for bit, on
    # every replay, with other eager work between the calls
    say(f"[merged batch] graph={use_graph} complex={complex_orbitals}")
    systems, psis, occs = _merge_inputs(MERGE_CASES, complex_orbitals)
    grids = [grid_of(s) for s in systems]
    ns = [s.n_orb for s in systems]
    ref = exx.Batch(grids, ns, "fp32", use_graph=False, complex_orbitals=complex_orbitals)
    want = [(e.item(), k.clone()) for e, k in ref.compute(psis, occs, "energy_kpsi")]
    del ref
    b = exx.Batch(grids, ns, "fp32", use_graph=use_graph, complex_orbitals=complex_orbitals,
                  merge=True)
    outs = None
    for rep in range(3):
        outs = b.compute(psis, occs, "energy_kpsi", outputs=outs)
        torch.cuda.synchronize()
        for (ex, kp), (E1, K1) in zip(outs, want):
            assert ex.item() == E1
            assert torch.equal(kp, K1)
        x = torch.randn(1 << 20, device=psis[0].device)
        (x * 2).sum().item()
        for ex, kp in outs:
            kp.fill_(123.0)
            ex.fill_(7.0)
    # K psi only, and accumulation into K psi
    outs = b.compute(psis, occs, "kpsi", outputs=outs)
    torch.cuda.synchronize()
    for (_, kp), (_, K1) in zip(outs, want):
        assert torch.equal(kp, K1)


def test_merged_batch_matches_oracle_and_limits():
    say("[merged batch] oracle, 34 systems on one grid, refusals")
    cases = [("free", 16, 1 + k % 3, 200 + k) for k in range(34)] + [("free", 32, 5, 91)]
    systems, psis, occs = _merge_inputs(cases)
    b = exx.Batch([grid_of(s) for s in systems], [s.n_orb for s in systems], "fp32",
                  use_graph=True, merge=True)
    outs = b.compute(psis, occs, "energy_kpsi")
    torch.cuda.synchronize()
    for k in (0, 17, 33, 34):  # both 16^3 classes (32 + 2 systems) and the 32^3 one
        s = systems[k]
        ref = oracle.exx(s.psi, s.occ, s.h, s.bc, symmetric=True)
        E, K = outs[k][0].item(), outs[k][1].cpu().numpy()
        assert abs(E - ref["E"]) / s.n_orb < 1e-6
        assert np.max(np.abs(K - ref["kpsi"])) <= 1e-5 * np.max(np.abs(ref["kpsi"]))
    with pytest.raises(exx.ExxError):
        b.compute(psis, occs, "energy")
    with pytest.raises(exx.ExxError):
        exx.Batch([grid_of(s) for s in systems[:2]], [1, 1], "fp64_fused", merge=True)
