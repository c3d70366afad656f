"""GPU parity for complex orbitals (rho_ij = conj(psi_j) psi_i, Eq. 2): the HIP
paths through the C ABI against the FP64 oracle.

Cases cover the four boundaries, several pair tiles with a ragged last tile
(N not a multiple of the complex tile edge: 8 up to n = 64 and 4 beyond on the
FP32 path; 8, 4, 2 on the FP64 fused one), the mixed radices 3 and 5, the
three-launch pass B of large FP32 slabs, the energy-only (Parseval) and K psi
only modes, several launch chunks, the overlapped-stream pipeline and the
autograd gradient (PyTorch's complex convention: dE/dRe + i dE/dIm).
"""
import numpy as np
import pytest
import torch

from gpu_common import (TOL_FP32_E_PER_ORB, TOL_FP32_K, TOL_FP64_E, TOL_FP64_K, grid_of,
                        kpsi_rel_err, oracle_result, say)

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")

KMAX = 1.0
CASES = [
    # (bc, n, N, seed, frac)
    ("periodic", 16, 5, 61, 1),
    ("free", 16, 9, 62, 2),
    ("surface", 16, 4, 63, 0),
    ("wire", 16, 4, 64, 1),
    ("free", 32, 10, 65, 0),
    ("periodic", 48, 4, 66, 0),
    ("free", 64, 3, 67, 0),
    ("surface", 64, 3, 68, 0),
    ("periodic", 80, 5, 69, 0),
    ("free", 96, 3, 70, 0),
]
SPLIT_CASES = [("free", 112, 5, 71, 0), ("surface", 112, 2, 72, 0)]


def ref_of(case):
    bc, n, N, seed, frac = case
    return oracle_result(bc, n, N, seed, frac, kmax=KMAX)


def tensors(s):
    dev = torch.device("cuda", 0)
    return torch.from_numpy(s.psi).to(dev), torch.from_numpy(s.occ).to(dev)


def run(s, precision, pair_e=True, tuning=None):
    psi, occ = tensors(s)
    assert psi.dtype == torch.complex128
    plan = exx.Plan(grid_of(s), precision, n_orb_max=s.n_orb, complex_orbitals=True)
    if tuning:
        plan.set_tuning(**tuning)
    pe = torch.empty((s.n_orb, s.n_orb), dtype=torch.float64, device=psi.device) if pair_e else None
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    torch.cuda.synchronize()
    return float(ex.item()), kpsi.cpu().numpy(), (pe.cpu().numpy() if pe is not None else None)


def check(precision, s, ref, E, K, P):
    N = s.n_orb
    if precision == "fp32":
        assert abs(E - ref["E"]) / N < TOL_FP32_E_PER_ORB
        assert kpsi_rel_err(K, ref["kpsi"]) < TOL_FP32_K
        if P is not None:
            assert np.max(np.abs(P - ref["pair_e"])) <= 1e-6 * np.max(np.abs(ref["pair_e"]))
    else:
        assert abs(E - ref["E"]) <= TOL_FP64_E * abs(ref["E"])
        assert kpsi_rel_err(K, ref["kpsi"]) <= TOL_FP64_K
        if P is not None:
            assert np.max(np.abs(P - ref["pair_e"])) <= 1e-12 * np.max(np.abs(ref["pair_e"]))


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused", "fp64_plain"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_complex_paths_match_oracle(case, precision):
    bc, n, N, seed, frac = case
    say(f"[complex parity] {precision} {bc} n={n} N={N} seed={seed}")
    s, ref = ref_of(case)
    assert np.abs(ref["kpsi"].imag).max() > 1e-2 * np.abs(ref["kpsi"]).max()  # genuinely complex
    E, K, P = run(s, precision)
    check(precision, s, ref, E, K, P)


@pytest.mark.parametrize("case", SPLIT_CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}")
def test_complex_split_pass_b(case):
    bc, n, N, seed, frac = case
    say(f"[complex parity split] fp32 {bc} n={n} N={N} seed={seed}")
    s, ref = ref_of(case)
    E, K, P = run(s, "fp32")
    check("fp32", s, ref, E, K, P)


@pytest.mark.parametrize("bc", ["free", "periodic"])
@pytest.mark.parametrize("precision", ["fp32", "fp64_fused", "fp64_plain"])
def test_complex_energy_only_and_kpsi_only_modes(precision, bc):
    say(f"[complex modes] {precision} {bc}")
    case = (bc, 32, 10, 65, 0) if bc == "free" else ("periodic", 16, 5, 61, 1)
    s, ref = ref_of(case)
    psi, occ = tensors(s)
    plan = exx.Plan(grid_of(s), precision, n_orb_max=s.n_orb, complex_orbitals=True)
    ex, _, _ = plan.compute(psi, occ, "energy")  # Parseval route on the fused paths
    _, kpsi, _ = plan.compute(psi, occ, "kpsi")
    ex2, _, _ = plan.compute(psi, occ, "energy_kpsi")  # energies from pass C, no pair matrix
    torch.cuda.synchronize()
    tolE = TOL_FP64_E * abs(ref["E"]) if precision != "fp32" else TOL_FP32_E_PER_ORB * s.n_orb
    assert abs(ex.item() - ref["E"]) <= tolE
    assert abs(ex2.item() - ref["E"]) <= tolE
    tolK = TOL_FP64_K if precision != "fp32" else TOL_FP32_K
    assert kpsi_rel_err(kpsi.cpu().numpy(), ref["kpsi"]) <= tolK


@pytest.mark.parametrize("streams", [1, 3])
def test_complex_chunks_and_streams_are_bitwise_neutral(streams):
    # several launch chunks (batch_slots below one tile pair's slots is raised to
    # a whole tile pair) and the overlapped rounds give the default's bits
    say(f"[complex chunks] fp32 streams={streams}")
    s, ref = ref_of(("free", 32, 10, 65, 0))
    E0, K0, P0 = run(s, "fp32")
    E1, K1, P1 = run(s, "fp32", tuning={"batch_slots": 40, "streams": streams})
    assert E1 == E0
    assert np.array_equal(K1, K0) and np.array_equal(P1, P0)
    check("fp32", s, ref, E1, K1, P1)


def test_complex_plan_rejects_real_tensors_and_unknown_flags():
    say("[complex plan] dtype checks")
    s, _ = ref_of(("periodic", 16, 5, 61, 1))
    psi, occ = tensors(s)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=8, complex_orbitals=True)
    with pytest.raises(TypeError):
        plan.compute(psi.real.contiguous(), occ, "energy")
    real_plan = exx.Plan(grid_of(s), "fp32", n_orb_max=8)
    with pytest.raises(TypeError):
        real_plan.compute(psi, occ, "energy")


def test_complex_autograd_gradient():
    say("[complex autograd] fp32 free")
    import oracle
    s, ref = ref_of(("free", 16, 9, 62, 2))
    psi, occ = tensors(s)
    psi.requires_grad_(True)
    E = exx.exchange_energy(psi, occ, grid_of(s), "fp32")
    E.backward()
    torch.cuda.synchronize()
    g_ref = oracle.exx_grad_psi(ref["kpsi"], s.occ, s.h)
    g = psi.grad.cpu().numpy()
    assert abs(E.item() - ref["E"]) / s.n_orb < TOL_FP32_E_PER_ORB
    assert kpsi_rel_err(g, g_ref) < TOL_FP32_K


@pytest.mark.parametrize("use_graph", [False, True])
def test_spin_polarized_complex_batch(use_graph):
    # two spin channels (Eq. 2's sum over sigma): own orbitals and occupations on
    # one grid, one batched call (graph replays included) against the oracle
    # and bitwise against single-channel calls
    say(f"[complex spin batch] fp32 graph={use_graph}")
    chans = [ref_of(("free", 32, 10, 65, 0)), ref_of(("free", 32, 7, 73, 3))]
    dev = torch.device("cuda", 0)
    psis = [torch.from_numpy(s.psi).to(dev) for s, _ in chans]
    occs = [torch.from_numpy(s.occ).to(dev) for s, _ in chans]
    single = []
    for (s, _), p, o in zip(chans, psis, occs):
        plan = exx.Plan(grid_of(s), "fp32", n_orb_max=s.n_orb, complex_orbitals=True)
        ex, kp, _ = plan.compute(p, o, "energy_kpsi")
        single.append((ex.item(), kp.cpu().numpy()))
    b = exx.Batch([grid_of(s) for s, _ in chans], [s.n_orb for s, _ in chans], "fp32",
                  use_graph=use_graph, complex_orbitals=True)
    outs = None
    for rep in range(3):
        outs = b.compute(psis, occs, "energy_kpsi", outputs=outs)
        torch.cuda.synchronize()
        E_total = 0.0
        for (ex, kp), (E1, K1), (s, ref) in zip(outs, single, chans):
            assert ex.item() == E1
            assert np.array_equal(kp.cpu().numpy(), K1)
            check("fp32", s, ref, ex.item(), kp.cpu().numpy(), None)
            E_total += ex.item()
        assert abs(E_total - sum(r["E"] for _, r in chans)) / 17 < TOL_FP32_E_PER_ORB
        for ex, kp in outs:  # clobber the outputs between replays
            kp.fill_(3.0)
            ex.fill_(7.0)


@pytest.mark.parametrize("precision", ["fp32", "fp64_fused"])
def test_complex_orbitals_with_the_screened_kernel(precision):
    # the kernel is independent of the orbitals' type: erfc(omega r)/r on a
    # periodic grid with complex orbitals
    say(f"[complex screened] {precision}")
    import oracle
    from gpu_common import small_system
    s = small_system("periodic", 32, 6, 74, kmax=KMAX)
    omega = 0.4
    ref = oracle.exx(s.psi, s.occ, s.h, "periodic", omega=omega, symmetric=True)
    psi, occ = tensors(s)
    g = exx.Grid(n=s.n, h=s.h, bc="periodic", kernel="screened", omega=omega)
    plan = exx.Plan(g, precision, n_orb_max=s.n_orb, complex_orbitals=True)
    pe = torch.empty((s.n_orb, s.n_orb), dtype=torch.float64, device=psi.device)
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    torch.cuda.synchronize()
    check(precision, s, ref, float(ex.item()), kpsi.cpu().numpy(), pe.cpu().numpy())
