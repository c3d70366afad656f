"""Overlapped rounds (passes A, B, C on three streams) against the serial order.

Pass C launches keep their round order on one stream and every slot's energy
partial has a fixed place, so the overlapped evaluation must reproduce the
serial one bit for bit, in every mode, with several chunks and with
accumulation into K psi.
"""
import numpy as np
import pytest
import torch

from gpu_common import grid_of, say, small_system

pytestmark = pytest.mark.gpu

exx = pytest.importorskip("paper_1712_07973_amd")

CASES = [("free", 32, 11, 61, "fp32", 4, 0), ("free", 48, 9, 62, "fp32", 4, 8),
         ("periodic", 32, 13, 63, "fp32", 8, 0), ("free", 32, 10, 64, "fp64_fused", 4, 8)]


def _run(plan, psi, occ, mode, pair=False, accumulate=False, kp0=None):
    dev = psi.device
    pe = torch.empty((psi.shape[0],) * 2, dtype=torch.float64, device=dev) if pair else None
    kp = kp0.clone() if kp0 is not None else None
    ex, kp, pe = plan.compute(psi, occ, mode, kpsi=kp, pair_e=pe, accumulate=accumulate)
    torch.cuda.synchronize()
    out = [ex.item() if ex is not None else None]
    if kp is not None:
        out.append(kp.cpu().numpy())
    if pe is not None:
        out.append(pe.cpu().numpy())
    return out


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}_N{c[2]}_{c[4]}_t{c[5]}_b{c[6]}")
def test_overlapped_rounds_match_serial(case):
    bc, n, N, seed, prec, tile, batch = case
    say(f"[streams] {case}")
    s = small_system(bc, n, N, seed)
    dev = torch.device("cuda", 0)
    psi = torch.from_numpy(s.psi).to(dev)
    occ = torch.from_numpy(s.occ).to(dev)
    kp0 = torch.from_numpy(np.random.default_rng(seed).standard_normal(s.psi.shape)).to(dev)
    res = {}
    for streams in (1, 3):
        plan = exx.Plan(grid_of(s), prec, n_orb_max=N)
        plan.set_tuning(tile=tile, batch_slots=batch, streams=streams)
        assert plan.tuning["streams"] == streams
        res[streams] = [
            _run(plan, psi, occ, "energy_kpsi"),
            _run(plan, psi, occ, "energy_kpsi", pair=True),
            _run(plan, psi, occ, "energy"),
            _run(plan, psi, occ, "kpsi", accumulate=True, kp0=kp0),
        ]
    for a, b in zip(res[1], res[3]):
        for x, y in zip(a, b):
            assert np.array_equal(np.asarray(x), np.asarray(y))


def test_streams_setting_is_validated():
    s = small_system("free", 16, 3, 65)
    plan = exx.Plan(grid_of(s), "fp32", n_orb_max=3)
    with pytest.raises(exx.ExxError):
        plan.set_tuning(streams=2)
    with pytest.raises(exx.ExxError):
        plan.set_tuning(slab_threads=300)
