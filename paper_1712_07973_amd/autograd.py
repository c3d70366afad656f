"""E_x as a differentiable function of the orbitals (and occupations).

Forward: E_x alone (exx_compute in ENERGY mode, no pair potential stored).
Backward: exx_gradient, which recomputes every pair potential (KPSI mode) and
returns, scaled on the device by the upstream derivative, the exact gradient
of the grid function,

    dE_x / dpsi_k(r) = -2 f_k h^3 (K psi)_k(r),
    dE_x / df_k      = -sum_j f_j e_kj,

where (K psi)_k = sum_j f_j V_kj psi_j is minus the Fock action of Eq. 3 of
arXiv:1712.07973 and e_kj the pair energies (Eq. 5).  For complex orbitals
(complex128 psi) the first line is the gradient with respect to Re psi plus i
times the one with respect to Im psi, which is PyTorch's convention for a real
function of complex inputs.  E_x is a homogeneous quartic in psi and quadratic
in f, which the tests use.
"""
from __future__ import annotations

import torch

from .api import Grid, get_plan


class ExchangeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi: torch.Tensor, occ: torch.Tensor, grid: Grid, precision: str):
        psi_c = psi.detach().contiguous()
        occ_c = occ.detach().contiguous()
        plan = get_plan(grid, precision, psi_c.shape[0], psi_c.device, psi_c.is_complex())
        ex, _, _ = plan.compute(psi_c, occ_c, "energy")
        ctx.save_for_backward(psi_c, occ_c)
        ctx.grid = grid
        ctx.precision = precision
        return ex.clone()

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        psi, occ = ctx.saved_tensors
        grid, precision = ctx.grid, ctx.precision
        plan = get_plan(grid, precision, psi.shape[0], psi.device, psi.is_complex())
        need_psi, need_occ = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_psi or need_occ):
            return None, None, None, None
        gbar = g.detach().to(device=psi.device, dtype=torch.float64).contiguous()
        # the library recomputes K psi and scales it (exx_gradient)
        gpsi, gocc = plan.gradient(psi, occ, gbar, want_occ=need_occ)
        return (gpsi if need_psi else None), gocc, None, None


def exchange_energy(psi: torch.Tensor, occ: torch.Tensor, grid: Grid,
                    precision: str = "fp32") -> torch.Tensor:
    """Differentiable E_x (float64 0-dim tensor)."""
    return ExchangeEnergy.apply(psi, occ, grid, precision)
