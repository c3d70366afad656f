"""MI355X exact-exchange operator (arXiv:1712.07973, Section 2) over libexx.so.

``energy_and_kpsi`` returns E_x and K psi; ``exchange_energy`` is the
differentiable E_x (autograd backward = recomputed K psi); ``Plan`` exposes
the C ABI (precisions 'fp32', 'fp64_plain', 'fp64_fused', tuning, autotune);
``Batch`` evaluates many independent systems in one captured HIP graph.
"""
from ._lib import ExxError
from .api import Grid, Plan, energy_and_kpsi, get_plan, library_version
from .autograd import ExchangeEnergy, exchange_energy
from .batch import Batch

__all__ = ["Grid", "Plan", "Batch", "energy_and_kpsi", "exchange_energy", "ExchangeEnergy",
           "ExxError", "get_plan", "library_version"]
