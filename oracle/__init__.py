"""FP64 CPU oracle (test infrastructure only; never on the product path)."""
from .exx_oracle import (FREE, PERIODIC, brute_force_potential, co_density, default_radius,
                         embed, exx, exx_grad_occ, exx_grad_psi, fft_size, kernel_hat,
                         kpsi_rows, pair_energies, pair_energy, realspace_kernel,
                         solve_poisson, wavevector_sq)

__all__ = [
    "FREE", "PERIODIC", "brute_force_potential", "co_density", "default_radius", "embed", "exx",
    "exx_grad_occ", "exx_grad_psi", "fft_size", "kernel_hat", "kpsi_rows", "pair_energies",
    "pair_energy", "realspace_kernel", "solve_poisson", "wavevector_sq",
]
