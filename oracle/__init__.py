"""FP64 CPU oracle (test infrastructure only; never on the product path)."""
from .exx_oracle import (FREE, PERIODIC, SURFACE, WIRE, brute_force_potential, co_density,
                         default_radius, embed, exx, exx_grad_occ, exx_grad_psi, fft_shape,
                         fft_size, kernel_hat, kpsi_rows, pair_energies, pair_energy,
                         realspace_kernel, solve_poisson, surface_kernel, wavevector_components,
                         wavevector_sq, wire_kernel)

__all__ = [
    "FREE", "PERIODIC", "SURFACE", "WIRE", "brute_force_potential", "co_density", "default_radius",
    "embed", "exx", "exx_grad_occ", "exx_grad_psi", "fft_shape", "fft_size", "kernel_hat",
    "kpsi_rows", "pair_energies", "pair_energy", "realspace_kernel", "solve_poisson",
    "surface_kernel", "wavevector_components", "wavevector_sq", "wire_kernel",
]
