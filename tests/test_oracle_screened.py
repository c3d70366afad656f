"""Pins of the oracle's screened (erfc(omega r)/r) kernel, the short-range
kernel of screened hybrids (only the Poisson filter changes, Section 3.2.3)."""
import math

import numpy as np
import pytest

import closed_forms as cf
import oracle


def _periodic_gaussian(n, h, P, c):
    L = n * h
    rho = np.zeros((n, n, n))
    for tx in (-1, 0, 1):
        for ty in (-1, 0, 1):
            for tz in (-1, 0, 1):
                rho += cf.normalised_gaussian(n, h, P + L * np.array([tx, ty, tz]), c)
    return rho


@pytest.mark.parametrize("omega", [0.3, 0.8])
def test_screened_pair_energy_reciprocal_sum(omega):
    n, h, c = 32, 0.4, 1.1
    rho = _periodic_gaussian(n, h, np.array([3.0, 7.1, 9.4]), c)
    V = oracle.solve_poisson(rho, h, "periodic", omega=omega)
    e = oracle.pair_energy(rho, V, h)
    assert e == pytest.approx(cf.periodic_screened_pair_energy(1.0, c, n * h, omega, 40), rel=1e-11)


def test_screened_tends_to_free_space_for_short_range():
    # omega = 1.2: erfc(omega L/2)/(L/2) ~ 1e-15, so periodic images do not matter
    n, h, c, omega = 32, 0.4, 1.0, 1.2
    rho = _periodic_gaussian(n, h, np.array([6.4, 6.4, 6.4]), c)
    e = oracle.pair_energy(rho, oracle.solve_poisson(rho, h, "periodic", omega=omega), h)
    assert e == pytest.approx(cf.screened_self_energy_normalised(c, omega), rel=1e-10)


def test_screened_kernel_limits():
    K = oracle.kernel_hat(16, 0.5, "periodic", omega=0.7)
    assert K[0, 0, 0] == pytest.approx(math.pi / 0.49, rel=1e-15)
    Kc = oracle.kernel_hat(16, 0.5, "periodic")
    G2 = oracle.wavevector_sq(16, 0.5)
    # screened = Coulomb * (1 - exp(-G^2/4w^2)) away from G = 0
    nz = G2 > 0
    assert np.allclose(K[nz], Kc[nz] * (1 - np.exp(-G2[nz] / (4 * 0.49))), rtol=1e-14)
