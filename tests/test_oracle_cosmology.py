"""Pins of the oracle's distance-redshift relation (CPU)."""
import numpy as np
from scipy import integrate

from oracle import cosmology as cz


def test_einstein_de_sitter_closed_form():
    z = np.array([0.0, 0.5, 1.8, 2.5, 3.6, 5.0])
    exact = 2.0 * cz.C_OVER_H0 * (1.0 - 1.0 / np.sqrt(1.0 + z))
    np.testing.assert_allclose(cz.chi_of_z(z, omega_m=1.0), exact, rtol=1e-13, atol=1e-10)


def test_pure_lambda_closed_form():
    z = np.array([0.1, 1.0, 3.0])
    np.testing.assert_allclose(cz.chi_of_z(z, omega_m=0.0), cz.C_OVER_H0 * z, rtol=1e-14)


def test_against_scipy_quad():
    for z in (1.6, 1.8, 2.5, 3.6, 3.8):
        ref = cz.C_OVER_H0 * integrate.quad(lambda t: 1.0 / np.sqrt(
            0.3147 * (1 + t) ** 3 + 0.6853), 0.0, z, epsabs=0, epsrel=1e-13)[0]
        assert abs(cz.chi_of_z(z) - ref) < 1e-9 * ref


def test_inverse_roundtrip():
    z = np.linspace(0.01, 4.5, 301)
    np.testing.assert_allclose(cz.z_of_chi(cz.chi_of_z(z)), z, rtol=1e-12, atol=1e-13)


def test_forest_distance_scale():
    # order-of-magnitude anchors for the workload geometry (Mpc/h)
    assert 3300 < cz.chi_of_z(1.8) < 3450
    assert 4650 < cz.chi_of_z(3.6) < 4850


def test_velocity_conversion():
    # dv/dchi = H(z)/(1+z) in km/s per Mpc/h; at z=0 it is 100 (H0 = 100 h)
    assert abs(cz.dv_per_dchi(0.0) - 100.0) < 1e-12
    z = 2.5
    assert abs(cz.dv_per_dchi(z) - 100 * np.sqrt(0.3147 * 3.5 ** 3 + 0.6853) / 3.5) < 1e-10
