"""Pins of the oracle's FGPA and mean-flux reduction (CPU)."""
import numpy as np

from oracle import cosmology, fgpa


def test_closed_form_special_values():
    coef = [[0.5, 0.0, 0.0], [1.6, 0.0, 0.0], [1.0, 0.0, 0.0]]
    z = np.full(3, 2.5)
    # g = 0 -> F = exp(-a)
    assert fgpa.flux(np.zeros(3), np.zeros(3), z, coef)[0] == np.exp(-0.5)
    # a = 0 -> F = 1
    coef0 = [[0.0, 0.0, 0.0], [1.6, 0.0, 0.0], [1.0, 0.0, 0.0]]
    assert np.all(fgpa.flux(np.ones(3), np.ones(3), z, coef0) == 1.0)
    # g = delta + c eta: only the sum matters
    np.testing.assert_allclose(fgpa.flux(np.array([0.3]), np.array([0.2]), z[:1], coef),
                               fgpa.flux(np.array([0.5]), np.array([0.0]), z[:1], coef))
    # b = 0 -> F = exp(-a) for any g
    coefb = [[0.7, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]]
    np.testing.assert_allclose(fgpa.flux(np.array([3.0]), np.array([-2.0]), z[:1], coefb), np.exp(-0.7))


def test_monotone_decreasing_in_g():
    coef = [[0.5, 0.0, 0.0], [1.6, 0.0, 0.0], [1.0, 0.0, 0.0]]
    g = np.linspace(-3, 3, 101)
    F = fgpa.flux(g, np.zeros_like(g), np.full_like(g, 2.5), coef)
    assert np.all(np.diff(F) < 0)


def test_quadratic_coefficients():
    coef = [[1.0, 2.0, 3.0], [0.5, 0.0, 0.0], [0.0, 0.0, 1.0]]
    a, b, c = fgpa.coeff_eval(coef, 2.0)    # 1+z = 3
    assert (a, b, c) == (1 + 6 + 27, 0.5, 9.0)


def test_gauss_hermite_mean_flux_vs_sampling():
    rng = np.random.default_rng(3)
    a, b, sig = 0.4, 1.3, 0.8
    g = rng.normal(0, sig, 4_000_000)
    mc = np.mean(np.exp(-a * np.exp(b * g)))
    assert abs(mc - fgpa.gauss_hermite_mean_flux(a, b, sig)) < 5 * 0.3 / np.sqrt(g.size)
    # depends only on (a, b*sigma)
    assert abs(fgpa.gauss_hermite_mean_flux(a, b, sig) - fgpa.gauss_hermite_mean_flux(a, b * 2, sig / 2)) < 1e-15


def test_pixel_chi_and_bins():
    sk = dict(npix=np.array([4, 2]), offset=np.array([2, 0]), chi0=np.array([100.0, 50.0]), dchi=0.5)
    chi = fgpa.pixel_chi(sk)
    np.testing.assert_array_equal(chi, [50.0, 49.5, 100.0, 99.5, 99.0, 98.5])
    edges = np.array([49.5, 50.0, 99.0, 100.0])
    F = np.arange(6, dtype=np.float64)
    s, c = fgpa.mean_flux_bins(F, chi, edges)
    # bin0: [49.5, 50) -> 49.5 ; bin1: [50, 99) -> 50.0, 98.5 ; bin2: [99,100) -> 99.5, 99.0 ; 100.0 out
    np.testing.assert_array_equal(c, [1, 2, 2])
    np.testing.assert_array_equal(s, [1.0, 0.0 + 5.0, 3.0 + 4.0])


def test_apply_fgpa_uses_pixel_redshift():
    sk = dict(npix=np.array([3]), offset=np.array([0]), chi0=np.array([cosmology.chi_of_z(2.5)]), dchi=0.2)
    coef = [[0.0, 0.1, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]]   # a = 0.1 (1+z)
    F, z = fgpa.apply_fgpa(np.zeros(3), np.zeros(3), sk, coef)
    assert abs(z[0] - 2.5) < 1e-12 and z[1] < z[0]
    np.testing.assert_allclose(F, np.exp(-0.1 * (1 + z)), rtol=1e-15)
