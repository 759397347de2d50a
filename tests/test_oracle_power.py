"""Pins of the oracle's P(k), sigma8 normalisation and amplitude table (CPU)."""
import numpy as np
from scipy import integrate

from oracle import power


def test_bbks_small_q_expansion():
    # T(q) = 1 - (2.34/2 + 3.89/4) q + c2 q^2 + ..., with (derived by hand)
    # c2 = 2.34^2/3 - 16.1^2/4 + 5*3.89^2/32 + (2.34/2)(3.89/4)
    c1 = 2.34 / 2 + 3.89 / 4
    c2 = 2.34 ** 2 / 3 - 16.1 ** 2 / 4 + 5 * 3.89 ** 2 / 32 + (2.34 / 2) * (3.89 / 4)
    for q in (1e-5, 3e-5):
        t = power.t_bbks(q)
        assert abs((1.0 - t) / q - c1) < 2e-3 * c1 + 1e-9
        est_c2 = (t - 1.0 + c1 * q) / q ** 2
        assert abs(est_c2 - c2) < 0.02 * abs(c2)


def test_bbks_large_q_asymptote():
    q = 1e6
    t = power.t_bbks(q)
    lead = np.log1p(2.34 * q) / (2.34 * q) / (6.71 * q)
    assert abs(t / lead - 1.0) < 1e-6


def test_tophat_white_noise_variance():
    # white noise P = 1: sigma_R^2 = 1 / V_sphere = 3 / (4 pi R^3)
    for r in (8.0, 20.0):
        got = power.sigma_r2(lambda k: np.ones_like(k), r)
        assert abs(got / (3.0 / (4.0 * np.pi * r ** 3)) - 1.0) < 3e-4


def test_sigma8_against_quad():
    pk = power.PowerSpectrum()
    f = lambda lnk: (np.exp(lnk) ** 3 * pk(np.exp(lnk))
                     * power.w_tophat(8.0 * np.exp(lnk)) ** 2)
    pts = np.log(np.logspace(-5, 3, 400))
    val = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-12, limit=200)[0]
              for a, b in zip(pts[:-1], pts[1:]))
    s8 = np.sqrt(val / (2 * np.pi ** 2))
    assert abs(s8 - 0.8) < 1e-9


def test_power_law_slope_at_small_k():
    pk = power.PowerSpectrum()
    k1, k2 = 1e-5, 2e-5
    slope = np.log(pk(k2) / pk(k1)) / np.log(2.0)
    assert abs(slope - 0.96) < 1e-3


def test_tophat_series_matches_closed_form():
    x = np.array([0.009, 0.011, 0.5, 3.0])
    closed = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    np.testing.assert_allclose(power.w_tophat(x), closed, rtol=1e-9)


def test_amplitude_table():
    pk = power.PowerSpectrum()
    n, dx = 16, 2.19
    tab = power.amplitude_table(pk, n, dx)
    assert tab.shape == (3 * 64 + 1,)
    assert tab[0] == 0.0
    L = n * dx
    k = 2 * np.pi * np.sqrt(5.0) / L
    assert abs(tab[5] - np.sqrt(pk(k) / L ** 3)) < 1e-15 * tab[5] * 10
    sm = power.amplitude_table(pk, n, dx, smooth=dx)
    assert abs(sm[5] / tab[5] - np.exp(-0.5 * (k * dx) ** 2)) < 1e-14


def test_tabulated_power_nodes_and_power_laws():
    k = np.geomspace(1e-3, 10.0, 40)
    pk = power.PowerSpectrum()
    tab = power.TabulatedPower(k, pk(k))
    np.testing.assert_allclose(tab(k), pk(k), rtol=1e-13)           # exact at the nodes
    # a pure power law is a straight line in log-log: reproduced everywhere,
    # extrapolation included
    law = power.TabulatedPower(k, 3.0 * k ** -1.7)
    kk = np.geomspace(1e-5, 1e3, 101)
    np.testing.assert_allclose(law(kk), 3.0 * kk ** -1.7, rtol=1e-12)


def test_dense_table_reproduces_the_analytic_amplitudes():
    pk = power.PowerSpectrum()
    k = np.geomspace(1e-4, 1e2, 20000)
    tab = power.TabulatedPower(k, pk(k))
    a = power.amplitude_table(pk, 64, 2.19)
    b = power.amplitude_table(tab, 64, 2.19)
    np.testing.assert_allclose(b[1:], a[1:], rtol=2e-6)
