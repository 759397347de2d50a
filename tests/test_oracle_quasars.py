"""Pins of the oracle's lognormal quasar field (section "Quasar generation",
Appendix A)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import cosmology, power, quasars

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def test_bias_and_alpha():
    np.testing.assert_allclose(quasars.bias_qso(2.33), 3.7, rtol=1e-14)
    np.testing.assert_allclose(quasars.alpha_of_z(2.75, 2.75), 1.0, rtol=1e-14)
    # Appendix A: alpha = b_q(z)(1+z0) / (b_q(z0)(1+z))
    np.testing.assert_allclose(quasars.alpha_of_z(3.6, 1.9),
                               3.7 * (4.6 / 3.33) ** 1.7 * 2.9 / (3.7 * (2.9 / 3.33) ** 1.7 * 4.6), rtol=1e-14)


def test_growth_limits():
    # Einstein-de Sitter: G = 1/(1+z) exactly
    for z in (0.5, 2.0, 3.6):
        np.testing.assert_allclose(quasars.growth(z, omega_m=1.0), 1.0 / (1.0 + z), rtol=1e-10)
    g = quasars.growth(2.5)
    assert 1.0 / 3.5 < g < 0.4     # LCDM grows less than EdS since z = 2.5


def test_xi_of_a_gaussian_spectrum():
    # P(k) = A exp(-k^2 c^2) with smoothing s: the pair of a 3D Gaussian,
    # xi(r) = A / (8 pi^(3/2) w^3) exp(-r^2 / (4 w^2)), w^2 = c^2 + s^2
    A, c, s = 3.0e3, 4.0, 2.19
    pk = lambda k: A * np.exp(-(k * c) ** 2)
    r = np.array([0.0, 1.0, 5.0, 12.0, 30.0])
    w2 = c * c + s * s
    want = A / (8.0 * np.pi ** 1.5 * w2 ** 1.5) * np.exp(-r * r / (4.0 * w2))
    np.testing.assert_allclose(quasars.xi_of_r(pk, r, s), want, rtol=1e-9, atol=1e-14)


def test_lognormal_spectrum_linear_limit():
    # small b0: ln(1 + b0^2 xi) -> b0^2 xi, so P_q -> b0^2 P exp(-k^2 s^2)
    pk = power.PowerSpectrum()
    b0, s = 1e-3, 2.19
    k = np.array([0.01, 0.05, 0.2, 0.5])
    with np.errstate(all="ignore"):
        pq = quasars.lognormal_pk(pk, b0, s, k, rmax=800.0, nr=801)
    np.testing.assert_allclose(pq, b0 * b0 * pk(k) * np.exp(-(k * s) ** 2), rtol=2e-3)


def test_draw_decisions_and_positions():
    rng = np.random.default_rng(4)
    n, dx, z0 = 8, 40.0, 2.5
    dq = rng.normal(scale=0.5, size=(n, n, n))
    obs = np.array([n * dx / 2, n * dx / 2, -cosmology.chi_of_z(2.4)])
    zt = np.array([1.5, 2.5, 4.0])
    nb = np.array([2e-6, 5e-6, 1e-6])
    idx, fx, p, u, s2 = quasars.draw(dq, dx, obs, z0, zt, nb, 11)
    np.testing.assert_allclose(s2, np.mean(dq ** 2))
    # brute force on a few voxels, written out
    for lin in (0, 77, 300, 511):
        ix, iy, iz = lin // (n * n), (lin // n) % n, lin % n
        chi = np.sqrt((ix * dx - obs[0]) ** 2 + (iy * dx - obs[1]) ** 2 + (iz * dx - obs[2]) ** 2)
        z = cosmology.z_of_chi(np.array([chi]))[0]
        al = quasars.bias_qso(z) * (1 + z0) / (quasars.bias_qso(z0) * (1 + z))
        want = min(np.interp(z, zt, nb) * dx ** 3 * np.exp(al * dq[ix, iy, iz] - al * al * s2 / 2), 1.0)
        np.testing.assert_allclose(p[lin], want, rtol=1e-12)
    np.testing.assert_array_equal(idx, np.flatnonzero(u < p))
    cells = fx >> 32
    frac = fx - (cells << 32)
    # positions inside their voxel [m - 1/2, m + 1/2)
    centre = np.stack([idx // (n * n), (idx // n) % n, idx % n], axis=1)
    off = (fx - (centre << 32)).astype(np.float64) / 2 ** 32
    assert np.all(off >= -0.5) and np.all(off < 0.5)
    assert np.all((frac >= 0) & (frac < 2 ** 32))


def test_draw_mean_count():
    # with alpha delta_q normalised, the expected count is sum nbar dx^3
    rng = np.random.default_rng(5)
    n, dx, z0 = 16, 20.0, 2.5
    dq = rng.normal(scale=0.3, size=(n, n, n))
    obs = np.array([n * dx / 2, n * dx / 2, -cosmology.chi_of_z(2.49)])
    zt, nb = np.array([0.0, 10.0]), np.array([0.02 / dx ** 3, 0.02 / dx ** 3])
    counts = [len(quasars.draw(dq, dx, obs, z0, zt, nb, s)[0]) for s in range(6)]
    mean = np.mean(counts)
    expect = 0.02 * n ** 3 * np.mean(np.exp(quasars.alpha_of_z(2.5, z0) * dq - 0.5 * np.mean(dq ** 2)))
    assert abs(mean - expect) < 4 * np.sqrt(expect / 6) + 3
