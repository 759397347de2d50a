"""Pins of the oracle's 1D power spectrum (CPU)."""
import numpy as np

from oracle import cosmology, p1d


def _sk(npix, chi0=4000.0, dchi=0.2):
    npix = np.asarray(npix)
    off = np.concatenate([[0], np.cumsum(npix[:-1])]).astype(np.int64)
    return dict(npix=npix, offset=off, chi0=np.full(len(npix), chi0), dchi=dchi)


def test_single_cosine():
    n, m0, A, fbar = 256, 17, 0.3, 0.7
    j = np.arange(n)
    F = fbar * (1 + A * np.cos(2 * np.pi * m0 * j / n))
    sk = _sk([n + 40])          # prefix of 256 pixels is used
    F = np.concatenate([F, np.full(40, 5.0)])
    dv = p1d.dv_pixel(2.5, 0.2)
    k_edges = np.array([1e-6, 1.0])
    ps, cnt = p1d.p1d(F, sk, [0.0, 1e5], [fbar], k_edges, 2.5, 0.2)
    assert cnt[0] == n // 2
    np.testing.assert_allclose(ps[0], dv * A ** 2 * n / 4, rtol=1e-12)
    # only the mode m0 carries power: a bin around k_m0 alone
    k0 = 2 * np.pi * m0 / (n * dv)
    ps, cnt = p1d.p1d(F, sk, [0.0, 1e5], [fbar], [k0 * 0.999, k0 * 1.001], 2.5, 0.2)
    assert cnt[0] == 1
    np.testing.assert_allclose(ps[0], dv * A ** 2 * n / 4, rtol=1e-12)


def test_parseval_all_modes():
    rng = np.random.default_rng(0)
    n = 512
    d = rng.normal(size=n)
    d -= d.mean()
    F = 0.6 * (1 + d)
    ps, cnt = p1d.p1d(F, _sk([n]), [0.0, 1e5], [0.6], [1e-9, 1e9], 3.0, 0.2)
    dv = p1d.dv_pixel(3.0, 0.2)
    X = np.fft.rfft(d)
    # sum_{m=1}^{N/2} |X_m|^2 = (N sum d^2 - |X_0|^2 + |X_{N/2}|^2) / 2
    expect = dv / n * (n * np.sum(d ** 2) - abs(X[0]) ** 2 + abs(X[-1]) ** 2) / 2
    np.testing.assert_allclose(ps[0], expect, rtol=1e-12)
    assert cnt[0] == n // 2


def test_white_noise_level():
    rng = np.random.default_rng(1)
    n, S = 256, 400
    d = rng.normal(0, 0.5, (S, n))
    F = (0.8 * (1 + d)).ravel()
    edges = p1d.log_k_edges(8, 0.01, 0.1)
    ps, cnt = p1d.p1d(F, _sk([n] * S), [0.0, 1e5], [0.8], edges, 2.2, 0.2)
    dv = p1d.dv_pixel(2.2, 0.2)
    mean = ps[cnt > 0] / cnt[cnt > 0]
    assert np.all(np.abs(mean / (dv * 0.25) - 1) < 5 / np.sqrt(cnt[cnt > 0]))


def test_velocity_units_and_edges():
    e = p1d.log_k_edges(32)
    assert abs(e[0] - 0.001) < 1e-15 and abs(e[-1] - 0.05) < 1e-15 and len(e) == 33
    assert abs(p1d.dv_pixel(2.5, 0.2) - 0.2 * 100 * cosmology.hubble_e(2.5) / 3.5) < 1e-12


def test_per_bin_mean_flux_and_short_skewers():
    # pixels in two distance bins with different Fbar: delta_F uses its own bin
    n = 64
    sk = _sk([n, 1, 3], chi0=1000.0, dchi=1.0)
    F = np.concatenate([np.where(np.arange(n) < 32, 0.5, 0.25), [1.0], [0.5, 0.5, 0.3]])
    edges = [900.0, 968.5, 1100.0]    # pixels 0..31 at chi >= 969 -> bin 1
    ps, cnt = p1d.p1d(F, sk, edges, [0.25, 0.5], [1e-9, 1e9], 2.5, 1.0)
    np.testing.assert_allclose(ps[0], 0.0, atol=1e-20)   # delta_F == 0 everywhere
    assert cnt[0] == n // 2 + 1                            # 1-pixel skewer adds nothing, 3 -> 2 pixels
