"""Pins of the oracle's Gaussian box (CPU)."""
import numpy as np
import pytest

from oracle import field, lines, power

PK = power.PowerSpectrum()


def _table(n, dx=2.19, smooth=0.0):
    return power.amplitude_table(PK, n, dx, smooth)


def test_hermitian_noise():
    n = 8
    w = field.white_noise(n, 77)
    idx = np.arange(n)
    neg = (-idx) % n
    np.testing.assert_array_equal(w, np.conj(w[np.ix_(neg, neg, neg)]))
    # self-conjugate modes are real and distinct modes are not all real
    for i in [(0, 0, 0), (4, 0, 4), (4, 4, 4), (0, 4, 0)]:
        assert w[i].imag == 0.0
    assert np.mean(np.abs(w.imag) > 0) > 0.9


def test_noise_unit_variance():
    w = field.white_noise(32, 5)
    assert abs(np.mean(np.abs(w) ** 2) - 1.0) < 0.02


def test_brute_force_dft():
    n = 8
    tab = _table(n)
    x = field.spectrum(n, 3, tab, ("delta", "zz"))
    np.testing.assert_allclose(field.inverse_dft3(x), field.brute_force_field(n, x),
                               rtol=0, atol=1e-12 * np.abs(x).sum())


def test_fields_are_real():
    n = 16
    tab = _table(n)
    for comp in field.COMPONENTS:
        x = field.spectrum(n, 9, tab, (comp,), box_len=40.0)
        v = field.inverse_dft3(x)
        assert np.max(np.abs(v.imag)) <= 1e-12 * max(np.max(np.abs(v.real)), 1e-300)


def test_fixed_amplitude_variance_equals_power_sum():
    # |W| = 1: mean(delta^2) over the grid = sum_k s(n^2)^2 = sum P/V_box exactly
    n = 32
    tab = _table(n)
    box = field.make_box(n, 21, tab, ("delta",), fixed_amp=True)
    s = field.amplitudes(n, tab)
    np.testing.assert_allclose(np.mean(box.real ** 2), np.sum(s ** 2), rtol=1e-12)


def test_parseval_per_realisation():
    n = 16
    tab = _table(n)
    x = field.spectrum(n, 4, tab, ("delta", "zz"))
    box = field.inverse_dft3(x)
    np.testing.assert_allclose(np.sum(np.abs(box) ** 2), n ** 3 * np.sum(np.abs(x) ** 2), rtol=1e-12)


def test_single_shell_is_three_plane_waves():
    # keep only n^2 = 1: delta = sum of the +-x, +-y, +-z modes, eta_par only
    # the z pair, scaled by f mu_z^2 = f
    n, f = 16, 0.7
    tab = _table(n)
    box = field.make_box(n, 8, tab, ("delta", "zz"), f=f, only_n2=1)
    w = field.white_noise(n, 8)
    s1 = tab[1]
    m = np.arange(n)
    ph = np.exp(2j * np.pi * m / n)
    wx, wy, wz = w[1, 0, 0], w[0, 1, 0], w[0, 0, 1]
    ex = 2 * s1 * np.real(wx * ph)[:, None, None]
    ey = 2 * s1 * np.real(wy * ph)[None, :, None]
    ez = 2 * s1 * np.real(wz * ph)[None, None, :]
    np.testing.assert_allclose(box.real, ex + ey + ez + 0 * box.real, atol=1e-13)
    np.testing.assert_allclose(box.imag, f * ez + 0 * box.imag, atol=1e-13)


def test_eta_is_f_mu2_delta_in_k_space():
    n, f = 16, 0.9
    tab = _table(n)
    box = field.make_box(n, 12, tab, ("delta", "zz"), f=f)
    dk = np.fft.fftn(box.real)
    ek = np.fft.fftn(box.imag)
    nz = field.signed_freq(np.arange(n), n)
    g = np.meshgrid(nz, nz, nz, indexing="ij")
    n2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    mu2 = np.where(n2 > 0, g[2] ** 2 / np.where(n2 > 0, n2, 1), 0)
    np.testing.assert_allclose(ek, f * mu2 * dk, atol=1e-10 * np.abs(dk).max())


def test_power_recovered_by_forward_fft():
    # |FFT(delta)|^2 / N^6 * V_box = P(k) |W|^2 exactly; shell mean over seeds -> P(k)
    n, dx = 32, 2.19
    tab = _table(n, dx)
    L = n * dx
    acc = np.zeros(3 * (n // 2) ** 2 + 1)
    cnt = np.zeros_like(acc)
    for seed in range(6):
        box = field.make_box(n, 100 + seed, tab, ("delta",))
        pk_hat = np.abs(np.fft.fftn(box.real)) ** 2 / n ** 6 * L ** 3
        w = field.white_noise(n, 100 + seed)
        nn = field.signed_freq(np.arange(n), n)
        g = np.meshgrid(nn, nn, nn, indexing="ij")
        n2 = (g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
        k = 2 * np.pi * np.sqrt(n2) / L
        exact = np.where(n2 > 0, PK(np.where(n2 > 0, k, 1.0)) * np.abs(w) ** 2, 0)
        np.testing.assert_allclose(pk_hat, exact, rtol=1e-9, atol=1e-12 * exact.max())
        np.add.at(acc, n2.ravel(), pk_hat.ravel())
        np.add.at(cnt, n2.ravel(), 1)
    sel = (cnt > 500)
    n2v = np.nonzero(sel)[0]
    ratio = acc[sel] / cnt[sel] / PK(2 * np.pi * np.sqrt(n2v) / L)
    assert np.all(np.abs(ratio - 1) < 5 / np.sqrt(cnt[sel] / 2))


def test_c_lines_match_numpy_box():
    n = 16
    tab = _table(n)
    for comps, fixed in ((("delta", "zz"), False), (("xy", "yz"), True), (("xx",), False)):
        box = field.make_box(n, 31, tab, comps, f=0.8, fixed_amp=fixed)
        cols = [(0, 0), (3, 7), (8, 8), (15, 1)]
        re, im = lines.field_lines(n, 31, tab, cols, comps, f=0.8, fixed_amp=fixed, nthreads=2)
        for l, (mx, my) in enumerate(cols):
            np.testing.assert_allclose(re[l] + 1j * im[l], box[mx, my, :],
                                       atol=1e-11 * np.abs(box).max())


def test_c_lines_only_shell():
    n = 16
    tab = _table(n)
    box = field.make_box(n, 2, tab, ("delta", "zz"), only_n2=1)
    re, im = lines.field_lines(n, 2, tab, [(5, 6)], only_n2=1, nthreads=1)
    np.testing.assert_allclose(re[0] + 1j * im[0], box[5, 6], atol=1e-12)


@pytest.mark.parametrize("n,s2", [(16, 1), (16, 6), (32, 27), (32, 50)])
def test_shell_direct_sum_matches_box(n, s2):
    # the single-shell evaluator (a direct sum over the shell's modes at any
    # voxel) reproduces the FFT box with only that shell kept
    tab = _table(n)
    box = field.make_box(n, 9, tab, ("delta", "zz"), f=0.8, only_n2=s2)
    freqs, coef = field.shell_modes(n, 9, tab, s2, f=0.8)
    assert len(freqs) > 0
    ix, iy, iz = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    got = field.shell_field_at(n, freqs, coef, ix, iy, iz, chunk=999)
    np.testing.assert_allclose(got, box, atol=1e-12 * np.abs(box).max())


def test_velocity_continuity_and_reality():
    # eq:velocity: v_hat = i f aH k / k^2 delta_hat, so i k . v_hat = -f aH delta_hat
    # (linear continuity), checked on the forward FFT of the real-space boxes
    n, dx, f = 16, 5.0, 0.7
    L = n * dx
    tab = power.amplitude_table(power.PowerSpectrum(), n, dx)
    vxy = field.make_box(n, 3, tab, ("vx", "vy"), f=f, box_len=L)
    vz = field.make_box(n, 3, tab, ("vz",), f=f, box_len=L)
    delta = field.make_box(n, 3, tab, ("delta",)).real
    assert np.max(np.abs(vz.imag)) < 1e-9 * np.max(np.abs(vz.real))   # a real field
    k1 = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    kx, ky, kz = np.meshgrid(k1, k1, k1, indexing="ij")
    div = 1j * (kx * np.fft.fftn(vxy.real) + ky * np.fft.fftn(vxy.imag) + kz * np.fft.fftn(vz.real))
    want = -f * 100.0 * np.fft.fftn(delta)
    nyq = (np.abs(np.fft.fftfreq(n) * n) == n // 2)
    off = ~(nyq[:, None, None] | nyq[None, :, None] | nyq[None, None, :])
    np.testing.assert_allclose(div[off], want[off], rtol=0, atol=1e-9 * np.abs(want).max())
    # the Nyquist plane of v_j carries nothing
    vx_hat = np.fft.fftn(vxy.real)
    assert np.max(np.abs(vx_hat[n // 2])) < 1e-9 * np.abs(vx_hat).max()


@pytest.mark.parametrize("n,s2", [(16, 6), (32, 27)])
def test_shell_direct_sum_of_velocities(n, s2):
    tab = _table(n)
    box = field.make_box(n, 9, tab, ("vx", "vy"), f=1.0, only_n2=s2, box_len=40.0)
    freqs, coef = field.shell_modes(n, 9, tab, s2, comps=("vx", "vy"), f=1.0, box_len=40.0)
    ix, iy, iz = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    got = field.shell_field_at(n, freqs, coef, ix, iy, iz, chunk=999)
    np.testing.assert_allclose(got, box, atol=1e-12 * np.abs(box).max())
