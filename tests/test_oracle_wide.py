"""Pins of the oracle's wide-angle line-of-sight velocity gradient
(eta_par = u_p u_q eta^{pq}, section "Mock generation" after eq:eta)."""
import numpy as np
import pytest

from oracle import field, power, skewers

PK = power.PowerSpectrum()


def _grids(n, seed, f, **kw):
    tab = power.amplitude_table(PK, n, 2.19)
    a = field.make_box(n, seed, tab, ("delta", "zz"), f=f, **kw)
    b = field.make_box(n, seed, tab, ("xx", "yy"), f=f, **kw)
    c = field.make_box(n, seed, tab, ("xy", "xz"), f=f, **kw)
    d = field.make_box(n, seed, tab, ("yz",), f=f, **kw)
    delta = a.real
    eta6 = [b.real, b.imag, a.imag, c.real, c.imag, d.real]
    return delta, eta6


def test_trace_is_f_delta():
    # sum_p k_p^2 / k^2 = 1 for every mode: eta_xx + eta_yy + eta_zz = f delta
    n, f = 16, 0.8
    delta, eta6 = _grids(n, 3, f)
    np.testing.assert_allclose(eta6[0] + eta6[1] + eta6[2], f * delta, atol=1e-12 * np.abs(delta).max())


def test_single_shell_closed_form():
    # only |n|^2 = 1 kept: the six modes +-x, +-y, +-z are plane waves along
    # the axes, eta_pq is diagonal (k_p k_q = 0 for p != q), so
    # eta_par = f (u_x^2 delta_x + u_y^2 delta_y + u_z^2 delta_z) for any u
    n, f, seed = 16, 0.7, 8
    tab = power.amplitude_table(PK, n, 2.19)
    delta, eta6 = _grids(n, seed, f, only_n2=1)
    w = field.white_noise(n, seed)
    m = np.arange(n)
    ph = np.exp(2j * np.pi * m / n)
    dx = 2 * tab[1] * np.real(w[1, 0, 0] * ph)[:, None, None] + 0 * delta
    dy = 2 * tab[1] * np.real(w[0, 1, 0] * ph)[None, :, None] + 0 * delta
    dz = 2 * tab[1] * np.real(w[0, 0, 1] * ph)[None, None, :] + 0 * delta
    for u in ([0.0, 0.0, 1.0], [0.6, 0.0, 0.8], [1 / np.sqrt(3)] * 3, [0.2, -0.5, np.sqrt(1 - 0.29)]):
        u = np.asarray(u)
        got = skewers.eta_par_from_components(eta6, u)
        want = f * (u[0] ** 2 * dx + u[1] ** 2 * dy + u[2] ** 2 * dz)
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_rotation_of_the_line_of_sight():
    # u along x gives eta_xx; u in the x-y diagonal gives (xx + yy)/2 + xy
    n = 16
    delta, eta6 = _grids(n, 5, 1.0)
    np.testing.assert_allclose(skewers.eta_par_from_components(eta6, np.array([1.0, 0, 0])), eta6[0], atol=1e-14)
    diag = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    np.testing.assert_allclose(skewers.eta_par_from_components(eta6, diag),
                               0.5 * (eta6[0] + eta6[1]) + eta6[3], atol=1e-13)


def test_fixed_amplitude_variance_of_eta_par():
    # with |W| = 1 the grid mean of eta_par^2 is sum_k |m(k)|^2 s(n^2)^2, where
    # m(k) = f (k.u)^2/k^2 (a Nyquist component drops the cross terms that
    # involve it): Parseval for the combined field, whatever the phases
    n, f = 16, 0.9
    tab = power.amplitude_table(PK, n, 2.19)
    delta, eta6 = _grids(n, 2, f, fixed_amp=True)
    u = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])
    e = skewers.eta_par_from_components(eta6, u)
    v = np.fft.fftfreq(n, 1.0 / n)
    nx, ny, nz = np.meshgrid(v, v, v, indexing="ij")
    n2 = nx ** 2 + ny ** 2 + nz ** 2
    nyq = -(n // 2)
    cross = 0.0
    for (pa, pb, up) in ((nx, ny, u[0] * u[1]), (nx, nz, u[0] * u[2]), (ny, nz, u[1] * u[2])):
        cross = cross + 2 * up * np.where((pa == nyq) | (pb == nyq), 0.0, pa * pb)
    num = u[0] ** 2 * nx ** 2 + u[1] ** 2 * ny ** 2 + u[2] ** 2 * nz ** 2 + cross
    mult = f * np.where(n2 > 0, num / np.where(n2 > 0, n2, 1), 0.0)
    s = tab[n2.astype(np.int64)]
    np.testing.assert_allclose(np.mean(e ** 2), np.sum((mult * s) ** 2), rtol=1e-10)


def test_draw_skewers_wide_reduces_to_the_axis_boxes():
    # a skewer along z reproduces draw_skewers on {delta, eta_zz}; along x it
    # interpolates eta_xx
    n = 16
    delta, eta6 = _grids(n, 7, 1.0)
    two32 = 2 ** 32
    sk = dict(origin_fx=np.array([[int(1.25 * two32), int(3.5 * two32), int(0.75 * two32)],
                                  [int(2.5 * two32), int(7.125 * two32), int(5.0 * two32)]], dtype=np.int64),
              step_fx=np.array([[0, 0, int(0.3 * two32)], [int(-0.4 * two32), 0, 0]], dtype=np.int64),
              npix=np.array([40, 33], dtype=np.int32), offset=np.array([0, 40], dtype=np.int64), id_base=0)
    d_w, e_w = skewers.draw_skewers_wide(delta, eta6, sk, 1, ps_amp=0.5)
    d_z, e_z = skewers.draw_skewers(delta, eta6[2], sk, 1, ps_amp=0.5)
    np.testing.assert_allclose(d_w, d_z, atol=1e-13)
    np.testing.assert_allclose(e_w[:40], e_z[:40], atol=1e-13)
    _, e_x = skewers.draw_skewers(delta, eta6[0], sk, 1)
    np.testing.assert_allclose(e_w[40:], e_x[40:], atol=1e-13)
