"""Pins of the oracle's line-of-sight stage (CPU)."""
import numpy as np

from oracle import field, power, skewers

T32 = 2 ** 32


def _fx(cells):
    return np.round(np.asarray(cells, dtype=np.float64) * T32).astype(np.int64)


def test_trilinear_reproduces_multilinear_fields():
    n = 16
    m = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(m, m, m, indexing="ij")
    grid = 0.3 + 1.1 * X - 0.7 * Y + 0.25 * Z + 0.05 * X * Y - 0.02 * Y * Z + 0.01 * X * Y * Z
    rng = np.random.default_rng(0)
    p = rng.uniform(0.0, n - 1.0, (200, 3))
    pos = _fx(p)
    x = pos.astype(np.float64) / T32   # exact positions used by the oracle
    ref = (0.3 + 1.1 * x[:, 0] - 0.7 * x[:, 1] + 0.25 * x[:, 2] + 0.05 * x[:, 0] * x[:, 1]
           - 0.02 * x[:, 1] * x[:, 2] + 0.01 * x[:, 0] * x[:, 1] * x[:, 2])
    np.testing.assert_allclose(skewers.trilinear(grid, pos), ref, rtol=0, atol=1e-12)


def test_grid_points_and_periodic_wrap():
    n = 8
    rng = np.random.default_rng(1)
    grid = rng.normal(size=(n, n, n))
    idx = rng.integers(0, n, (50, 3))
    pos = idx.astype(np.int64) * T32
    np.testing.assert_array_equal(skewers.trilinear(grid, pos), grid[idx[:, 0], idx[:, 1], idx[:, 2]])
    # shifting by whole periods (positive or negative) changes nothing
    frac = _fx(rng.uniform(0, n, (50, 3)))
    for shift in (n, -n, -3 * n):
        np.testing.assert_array_equal(skewers.trilinear(grid, frac + shift * T32),
                                      skewers.trilinear(grid, frac))


def test_interpolation_axis_order():
    n = 8
    grid = np.zeros((n, n, n))
    grid[2, 5, 7] = 1.0
    # half a cell towards +x from (2,5,7): weight 1/2
    pos = np.array([[int(2.5 * T32), 5 * T32, 7 * T32]], dtype=np.int64)
    assert skewers.trilinear(grid, pos)[0] == 0.5
    pos = np.array([[2 * T32, int(4.75 * T32), 7 * T32]], dtype=np.int64)
    assert skewers.trilinear(grid, pos)[0] == 0.75


def test_delta_s_brute_force_dft():
    seed, q, npix, dpix = 17, 5, 100, 0.2
    ds = skewers.delta_s(seed, q, npix, dpix, 1.3, 1.5)
    ns = 128
    m = np.arange(ns // 2 + 1)
    k = 2 * np.pi * m / (ns * dpix)
    a = np.sqrt(1.3 * np.exp(-(k / 1.5) ** 2) / (ns * dpix))
    a[0] = 0
    from oracle import philox
    z1, z2 = philox.normal_pair(seed, 1, (np.uint64(q) << np.uint64(33)) + m.astype(np.uint64))
    w = (z1 + 1j * z2) / np.sqrt(2)
    w[-1] = z1[-1]
    j = np.arange(npix)
    ref = np.zeros(npix, dtype=np.complex128)
    for mm in range(-ns // 2 + 1, ns // 2 + 1):
        c = a[abs(mm)] * (w[mm] if mm >= 0 else np.conj(w[-mm]))
        ref += c * np.exp(2j * np.pi * mm * j / ns)
    assert np.max(np.abs(ref.imag)) < 1e-12
    np.testing.assert_allclose(ds, ref.real, atol=1e-12)


def test_delta_s_fixed_amplitude_variance():
    npix, dpix = 256, 0.2
    ds = skewers.delta_s(3, 9, npix, dpix, 1.0, 1.5, fixed_amp=True)
    m = np.arange(npix // 2 + 1)
    k = 2 * np.pi * m / (npix * dpix)
    p = np.exp(-(k / 1.5) ** 2) / (npix * dpix)
    expect = 2 * np.sum(p[1:-1]) + p[-1]
    np.testing.assert_allclose(np.mean(ds ** 2), expect, rtol=1e-12)


def test_delta_s_periodogram_recovers_ps():
    npix, dpix, amp = 512, 0.2, 2.0
    acc = np.zeros(npix // 2 + 1)
    for q in range(40):
        ds = skewers.delta_s(11, q, npix, dpix, amp, 1.5, fixed_amp=True)
        acc += np.abs(np.fft.rfft(ds)) ** 2 * dpix / npix
    acc /= 40
    k = 2 * np.pi * np.arange(npix // 2 + 1) / (npix * dpix)
    np.testing.assert_allclose(acc[1:], amp * np.exp(-(k[1:] / 1.5) ** 2), rtol=1e-10, atol=1e-14)


def test_axis_aligned_skewers_discrete_p1d():
    # Skewers along +z through grid points with pixel = voxel: the mean
    # periodogram equals sum_{n_perp} P(k)/(L_x L_y) at each k_z when |W| = 1,
    # the discrete form of eq:P1D.
    n, dx = 16, 2.19
    pk = power.PowerSpectrum()
    tab = power.amplitude_table(pk, n, dx)
    box = field.make_box(n, 44, tab, ("delta",), fixed_amp=True).real
    L = n * dx
    sk = dict(origin_fx=np.array([[mx * T32, my * T32, 3 * T32] for mx in range(n) for my in range(n)]),
              step_fx=np.tile(np.array([[0, 0, T32]], dtype=np.int64), (n * n, 1)),
              npix=np.full(n * n, n), offset=np.arange(n * n) * n, id_base=0)
    dens, _ = skewers.draw_skewers(box, np.zeros_like(box), sk, seed=1)
    per = np.abs(np.fft.fft(dens.reshape(n * n, n), axis=1)) ** 2 * dx / n
    mean = per.mean(axis=0)
    nn = field.signed_freq(np.arange(n), n)
    g = np.meshgrid(nn, nn, nn, indexing="ij")
    n2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    pgrid = np.where(n2 > 0, pk(2 * np.pi * np.sqrt(np.where(n2 > 0, n2, 1)) / L), 0.0)
    expect = pgrid.sum(axis=(0, 1)) / L ** 2   # indexed by z index
    np.testing.assert_allclose(mean, expect, rtol=1e-10)
    # and every pixel is exactly the voxel it sits on
    np.testing.assert_array_equal(dens.reshape(n, n, n), np.roll(box, -3, axis=2))


def test_draw_skewers_layout_and_small_scale_added():
    n = 8
    rng = np.random.default_rng(2)
    d = rng.normal(size=(n, n, n))
    e = rng.normal(size=(n, n, n))
    sk = dict(origin_fx=_fx(rng.uniform(0, n, (3, 3))), step_fx=_fx(rng.normal(size=(3, 3)) * 0.1),
              npix=np.array([5, 9, 3]), offset=np.array([10, 0, 20]), id_base=7)
    dens0, et0 = skewers.draw_skewers(d, e, sk, seed=5)
    dens1, et1 = skewers.draw_skewers(d, e, sk, seed=5, ps_amp=1.0, ps_kcut=1.5)
    assert dens0.shape == (23,)
    np.testing.assert_array_equal(et0, et1)
    np.testing.assert_allclose(dens1[10:15] - dens0[10:15], skewers.delta_s(5, 7, 5, 0.2, 1.0, 1.5))
    np.testing.assert_allclose(dens1[0:9] - dens0[0:9], skewers.delta_s(5, 8, 9, 0.2, 1.0, 1.5))
    assert np.all(dens0[15:20] == 0)
