"""Pins of the oracle's 7^3 Gaussian-kernel average (section "Gaussian fields
along lines of sight": standard deviation one voxel, three voxels each way)."""
import numpy as np

from oracle import skewers

T32 = 2 ** 32


def _fx(u):
    """Fixed-point positions (cell units x 2^32) of real cell coordinates."""
    return np.floor(np.asarray(u, dtype=np.float64) * T32).astype(np.int64)


def test_constant_field():
    g = np.full((8, 8, 8), 2.5)
    u = np.random.default_rng(0).uniform(-20, 20, (50, 3))
    np.testing.assert_allclose(skewers.gauss7(g, _fx(u)), 2.5, rtol=1e-14)


def test_brute_force_in_physical_units():
    # an independent direct sum: positions in Mpc/h, the pixel's voxel by
    # rounding, weights exp(-d^2 / (2 dx^2)) over the 7^3 neighbours
    rng = np.random.default_rng(1)
    n, dx = 8, 2.19
    g = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    pos = _fx(rng.uniform(-3 * n, 3 * n, (20, 3)))
    got = skewers.gauss7(g, pos)
    for p, val in zip(pos, got):
        x = p.astype(np.float64) / T32 * dx
        centre = [int(np.floor(x[a] / dx + 0.5)) for a in range(3)]
        num, den = 0.0, 0.0
        for i in range(centre[0] - 3, centre[0] + 4):
            for j in range(centre[1] - 3, centre[1] + 4):
                for k in range(centre[2] - 3, centre[2] + 4):
                    d2 = (i * dx - x[0]) ** 2 + (j * dx - x[1]) ** 2 + (k * dx - x[2]) ** 2
                    w = np.exp(-d2 / (2 * dx * dx))
                    num += w * g[i % n, j % n, k % n]
                    den += w
        np.testing.assert_allclose(val, num / den, rtol=1e-12)


def test_linear_field_on_grid_points():
    # at a grid point the truncated kernel is symmetric: a linear field keeps
    # its value there (away from the periodic seam)
    n = 32
    m = np.arange(n, dtype=np.float64)
    g = 1.5 + 0.25 * m[:, None, None] - 0.5 * m[None, :, None] + 0.125 * m[None, None, :]
    c = np.array([[10, 12, 14], [5, 20, 9], [16, 16, 16]])
    got = skewers.gauss7(g, c.astype(np.int64) * T32)
    want = 1.5 + 0.25 * c[:, 0] - 0.5 * c[:, 1] + 0.125 * c[:, 2]
    np.testing.assert_allclose(got, want, rtol=1e-13)


def test_product_field_factorises():
    rng = np.random.default_rng(2)
    n = 16
    a, b, c = rng.normal(size=(3, n))
    g = a[:, None, None] * b[None, :, None] * c[None, None, :]
    u = rng.uniform(0, n, (30, 3))
    got = skewers.gauss7(g, _fx(u))
    uu = _fx(u).astype(np.float64) / T32
    cen = np.floor(uu + 0.5).astype(int)
    for q in range(len(u)):
        f = 1.0
        for axis, vec in enumerate((a, b, c)):
            o = np.arange(-3, 4)
            w = np.exp(-((cen[q, axis] + o - uu[q, axis]) ** 2) / 2)
            f *= np.sum(w * vec[(cen[q, axis] + o) % n]) / np.sum(w)
        np.testing.assert_allclose(got[q], f, rtol=1e-12, atol=1e-14)


def test_transfer_of_a_long_wave():
    # a wave of wavenumber k is damped by exp(-k^2 dx^2 / 2) (the paper's
    # window W^2 = exp(-dx^2 k^2)); the 3-sigma truncation and the grid
    # change that by far less than 1e-3 for long waves
    n = 64
    i = np.arange(n)
    for m in (1, 2, 4):
        g = np.cos(2 * np.pi * m * i / n)[:, None, None] * np.ones((1, n, n))
        got = skewers.gauss7(g, np.array([[7 * T32, 3 * T32, 5 * T32]], dtype=np.int64))[0]
        k = 2 * np.pi * m / n
        np.testing.assert_allclose(got, np.cos(2 * np.pi * m * 7 / n) * np.exp(-k * k / 2), rtol=1e-3)
