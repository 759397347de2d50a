"""Lines of sight through the box (oracle, FP64).

Follows section "Gaussian fields along lines of sight":

* each quasar line of sight is cut into pixels of 0.2 Mpc/h;
* delta_L and eta_par at a pixel come from the voxel values of the boxes;
* delta_S is an independent 1D Gaussian field per line of sight, generated
  like the 3D box: Fourier modes of a Gaussian field defined over the pixel
  range, scaled by the square root of the wanted 1D spectrum P_s(k), then
  inverse Fourier transformed.

Readings (paper silent or superseded):

* Interpolation: periodic trilinear interpolation of the grid values (grid
  point m at x = m dx) replaces the paper's 7^3 Gaussian-kernel average on
  the hot path; gauss7 is that average (draw_skewers(interp=gauss7)), with
  the pixel's voxel read as its nearest grid point.
* Geometry: pixel j of a skewer sits at the fixed-point position
  p_j = origin + j step (integers, cell units times 2^32); the voxel index is
  floor(p_j / 2^32) mod N per axis, and the fractional offset is
  (p_j mod 2^32) 2^-32.  Those integers are the input, so the oracle uses them
  exactly (Python/numpy int64) and interpolates in FP64.
* delta_S: length N_S = next power of two >= n_q, spacing dpix; modes
  m = 0..N_S/2, k_m = 2 pi m /(N_S dpix); amplitude sqrt(P_s(k_m)/(N_S dpix));
  m = 0 carries nothing, m = N_S/2 is real; normals from
  oracle.philox.normal_pair(seed, 1, (q << 33) + m) for quasar id q;
  delta_S(j) = sum over +-m of the modes exp(2 pi i m j / N_S), first n_q
  values.  P_s(k) = amp exp(-(k/kcut)^2) (the configuration's shape; the
  paper only says "proportional to").
* Line of sight of eta_par: draw_skewers takes eta_par from a box built for
  the z axis (the distant-observer reading, eta_zz); draw_skewers_wide forms
  eta_par = u_p u_q eta^{pq} at each pixel from the six components, with u
  the skewer's own direction (a straight radial line keeps one direction).
"""
import numpy as np

from . import philox

TWO32 = 2 ** 32


def next_pow2(n):
    p = 1
    while p < n:
        p *= 2
    return p


def pixel_positions(origin_fx, step_fx, npix):
    """Fixed-point positions [npix, 3] of one skewer (int64, exact)."""
    j = np.arange(npix, dtype=np.int64)[:, None]
    return np.asarray(origin_fx, dtype=np.int64)[None, :] + \
        j * np.asarray(step_fx, dtype=np.int64)[None, :]


def trilinear(grid, pos_fx):
    """Periodic trilinear interpolation of grid [N,N,N] (real or complex) at
    fixed-point positions pos_fx [..., 3]."""
    n = grid.shape[0]
    pos = np.asarray(pos_fx, dtype=np.int64)
    cell = pos >> 32                     # arithmetic shift: floor
    frac = (pos & (TWO32 - 1)).astype(np.float64) / TWO32
    i0 = cell % n
    i1 = (cell + 1) % n
    tx, ty, tz = frac[..., 0], frac[..., 1], frac[..., 2]
    out = 0.0
    for a, wa in ((i0[..., 0], 1.0 - tx), (i1[..., 0], tx)):
        for b, wb in ((i0[..., 1], 1.0 - ty), (i1[..., 1], ty)):
            for c, wc in ((i0[..., 2], 1.0 - tz), (i1[..., 2], tz)):
                out = out + (wa * wb * wc) * grid[a, b, c]
    return out


def gauss7(grid, pos_fx, sigma=1.0, reach=3):
    """Gaussian-kernel average of grid [N,N,N] (real or complex) at fixed-point
    positions pos_fx [..., 3] (section "Gaussian fields along lines of
    sight": standard deviation one voxel side, three voxels each way of the
    pixel's voxel, 7^3 = 343 voxels).  Reading: the pixel's voxel is its
    nearest grid point c = floor(u + 1/2) per axis (u in cell units); voxel
    c + o, o in [-reach, reach]^3, periodic, weighs exp(-|c + o - u|^2 /
    (2 sigma^2)); the average divides by the sum of the 343 weights."""
    n = grid.shape[0]
    pos = np.asarray(pos_fx, dtype=np.int64)
    cell = pos >> 32
    frac = (pos & (TWO32 - 1)).astype(np.float64) / TWO32
    up = frac >= 0.5                       # nearest grid point
    c = cell + up
    t = frac - up                          # u - c, in [-1/2, 1/2)
    num = 0.0
    den = 0.0
    rng = range(-reach, reach + 1)
    for ox in rng:
        wx = np.exp(-((ox - t[..., 0]) ** 2) / (2.0 * sigma ** 2))
        ix = (c[..., 0] + ox) % n
        for oy in rng:
            wy = np.exp(-((oy - t[..., 1]) ** 2) / (2.0 * sigma ** 2))
            iy = (c[..., 1] + oy) % n
            for oz in rng:
                wz = np.exp(-((oz - t[..., 2]) ** 2) / (2.0 * sigma ** 2))
                iz = (c[..., 2] + oz) % n
                w = wx * wy * wz
                num = num + w * grid[ix, iy, iz]
                den = den + w
    return num / den


def ps_gauss(k, amp, kcut):
    return amp * np.exp(-(np.asarray(k) / kcut) ** 2)


def delta_s(seed, qid, npix, dpix, amp, kcut, fixed_amp=False):
    """Small-scale field of quasar qid, first npix pixels (FP64)."""
    ns = next_pow2(npix)
    m = np.arange(ns // 2 + 1, dtype=np.int64)
    k = 2.0 * np.pi * m / (ns * dpix)
    a = np.sqrt(ps_gauss(k, amp, kcut) / (ns * dpix))
    a[0] = 0.0
    lin = (np.uint64(qid) << np.uint64(33)) + m.astype(np.uint64)
    z1, z2 = philox.normal_pair(seed, 1, lin)
    w = (z1 + 1j * z2) / np.sqrt(2.0)
    w[-1] = z1[-1]
    if fixed_amp:
        w = w / np.abs(w)
    spec = a * w
    full = np.fft.irfft(spec, n=ns) * ns
    return full[:npix]


def draw_skewers(delta, eta, sk, seed, ps_amp=0.0, ps_kcut=1.5, dpix=0.2,
                 fixed_amp_s=False, interp=None):
    """Pre-FGPA pixels of every skewer.

    delta, eta: real grids [N,N,N] (FP64).  sk: dict with origin_fx [S,3],
    step_fx [S,3], npix [S], offset [S], id_base.  Returns flat arrays
    (dens = delta_L + delta_S, eta) of length sum(npix) laid out by offset."""
    npix = np.asarray(sk["npix"])
    off = np.asarray(sk["offset"])
    total = int(np.max(off + npix)) if len(npix) else 0
    dens = np.zeros(total)
    et = np.zeros(total)
    grid = delta + 1j * eta
    for q in range(len(npix)):
        nq = int(npix[q])
        pos = pixel_positions(sk["origin_fx"][q], sk["step_fx"][q], nq)
        v = (interp or trilinear)(grid, pos)
        d = v.real.copy()
        if ps_amp > 0.0:
            d += delta_s(seed, int(sk["id_base"]) + q, nq, dpix, ps_amp,
                         ps_kcut, fixed_amp_s)
        o = int(off[q])
        dens[o:o + nq] = d
        et[o:o + nq] = v.imag
    return dens, et


WIDE_COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


def los_unit(step_fx):
    """Unit vector of a straight line of sight from its fixed-point step
    (FP64; the sign is irrelevant to eta_par, which is quadratic in u)."""
    u = np.asarray(step_fx, dtype=np.float64)
    return u / np.sqrt(np.sum(u * u))


def eta_par_from_components(eta6, u):
    """eta_par = u_p u_q eta^{pq} (section "Mock generation", after eq:eta) from
    the six components in the order xx, yy, zz, xy, xz, yz (arrays of any
    common shape); the off-diagonal terms appear twice in the double sum."""
    ux, uy, uz = u
    xx, yy, zz, xy, xz, yz = eta6
    return (ux * ux * xx + uy * uy * yy + uz * uz * zz
            + 2.0 * (ux * uy * xy + ux * uz * xz + uy * uz * yz))


def draw_skewers_wide(delta, eta6, sk, seed, ps_amp=0.0, ps_kcut=1.5, dpix=0.2, fixed_amp_s=False):
    """Pre-FGPA pixels with the wide-angle line-of-sight velocity gradient:
    as draw_skewers, but eta_par at each pixel is u_p u_q eta^{pq} with u the
    skewer's own direction, from the six real grids eta6 (order xx, yy, zz,
    xy, xz, yz), each interpolated trilinearly like delta."""
    npix = np.asarray(sk["npix"])
    off = np.asarray(sk["offset"])
    total = int(np.max(off + npix)) if len(npix) else 0
    dens = np.zeros(total)
    et = np.zeros(total)
    for q in range(len(npix)):
        nq = int(npix[q])
        pos = pixel_positions(sk["origin_fx"][q], sk["step_fx"][q], nq)
        d = trilinear(delta, pos)
        comps = [trilinear(g, pos) for g in eta6]
        e = eta_par_from_components(comps, los_unit(sk["step_fx"][q]))
        if ps_amp > 0.0:
            d = d + delta_s(seed, int(sk["id_base"]) + q, nq, dpix, ps_amp, ps_kcut, fixed_amp_s)
        o = int(off[q])
        dens[o:o + nq] = d
        et[o:o + nq] = e
    return dens, et
