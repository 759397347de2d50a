"""Lognormal quasar field (oracle, FP64).

TEST INFRASTRUCTURE ONLY: used by tests/, not by the library.

Follows section "Quasar generation" and the single-box form of Appendix A:

* the quasar bias b_q(z) = 3.7 ((1+z)/(1+2.33))^1.7;
* the quasar-density spectrum P_q(k) is the Fourier transform of
  ln[1 + b_0^2 xi_m(r)], xi_m the matter correlation function, b_0 the bias
  at the box redshift z_0 times the linear growth G(z_0) (the boxes are at
  z = 0, so xi_m(r, z_0) = G(z_0)^2 xi_m(r, 0));
* delta_q is the box of P_q on the same Philox modes as delta (the paper
  derives its modes from the original delta-hat);
* a voxel hosts a quasar with probability proportional to exp(alpha(z) delta_q),
  alpha(z) = b_q(z) (1+z_0) / (b_q(z_0) (1+z)) (Appendix A), and the quasar
  sits uniformly inside the voxel.

Readings (the paper is silent on these):

* xi_m comes from the smoothed spectrum P(k) exp(-k^2 s^2) (s the smoothing
  length, normally the voxel side, the paper's window W^2 = exp(-dx^2 k^2));
  without a cut-off the transform of a CDM-like P diverges at r -> 0;
* G is the growing mode of flat LCDM, D(a) proportional to
  E(a) int_0^a da' / (a' E(a'))^3, normalised to G(0) = 1;
* the probability of voxel m (grid point, x = m dx) is
  p = nbar(z) dx^3 exp(alpha delta_q - alpha^2 sigma_q^2 / 2), capped at 1, with
  z = z(|x - O|) for the observer O, nbar a tabulated comoving density
  (linear in z, zero outside the table) and sigma_q^2 the grid variance of
  delta_q (so the mean of the exponential factor is one);
* Philox4x32-10 stream 2, counter = the voxel's linear index m_x N^2 +
  m_y N + m_z: word 0 as the uniform u = ((w >> 9) + 1/2) 2^-23 decides
  (u < p); words 1-3 give the position in cell units times 2^32,
  (m << 32) - 2^31 + w, uniform over the voxel [m - 1/2, m + 1/2).
"""
import numpy as np
from scipy import integrate

from . import cosmology, philox


def bias_qso(z):
    return 3.7 * ((1.0 + np.asarray(z, dtype=np.float64)) / 3.33) ** 1.7


def alpha_of_z(z, z0):
    return bias_qso(z) * (1.0 + z0) / (bias_qso(z0) * (1.0 + np.asarray(z, dtype=np.float64)))


def growth(z, omega_m=cosmology.OMEGA_M):
    """Linear growth factor G(z)/G(0) of flat LCDM."""
    def d(a):
        e = lambda x: np.sqrt(omega_m / x ** 3 + 1.0 - omega_m)
        return e(a) * integrate.quad(lambda x: 1.0 / (x * e(x)) ** 3, 0.0, a, epsabs=0, epsrel=1e-13)[0]
    return d(1.0 / (1.0 + z)) / d(1.0)


def xi_of_r(pk, r, smooth):
    """(1 / 2 pi^2) int_0^inf P(k) exp(-k^2 s^2) k^2 sin(kr)/(kr) dk, by
    adaptive quadrature (scipy QAWO sine weight) on [0, 12/s]."""
    kmax = 12.0 / smooth
    f = lambda k: pk(k) * np.exp(-(k * smooth) ** 2) * k
    out = []
    for rr in np.atleast_1d(r):
        if rr == 0.0:
            v = integrate.quad(lambda k: f(k) * k, 0.0, kmax, epsabs=0, epsrel=1e-12, limit=2000)[0]
        else:
            v = integrate.quad(f, 0.0, kmax, weight="sin", wvar=rr, epsabs=0, epsrel=1e-12, limit=2000)[0] / rr
        out.append(v / (2.0 * np.pi ** 2))
    return np.array(out)


def pq_of_k(g_of_r, k, rmax):
    """4 pi int_0^rmax G(r) r^2 sin(kr)/(kr) dr for the given G (callable)."""
    out = []
    for kk in np.atleast_1d(k):
        v = integrate.quad(lambda r: g_of_r(r) * r, 0.0, rmax, weight="sin", wvar=kk, epsabs=0,
                           epsrel=1e-11, limit=4000)[0]
        out.append(4.0 * np.pi * v / kk)
    return np.array(out)


def lognormal_pk(pk, b0, smooth, k, rmax=2000.0, nr=4001):
    """P_q(k) for ln(1 + b0^2 xi): xi on a grid in r (quadrature above), G(r)
    interpolated by a cubic spline, then the transform back."""
    from scipy.interpolate import CubicSpline
    r = np.linspace(0.0, rmax, nr)
    xi = xi_of_r(pk, r, smooth)
    g = np.log1p(b0 * b0 * xi)
    spl = CubicSpline(r, g)
    return pq_of_k(spl, k, rmax)


def draw(delta_q, dx, observer, z0, nbar_z, nbar, seed, omega_m=cosmology.OMEGA_M):
    """Selected voxels and quasar positions.  Returns (lin index sorted,
    positions fx [M, 3] int64, probability p and uniform u of every voxel)."""
    n = delta_q.shape[0]
    m = np.arange(n)
    gx, gy, gz = np.meshgrid(m, m, m, indexing="ij")
    pos = np.stack([gx, gy, gz], axis=-1).astype(np.float64) * dx
    chi = np.sqrt(np.sum((pos - np.asarray(observer, dtype=np.float64)) ** 2, axis=-1))
    z = cosmology.z_of_chi(chi.ravel(), omega_m).reshape(chi.shape)
    al = alpha_of_z(z, z0)
    s2 = float(np.mean(delta_q ** 2))
    nb = np.interp(z, nbar_z, nbar, left=0.0, right=0.0)
    p = np.minimum(nb * dx ** 3 * np.exp(al * delta_q - 0.5 * al * al * s2), 1.0)
    lin = ((gx.astype(np.int64) * n + gy) * n + gz).ravel()
    w = philox.words(seed, 2, lin)          # [V, 4], 32-bit values
    u = ((w[:, 0] >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    sel = u < p.ravel()
    idx = lin[sel]
    cells = np.stack([gx.ravel()[sel], gy.ravel()[sel], gz.ravel()[sel]], axis=1).astype(np.int64)
    fx = (cells << 32) - (1 << 31) + w[sel][:, 1:4].astype(np.int64)
    return idx, fx, p.ravel(), u, s2
