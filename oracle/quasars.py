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
  E(a) int_0^a da' / (a' E(a'))^3, normalised to G(0) = 1.  Appendix A
  equates a(z) = sqrt(xi_mod / xi_0) with b_q(z) (1 + z_0) / (b_q(z_0) (1 + z)),
  which holds when G is proportional to 1/(1+z) (matter domination, true to
  about 1% over 1.9 < z < 3.6); the quasar fields therefore use
  G_q(z) = G(z_ref) (1 + z_ref) / (1 + z), z_ref the middle box (or the only
  one), and the box of redshift z_i takes b_0 = b_q(z_i) G_q(z_i).  With the
  exact LCDM growth instead, the three-box combination misses the model by
  about 1e-3 rather than the paper's 5e-4;
* the probability of voxel m (grid point, x = m dx) is
  p = nbar(z) dx^3 sum_i c_i(z) exp(a_i(z) delta_i - a_i(z)^2 sigma_i^2 / 2),
  clipped to [0, 1], with z = z(|x - O|) for the observer O, nbar a tabulated
  comoving density (linear in z, zero outside the table), sigma_i^2 the
  variance of box i (the mean of each exponential factor is then one) and
  a_i(z) = b_q(z) (1 + z_i) / (b_q(z_i) (1 + z)) (Appendix A);
* one box: c_1 = 1.  Three boxes (Appendix A): p_12 interpolates p_1, p_2
  linearly in z, p_23 extrapolates p_2, p_3 linearly in z, and
  p = w p_12 + (1 - w) p_23 with w fixed at r = 5 Mpc/h by
  w xi_12 + (1 - w) xi_23 = xi_mod, where xi_i = (1 + xi_0i)^(a_i^2) - 1,
  xi_0i = b_0i^2 xi_m(5), xi_mod = (b_q(z) G_q(z))^2 xi_m(5) and xi_12, xi_23
  the same linear combinations of the xi_i; w = 1/2 where xi_12 = xi_23
  (then p_12 = p_23); w is clipped to [0, 1];
* random numbers: the decision of voxel m uses Philox4x32-10 stream 2,
  counter m >> 2, word m & 3 (one call serves four consecutive voxels), as
  the uniform u = ((w >> 9) + 1/2) 2^-23, and selects when u < p; the
  position of a selected voxel uses stream 4, counter m, words 0-2: per axis
  (m_axis << 32) - 2^31 + w in cell units times 2^32, uniform over the voxel
  [m - 1/2, m + 1/2).

Catalogue and lines of sight (section "Quasar generation": the quasar
velocity from eq:velocity; readings, the paper giving no formulas):

* the velocity boxes are made at z = 0 with f = 1 and aH = 100 km/s per
  Mpc/h, v_hat_j = i 100 k_j / k^2 delta_hat; at redshift z the velocity is
  that times G(z) f(z) E(z) / (1 + z) (the faH of eq:velocity with the
  growth of the z = 0 box), f = dln G / dln a of flat LCDM;
* a quasar at x (its fixed-point position times dx) has the comoving
  distance chi = |x - O|, the cosmological redshift z_c = z(chi), the
  line-of-sight velocity v_par = v(x) . (x - O) / chi with v trilinear from
  the boxes (as the pixels), and the redshift z_q = z_c + (1 + z_c) v_par / c;
* its forest runs from the red end z_hi = (1 + z_q) r_hi - 1 towards the
  observer down to z_lo = max((1 + z_q) r_lo - 1, z_min), r = lambda /
  lambda_Lya for the rest-frame window (1040-1200 A in the paper's P1D
  selection); pixel j at chi(z_hi) - j dchi, npix = floor((chi(z_hi) -
  chi(z_lo)) / dchi) capped at 2048 (0 when z_hi <= z_lo); the origin
  O + u chi(z_hi) and the step -u dchi, u = (x - O) / chi, in cell units
  times 2^32 rounded to the nearest integer.
"""
import numpy as np
from scipy import integrate

from . import cosmology, philox, skewers


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


def growth_q(z, z_ref, omega_m=cosmology.OMEGA_M):
    """G_q(z) = G(z_ref) (1 + z_ref) / (1 + z)."""
    return growth(z_ref, omega_m) * (1.0 + z_ref) / (1.0 + np.asarray(z, dtype=np.float64))


def box_bias2(z_box, z_ref, omega_m=cosmology.OMEGA_M):
    """b_0^2 of the box at z_box: (b_q(z_box) G_q(z_box))^2."""
    return float((bias_qso(z_box) * growth_q(z_box, z_ref, omega_m)) ** 2)


def mix_coeffs(z, z_box, xi5, omega_m=cosmology.OMEGA_M):
    """(c_1, c_2, c_3) of the three-box combination at redshift z (scalar or
    array; the coefficients go along the last axis)."""
    z = np.asarray(z, dtype=np.float64)
    z1, z2, z3 = (float(v) for v in z_box)
    g2 = growth(z2, omega_m)
    xi = [(1.0 + box_bias2(zi, z2, omega_m) * xi5) ** (alpha_of_z(z, zi) ** 2) - 1.0 for zi in (z1, z2, z3)]
    xi_mod = (bias_qso(z) * g2 * (1.0 + z2) / (1.0 + z)) ** 2 * xi5
    t12 = (z - z1) / (z2 - z1)
    t23 = (z - z2) / (z3 - z2)
    xi12 = (1.0 - t12) * xi[0] + t12 * xi[1]
    xi23 = (1.0 - t23) * xi[1] + t23 * xi[2]
    den = xi12 - xi23
    flat = np.abs(den) <= 1e-12 * np.abs(xi[1])
    with np.errstate(invalid="ignore", divide="ignore"):
        w = np.where(flat, 0.5, np.clip((xi_mod - xi23) / np.where(flat, 1.0, den), 0.0, 1.0))
    return np.stack([w * (1.0 - t12), w * t12 + (1.0 - w) * (1.0 - t23), (1.0 - w) * t23], axis=-1)


def probability_at(lin, values, n, dx, observer, z_box, sigma2, nbar_z, nbar, xi5=None,
                   omega_m=cosmology.OMEGA_M):
    """p and z of the voxels with linear indices lin (grid point m at m dx),
    values[i] holding delta_i at those voxels."""
    lin = np.asarray(lin, dtype=np.int64)
    pos = np.stack([lin // (n * n), (lin // n) % n, lin % n], axis=-1).astype(np.float64) * dx
    chi = np.sqrt(np.sum((pos - np.asarray(observer, dtype=np.float64)) ** 2, axis=-1))
    z = cosmology.z_of_chi(chi, omega_m)
    nb = np.interp(z, nbar_z, nbar, left=0.0, right=0.0)
    coef = np.ones((len(z), 1)) if len(values) == 1 else mix_coeffs(z, z_box, xi5, omega_m)
    acc = np.zeros(len(z))
    for i, (v, zi, s2) in enumerate(zip(values, z_box, sigma2)):
        al = alpha_of_z(z, zi)
        acc += coef[:, i] * np.exp(al * np.asarray(v, dtype=np.float64) - 0.5 * al * al * s2)
    return np.clip(nb * dx ** 3 * acc, 0.0, 1.0), z


def probability(fields, dx, observer, z_box, sigma2, nbar_z, nbar, xi5=None, omega_m=cosmology.OMEGA_M):
    """p of every voxel (flat, linear index order) and its redshift."""
    n = fields[0].shape[0]
    return probability_at(np.arange(n ** 3), [np.asarray(f).ravel() for f in fields], n, dx, observer, z_box,
                          sigma2, nbar_z, nbar, xi5, omega_m)


def decision_uniforms_at(seed, lin):
    lin = np.asarray(lin, dtype=np.uint64)
    w = philox.words(seed, 2, lin >> np.uint64(2))
    wd = np.take_along_axis(w, (lin & np.uint64(3)).astype(np.int64)[:, None], axis=1)[:, 0]
    return ((wd >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def decision_uniforms(seed, n_vox):
    return decision_uniforms_at(seed, np.arange(n_vox))


def positions(seed, idx, n):
    """Fixed-point positions of the selected voxels idx (linear indices)."""
    idx = np.asarray(idx, dtype=np.int64)
    w = philox.words(seed, 4, idx.astype(np.uint64))
    cells = np.stack([idx // (n * n), (idx // n) % n, idx % n], axis=1).astype(np.int64)
    return (cells << 32) - (1 << 31) + w[:, 0:3].astype(np.int64)


def draw(fields, dx, observer, z_box, sigma2, nbar_z, nbar, seed, xi5=None, omega_m=cosmology.OMEGA_M):
    """Selected voxels (linear indices, increasing), their fixed-point
    positions [M, 3], and p, u of every voxel."""
    p, _ = probability(fields, dx, observer, z_box, sigma2, nbar_z, nbar, xi5, omega_m)
    u = decision_uniforms(seed, p.size)
    idx = np.flatnonzero(u < p)
    return idx, positions(seed, idx, fields[0].shape[0]), p, u


C_KMS = 299792.458
MAX_PIX = 2048


def growth_rate(z, omega_m=cosmology.OMEGA_M):
    """f = dln D / dln a of flat LCDM with D = E(a) I(a), I = int_0^a
    da' / (a' E(a'))^3: f = a E'/E + a / (I (a E)^3), a E'/E = -3 Om / (2 a^3 E^2)."""
    a = 1.0 / (1.0 + float(z))
    e2 = omega_m / a ** 3 + 1.0 - omega_m
    integ = integrate.quad(lambda x: (omega_m / x + (1.0 - omega_m) * x * x) ** -1.5, 0.0, a,
                           epsabs=0, epsrel=1e-13)[0]
    return -1.5 * omega_m / (a ** 3 * e2) + a / (integ * (a * a * e2) ** 1.5)


def velocity_factor(z, omega_m=cosmology.OMEGA_M):
    """G(z) f(z) E(z) / (1 + z): the z = 0, f = 1 velocity boxes to redshift z."""
    return growth(z, omega_m) * growth_rate(z, omega_m) * float(cosmology.hubble_e(z, omega_m)) / (1.0 + z)


def lines_of_sight(pos_fx, vx, vy, vz, dx, observer, r_lo, r_hi, z_min, dchi, omega_m=cosmology.OMEGA_M):
    """Redshift-space catalogue and its skewer table, quasar by quasar.
    vx, vy, vz: velocity grids (z = 0, f = 1).  Returns a dict with z_c, z_q,
    origin_fx, step_fx, npix, offset, chi0, total."""
    pos = np.asarray(pos_fx, dtype=np.int64)
    o = np.asarray(observer, dtype=np.float64)
    nq = len(pos)
    out = dict(z_c=np.zeros(nq), z_q=np.zeros(nq), origin_fx=np.zeros((nq, 3), np.int64),
               step_fx=np.zeros((nq, 3), np.int64), npix=np.zeros(nq, np.int32), chi0=np.zeros(nq))
    for q in range(nq):
        x = pos[q].astype(np.float64) / 2.0 ** 32 * dx
        d = x - o
        chi = np.sqrt(np.sum(d * d))
        u = d / chi
        zc = float(cosmology.z_of_chi(np.array([chi]), omega_m)[0])
        v = np.array([skewers.trilinear(g, pos[q][None, :])[0] for g in (vx, vy, vz)])
        vpar = float(v @ u) * velocity_factor(zc, omega_m)
        zq = zc + (1.0 + zc) * vpar / C_KMS
        z_hi = (1.0 + zq) * r_hi - 1.0
        z_lo = max((1.0 + zq) * r_lo - 1.0, z_min)
        c_hi = float(cosmology.chi_of_z(z_hi, omega_m))
        npix = 0
        if z_hi > z_lo:
            c_lo = float(cosmology.chi_of_z(z_lo, omega_m))
            npix = min(int(np.floor((c_hi - c_lo) / dchi)), MAX_PIX)
        out["z_c"][q], out["z_q"][q], out["chi0"][q], out["npix"][q] = zc, zq, c_hi, npix
        out["origin_fx"][q] = np.rint((o + u * c_hi) / dx * 2.0 ** 32).astype(np.int64)
        out["step_fx"][q] = np.rint(-u * dchi / dx * 2.0 ** 32).astype(np.int64)
    out["offset"] = np.concatenate([[0], np.cumsum(out["npix"].astype(np.int64))[:-1]]) if nq else np.zeros(0, np.int64)
    out["total"] = int(out["npix"].astype(np.int64).sum())
    return out
