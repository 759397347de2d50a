"""Flat LCDM background for pixel redshifts (oracle, FP64).

Follows Table cosmoparams (flat LCDM, Omega_M = 0.3147) and the statement in
section "FGPA" that each pixel's wavelength uses the unperturbed cosmological
redshift.  Reading: radiation is not mentioned, so E(z)^2 = Om (1+z)^3 + 1 - Om.
Distances are in Mpc/h, so h cancels and c/H0 = 2997.92458 Mpc/h.

chi(z) = (c/H0) * int_0^z dz'/E(z') is evaluated with 64-node Gauss-Legendre
quadrature on [0, z] (numpy.polynomial.legendre.leggauss); z(chi) inverts it by
Newton iteration, d chi/dz = (c/H0)/E(z), started from a linear interpolation
in a table of chi(z).

Pins: the Einstein-de Sitter closed form (Om = 1), the pure-Lambda closed form
(Om = 0), scipy.integrate.quad at sample redshifts, and z(chi(z)) = z.
"""
import numpy as np

C_OVER_H0 = 2997.92458  # Mpc/h
OMEGA_M = 0.3147        # Table cosmoparams

_GL_X, _GL_W = np.polynomial.legendre.leggauss(64)


def hubble_e(z, omega_m=OMEGA_M):
    """E(z) = H(z)/H0 for flat LCDM."""
    zp1 = 1.0 + np.asarray(z, dtype=np.float64)
    return np.sqrt(omega_m * zp1 ** 3 + (1.0 - omega_m))


def chi_of_z(z, omega_m=OMEGA_M):
    """Comoving distance in Mpc/h (vectorised over z)."""
    z = np.asarray(z, dtype=np.float64)
    half = 0.5 * z[..., None]
    nodes = half * (_GL_X + 1.0)
    integrand = 1.0 / hubble_e(nodes, omega_m)
    return C_OVER_H0 * half[..., 0] * np.sum(_GL_W * integrand, axis=-1)


def z_of_chi(chi, omega_m=OMEGA_M, iters=60, chunk=1 << 15):
    """Inverse of chi_of_z by Newton iteration (vectorised).  Each value stops
    at its first step below 1e-15 (1 + z); values are processed in chunks so
    that the quadrature arrays stay small."""
    chi = np.asarray(chi, dtype=np.float64)
    flat = chi.reshape(-1)
    out = np.empty_like(flat)
    # starting values: linear interpolation in a table of chi_of_z itself
    z_tab = np.linspace(0.0, 12.0, 4801)
    chi_tab = chi_of_z(z_tab, omega_m)
    for s in range(0, flat.size, chunk):
        c = flat[s:s + chunk]
        z = np.interp(c, chi_tab, z_tab, right=z_tab[-1])
        active = np.arange(c.size)
        for _ in range(iters):
            za = z[active]
            dz = (chi_of_z(za, omega_m) - c[active]) * hubble_e(za, omega_m) / C_OVER_H0
            zn = za - dz
            z[active] = zn
            active = active[np.abs(dz) >= 1e-15 * (1.0 + np.abs(zn))]
            if active.size == 0:
                break
        out[s:s + chunk] = z
    return out.reshape(chi.shape)


def dv_per_dchi(z, omega_m=OMEGA_M):
    """Velocity per comoving length, km/s per Mpc/h: 100 E(z)/(1+z)."""
    z = np.asarray(z, dtype=np.float64)
    return 100.0 * hubble_e(z, omega_m) / (1.0 + z)
