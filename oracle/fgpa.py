"""Fluctuating Gunn-Peterson transform and mean flux (oracle, FP64).

Follows eq:gfield and eq:FGPA:

    g = delta_L + delta_S + c(z) eta_par,    F = exp(-a(z) exp(b(z) g)),

with the pixel redshift the unperturbed cosmological one (section "FGPA").
Reading: a, b, c are quadratics in (1+z), coef[p][i] multiplying (1+z)^i for
p = a, b, c (the workload states them this way; the paper tunes them at five
redshifts and interpolates).

Pixel distance: pixel j of a skewer is at chi_j = chi0 - j dchi, evaluated as
chi0 - (j * dchi) with both operations rounded in FP64 (no fused multiply-add),
so that a redshift bin decision, which compares chi_j against bin edges, is
the same in any implementation that forms chi_j this way.

Mean flux (section "Analysis procedure of forest correlations": the mean
transmission is the average of F over forests in small wavelength ranges):
here per redshift bin, a pixel falling in bin b when
edges[b] <= chi_j < edges[b+1], edges being comoving distances of the bin's
redshift limits.  The host-quasar correction discussed there is not applied.
"""
import numpy as np

from . import cosmology


def coeff_eval(coef, z):
    """(a, b, c) at redshift z from coef[3][3]."""
    coef = np.asarray(coef, dtype=np.float64)
    x = 1.0 + np.asarray(z, dtype=np.float64)
    return tuple(coef[p, 0] + coef[p, 1] * x + coef[p, 2] * x * x for p in range(3))


def flux(dens, eta, z, coef):
    a, b, c = coeff_eval(coef, z)
    g = dens + c * eta
    return np.exp(-a * np.exp(b * g))


def pixel_chi(sk, total=None):
    """Flat FP64 chi of every pixel (chi0 - (j * dchi))."""
    npix = np.asarray(sk["npix"])
    off = np.asarray(sk["offset"])
    if total is None:
        total = int(np.max(off + npix)) if len(npix) else 0
    chi = np.zeros(total)
    for q in range(len(npix)):
        j = np.arange(int(npix[q]), dtype=np.float64)
        o = int(off[q])
        chi[o:o + int(npix[q])] = sk["chi0"][q] - (j * sk["dchi"])
    return chi


def apply_fgpa(dens, eta, sk, coef, omega_m=cosmology.OMEGA_M):
    chi = pixel_chi(sk, len(dens))
    z = cosmology.z_of_chi(chi, omega_m)
    return flux(dens, eta, z, coef), z


def chi_edges_for_z(z_edges, omega_m=cosmology.OMEGA_M):
    return cosmology.chi_of_z(np.asarray(z_edges, dtype=np.float64), omega_m)


def mean_flux_bins(F, chi, chi_edges, valid=None):
    """Per-bin sum of F and pixel count (FP64 sums, int64 counts)."""
    edges = np.asarray(chi_edges, dtype=np.float64)
    nb = len(edges) - 1
    b = np.searchsorted(edges, chi, side="right") - 1
    ok = (b >= 0) & (b < nb)
    if valid is not None:
        ok &= valid
    fsum = np.zeros(nb)
    cnt = np.zeros(nb, dtype=np.int64)
    np.add.at(fsum, b[ok], F[ok])
    np.add.at(cnt, b[ok], 1)
    return fsum, cnt


def gauss_hermite_mean_flux(a, b, sigma_g, nodes=64):
    """<F> for Gaussian g of variance sigma_g^2 (statistical pin):
    int exp(-a e^{b g}) N(g; 0, sigma_g^2) dg by Gauss-Hermite."""
    x, w = np.polynomial.hermite.hermgauss(nodes)
    g = np.sqrt(2.0) * sigma_g * x
    return np.sum(w * np.exp(-a * np.exp(b * g))) / np.sqrt(np.pi)
