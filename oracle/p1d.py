"""1D flux power spectrum (oracle, FP64).

The paper tunes its mocks so that the 1D power spectrum of the flux contrast
matches a measured one (section "Adjusting mock parameters"), with the flux
contrast delta_F = F / Fbar - 1 of equation::definition_delta (section
"Analysis procedure of forest correlations").  The estimator itself is not
given in the paper; the reading taken here is a plain periodogram:

* per skewer, the first N_P = min(2^floor(log2 n_q), 2048) pixels (n_q >= 2);
* delta_F = F / Fbar(bin) - 1, Fbar given per redshift bin (bins in comoving
  distance as for the mean-flux reduction; a pixel outside the bins takes
  the nearest one);
* velocity pixel Dv = dpix 100 E(z_ref) / (1 + z_ref) km/s at one reference
  redshift z_ref for the whole call (the paper tunes at fixed z_t);
* DFT X_m = sum_j delta_F(j) exp(-2 pi i m j / N_P), modes m = 1..N_P/2,
  k_m = 2 pi m / (N_P Dv) in s/km, P(k_m) = Dv |X_m|^2 / N_P;
* modes are binned by k_edges[b] <= k_m < k_edges[b+1]; the result is the
  sum of P and the number of modes per bin (mean = sum / count).

Pins: Parseval (sum over all modes of the periodogram), the white-noise
expectation, and a single cosine, each checked in tests/test_oracle_p1d.py.
"""
import numpy as np

from . import cosmology, fgpa


def log_k_edges(n_bins=32, kmin=0.001, kmax=0.05):
    return kmin * (kmax / kmin) ** (np.arange(n_bins + 1) / n_bins)


def dv_pixel(z_ref, dpix, omega_m=cosmology.OMEGA_M):
    return dpix * cosmology.dv_per_dchi(z_ref, omega_m)


def p1d(flux, sk, chi_edges, fmean, k_edges, z_ref, dpix, omega_m=cosmology.OMEGA_M):
    """Per-bin sum of P and mode count over all skewers of sk."""
    k_edges = np.asarray(k_edges, dtype=np.float64)
    nk = len(k_edges) - 1
    psum = np.zeros(nk)
    cnt = np.zeros(nk, dtype=np.int64)
    edges = np.asarray(chi_edges, dtype=np.float64)
    nb = len(edges) - 1
    fmean = np.asarray(fmean, dtype=np.float64)
    dv = dv_pixel(z_ref, dpix, omega_m)
    chi_all = fgpa.pixel_chi(sk, len(flux))
    for q in range(len(sk["npix"])):
        nq = int(sk["npix"][q])
        if nq < 2:
            continue
        n_p = min(1 << int(np.floor(np.log2(nq))), 2048)
        o = int(sk["offset"][q])
        F = np.asarray(flux[o:o + n_p], dtype=np.float64)
        b = np.searchsorted(edges, chi_all[o:o + n_p], side="right") - 1
        b = np.clip(b, 0, nb - 1)
        d = F / fmean[b] - 1.0
        X = np.fft.rfft(d)
        m = np.arange(1, n_p // 2 + 1)
        P = dv * np.abs(X[1:]) ** 2 / n_p
        k = 2.0 * np.pi * m / (n_p * dv)
        kb = np.searchsorted(k_edges, k, side="right") - 1
        ok = (kb >= 0) & (kb < nk)
        np.add.at(psum, kb[ok], P[ok])
        np.add.at(cnt, kb[ok], 1)
    return psum, cnt
