"""Small-scale power iteration of the tuning (oracle, FP64).

TEST INFRASTRUCTURE ONLY: used by tests/, not by the library.

Follows section "Adjusting mock parameters": at each tuning redshift z_t,

1. a and s = b sigma_g are fixed so that a Gaussian g gives the target mean
   flux Fbar_t and the target flux dispersion sigma_F,t (both depend only on
   a and b sigma_g);
2. sigma_g^2 = sigma_L^2 + sigma_s^2 + c^2 sigma_eta^2 + 2 c cov(delta_L,
   eta_par), with sigma_L, sigma_eta and the covariance measured on the
   mock and sigma_s from the current P_s, gives b = s / sigma_g;
3. the spectra are drawn again with that P_s, passed through eq:FGPA, and
   their 1D flux power P1D measured; in each k bin
   P_s^{n+1} = P_s^n P_target / P1D;
4. ten iterations (the paper's number; an argument here).

Readings (the paper is silent or states these loosely):

* sigma_F,t comes from the target P1D integrated over its own bins (unless
  the caller knows the target dispersion itself, as for a synthetic truth):
  sigma_F,t^2 = Fbar_t^2 sum_b P_t,b (k_{b+1} - k_b) / pi (delta_F is
  F/Fbar - 1, and the 1D power of a real field integrates to its variance
  as (1/pi) int_0^inf P dk); bins with no target value add nothing;
* the Gaussian averages use adaptive quadrature (scipy.integrate.quad);
* P_s^n(k) = P_s^0(k) r_n(bin of k): P_s^0 the configuration's form
  amp exp(-(k/kcut)^2), r_0 = 1, the bins those of the P1D converted to
  h/Mpc at z_t (k = k_v dv/dchi, dv/dchi = 100 E(z_t)/(1+z_t)); wavenumbers
  below the first edge take the first bin's ratio and those above the last
  edge the last one's;
* sigma_s^2 = (1/pi) int_0^{pi/dpix} P_s(k) dk (the variance of the 1D field
  up to the pixel Nyquist wavenumber), piecewise in closed form with erf;
* the statistics of an iteration use every stored pixel under constant
  (a, b, c): Fbar = mean F and the P1D of delta_F = F/Fbar - 1 in velocity
  units at z_t (oracle.tune.evaluate's convention);
* delta_L and eta_par are the stored pixels without delta_S; delta_S is
  drawn per skewer exactly as oracle.skewers.delta_s (Philox stream 1,
  counter (q << 33) + m) with the amplitude sqrt(P_s^n(k_m) / (N_S dpix)).
The outer loop of the paper (adjusting a and b against the bias of the
correlation-function prediction) is not part of this reading.
"""
import numpy as np
from scipy import integrate, optimize, special

from . import cosmology, philox
from . import p1d as op1d
from .skewers import next_pow2


def gauss_fbar_sigf(a, s):
    """(Fbar, sigma_F) of F = exp(-a exp(s x)), x a unit normal: adaptive
    quadrature over [-12, 12] with a break point where a exp(s x) = 1 (F
    turns over there, steeply for large s)."""
    pdf = lambda x: np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)
    x0 = float(np.clip(-np.log(a) / s, -11.0, 11.0)) if s > 0 else 0.0
    f1 = integrate.quad(lambda x: np.exp(-a * np.exp(s * x)) * pdf(x), -12.0, 12.0, points=[x0],
                        epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    f2 = integrate.quad(lambda x: np.exp(-2.0 * a * np.exp(s * x)) * pdf(x), -12.0, 12.0, points=[x0],
                        epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    return f1, np.sqrt(max(f2 - f1 * f1, 0.0))


def fit_a_s(fbar_t, sigf_t, x0=(0.3, 0.5)):
    """(a, s) with gauss_fbar_sigf(a, s) = (fbar_t, sigf_t), solved in (ln a, ln s)."""
    def resid(t):
        f, sf = gauss_fbar_sigf(np.exp(t[0]), np.exp(t[1]))
        return [np.log(f / fbar_t), np.log(sf / sigf_t)]

    sol = optimize.root(resid, np.log(np.asarray(x0, dtype=np.float64)), method="hybr", tol=1e-14)
    return float(np.exp(sol.x[0])), float(np.exp(sol.x[1]))


def sigma_df2_target(pk_t, k_edges):
    """Variance of delta_F implied by the target P1D over its bins."""
    pk_t = np.asarray(pk_t, dtype=np.float64)
    dk = np.diff(np.asarray(k_edges, dtype=np.float64))
    ok = np.isfinite(pk_t)
    return float(np.sum(pk_t[ok] * dk[ok]) / np.pi)


def dv_per_dchi(z_t, omega_m=cosmology.OMEGA_M):
    return float(cosmology.dv_per_dchi(z_t, omega_m))


def ratio_of_k(k, ratio, edges_k):
    """r(bin of k) with the ends clamped."""
    b = np.searchsorted(np.asarray(edges_k, dtype=np.float64), k, side="right") - 1
    return np.asarray(ratio, dtype=np.float64)[np.clip(b, 0, len(ratio) - 1)]


def ps_of_k(k, amp, kcut, ratio, edges_k):
    return amp * np.exp(-(np.asarray(k, dtype=np.float64) / kcut) ** 2) * ratio_of_k(k, ratio, edges_k)


def sigma_s2(amp, kcut, ratio, edges_k, dpix):
    """(1/pi) int_0^{pi/dpix} P_s(k) dk for the piecewise form above."""
    kmax = np.pi / dpix
    e = np.asarray(edges_k, dtype=np.float64)
    cuts = np.concatenate([[0.0], np.clip(e, 0.0, kmax), [kmax]])
    rs = np.concatenate([[ratio[0]], ratio, [ratio[-1]]])
    tot = 0.0
    for i in range(len(cuts) - 1):
        lo, hi = cuts[i], cuts[i + 1]
        if hi > lo:
            tot += rs[i] * amp * kcut * np.sqrt(np.pi) / 2.0 * (special.erf(hi / kcut) - special.erf(lo / kcut))
    return tot / np.pi


def delta_s_tab(seed, qid, npix, dpix, amp, kcut, ratio, edges_k):
    """delta_S of quasar qid with P_s = amp exp(-(k/kcut)^2) r(bin of k)."""
    ns = next_pow2(npix)
    m = np.arange(ns // 2 + 1, dtype=np.int64)
    k = 2.0 * np.pi * m / (ns * dpix)
    a = np.sqrt(ps_of_k(k, amp, kcut, ratio, edges_k) / (ns * dpix))
    a[0] = 0.0
    lin = (np.uint64(qid) << np.uint64(33)) + m.astype(np.uint64)
    z1, z2 = philox.normal_pair(seed, 1, lin)
    w = (z1 + 1j * z2) / np.sqrt(2.0)
    w[-1] = z1[-1]
    full = np.fft.irfft(a * w, n=ns) * ns
    return full[:npix]


def moments(dl, eta):
    """(sigma_L^2, sigma_eta^2, cov) over all pixels."""
    dl = np.asarray(dl, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    ml, me = dl.mean(), eta.mean()
    return float(np.mean(dl * dl) - ml * ml), float(np.mean(eta * eta) - me * me), float(np.mean(dl * eta) - ml * me)


def iterate(dl, eta, sk, seed, z_t, c_t, fbar_t, pk_t, k_edges, dpix, amp0, kcut0, n_iter=10,
            omega_m=cosmology.OMEGA_M, sigf_t=None):
    """The procedure above at one z_t.  Returns a, b of the last iteration, the
    ratios it used, and per iteration (Fbar, P1D, sigma_g).  sigf_t, when
    given, is the target flux dispersion itself (a synthetic truth knows it);
    otherwise it comes from the target P1D over its bins."""
    k_edges = np.asarray(k_edges, dtype=np.float64)
    nk = len(k_edges) - 1
    edges_k = k_edges * dv_per_dchi(z_t, omega_m)
    if sigf_t is None:
        sigf_t = fbar_t * np.sqrt(sigma_df2_target(pk_t, k_edges))
    a, s = fit_a_s(fbar_t, sigf_t)
    sl2, se2, cov = moments(dl, eta)
    ratio = np.ones(nk)
    npix = np.asarray(sk["npix"])
    off = np.asarray(sk["offset"])
    hist = []
    for it in range(n_iter):
        used = ratio.copy()
        ss2 = sigma_s2(amp0, kcut0, used, edges_k, dpix)
        sg = np.sqrt(sl2 + ss2 + c_t * c_t * se2 + 2.0 * c_t * cov)
        b = s / sg
        dens = np.array(dl, dtype=np.float64, copy=True)
        for q in range(len(npix)):
            o, nq = int(off[q]), int(npix[q])
            if nq > 0:
                dens[o:o + nq] += delta_s_tab(seed, int(sk["id_base"]) + q, nq, dpix, amp0, kcut0, used, edges_k)
        F = np.exp(-a * np.exp(b * (dens + c_t * np.asarray(eta, dtype=np.float64))))
        fbar = float(np.mean(F))
        ps, cnt = op1d.p1d(F, sk, [-1e30, 1e30], [fbar], k_edges, z_t, dpix, omega_m)
        with np.errstate(invalid="ignore", divide="ignore"):
            pk = np.where(cnt > 0, ps / np.maximum(cnt, 1), np.nan)
        hist.append(dict(fbar=fbar, p1d=pk, sigma_g=float(sg), b=float(b), ratio=used))
        upd = np.isfinite(pk_t) & np.isfinite(pk) & (pk > 0)
        ratio = used.copy()
        ratio[upd] = used[upd] * np.asarray(pk_t)[upd] / pk[upd]
    return dict(a=a, s=s, b=hist[-1]["b"], ratio=hist[-1]["ratio"], hist=hist,
                moments=(sl2, se2, cov))
