"""Plain parameter tuning of the FGPA (oracle, FP64).

Follows section "Adjusting mock parameters": at each tuning redshift z_t the
FGPA parameters are chosen so that the mocks reproduce a target mean
transmission and 1D flux power spectrum, then interpolated in redshift.

Readings (the paper uses Minuit and an iterative P_s update that is out of
scope here):

* c_GP(z_t) is fixed (c = beta/f, the paper's RSD relation);
* the model statistics at z_t come from the stored pre-FGPA pixels with
  constant (a, b, c) over every pixel (the paper's post-production reuse):
  Fbar = mean F, and P1D by oracle.p1d with velocity units at z_t and
  delta_F = F / Fbar - 1;
* the objective is chi^2 = ((Fbar - Fbar_t)/(s Fbar_t))^2
  + sum_bins ((P_b - P_t,b)/(s P_t,b))^2 with s = 0.002, minimised over
  (ln a, ln b) by Nelder-Mead (scipy.optimize.minimize);
* a(z), b(z), c(z) are then least-squares quadratics in (1+z) through the
  tuned points (numpy.polyfit).
"""
import numpy as np
from scipy import optimize

from . import p1d as op1d

SIGMA_REL = 0.002


def evaluate(dens, eta, sk, a, b, c, z_ref, k_edges, dpix, omega_m=0.3147):
    """(Fbar, P1D per bin) of the pixels under constant (a, b, c)."""
    F = np.exp(-a * np.exp(b * (np.asarray(dens, np.float64) + c * np.asarray(eta, np.float64))))
    fbar = float(np.mean(F))
    ps, cnt = op1d.p1d(F, sk, [-1e30, 1e30], [fbar], k_edges, z_ref, dpix, omega_m)
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = np.where(cnt > 0, ps / np.maximum(cnt, 1), np.nan)
    return fbar, pk


def chi2(fbar, pk, fbar_t, pk_t):
    ok = np.isfinite(pk_t) & np.isfinite(pk)
    r = ((fbar - fbar_t) / (SIGMA_REL * fbar_t)) ** 2
    r += np.sum(((pk[ok] - pk_t[ok]) / (SIGMA_REL * pk_t[ok])) ** 2)
    return float(r)


def tune_one(dens, eta, sk, z_t, c_t, fbar_t, pk_t, k_edges, dpix, x0=(0.3, 1.5), omega_m=0.3147,
             xatol=1e-6, fatol=1e-8, maxfev=400):
    """Nelder-Mead over (ln a, ln b); returns a, b, Fbar, P1D, evaluations."""
    nfev = [0]

    def f(t):
        nfev[0] += 1
        fb, pk = evaluate(dens, eta, sk, np.exp(t[0]), np.exp(t[1]), c_t, z_t, k_edges, dpix, omega_m)
        return chi2(fb, pk, fbar_t, pk_t)

    res = optimize.minimize(f, np.log(np.asarray(x0, dtype=np.float64)), method="Nelder-Mead",
                            options=dict(xatol=xatol, fatol=fatol, maxfev=maxfev,
                                         initial_simplex=np.log(np.asarray(x0))[None, :]
                                         + np.array([[0, 0], [0.3, 0], [0, 0.3]])))
    a, b = float(np.exp(res.x[0])), float(np.exp(res.x[1]))
    fb, pk = evaluate(dens, eta, sk, a, b, c_t, z_t, k_edges, dpix, omega_m)
    return dict(a=a, b=b, fbar=fb, p1d=pk, nfev=nfev[0], chi2=float(res.fun))


def fit_quadratics(z_t, a_t, b_t, c_t):
    """coef[p][i] of a, b, c = sum_i coef[p][i] (1+z)^i (least squares)."""
    x = 1.0 + np.asarray(z_t, dtype=np.float64)
    out = []
    for vals in (a_t, b_t, c_t):
        p = np.polyfit(x, np.asarray(vals, dtype=np.float64), 2)   # highest power first
        out.append([p[2], p[1], p[0]])
    return out
