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

A second per-bin update (not in the paper; update="secant"): the paper's
rule multiplies each bin's P_s by P_t/P1D as if the bin's P1D answered one
to one, while with b sigma_g fixed it answers less.  From the second
iteration of a run on, each bin's response gamma = d ln P1D / d ln r is
estimated from the last two iterations (the secant) and the step becomes
r <- r (P_t/P1D)^w with w = 1/gamma clipped to [1, 3] (w = 1 where the
secant is undefined: the ratio moved by 1e-6 or less in log, or gamma
<= 0.05).  Each outer step starts a new run (no secant across a change of
(a, s)).

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

The outer loop (the paper adjusts a and b so that the bias its
correlation-function prediction implies approaches the target while Fbar
stays, then runs the P_s iteration again; five times), read as:

* the large-scale flux bias with respect to delta_L is the first term of the
  bivariate-Gaussian expansion of the flux correlation: b_F = E[dF/dg] /
  Fbar = -(a s / sigma_g) E[e^{s x} F] / Fbar (Stein's identity; g =
  delta_L + delta_S + c eta_par responds one to one to a long delta_L mode,
  delta_S being uncorrelated), beta_F = f c (the paper's f c(z_t) = beta);
  the target is the effective bias |b_F| (1 + 2 beta/3 + beta^2/5)^(1/2);
* outer step o >= 1: sigma_g from the current P_s (the ratios after the last
  update), (a, s) solve Fbar(a, s) = Fbar_t and b_eff(a, s; sigma_g) =
  b_eff,t, and the P_s iteration runs again from the current ratios; outer
  step 0 is the (Fbar, sigma_F) fit above;
* at fixed Fbar the bias tends to phi(x_0) / (sigma_g Fbar), x_0 =
  Phi^{-1}(Fbar), as s grows (F becomes a step), so a target beyond what the
  current sigma_g allows has no solution: the outer loop then stops and keeps
  the last step (a poor first step, e.g. sigma_F from a binned P1D that
  misses most of the power, leads there).

The emulator mode of the library (not in the paper) solves, at each z_t, the
problem the iteration approaches: P_s keeps the configuration's form
amp exp(-(k/kcut)^2) with (amp, kcut) free, (a, s) follow from (Fbar_t,
sigma_F,t), or with the outer loop from (Fbar_t, b_eff,t) at the sigma_g of
(amp, kcut), b = s / sigma_g, and (amp, kcut) minimise
sum_b (P1D_b / P_t,b - 1)^2 over the bins with a target.  ps_fit_problem
states that objective; statistics_ps is one evaluation of it (and one
emulator training label).
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


def flux_bias(a, s, sigma_g):
    """b_F = -(a s / sigma_g) E[e^{s x} F(x)] / Fbar, F = exp(-a exp(s x))."""
    pdf = lambda x: np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)
    x0 = float(np.clip(-np.log(a) / s, -11.0, 11.0)) if s > 0 else 0.0
    m = integrate.quad(lambda x: np.exp(s * x - a * np.exp(s * x)) * pdf(x), -12.0, 12.0, points=[x0],
                       epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    fbar = gauss_fbar_sigf(a, s)[0]
    return -(a * s / sigma_g) * m / fbar


def kaiser_factor(beta):
    """(1 + 2 beta/3 + beta^2/5)^(1/2): the monopole of (1 + beta mu^2)^2."""
    return float(np.sqrt(1.0 + 2.0 * beta / 3.0 + beta * beta / 5.0))


def effective_bias(a, s, sigma_g, beta):
    return abs(flux_bias(a, s, sigma_g)) * kaiser_factor(beta)


def fit_a_s_bias(fbar_t, beff_t, sigma_g, beta, x0=(0.3, 0.5)):
    """(a, s) with Fbar(a, s) = fbar_t and b_eff(a, s; sigma_g) = beff_t, or
    None when the solve fails."""
    def resid(t):
        a, s = np.exp(t[0]), np.exp(t[1])
        return [np.log(gauss_fbar_sigf(a, s)[0] / fbar_t), np.log(effective_bias(a, s, sigma_g, beta) / beff_t)]

    sol = optimize.root(resid, np.log(np.asarray(x0, dtype=np.float64)), method="hybr", tol=1e-14)
    if not np.all(np.isfinite(sol.x)) or np.max(np.abs(resid(sol.x))) > 1e-9:
        return None
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


def sigma_s2_gauss(amp, kcut, dpix):
    """(1/pi) int_0^{pi/dpix} amp exp(-(k/kcut)^2) dk in closed form:
    amp kcut erf(pi / (dpix kcut)) / (2 sqrt(pi))."""
    return float(amp * kcut * special.erf(np.pi / (dpix * kcut)) / (2.0 * np.sqrt(np.pi)))


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


def update_ratio(ratio, pk, pk_t, prev=None, update="paper"):
    """The per-bin update of step 3 (update="paper") or the secant form
    above (update="secant"; prev = (ratio, P1D) of the previous iteration of
    the run, None at its first).  Bins without a finite positive P1D and a
    finite target keep their ratio."""
    ratio = np.asarray(ratio, dtype=np.float64)
    pk = np.asarray(pk, dtype=np.float64)
    pk_t = np.asarray(pk_t, dtype=np.float64)
    upd = np.isfinite(pk_t) & np.isfinite(pk) & (pk > 0)
    w = np.ones_like(ratio)
    if update == "secant" and prev is not None:
        r0, p0 = (np.asarray(x, dtype=np.float64) for x in prev)
        for b in np.flatnonzero(upd):
            if not (np.isfinite(p0[b]) and p0[b] > 0):
                continue
            dr = np.log(ratio[b]) - np.log(r0[b])
            if abs(dr) <= 1e-6:
                continue
            gam = (np.log(pk[b]) - np.log(p0[b])) / dr
            if gam > 0.05:
                w[b] = min(max(1.0 / gam, 1.0), 3.0)
    elif update not in ("paper", "secant"):
        raise ValueError("update is 'paper' or 'secant'")
    out = ratio.copy()
    out[upd] = ratio[upd] * (pk_t[upd] / pk[upd]) ** w[upd]
    return out


def iterate(dl, eta, sk, seed, z_t, c_t, fbar_t, pk_t, k_edges, dpix, amp0, kcut0, n_iter=10,
            omega_m=cosmology.OMEGA_M, sigf_t=None, n_outer=1, beff_t=None, f=1.0, update="paper"):
    """The procedure above at one z_t.  Returns a, b of the last iteration, the
    ratios it used, and per iteration (Fbar, P1D, sigma_g).  sigf_t, when
    given, is the target flux dispersion itself (a synthetic truth knows it);
    otherwise it comes from the target P1D over its bins.  n_outer > 1 adds
    outer steps (target effective bias beff_t, beta = f c_t); "beff" holds
    the predicted effective bias after each outer step run and "hist" the
    iterations of the last one."""
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
    beta = f * c_t
    sg_of = lambda r: np.sqrt(sl2 + sigma_s2(amp0, kcut0, r, edges_k, dpix) + c_t * c_t * se2 + 2.0 * c_t * cov)
    beff = []
    for o in range(n_outer):
        if o > 0:
            fit = fit_a_s_bias(fbar_t, beff_t, sg_of(ratio), beta, x0=(a, s))
            if fit is None:
                break
            a, s = fit
        hist, ratio = _inner(dl, eta, sk, seed, z_t, c_t, pk_t, k_edges, edges_k, dpix, amp0, kcut0, n_iter,
                             omega_m, a, s, ratio, sl2, se2, cov, npix, off, update)
        beff.append(effective_bias(a, s, hist[-1]["sigma_g"], beta))
    return dict(a=a, s=s, b=hist[-1]["b"], ratio=hist[-1]["ratio"], hist=hist,
                moments=(sl2, se2, cov), beff=beff)


def _inner(dl, eta, sk, seed, z_t, c_t, pk_t, k_edges, edges_k, dpix, amp0, kcut0, n_iter, omega_m, a, s, ratio,
           sl2, se2, cov, npix, off, update="paper"):
    """n_iter P_s iterations from the given ratios; returns their history and
    the ratios after the last update."""
    hist = []
    prev = None
    for it in range(n_iter):
        used = ratio.copy()
        ss2 = sigma_s2(amp0, kcut0, used, edges_k, dpix)
        sg = np.sqrt(sl2 + ss2 + c_t * c_t * se2 + 2.0 * c_t * cov)
        b = s / sg
        fbar, pk = _statistics(dl, eta, sk, seed, z_t, c_t, a, b, amp0, kcut0, used, edges_k, k_edges, dpix, omega_m)
        hist.append(dict(fbar=fbar, p1d=pk, sigma_g=float(sg), b=float(b), ratio=used))
        ratio = update_ratio(used, pk, pk_t, prev, update)
        prev = (used, pk)
    return hist, ratio


def _statistics(dl, eta, sk, seed, z_t, c_t, a, b, amp, kcut, ratio, edges_k, k_edges, dpix, omega_m):
    """Fbar and the P1D per bin of the stored pixels with delta_S of
    P_s = amp exp(-(k/kcut)^2) r(bin of k) added, under constant (a, b, c_t)."""
    npix = np.asarray(sk["npix"])
    off = np.asarray(sk["offset"])
    dens = np.array(dl, dtype=np.float64, copy=True)
    for q in range(len(npix)):
        o, nq = int(off[q]), int(npix[q])
        if nq > 0:
            dens[o:o + nq] += delta_s_tab(seed, int(sk["id_base"]) + q, nq, dpix, amp, kcut, ratio, edges_k)
    F = np.exp(-a * np.exp(b * (dens + c_t * np.asarray(eta, dtype=np.float64))))
    fbar = float(np.mean(F))
    ps, cnt = op1d.p1d(F, sk, [-1e30, 1e30], [fbar], k_edges, z_t, dpix, omega_m)
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = np.where(cnt > 0, ps / np.maximum(cnt, 1), np.nan)
    return fbar, pk


def statistics_ps(dl, eta, sk, seed, z_t, c_t, a, b, amp, kcut, k_edges, dpix, omega_m=cosmology.OMEGA_M):
    """(Fbar, P1D per bin) with delta_S of P_s = amp exp(-(k/kcut)^2) (no
    table) redrawn on every skewer and constant (a, b, c_t) at z_t."""
    k_edges = np.asarray(k_edges, dtype=np.float64)
    one = np.ones(len(k_edges) - 1)
    return _statistics(dl, eta, sk, seed, z_t, c_t, a, b, amp, kcut, one, k_edges * dv_per_dchi(z_t, omega_m),
                       k_edges, dpix, omega_m)


def ps_fit_problem(dl, eta, sk, seed, z_t, c_t, fbar_t, pk_t, k_edges, dpix, omega_m=cosmology.OMEGA_M,
                   sigf_t=None, beff_t=None, f=1.0):
    """The emulator mode's problem at one z_t as a function of
    th = (ln amp, ln kcut): returns a callable giving (a, b, s, Fbar, P1D,
    objective) at th, the objective sum_b (P1D_b / P_t,b - 1)^2 over the bins
    with a finite target.  (a, s) from (fbar_t, sigma_F,t) when beff_t is
    None, else from (fbar_t, beff_t) at sigma_g(th) (beta = f c_t)."""
    k_edges = np.asarray(k_edges, dtype=np.float64)
    pk_t = np.asarray(pk_t, dtype=np.float64)
    if sigf_t is None:
        sigf_t = fbar_t * np.sqrt(sigma_df2_target(pk_t, k_edges))
    sl2, se2, cov = moments(dl, eta)
    sig0 = sl2 + c_t * c_t * se2 + 2.0 * c_t * cov
    a0, s0 = fit_a_s(fbar_t, sigf_t)
    ok = np.isfinite(pk_t)

    def at(th):
        amp, kcut = float(np.exp(th[0])), float(np.exp(th[1]))
        sg = np.sqrt(sig0 + sigma_s2_gauss(amp, kcut, dpix))
        if beff_t is None:
            a, s = a0, s0
        else:
            fit = fit_a_s_bias(fbar_t, beff_t, sg, f * c_t, x0=(a0, s0))
            if fit is None:
                return None
            a, s = fit
        b = s / sg
        fbar, pk = statistics_ps(dl, eta, sk, seed, z_t, c_t, a, b, amp, kcut, k_edges, dpix, omega_m)
        obj = float(np.sum((pk[ok] / pk_t[ok] - 1.0) ** 2))
        return dict(a=a, b=b, s=s, sigma_g=float(sg), fbar=fbar, p1d=pk, objective=obj)

    return at
