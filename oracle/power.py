"""Linear matter power spectrum and the per-mode amplitude table (oracle, FP64).

The paper scales unit white noise by sqrt(P_m(k)/V) in k-space (eq:deltaL and
section "Mock generation"), with P_m from CAMB.  CAMB is not available, so the
workload stand-in is analytic:

    P(k) = A k^ns T_BBKS(k/Gamma)^2 (1 + w_amp sin(k r_w) exp(-(k/k_d)^2))

with the BBKS transfer function (Bardeen, Bond, Kaiser & Szalay 1986)

    T(q) = ln(1 + 2.34 q)/(2.34 q) [1 + 3.89 q + (16.1 q)^2 + (5.46 q)^3 + (6.71 q)^4]^(-1/4)

and A fixed by sigma8: sigma_R^2 = 1/(2 pi^2) int k^3 P(k) W_TH(kR)^2 dln k,
R = 8 Mpc/h, W_TH(x) = 3 (sin x - x cos x)/x^3 (the sphere window quoted in
section "The expected auto-correlation function of the mocks").

Reading of the normalisation (paper ambiguous): eq:deltaL divides by the box
volume V while the text multiplies real-space unit noise by sqrt(P/V_vox).
Both give the same field; with unit-variance complex k-space noise W the
per-mode amplitude is s(n^2) = sqrt(P(k)/V_box), k = 2 pi |n| / L, and s(0)=0.

Quadrature (paper silent): composite Simpson in ln k over [1e-5, 1e3] h/Mpc
with 2**16 + 1 nodes.

Optional smoothing: the Gaussian window of Appendix B, W^2 = exp(-dx^2 k^2),
applied to the amplitude as exp(-k^2 sigma^2 / 2) with sigma = smooth.

Pins: small-q Taylor coefficients of T (first and second order, derived by
hand), the large-q asymptote, the white-noise top-hat variance 3/(4 pi R^3),
and scipy.integrate.quad on the sigma8 integral.  The 5.46 coefficient only
enters at third order and is not separately pinned.
"""
import numpy as np

LNK_MIN = np.log(1e-5)
LNK_MAX = np.log(1e3)
N_SIMPSON = 2 ** 16 + 1


def t_bbks(q):
    q = np.asarray(q, dtype=np.float64)
    x = 2.34 * q
    lead = np.where(x > 0, np.log1p(x) / np.where(x > 0, x, 1.0), 1.0)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return lead * poly ** -0.25


def pk_shape(k, ns=0.96, gamma=0.21, wig_amp=0.05, wig_r=105.0, wig_kd=0.2):
    """P(k)/A for the analytic stand-in spectrum (k in h/Mpc)."""
    k = np.asarray(k, dtype=np.float64)
    wig = 1.0 + wig_amp * np.sin(k * wig_r) * np.exp(-(k / wig_kd) ** 2)
    return k ** ns * t_bbks(k / gamma) ** 2 * wig


def w_tophat(x):
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-2
    xs = np.where(small, 1.0, x)
    full = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    series = 1.0 - x ** 2 / 10.0 + x ** 4 / 280.0
    return np.where(small, series, full)


def sigma_r2(pk_func, r=8.0):
    """sigma_R^2 by Simpson's rule in ln k (2**16+1 nodes on [1e-5, 1e3])."""
    lnk = np.linspace(LNK_MIN, LNK_MAX, N_SIMPSON)
    k = np.exp(lnk)
    f = k ** 3 * pk_func(k) * w_tophat(k * r) ** 2
    h = (LNK_MAX - LNK_MIN) / (N_SIMPSON - 1)
    wts = np.ones(N_SIMPSON)
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    return h / 3.0 * np.sum(wts * f) / (2.0 * np.pi ** 2)


class PowerSpectrum:
    """Analytic P(k) normalised to sigma8."""

    def __init__(self, sigma8=0.8, ns=0.96, gamma=0.21, wig_amp=0.05,
                 wig_r=105.0, wig_kd=0.2):
        self.params = dict(ns=ns, gamma=gamma, wig_amp=wig_amp, wig_r=wig_r,
                           wig_kd=wig_kd)
        self.sigma8 = sigma8
        s2 = sigma_r2(lambda k: pk_shape(k, **self.params), 8.0)
        self.amp = sigma8 ** 2 / s2

    def __call__(self, k):
        return self.amp * pk_shape(k, **self.params)


class TabulatedPower:
    """P(k) from a table (the paper's CAMB spectrum is one): ln P linear in
    ln k between the nodes, the end intervals' power laws continued outside."""

    def __init__(self, k_tab, p_tab):
        self.lk = np.log(np.asarray(k_tab, dtype=np.float64))
        self.lp = np.log(np.asarray(p_tab, dtype=np.float64))

    def __call__(self, k):
        x = np.log(np.asarray(k, dtype=np.float64))
        i = np.clip(np.searchsorted(self.lk, x, side="right") - 1, 0, len(self.lk) - 2)
        t = (x - self.lk[i]) / (self.lk[i + 1] - self.lk[i])
        return np.exp(self.lp[i] + t * (self.lp[i + 1] - self.lp[i]))


def amplitude_table(pk, n, dx, smooth=0.0):
    """s(n^2) for every integer n^2 in [0, 3 (n/2)^2] (index = n^2)."""
    L = n * dx
    vbox = L ** 3
    nmax = 3 * (n // 2) ** 2
    n2 = np.arange(nmax + 1, dtype=np.float64)
    k = 2.0 * np.pi * np.sqrt(n2) / L
    kk = np.where(n2 > 0, k, 1.0)
    s = np.sqrt(pk(kk) / vbox)
    if smooth > 0.0:
        s = s * np.exp(-0.5 * (kk * smooth) ** 2)
    s[0] = 0.0
    return s
