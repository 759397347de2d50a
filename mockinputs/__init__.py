"""Seeded synthetic workloads for the Lyman-alpha mock hot path.

This module only builds inputs: box and spectrum parameters, quasar lines of
sight (the skewer table) and parameter draws.  It holds none of the method's
arithmetic (no field, no interpolation, no flux), so both the HIP path and the
oracle can take their inputs from here.  Random numbers used to lay out the
inputs come from numpy's seeded Generator; random numbers the method itself
draws (box noise, small-scale fields) are not made here.

Workloads (stand-ins for the paper's DESI/eBOSS footprint, which is not
available; shapes follow the paper: 2.19 Mpc/h voxels, 0.2 Mpc/h pixels,
redshifts 1.8-3.8):

tiny       64^3 box, 500 skewers of 256 pixels, origins uniform in the box,
           directions radial from a fixed observer, constant (a, b, c).
mid        512^3 box, 50,000 skewers, z_q ~ U[1.8, 3.6], 200-1200 pixels.
big        2048^3 box, 1,000,000 skewers, z_q ~ (1+z)^2 exp(-((z-2.3)/0.6)^2)
           on [1.8, 3.8], 200-2000 pixels.
precision  1024^3 box, 200,000 skewers, z_q ~ U[1.8, 3.6], 200-1200 pixels.
emulator   256^3 box, 20,000 skewers, z_q ~ U[1.8, 3.6], 200-1200 pixels.

Geometry: the observer sits at (L/2, L/2, -chi_obs) with chi_obs the comoving
distance to z = 2.5; a quasar at redshift z_q lies at distance chi(z_q) along
a direction within 5 degrees of +z; its forest starts at the red end
z_hi = (1 + z_q) 1200/1215.67 - 1 and runs towards the observer, one pixel
every 0.2 Mpc/h, for n_q pixels with n_q affine in z_q between the
workload's minimum and maximum.  Positions are handed over as int64 fixed
point (cell units times 2^32); the comoving distance of pixel 0 as FP64.
"""
import numpy as np

C_OVER_H0 = 2997.92458
OMEGA_M = 0.3147
DPIX = 0.2
LYA_A = 1215.67

PK_DEFAULT = dict(sigma8=0.8, ns=0.96, gamma=0.21, wig_amp=0.05, wig_r=105.0,
                  wig_kd=0.2)


def _quad_in_1pz(c0, c1, c2, x0=3.5):
    """Coefficients in powers of (1+z) of c0 + c1 x + c2 x^2, x = (1+z) - x0."""
    return [c0 - c1 * x0 + c2 * x0 * x0, c1 - 2.0 * c2 * x0, c2]


FGPA_CONST_TINY = [[0.5, 0.0, 0.0], [1.6, 0.0, 0.0], [1.0, 0.0, 0.0]]
FGPA_MID = [_quad_in_1pz(0.5, 0.4, 0.1), _quad_in_1pz(1.6, -0.1, 0.0),
            _quad_in_1pz(1.535, -1.018, 0.483)]

Z_EDGES = np.round(np.linspace(1.6, 3.8, 23), 10)

CONFIGS = {
    "tiny": dict(n=64, dx=2.19, seed=1234, n_sk=500, geometry="box",
                 npix_min=256, npix_max=256, fgpa=FGPA_CONST_TINY,
                 ps_amp=1.0, ps_kcut=1.5),
    "mid": dict(n=512, dx=2.19, seed=1234, n_sk=50_000, geometry="zq_uniform",
                zq_lo=1.8, zq_hi=3.6, npix_min=200, npix_max=1200,
                fgpa=FGPA_MID, ps_amp=1.0, ps_kcut=1.5),
    "big": dict(n=2048, dx=2.19, seed=1234, n_sk=1_000_000, geometry="zq_nz",
                zq_lo=1.8, zq_hi=3.8, npix_min=200, npix_max=2000,
                fgpa=FGPA_MID, ps_amp=1.0, ps_kcut=1.5),
    "precision": dict(n=1024, dx=2.19, seed=1234, n_sk=200_000,
                      geometry="zq_uniform", zq_lo=1.8, zq_hi=3.6,
                      npix_min=200, npix_max=1200, fgpa=FGPA_MID, ps_amp=1.0,
                      ps_kcut=1.5),
    "emulator": dict(n=256, dx=2.19, seed=1234, n_sk=20_000,
                     geometry="zq_uniform", zq_lo=1.8, zq_hi=3.6,
                     npix_min=200, npix_max=1200, fgpa=FGPA_MID, ps_amp=1.0,
                     ps_kcut=1.5),
}


# Lognormal quasar field: the paper's three box redshifts, the r range and
# nodes of the P_q transform (5 Mpc/h is node 100), a quasar density in
# (h/Mpc)^3 with the shape of the skewer n(z) peaking at 1e-5, and the
# observer of the quasar draw at (L/2, L/2, -chi(1.8)).
QSO_Z_BOXES = (1.9, 2.75, 3.6)
QSO_RMAX = 2000.0
QSO_NR = 40001
QSO_Z_OBS = 1.8


def qso_nbar():
    z = np.round(np.linspace(1.7, 4.0, 24), 10)
    shape = (1 + z) ** 2 * np.exp(-((z - 2.3) / 0.6) ** 2)
    return z, 1e-5 * shape / shape.max()


def qso_k_nodes(n, dx, count=512):
    """k nodes (h/Mpc) of the tabulated P_q: from half the fundamental mode to
    just past the box's largest |k|."""
    L = n * dx
    return np.geomspace(np.pi / L, 1.05 * np.sqrt(3.0) * np.pi / dx, count)


def qso_observer(n, dx):
    return np.array([n * dx / 2, n * dx / 2, -_Distance().chi_of(QSO_Z_OBS)])


def config(name, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    c["pk"] = dict(PK_DEFAULT)
    c["f"] = 1.0
    c["dpix"] = DPIX
    c["omega_m"] = OMEGA_M
    c["z_edges"] = Z_EDGES.copy()
    return c


class _Distance:
    """Comoving distance on a fine grid, only to place quasars (input
    layout; the method computes its own pixel redshifts)."""

    def __init__(self, zmax=6.0, n=200_001):
        z = np.linspace(0.0, zmax, n)
        inv_e = 1.0 / np.sqrt(OMEGA_M * (1 + z) ** 3 + 1 - OMEGA_M)
        chi = np.concatenate([[0.0], np.cumsum(0.5 * (inv_e[1:] + inv_e[:-1])
                                               * np.diff(z))]) * C_OVER_H0
        self.z, self.chi = z, chi

    def chi_of(self, z):
        return np.interp(z, self.z, self.chi)


def _to_fixed(cells):
    return np.round(np.asarray(cells, dtype=np.float64) * 2.0 ** 32).astype(np.int64)


def _draw_zq(rng, geometry, n, lo, hi):
    if geometry == "zq_uniform":
        return rng.uniform(lo, hi, n)
    # n(z) ~ (1+z)^2 exp(-((z-2.3)/0.6)^2) on [lo, hi] by inverse CDF
    zg = np.linspace(lo, hi, 20001)
    pdf = (1 + zg) ** 2 * np.exp(-((zg - 2.3) / 0.6) ** 2)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(zg))])
    cdf /= cdf[-1]
    return np.interp(rng.uniform(0.0, 1.0, n), cdf, zg)


def skewer_table(cfg, n_sk=None, seed=None, sort_by_length=True):
    """Skewer table (numpy arrays) for workload cfg.

    Keys: origin_fx [S,3] int64, step_fx [S,3] int64, npix [S] int32,
    offset [S] int64, chi0 [S] float64, dchi, id_base, total (pixels).
    Skewers are ordered by decreasing length when sort_by_length (longest
    first balances a work queue)."""
    n_sk = cfg["n_sk"] if n_sk is None else n_sk
    seed = cfg["seed"] if seed is None else seed
    rng = np.random.default_rng([seed, 2])
    n, dx = cfg["n"], cfg["dx"]
    L = n * dx
    dist = _Distance()
    obs = np.array([L / 2, L / 2, -dist.chi_of(2.5)])
    if cfg["geometry"] == "box":
        x0 = rng.uniform(0.0, L, (n_sk, 3))
        d = x0 - obs
        chi0 = np.linalg.norm(d, axis=1)
        u = d / chi0[:, None]
        npix = np.full(n_sk, cfg["npix_min"], dtype=np.int32)
    else:
        zq = _draw_zq(rng, cfg["geometry"], n_sk, cfg["zq_lo"], cfg["zq_hi"])
        cos_t = rng.uniform(np.cos(np.radians(5.0)), 1.0, n_sk)
        phi = rng.uniform(0.0, 2 * np.pi, n_sk)
        sin_t = np.sqrt(1.0 - cos_t ** 2)
        u = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)
        z_red = (1.0 + zq) * 1200.0 / LYA_A - 1.0
        chi0 = dist.chi_of(z_red)
        x0 = obs[None, :] + chi0[:, None] * u
        frac = (zq - cfg["zq_lo"]) / (cfg["zq_hi"] - cfg["zq_lo"])
        npix = np.round(cfg["npix_min"] + (cfg["npix_max"] - cfg["npix_min"])
                        * frac).astype(np.int32)
    if sort_by_length:
        order = np.argsort(-npix, kind="stable")
        x0, u, chi0, npix = x0[order], u[order], chi0[order], npix[order]
    offset = np.zeros(n_sk, dtype=np.int64)
    if n_sk > 1:
        offset[1:] = np.cumsum(npix[:-1].astype(np.int64))
    return dict(origin_fx=_to_fixed(x0 / dx), step_fx=_to_fixed(-DPIX * u / dx),
                npix=np.ascontiguousarray(npix, dtype=np.int32), offset=offset,
                chi0=np.ascontiguousarray(chi0, dtype=np.float64), dchi=DPIX,
                id_base=0, total=int(npix.astype(np.int64).sum()))


EMULATOR_RANGES = ((0.1, 2.0), (1.0, 2.2), (0.5, 2.0), (1.8, 3.6))
# Ranges that cover the tuning workload's solutions (a from ~0.008 at z=1.8 to
# ~2.7 at z=3.6 and c(1.8)=2.48 on these z=0 boxes), a drawn log-uniform
TUNE_EMULATOR_RANGES = ((1e-3, 5.0), (1.0, 2.2), (0.5, 2.6), (1.8, 3.6))


def emulator_draws(n, seed=1234, ranges=EMULATOR_RANGES, log_a=False):
    """(a, b, c, z) uniform in the given ranges (a log-uniform if log_a)."""
    rng = np.random.default_rng([seed, 3])
    (a0, a1), (b0, b1), (c0, c1), (z0, z1) = ranges
    a = np.exp(rng.uniform(np.log(a0), np.log(a1), n)) if log_a else rng.uniform(a0, a1, n)
    return np.stack([a, rng.uniform(b0, b1, n), rng.uniform(c0, c1, n), rng.uniform(z0, z1, n)], axis=1)


# ---------------------------------------------------------------- tuning workload
TUNE_Z = [1.8, 2.2, 2.6, 3.0, 3.6]
TUNE_K_BINS = (32, 0.001, 0.05)      # 32 log-spaced P1D bins over [0.001, 0.05] s/km


def fbar_target(z, f_lo=0.75, f_hi=0.35, z_lo=1.8, z_hi=3.6):
    """Target mean transmission of the tuning workload: log-linear in z from
    f_lo at z_lo to f_hi at z_hi."""
    t = (np.asarray(z, dtype=np.float64) - z_lo) / (z_hi - z_lo)
    return np.exp(np.log(f_lo) + t * (np.log(f_hi) - np.log(f_lo)))


def tune_c(z):
    """c(z_t) held fixed while tuning: the mid workload's c(z) quadratic."""
    x = 1.0 + np.asarray(z, dtype=np.float64)
    c = FGPA_MID[2]
    return c[0] + c[1] * x + c[2] * x * x


def paper_targets(z):
    """The paper's tuning targets at redshift z (section "Adjusting mock
    parameters"): the effective bias b_eff = 0.183 ((1+z)/3.3)^3.47 and the
    distortion parameter beta = 1.76 ((1+z)/3.3)^-2.32 of its power-law fits to
    the eBOSS DR16 forest, and the mean transmission exp(-0.0028 (1+z)^3.45)
    of the Calura et al. parameterisation.  Returns (b_eff, beta, Fbar)."""
    x = (1.0 + np.asarray(z, dtype=np.float64)) / 3.3
    b_eff = 0.183 * x ** 3.47
    beta = 1.76 * x ** -2.32
    fbar = np.exp(-0.0028 * (1.0 + np.asarray(z, dtype=np.float64)) ** 3.45)
    return b_eff, beta, fbar


def tune_k_edges():
    n, lo, hi = TUNE_K_BINS
    return lo * (hi / lo) ** (np.arange(n + 1) / n)


def tune_b_truth(z):
    """b(z_t) of the hidden parameters of the truth mock: the mid workload's
    b(z) quadratic."""
    x = 1.0 + np.asarray(z, dtype=np.float64)
    b = FGPA_MID[1]
    return b[0] + b[1] * x + b[2] * x * x
