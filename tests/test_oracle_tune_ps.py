"""Pins of the oracle's small-scale power iteration (section "Adjusting mock
parameters")."""
import numpy as np
import pytest
from scipy import integrate

import mockinputs
from oracle import field, fgpa, p1d, skewers, tune_ps
from tests.lyahelp import oracle_table


@pytest.mark.parametrize("a,s", [(0.2, 0.5), (1.0, 1.2), (3.0, 0.3)])
def test_gaussian_flux_moments_against_gauss_hermite(a, s):
    # an independent rule where it is accurate (moderate s): 100-node Gauss-Hermite
    f1, sf = tune_ps.gauss_fbar_sigf(a, s)
    x, w = np.polynomial.hermite.hermgauss(100)
    u = np.sqrt(2.0) * s * x
    g1 = np.sum(w * np.exp(-a * np.exp(u))) / np.sqrt(np.pi)
    g2 = np.sum(w * np.exp(-2 * a * np.exp(u))) / np.sqrt(np.pi)
    np.testing.assert_allclose(f1, g1, rtol=1e-10)
    np.testing.assert_allclose(sf, np.sqrt(g2 - g1 * g1), rtol=1e-8)


@pytest.mark.parametrize("a,s", [(0.37, 3.96), (0.05, 6.0)])
def test_gaussian_flux_moments_steep(a, s):
    # steep F(x): a fine Riemann sum (Simpson on 200,001 nodes) as the check
    f1, sf = tune_ps.gauss_fbar_sigf(a, s)
    x = np.linspace(-12, 12, 200001)
    pdf = np.exp(-0.5 * x * x) / np.sqrt(2 * np.pi)
    F = np.exp(-a * np.exp(s * x))
    g1 = integrate.simpson(F * pdf, x=x)
    g2 = integrate.simpson(F * F * pdf, x=x)
    np.testing.assert_allclose(f1, g1, rtol=1e-10)
    np.testing.assert_allclose(sf, np.sqrt(g2 - g1 * g1), rtol=1e-9)


def test_gaussian_flux_moments_limits():
    # s -> 0: F is the constant exp(-a)
    f1, sf = tune_ps.gauss_fbar_sigf(0.7, 1e-9)
    np.testing.assert_allclose(f1, np.exp(-0.7), rtol=1e-12)
    assert sf < 1e-8


def test_fit_recovers_a_and_s():
    for a, s in ((0.25, 0.7), (1.3, 1.9), (0.05, 0.4)):
        f1, sf = tune_ps.gauss_fbar_sigf(a, s)
        ra, rs = tune_ps.fit_a_s(f1, sf)
        np.testing.assert_allclose([ra, rs], [a, s], rtol=1e-8)


def test_sigma_s2_matches_numerical_integral():
    k_edges = p1d.log_k_edges()
    edges_k = k_edges * tune_ps.dv_per_dchi(2.4)
    ratio = 1.0 + 0.5 * np.sin(np.arange(len(k_edges) - 1))
    dpix = 0.2
    got = tune_ps.sigma_s2(1.3, 1.1, ratio, edges_k, dpix)
    pts = np.concatenate([[0.0], edges_k, [np.pi / dpix]])
    num = sum(integrate.quad(lambda k: tune_ps.ps_of_k(k, 1.3, 1.1, ratio, edges_k), lo, hi,
                             epsabs=1e-14, limit=200)[0] for lo, hi in zip(pts[:-1], pts[1:]))
    np.testing.assert_allclose(got, num / np.pi, rtol=1e-10)


def test_unit_ratios_reproduce_delta_s():
    k_edges = p1d.log_k_edges()
    edges_k = k_edges * tune_ps.dv_per_dchi(2.0)
    for q, n in ((3, 256), (9, 700), (12, 1)):
        a = tune_ps.delta_s_tab(77, q, n, 0.2, 1.0, 1.5, np.ones(len(k_edges) - 1), edges_k)
        b = skewers.delta_s(77, q, n, 0.2, 1.0, 1.5)
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def test_ratios_scale_the_mode_amplitudes():
    # a ratio r in one bin multiplies the modes inside it by sqrt(r)
    k_edges = p1d.log_k_edges()
    edges_k = k_edges * tune_ps.dv_per_dchi(2.0)
    n, dpix = 1024, 0.2
    r = np.ones(len(k_edges) - 1)
    r[20] = 4.0
    base = np.fft.rfft(tune_ps.delta_s_tab(5, 2, n, dpix, 1.0, 1.5, np.ones_like(r), edges_k))
    mod = np.fft.rfft(tune_ps.delta_s_tab(5, 2, n, dpix, 1.0, 1.5, r, edges_k))
    k = 2 * np.pi * np.arange(n // 2 + 1) / (n * dpix)
    inside = (k >= edges_k[20]) & (k < edges_k[21])
    assert inside.sum() > 0
    np.testing.assert_allclose(mod[inside], 2.0 * base[inside], rtol=1e-12)
    np.testing.assert_allclose(mod[~inside], base[~inside], rtol=1e-12, atol=1e-12)


def test_paper_update_is_the_ratio_of_target_to_measured_power():
    r = np.array([1.0, 2.0, 0.5, 1.5, 3.0])
    pk = np.array([2.0, 1.0, np.nan, 0.0, 4.0])
    pk_t = np.array([1.0, 3.0, 1.0, 1.0, np.nan])
    out = tune_ps.update_ratio(r, pk, pk_t)
    np.testing.assert_array_equal(out, [0.5, 6.0, 0.5, 1.5, 3.0])   # bins 2-4: no finite positive pair
    # the secant form at the first iteration of a run is the same step
    np.testing.assert_array_equal(tune_ps.update_ratio(r, pk, pk_t, None, "secant"), out)
    with pytest.raises(ValueError):
        tune_ps.update_ratio(r, pk, pk_t, None, "newton")


def test_secant_update_lands_on_the_target_for_a_power_law_response():
    # P1D_b = c_b r_b^gamma_b: the secant of two iterations is gamma_b exactly,
    # and the step (P_t/P1D)^(1/gamma) reaches the target in one move when
    # 1/gamma lies in [1, 3]; outside, the exponent is clipped (gamma = 2: the
    # paper's step; gamma = 0.1: exponent 3), and gamma <= 0.05 (here a
    # response that falls) or a ratio that did not move takes the paper's step
    c = np.array([2.0, 0.7, 1.3, 0.9, 1.1, 1.6, 0.8])
    gam = np.array([1.0, 0.5, 0.4, 2.0, 0.1, -0.3, 0.6])
    pk_t = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    P = lambda r: c * r ** gam
    r0 = np.ones(7)
    r1 = tune_ps.update_ratio(r0, P(r0), pk_t, None, "secant")
    r1[6] = r0[6] * (1 + 1e-8)             # this bin's ratio barely moved
    r2 = tune_ps.update_ratio(r1, P(r1), pk_t, (r0, P(r0)), "secant")
    p1, p2 = P(r1), P(r2)
    np.testing.assert_allclose(p2[:3], pk_t[:3], rtol=1e-12)
    np.testing.assert_allclose(p2[3], p1[3] * (pk_t[3] / p1[3]) ** 2, rtol=1e-12)
    np.testing.assert_allclose(p2[4], p1[4] * (pk_t[4] / p1[4]) ** 0.3, rtol=1e-12)
    np.testing.assert_allclose(r2[5], r1[5] * pk_t[5] / p1[5], rtol=1e-12)
    np.testing.assert_allclose(r2[6], r1[6] * pk_t[6] / p1[6], rtol=1e-12)


def test_iteration_converges_towards_a_target_from_another_small_scale_power():
    cfg = mockinputs.config("tiny")
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    box = field.make_box(n, seed, oracle_table(cfg["pk"], n, dx), ("delta", "zz"), f=cfg["f"])
    sk = mockinputs.skewer_table(cfg)
    dl, eta = skewers.draw_skewers(box.real, box.imag, sk, seed)          # no delta_S
    k_edges = p1d.log_k_edges()
    z_t, c_t = 2.4, 1.2
    # truth: delta_S of another amplitude and cut-off (and other draws), known FGPA
    truth = np.array(dl, copy=True)
    for q in range(len(sk["npix"])):
        o, m = int(sk["offset"][q]), int(sk["npix"][q])
        truth[o:o + m] += skewers.delta_s(seed + 1, q, m, cfg["dpix"], 1.8, 1.0)
    F = np.exp(-0.35 * np.exp(1.4 * (truth + c_t * eta)))
    fbar_t = float(F.mean())
    ps, cnt = p1d.p1d(F, sk, [-1e30, 1e30], [fbar_t], k_edges, z_t, cfg["dpix"])
    pk_t = np.where(cnt > 0, ps / np.maximum(cnt, 1), np.nan)
    # the truth knows its flux dispersion; the binned P1D integral would miss
    # the power outside the bins
    res = tune_ps.iterate(dl, eta, sk, seed, z_t, c_t, fbar_t, pk_t, k_edges, cfg["dpix"], 1.0, 1.5, n_iter=6,
                          sigf_t=float(F.std()))
    ok = np.isfinite(pk_t)
    err = [np.sqrt(np.mean((h["p1d"][ok] / pk_t[ok] - 1) ** 2)) for h in res["hist"]]
    print("P1D relative RMS error per iteration", ["%.3f" % e for e in err])
    assert all(e1 < e0 for e0, e1 in zip(err, err[1:]))
    assert err[-1] < 0.7 * err[0]
    assert abs(res["hist"][-1]["fbar"] / fbar_t - 1) < 0.03
    assert abs(res["b"] / 1.4 - 1) < 0.03
    # the secant update: the same first step, then larger ones
    sec = tune_ps.iterate(dl, eta, sk, seed, z_t, c_t, fbar_t, pk_t, k_edges, cfg["dpix"], 1.0, 1.5, n_iter=6,
                          sigf_t=float(F.std()), update="secant")
    err_s = [np.sqrt(np.mean((h["p1d"][ok] / pk_t[ok] - 1) ** 2)) for h in sec["hist"]]
    print("secant update: P1D relative RMS error per iteration", ["%.3f" % e for e in err_s])
    assert err_s[:2] == pytest.approx(err[:2], rel=1e-12)
    assert err_s[-1] < 0.8 * err[-1]


@pytest.mark.parametrize("a,s,sg", [(0.3, 0.8, 2.0), (0.05, 2.5, 3.1), (1.2, 0.4, 1.0)])
def test_flux_bias_is_the_mean_flux_response(a, s, sg):
    # b_F = (1/Fbar) dFbar/dmu for a long mode shifting g by mu: with b = s/sg,
    # F(g + mu) = exp(-a e^{b mu} e^{s x}), so Fbar(mu) = Fbar(a e^{b mu}, s)
    b = s / sg
    h = 1e-5
    fp = tune_ps.gauss_fbar_sigf(a * np.exp(b * h), s)[0]
    fm = tune_ps.gauss_fbar_sigf(a * np.exp(-b * h), s)[0]
    f0 = tune_ps.gauss_fbar_sigf(a, s)[0]
    np.testing.assert_allclose(tune_ps.flux_bias(a, s, sg), (fp - fm) / (2 * h) / f0, rtol=1e-7)
    assert tune_ps.flux_bias(a, s, sg) < 0


def test_flux_bias_step_limit():
    # s -> infinity at fixed x_0 = -ln(a)/s: F -> 1{x < x_0}, |b_F| -> phi(x_0)/(sigma_g Phi(x_0))
    from scipy import stats
    x0, sg = 0.3, 2.0
    lim = stats.norm.pdf(x0) / (sg * stats.norm.cdf(x0))
    got = [abs(tune_ps.flux_bias(np.exp(-s * x0), s, sg)) for s in (10.0, 20.0, 80.0)]
    assert abs(got[2] / lim - 1) < abs(got[1] / lim - 1) < abs(got[0] / lim - 1)
    assert abs(got[2] / lim - 1) < 0.01
    # a target far beyond any reachable bias has no solution
    assert tune_ps.fit_a_s_bias(0.6, 10.0 * lim, sg, 0.0) is None


def test_kaiser_monopole_factor():
    for beta in (0.0, 0.8, 1.6):
        mono = integrate.quad(lambda mu: (1 + beta * mu * mu) ** 2, 0.0, 1.0)[0]
        np.testing.assert_allclose(tune_ps.kaiser_factor(beta) ** 2, mono, rtol=1e-13)


def test_fit_with_the_bias_target_recovers_a_and_s():
    a0, s0, sg, beta = 0.4, 1.1, 2.2, 1.3
    fbar = tune_ps.gauss_fbar_sigf(a0, s0)[0]
    beff = tune_ps.effective_bias(a0, s0, sg, beta)
    a, s = tune_ps.fit_a_s_bias(fbar, beff, sg, beta)
    np.testing.assert_allclose([a, s], [a0, s0], rtol=1e-8)


def test_outer_steps_reach_the_bias_target():
    # a truth of known (a, b) and its predicted effective bias as the target;
    # from the (Fbar, sigma_F) start the outer steps bring the prediction to
    # the target and keep improving the P1D
    cfg = mockinputs.config("tiny")
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    box = field.make_box(n, seed, oracle_table(cfg["pk"], n, dx), ("delta", "zz"), f=cfg["f"])
    sk = mockinputs.skewer_table(cfg)
    dl, eta = skewers.draw_skewers(box.real, box.imag, sk, seed)
    k_edges = p1d.log_k_edges()
    z_t, c_t, a_true, b_true = 2.4, 1.2, 0.35, 1.4
    truth = np.array(dl, copy=True)
    for q in range(len(sk["npix"])):
        o, m = int(sk["offset"][q]), int(sk["npix"][q])
        truth[o:o + m] += skewers.delta_s(seed + 1, q, m, cfg["dpix"], 1.8, 1.0)
    g = truth + c_t * eta
    F = np.exp(-a_true * np.exp(b_true * g))
    fbar_t = float(F.mean())
    ps, cnt = p1d.p1d(F, sk, [-1e30, 1e30], [fbar_t], k_edges, z_t, cfg["dpix"])
    pk_t = np.where(cnt > 0, ps / np.maximum(cnt, 1), np.nan)
    sg = float(g.std())
    beff_t = tune_ps.effective_bias(a_true, b_true * sg, sg, cfg["f"] * c_t)
    ok = np.isfinite(pk_t)
    runs = {}
    for no in (1, 3):
        r = tune_ps.iterate(dl, eta, sk, seed, z_t, c_t, fbar_t, pk_t, k_edges, cfg["dpix"], 1.0, 1.5, n_iter=4,
                            sigf_t=float(F.std()), n_outer=no, beff_t=beff_t, f=cfg["f"])
        runs[no] = (r, np.sqrt(np.mean((r["hist"][-1]["p1d"][ok] / pk_t[ok] - 1) ** 2)))
    print("b_eff / target per outer step", ["%.4f" % (v / beff_t) for v in runs[3][0]["beff"]],
          "P1D error one / three steps %.3f %.3f" % (runs[1][1], runs[3][1]))
    assert len(runs[3][0]["beff"]) == 3
    assert abs(runs[3][0]["beff"][-1] / beff_t - 1) < 3e-3
    assert abs(runs[3][0]["beff"][-1] / beff_t - 1) < abs(runs[1][0]["beff"][-1] / beff_t - 1)
    assert runs[3][1] < runs[1][1]
    assert abs(runs[3][0]["hist"][-1]["fbar"] / fbar_t - 1) < 0.03


def test_sigma_s2_of_the_gaussian_form_in_closed_form():
    for amp, kc, dpix in ((1.0, 1.5, 0.2), (2.5, 0.4, 0.27375), (0.3, 8.0, 0.5)):
        num = integrate.quad(lambda k: amp * np.exp(-(k / kc) ** 2), 0.0, np.pi / dpix, epsabs=1e-15, limit=200)[0]
        np.testing.assert_allclose(tune_ps.sigma_s2_gauss(amp, kc, dpix), num / np.pi, rtol=1e-12)


def _tiny_subset(n_sk):
    """The tiny mock's stored pixels without delta_S (oracle box and skewers),
    restricted to its first n_sk skewers."""
    cfg = mockinputs.config("tiny")
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    box = field.make_box(n, seed, oracle_table(cfg["pk"], n, dx), ("delta", "zz"), f=cfg["f"])
    sk = mockinputs.skewer_table(cfg)
    dl, eta = skewers.draw_skewers(box.real, box.imag, sk, seed)
    sub = dict(sk)
    for key in ("npix", "offset", "chi0", "origin_fx", "step_fx"):
        if key in sub:
            sub[key] = np.asarray(sk[key])[:n_sk]
    used = int(sub["offset"][-1] + sub["npix"][-1])
    sub["total"] = used
    return cfg, sub, np.asarray(dl)[:used], np.asarray(eta)[:used]


def test_statistics_without_small_scale_power_are_the_plain_evaluation():
    from oracle import tune
    cfg, sk, dl, eta = _tiny_subset(120)
    k_edges = p1d.log_k_edges()
    a, b, c, z = 0.3, 1.5, 1.1, 2.6
    fb0, pk0 = tune.evaluate(dl, eta, sk, a, b, c, z, k_edges, cfg["dpix"])
    fb, pk = tune_ps.statistics_ps(dl, eta, sk, 7, z, c, a, b, 1e-300, 1.5, k_edges, cfg["dpix"])
    np.testing.assert_allclose(fb, fb0, rtol=1e-13)
    ok = np.isfinite(pk0)
    np.testing.assert_allclose(pk[ok], pk0[ok], rtol=1e-11)
    # with small-scale power present the 1D power moves
    fb2, pk2 = tune_ps.statistics_ps(dl, eta, sk, 7, z, c, a, b, 1.5, 1.2, k_edges, cfg["dpix"])
    assert np.max(np.abs(pk2[ok] / pk0[ok] - 1)) > 0.05


@pytest.mark.parametrize("outer", [False, True])
def test_small_scale_power_fit_recovers_a_truth_in_the_family(outer):
    # the truth: delta_S of (amp, kcut) = (1.8, 1.0) with the mock's own key
    # (skewers.delta_s), (a, s) = (0.3, 2.2), b = s / sigma_g with sigma_g from
    # the measured moments and a numerical integral of P_s, its P1D from
    # p1d.p1d; from P_s^0 = (1.0, 1.5) a least-squares solve of the problem
    # must find (1.8, 1.0)
    from scipy import optimize
    cfg, sk, dl, eta = _tiny_subset(120)
    k_edges = p1d.log_k_edges()
    dpix, seed, z_t, c_t, f = cfg["dpix"], 11, 2.4, 1.2, cfg["f"]
    amp, kc, a, s = 1.8, 1.0, 0.3, 2.2
    g = np.asarray(dl, dtype=np.float64) + c_t * eta
    ss2 = integrate.quad(lambda k: amp * np.exp(-(k / kc) ** 2), 0.0, np.pi / dpix, epsabs=1e-15)[0] / np.pi
    sg = np.sqrt(np.var(g) + ss2)
    dens = np.array(dl, dtype=np.float64, copy=True)
    for q in range(len(sk["npix"])):
        o, m = int(sk["offset"][q]), int(sk["npix"][q])
        dens[o:o + m] += skewers.delta_s(seed, q, m, dpix, amp, kc)
    F = np.exp(-a * np.exp((s / sg) * (dens + c_t * eta)))
    fb = float(F.mean())
    ps, cnt = p1d.p1d(F, sk, [-1e30, 1e30], [fb], k_edges, z_t, dpix)
    pk_t = np.where(cnt > 0, ps / np.maximum(cnt, 1), np.nan)
    f1, sf = tune_ps.gauss_fbar_sigf(a, s)
    kw = dict(beff_t=tune_ps.effective_bias(a, s, sg, f * c_t), f=f) if outer else {}
    at = tune_ps.ps_fit_problem(dl, eta, sk, seed, z_t, c_t, f1, pk_t, k_edges, dpix, sigf_t=sf, **kw)
    ok = np.isfinite(pk_t)

    def resid(th):
        r = at(th)
        return r["p1d"][ok] / pk_t[ok] - 1.0

    sol = optimize.least_squares(resid, [0.0, np.log(1.5)], xtol=1e-12, ftol=1e-14, gtol=1e-14)
    got = at(sol.x)
    print("fit (amp, kcut) = (%.6f, %.6f), objective %.2e" % (np.exp(sol.x[0]), np.exp(sol.x[1]), got["objective"]))
    np.testing.assert_allclose(np.exp(sol.x), [amp, kc], rtol=1e-5)
    np.testing.assert_allclose([got["a"], got["s"]], [a, s], rtol=1e-6)
    assert got["objective"] < 1e-12
