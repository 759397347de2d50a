"""GPU parity of the emulator mode of the small-scale power tuning
(lya_emulator_labels_ps, lya_tune_ps with LYA_TUNE_PS_EMULATOR; section
"Adjusting mock parameters" for the problem, the emulator itself is not in the
paper) against the FP64 oracle.  The stored pixels are the oracle's, rounded
to FP32, on both sides.  The truth lies in the (amp, kcut) family and uses the
mock's own delta_S key, so the fit problem has an exact solution, which the
oracle's statistics define (the target P1D comes from the oracle alone)."""
import time

import numpy as np
import pytest

import mockinputs
from oracle import field, p1d, skewers, tune_ps
from tests.lyahelp import oracle_table, rel_rms, skewer_tensors

pytestmark = pytest.mark.gpu
TOL = 1e-5
AMP_T, KC_T, A_T, S_T = 1.8, 1.0, 0.3, 2.2     # the truth
AMP0, KC0 = 1.0, 1.5                            # P_s^0, the start


@pytest.fixture(scope="module")
def L():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_18996_amd import lyamock
    lyamock.load()
    return lyamock


@pytest.fixture(scope="module")
def fam():
    cfg = mockinputs.config("tiny")
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    box = field.make_box(n, seed, oracle_table(cfg["pk"], n, dx), ("delta", "zz"), f=cfg["f"])
    sk = mockinputs.skewer_table(cfg)
    dl, eta = skewers.draw_skewers(box.real, box.imag, sk, seed)          # no delta_S
    dl = dl.astype(np.float32).astype(np.float64)
    eta = eta.astype(np.float32).astype(np.float64)
    k_edges = p1d.log_k_edges()
    z_t, c_t, dpix = 2.4, 1.2, cfg["dpix"]
    sl2, se2, cov = tune_ps.moments(dl, eta)
    sig0 = sl2 + c_t * c_t * se2 + 2.0 * c_t * cov
    sg = np.sqrt(sig0 + tune_ps.sigma_s2_gauss(AMP_T, KC_T, dpix))
    fbar_t, sigf_t = tune_ps.gauss_fbar_sigf(A_T, S_T)
    fb, pk_t = tune_ps.statistics_ps(dl, eta, sk, seed, z_t, c_t, A_T, S_T / sg, AMP_T, KC_T, k_edges, dpix)
    beff_t = tune_ps.effective_bias(A_T, S_T, sg, cfg["f"] * c_t)
    return dict(cfg=cfg, sk=sk, dl=dl, eta=eta, k_edges=k_edges, z_t=z_t, c_t=c_t, dpix=dpix, seed=seed,
                fbar_t=fbar_t, sigf_t=sigf_t, pk_t=np.ascontiguousarray(pk_t), beff_t=beff_t, sig0=sig0)


class Spec:
    """A one-redshift TunePsSpec over the mock's pixels (device copies kept alive)."""

    def __init__(self, L, fam, mode, emu=None, checks=8, n_outer=0, n_iter=10):
        import torch
        sk = fam["sk"]
        nk = len(fam["k_edges"]) - 1
        self.s, self.keep = skewer_tensors(L, sk)
        self.dl = torch.from_numpy(fam["dl"].astype(np.float32)).cuda()
        self.eta = torch.from_numpy(fam["eta"].astype(np.float32)).cuda()
        self.ke = torch.from_numpy(fam["k_edges"].astype(np.float64)).cuda()
        import ctypes
        sp = L.TunePsSpec()
        sp.sk = ctypes.pointer(self.s)
        sp.dens_l, sp.eta = self.dl.data_ptr(), self.eta.data_ptr()
        sp.n_pixels = int(sk["total"])
        sp.cosmo = L.Cosmo(0.3147)
        sp.seed = fam["seed"]
        sp.n_zt = 1
        sp.z_t[0], sp.c_t[0], sp.fbar_t[0], sp.sigf_t[0] = fam["z_t"], fam["c_t"], fam["fbar_t"], fam["sigf_t"]
        sp.p1d_t = fam["pk_t"].ctypes.data
        sp.p1d = L.P1dSpec(nk, self.ke.data_ptr(), fam["z_t"], fam["dpix"])
        sp.ps_amp, sp.ps_kcut, sp.n_iter = AMP0, KC0, n_iter
        sp.n_outer, sp.f = n_outer, fam["cfg"]["f"]
        sp.beff_t[0] = fam["beff_t"]
        sp.mode = mode
        if emu is not None:
            sp.emu[0] = emu.data_ptr()
        sp.emu_checks = checks
        self.spec = sp
        self.work = torch.empty(L.tune_ps_workspace_size(len(sk["npix"]), sk["total"], nk), dtype=torch.uint8,
                                device="cuda")


def test_labels_match_the_oracle(L, fam):
    import torch
    sp = Spec(L, fam, L.TUNE_PS_RATIOS)
    # eleven draws: a full pass of eight and a ragged one of three
    draws = np.array([[0.3, 1.0, 1.8, 1.0], [0.15, 1.3, 0.6, 2.5], [0.5, 0.8, 3.0, 0.7], [0.3, 1.1, 1e-3, 1.5],
                      [0.25, 0.9, 1.2, 1.2], [0.4, 1.2, 2.2, 0.9], [0.2, 1.0, 0.9, 1.8], [0.35, 0.7, 1.5, 1.1],
                      [0.3, 1.0, 1.8, 1.0], [0.1, 1.4, 4.0, 0.5], [0.6, 0.6, 0.5, 3.0]])
    nk = len(fam["k_edges"]) - 1
    y = torch.full((len(draws), 1 + nk), float("nan"), dtype=torch.float32, device="cuda")
    L.emulator_labels_ps(sp.spec, 0, draws, y, sp.work)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(y[0], y[8])       # the same draw in two passes
    for i, (a, b, amp, kc) in enumerate(draws):
        fb, pk = tune_ps.statistics_ps(fam["dl"], fam["eta"], fam["sk"], fam["seed"], fam["z_t"], fam["c_t"], a, b,
                                       amp, kc, fam["k_edges"], fam["dpix"])
        ok = np.isfinite(pk)
        np.testing.assert_array_equal(np.isfinite(y[i, 1:]), ok)
        e = rel_rms(y[i, 1:][ok], pk[ok])
        print("label %d (a %.2f b %.2f amp %.3g kcut %.2f): Fbar rel %.1e, P1D rel rms %.1e, max %.1e"
              % (i, a, b, amp, kc, abs(y[i, 0] / fb - 1), e, np.max(np.abs(y[i, 1:][ok] / pk[ok] - 1))), flush=True)
        assert abs(y[i, 0] / fb - 1) < TOL
        assert e < TOL and np.max(np.abs(y[i, 1:][ok] / pk[ok] - 1)) < 1e-4


def test_labels_reject_bad_input(L, fam):
    import torch
    sp = Spec(L, fam, L.TUNE_PS_RATIOS)
    nk = len(fam["k_edges"]) - 1
    y = torch.empty((1, 1 + nk), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LyaError):
        L.emulator_labels_ps(sp.spec, 1, np.array([[0.3, 1.0, 1.0, 1.0]]), y, sp.work)     # zi beyond n_zt
    with pytest.raises(L.LyaError):
        L.emulator_labels_ps(sp.spec, 0, np.array([[0.3, 1.0, 0.0, 1.0]]), y, sp.work)     # amp <= 0
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LyaError):
        L.emulator_labels_ps(sp.spec, 0, np.array([[0.3, 1.0, 1.0, 1.0]]), y, small)


def _draws(fam, n, rng):
    """Label draws (a, b, amp, kcut): (amp, kcut) log-uniform over the search
    box, (a, s) about their solution for that P_s (within +-25% in a and
    +-20% in s), b = s / sigma_g."""
    amp = np.exp(rng.uniform(np.log(0.5), np.log(4.0), n))
    kc = np.exp(rng.uniform(np.log(0.5), np.log(3.0), n))
    sg = np.sqrt(fam["sig0"] + np.array([tune_ps.sigma_s2_gauss(x, y, fam["dpix"]) for x, y in zip(amp, kc)]))
    a = A_T * np.exp(rng.uniform(-0.25, 0.25, n))
    s = S_T * np.exp(rng.uniform(-0.2, 0.2, n))
    return np.stack([a, s / sg, amp, kc], axis=1)


def _train(L, fam, n_lab=4000, steps=4000):
    import torch
    sp = Spec(L, fam, L.TUNE_PS_RATIOS)
    nk = len(fam["k_edges"]) - 1
    draws = _draws(fam, n_lab, np.random.default_rng(5))
    y = torch.empty((n_lab, 1 + nk), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    L.emulator_labels_ps(sp.spec, 0, draws, y, sp.work)
    torch.cuda.synchronize()
    t_lab = time.perf_counter() - t0
    lo = draws.min(axis=0) * 0.98
    hi = draws.max(axis=0) * 1.02
    emu = torch.zeros(L.emulator_bytes(1 + nk), dtype=torch.uint8, device="cuda")
    L.emulator_init(emu, 1 + nk, 1, 3, lo, hi, 0b1101)        # ln a, b, ln amp, ln kcut
    L.emulator_set_scaling(emu, y, n_lab)
    B = 256
    work = torch.empty(L.emulator_train_workspace_size(B, 1 + nk), dtype=torch.uint8, device="cuda")
    hist = torch.zeros(steps, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    L.emulator_train(emu, torch.from_numpy(draws.astype(np.float32)).cuda(), y, n_lab, steps, B, 1e-3, True, hist,
                     work)
    h = hist.cpu().numpy()
    print("labels %.2f s, training %.2f s, loss %.3g -> %.3g" % (t_lab, time.perf_counter() - t0, h[:10].mean(),
                                                                 h[-100:].mean()), flush=True)
    return emu


@pytest.fixture(scope="module")
def emu(L, fam):
    return _train(L, fam)


@pytest.mark.parametrize("outer", [False, True])
def test_emulator_mode_finds_the_truth(L, fam, emu, outer):
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=8, n_outer=3 if outer else 0)
    res = L.tune_ps(sp.spec, sp.work)
    nk = len(fam["k_edges"]) - 1
    amp, kc = res.ps_fit[0], res.ps_fit[1]
    gp = np.array(res.p1d[:nk])
    ok = np.isfinite(fam["pk_t"])
    err_t = rel_rms(gp[ok], fam["pk_t"][ok])
    print("emulator mode (outer %s): (amp, kcut) = (%.5f, %.5f), a %.5f b %.5f s %.5f; gpu evals %d fallback %d; "
          "P1D rel rms vs target %.2e; %.3f s" % (outer, amp, kc, res.a[0], res.b[0], res.s[0], res.gpu_evals[0],
                                                 res.fallback[0], err_t, res.seconds), flush=True)
    assert res.fallback[0] == 0 and 2 <= res.gpu_evals[0] <= 8
    assert abs(np.log(amp / AMP_T)) < 3e-3 and abs(np.log(kc / KC_T)) < 3e-3
    np.testing.assert_allclose([res.a[0], res.s[0]], [A_T, S_T], rtol=3e-3 if outer else 1e-7)
    assert err_t < 2e-3
    # what the result reports is the oracle's statistics at the parameters it returns
    fb, pk = tune_ps.statistics_ps(fam["dl"], fam["eta"], fam["sk"], fam["seed"], fam["z_t"], fam["c_t"], res.a[0],
                                   res.b[0], amp, kc, fam["k_edges"], fam["dpix"])
    assert abs(res.fbar[0] / fb - 1) < TOL
    assert rel_rms(gp[ok], pk[ok]) < TOL
    np.testing.assert_allclose(res.rms[0], np.sqrt(np.mean((gp[ok] / fam["pk_t"][ok] - 1) ** 2)), rtol=1e-12)
    if outer:
        sg = np.sqrt(fam["sig0"] + tune_ps.sigma_s2_gauss(amp, kc, fam["dpix"]))
        np.testing.assert_allclose(res.beff[0], fam["beff_t"], rtol=1e-7)
        np.testing.assert_allclose(res.b[0], res.s[0] / sg, rtol=1e-12)
    # the centre-of-bin ratios describe the fitted P_s
    ek = fam["k_edges"] * tune_ps.dv_per_dchi(fam["z_t"])
    kcen = np.sqrt(ek[:-1] * ek[1:])
    want = AMP0 ** -1 * amp * np.exp(-(kcen / kc) ** 2 + (kcen / KC0) ** 2)
    np.testing.assert_allclose(np.array(res.ratio[:nk]), want, rtol=1e-12)


def test_emulator_mode_beats_the_plain_iteration(L, fam, emu):
    pl = Spec(L, fam, L.TUNE_PS_RATIOS, n_iter=10)
    rp = L.tune_ps(pl.spec, pl.work)
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=8)
    re_ = L.tune_ps(sp.spec, sp.work)
    print("plain: P1D rel rms vs target %.2e after %d GPU evaluations (%.3f s); emulator: %.2e after %d (%.3f s)"
          % (rp.rms[9], rp.gpu_evals[0], rp.seconds, re_.rms[0], re_.gpu_evals[0], re_.seconds), flush=True)
    assert rp.gpu_evals[0] == 10
    assert re_.rms[0] < rp.rms[9] and re_.gpu_evals[0] < rp.gpu_evals[0]
    assert abs(re_.fbar[0] / rp.fbar[9] - 1) < 5e-3


def test_emulator_mode_hands_over_to_the_plain_iteration(L, fam):
    # an untrained emulator and one GPU check: the search cannot settle, so the
    # plain iteration runs, with exactly the plain mode's results
    import torch
    nk = len(fam["k_edges"]) - 1
    raw = torch.zeros(L.emulator_bytes(1 + nk), dtype=torch.uint8, device="cuda")
    L.emulator_init(raw, 1 + nk, 1, 9, (0.05, 0.2, 0.3, 0.3), (1.0, 3.0, 6.0, 4.0), 0b1101)
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=raw, checks=1, n_iter=4)
    re_ = L.tune_ps(sp.spec, sp.work)
    pl = Spec(L, fam, L.TUNE_PS_RATIOS, n_iter=4)
    rp = L.tune_ps(pl.spec, pl.work)
    assert re_.fallback[0] == 1 and rp.fallback[0] == 0
    assert re_.gpu_evals[0] == 1 + rp.gpu_evals[0] == 5
    for name in ("a", "b", "s"):
        assert getattr(re_, name)[0] == getattr(rp, name)[0]
    np.testing.assert_array_equal(np.array(re_.p1d[:nk]), np.array(rp.p1d[:nk]))
    np.testing.assert_array_equal(np.array(re_.fbar[:4]), np.array(rp.fbar[:4]))


@pytest.mark.parametrize("update", ["paper", "secant"])
def test_emulator_mode_refinement_matches_the_oracle(L, fam, emu, update):
    # three per-bin iterations after the fit: the oracle's iteration started
    # from the fitted form (its (a, s) come from the same mean flux and
    # dispersion targets) gives the same statistics
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=8)
    sp.spec.emu_refine = 3
    sp.spec.update = L.PS_UPDATE_SECANT if update == "secant" else L.PS_UPDATE_PAPER
    res = L.tune_ps(sp.spec, sp.work)
    plain_fit = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=8)
    r0 = L.tune_ps(plain_fit.spec, plain_fit.work)
    assert res.fallback[0] == 0 and res.gpu_evals[0] == r0.gpu_evals[0] + 3
    assert (res.ps_fit[0], res.ps_fit[1]) == (r0.ps_fit[0], r0.ps_fit[1])
    nk = len(fam["k_edges"]) - 1
    ref = tune_ps.iterate(fam["dl"], fam["eta"], fam["sk"], fam["seed"], fam["z_t"], fam["c_t"], fam["fbar_t"],
                          fam["pk_t"], fam["k_edges"], fam["dpix"], res.ps_fit[0], res.ps_fit[1], n_iter=3,
                          sigf_t=fam["sigf_t"], update=update)
    np.testing.assert_allclose([res.fbar[i] for i in range(3)], [h["fbar"] for h in ref["hist"]], rtol=TOL)
    last = ref["hist"][-1]
    ok = np.isfinite(last["p1d"])
    gp = np.array(res.p1d[:nk])
    print("refinement: P1D rel rms vs oracle %.2e; ratios %s" % (rel_rms(gp[ok], last["p1d"][ok]),
                                                                 np.round(np.array(res.ratio[:4]), 6)), flush=True)
    assert rel_rms(gp[ok], last["p1d"][ok]) < TOL
    np.testing.assert_allclose(np.array(res.ratio[:nk]), last["ratio"], rtol=1e-5)
    np.testing.assert_allclose(res.b[0], last["b"], rtol=1e-6)


def test_emulator_mode_at_two_redshifts(L, fam, emu):
    # two z_t with the same targets and emulator: each row is the
    # one-redshift result
    nk = len(fam["k_edges"]) - 1
    one = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=8)
    r1 = L.tune_ps(one.spec, one.work)
    two = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=8)
    sp = two.spec
    sp.n_zt = 2
    sp.z_t[1], sp.c_t[1], sp.fbar_t[1], sp.sigf_t[1] = sp.z_t[0], sp.c_t[0], sp.fbar_t[0], sp.sigf_t[0]
    pk2 = np.ascontiguousarray(np.concatenate([fam["pk_t"], fam["pk_t"]]))
    sp.p1d_t = pk2.ctypes.data
    sp.emu[1] = emu.data_ptr()
    r2 = L.tune_ps(sp, two.work)
    for z in (0, 1):
        assert r2.fallback[z] == 0 and r2.gpu_evals[z] == r1.gpu_evals[0]
        assert (r2.a[z], r2.b[z], r2.ps_fit[2 * z], r2.ps_fit[2 * z + 1]) == (r1.a[0], r1.b[0], r1.ps_fit[0],
                                                                            r1.ps_fit[1])
        np.testing.assert_array_equal(np.array(r2.p1d[64 * z:64 * z + nk]), np.array(r1.p1d[:nk]))


def test_emulator_mode_rejects_bad_input(L, fam, emu):
    import torch
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=None)
    with pytest.raises(L.LyaError):
        L.tune_ps(sp.spec, sp.work)                     # no emulator
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu, checks=0)
    with pytest.raises(L.LyaError):
        L.tune_ps(sp.spec, sp.work)                     # no GPU check allowed
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=emu)
    sp.spec.emu_refine = 17
    with pytest.raises(L.LyaError):
        L.tune_ps(sp.spec, sp.work)                     # refinement beyond 16 iterations
    sp = Spec(L, fam, 7, emu=emu)
    with pytest.raises(L.LyaError):
        L.tune_ps(sp.spec, sp.work)                     # unknown mode
    other = torch.zeros(L.emulator_bytes(5), dtype=torch.uint8, device="cuda")
    L.emulator_init(other, 5, 1, 1, (0.1, 0.1, 0.1, 0.1), (1.0, 1.0, 1.0, 1.0), 0)
    sp = Spec(L, fam, L.TUNE_PS_EMULATOR, emu=other)
    with pytest.raises(L.LyaError):
        L.tune_ps(sp.spec, sp.work)                     # outputs are not 1 + n_kbins
