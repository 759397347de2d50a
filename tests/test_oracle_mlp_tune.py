"""Pins of the oracle's emulator MLP and plain tuning loop (CPU)."""
import numpy as np
from scipy import stats

import mockinputs
from oracle import field, fgpa, mlp, p1d, power, skewers, tune


def test_gelu_matches_normal_cdf():
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mlp.gelu(x), x * stats.norm.cdf(x), rtol=1e-14, atol=1e-300)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_parameter_count():
    assert sum(p.size for p in mlp.init_params()) == 141345


def test_backward_against_finite_differences():
    sizes = (4, 7, 6, 5, 3)
    params = mlp.init_params(1, sizes)
    rng = np.random.default_rng(2)
    for p in params:
        p += rng.normal(0, 0.1, p.shape)
    x = rng.normal(size=(9, 4))
    t = rng.normal(size=(9, 3))
    _, grads = mlp.backward(params, x, t)
    h = 1e-6
    for pi, p in enumerate(params):
        flat = p.reshape(-1)
        for k in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[k]
            flat[k] = old + h
            lp = mlp.loss(params, x, t)
            flat[k] = old - h
            lm = mlp.loss(params, x, t)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            g = grads[pi].reshape(-1)[k]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (pi, k, fd, g)


def test_adam_first_step_is_lr_sign():
    params = [np.array([1.0, -2.0, 3.0])]
    opt = mlp.Adam(params, lr=0.01, eps=0.0)
    opt.step(params, [np.array([0.5, -3.0, 1e-3])])
    np.testing.assert_allclose(params[0], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=1e-14)


def test_training_fits_a_smooth_map():
    sizes = (4, 32, 32, 32, 2)
    params = mlp.init_params(3, sizes)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (256, 4))
    t = np.stack([np.sin(x[:, 0]) + x[:, 1] * x[:, 2], np.cos(x[:, 3])], axis=1)
    opt = mlp.Adam(params, lr=3e-3)
    l0 = mlp.loss(params, x, t)
    for _ in range(300):
        _, g = mlp.backward(params, x, t)
        opt.step(params, g)
    assert mlp.loss(params, x, t) < 0.05 * l0


def _mock(n=32, n_sk=60):
    cfg = mockinputs.config("mid", n=n, n_sk=n_sk)
    tab = power.amplitude_table(power.PowerSpectrum(**cfg["pk"]), n, cfg["dx"])
    box = field.make_box(n, 5, tab, ("delta", "zz"))
    sk = mockinputs.skewer_table(cfg)
    dens, eta = skewers.draw_skewers(box.real, box.imag, sk, 5, 0.5, 1.5, 0.2)
    return sk, dens, eta


def test_tuning_recovers_statistics_of_known_parameters():
    sk, dens, eta = _mock()
    k_edges = p1d.log_k_edges(16, 0.002, 0.05)
    a0, b0, c0, z = 0.35, 1.3, 1.2, 2.4
    fbar_t, pk_t = tune.evaluate(dens, eta, sk, a0, b0, c0, z, k_edges, 0.2)
    r = tune.tune_one(dens, eta, sk, z, c0, fbar_t, pk_t, k_edges, 0.2, x0=(0.25, 1.0))
    assert abs(r["fbar"] / fbar_t - 1) < 1e-3
    ok = np.isfinite(pk_t)
    assert np.max(np.abs(r["p1d"][ok] / pk_t[ok] - 1)) < 1e-3
    assert abs(r["a"] / a0 - 1) < 0.02 and abs(r["b"] / b0 - 1) < 0.02


def test_fit_quadratics_exact_for_quadratic_data():
    z = np.array([1.8, 2.2, 2.6, 3.0, 3.6])
    x = 1 + z
    a = 0.1 + 0.2 * x + 0.03 * x * x
    coef = tune.fit_quadratics(z, a, 2 * a, 3 * a)
    np.testing.assert_allclose(coef[0], [0.1, 0.2, 0.03], atol=1e-12)
    np.testing.assert_allclose(fgpa.coeff_eval(coef, z)[1], 2 * a, rtol=1e-12)


def test_fbar_target_endpoints():
    assert abs(mockinputs.fbar_target(1.8) - 0.75) < 1e-15 and abs(mockinputs.fbar_target(3.6) - 0.35) < 1e-15
