"""GPU parity of lya_make_box / lya_make_eta against the FP64 oracle."""
import numpy as np
import pytest

import mockinputs
from oracle import field, lines
from tests.lyahelp import bf16_to_f32, gpu_box, oracle_table, rel_rms

pytestmark = pytest.mark.gpu

PK = mockinputs.PK_DEFAULT
TOL = 1e-5   # relative RMS, FP32 path vs FP64 oracle


@pytest.fixture(scope="module")
def L():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_18996_amd import lyamock
    lyamock.load()
    return lyamock


@pytest.mark.parametrize("two_buffer", [False, True])
@pytest.mark.parametrize("n", [32, 64, 128])
def test_box_matches_oracle(L, n, two_buffer):
    dx, seed, f = 2.19, 1234, 1.0
    print("box parity n=%d seed=%d two-buffer %s" % (n, seed, two_buffer), flush=True)
    g = gpu_box(L, n, dx, seed, f, two_buffer=two_buffer, **PK).cpu().numpy().astype(np.float64)
    tab = oracle_table(PK, n, dx)
    ref = field.make_box(n, seed, tab, ("delta", "zz"), f=f)
    e_d = rel_rms(g[..., 0], ref.real)
    e_e = rel_rms(g[..., 1], ref.imag)
    print("rel rms delta %.3e eta %.3e" % (e_d, e_e))
    assert e_d < TOL and e_e < TOL


def test_box_without_eta_and_f(L):
    n, dx = 64, 2.19
    g = gpu_box(L, n, dx, 77, 0.6, with_eta=False, **PK).cpu().numpy()
    assert np.all(g[..., 1] == 0.0)
    g2 = gpu_box(L, n, dx, 77, 0.6, with_eta=True, **PK).cpu().numpy()
    # the same delta whether or not eta rides along (FFT rounding differs)
    assert rel_rms(g[..., 0], g2[..., 0]) < 1e-6
    tab = oracle_table(PK, n, dx)
    ref = field.make_box(n, 77, tab, ("delta", "zz"), f=0.6)
    assert rel_rms(g2[..., 1], ref.imag) < TOL


@pytest.mark.parametrize("two_buffer", [False, True])
@pytest.mark.parametrize("comps", [("xy", "yz"), ("xx", "yy"), ("xz", "none"), ("zz", "delta")])
def test_make_eta_components(L, comps, two_buffer):
    n, dx = 64, 2.19
    g = gpu_box(L, n, dx, 5, 0.9, comps=comps, two_buffer=two_buffer, **PK).cpu().numpy().astype(np.float64)
    tab = oracle_table(PK, n, dx)
    oc = (comps[0],) if comps[1] == "none" else comps
    ref = field.make_box(n, 5, tab, oc, f=0.9)
    assert rel_rms(g[..., 0], ref.real) < TOL
    if comps[1] == "none":
        assert np.all(g[..., 1] == 0.0)
    else:
        assert rel_rms(g[..., 1], ref.imag) < TOL


def test_fixed_amplitude_and_single_shell(L):
    n, dx = 64, 2.19
    tab = oracle_table(PK, n, dx)
    g = gpu_box(L, n, dx, 9, 1.0, fixed_amp=True, **PK).cpu().numpy().astype(np.float64)
    ref = field.make_box(n, 9, tab, ("delta", "zz"), fixed_amp=True)
    assert rel_rms(g[..., 0], ref.real) < TOL
    # variance identity holds on the GPU field too
    s = field.amplitudes(n, tab)
    assert abs(np.mean(g[..., 0] ** 2) / np.sum(s ** 2) - 1) < 1e-5
    g1 = gpu_box(L, n, dx, 9, 1.0, only_n2=1, **PK).cpu().numpy().astype(np.float64)
    ref1 = field.make_box(n, 9, tab, ("delta", "zz"), only_n2=1)
    assert rel_rms(g1[..., 0], ref1.real) < TOL and rel_rms(g1[..., 1], ref1.imag) < TOL


def test_smoothing(L):
    n, dx = 64, 2.19
    tab = oracle_table(PK, n, dx, smooth=dx)
    g = gpu_box(L, n, dx, 3, 1.0, smooth=dx, **PK).cpu().numpy().astype(np.float64)
    ref = field.make_box(n, 3, tab, ("delta", "zz"))
    assert rel_rms(g[..., 0], ref.real) < TOL and rel_rms(g[..., 1], ref.imag) < TOL


def test_bf16_storage_error_reported(L):
    n, dx = 64, 2.19
    g = bf16_to_f32(gpu_box(L, n, dx, 1234, 1.0, storage=L.LYA_BF16, **PK)).astype(np.float64)
    tab = oracle_table(PK, n, dx)
    ref = field.make_box(n, 1234, tab, ("delta", "zz"))
    e = rel_rms(g[..., 0], ref.real), rel_rms(g[..., 1], ref.imag)
    print("bf16 storage rel rms delta %.3e eta %.3e" % e)
    assert max(e) < 4e-3     # bf16 has 8 significant bits: ~2^-9 relative


def test_deterministic(L):
    a = gpu_box(L, 64, 2.19, 42, **PK).cpu().numpy()
    b = gpu_box(L, 64, 2.19, 42, **PK).cpu().numpy()
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("two_buffer", [False, True])
@pytest.mark.parametrize("n", [256, 512])
def test_box_lines_against_c_oracle(L, n, two_buffer):
    """Sampled whole z-lines (exact FP64, plain C oracle) plus Parseval."""
    dx, seed = 2.19, 1234
    print("line parity n=%d two-buffer %s" % (n, two_buffer), flush=True)
    gt = gpu_box(L, n, dx, seed, 1.0, two_buffer=two_buffer, **PK)   # [n, n, n, 2] view of the padded box
    cols = [(0, 0), (1, n - 1), (n // 2, 3), (n - 1, n // 2)]
    tab = oracle_table(PK, n, dx)
    re, im = lines.field_lines(n, seed, tab, cols)
    for l, (mx, my) in enumerate(cols):
        line = gt[mx, my].cpu().numpy().astype(np.float64)
        assert rel_rms(line[:, 0], re[l]) < TOL, (mx, my)
        assert rel_rms(line[:, 1], im[l]) < TOL, (mx, my)


def test_tabulated_power_spectrum(L):
    # a table unlike the analytic form (a log-periodic modulation) through
    # lya_pk.k_tab / p_tab against the oracle's box from the same table
    import torch
    from oracle import power
    n, dx, seed = 64, 2.19, 21
    k = np.geomspace(1e-3, 20.0, 400)
    p = power.PowerSpectrum()(k) * (1.0 + 0.3 * np.sin(3.0 * np.log(k)))
    kt = torch.from_numpy(k).cuda()
    pt = torch.from_numpy(p).cuda()
    got = gpu_box(L, n, dx, seed, 1.0, k_tab=kt, p_tab=pt).cpu().numpy()
    ref = field.make_box(n, seed, power.amplitude_table(power.TabulatedPower(k, p), n, dx), ("delta", "zz"))
    e = (rel_rms(got[..., 0], ref.real), rel_rms(got[..., 1], ref.imag))
    print("tabulated P(k) rel rms delta %.2e eta %.2e" % e)
    assert max(e) < 1e-5
    with pytest.raises(ValueError):
        L.pk_struct(k_tab=kt)
    with pytest.raises(L.LyaError):
        gpu_box(L, n, dx, seed, 1.0, k_tab=kt[:1], p_tab=pt[:1])


@pytest.mark.parametrize("n", [64, 1024])
def test_two_buffer_order_against_in_place(L, n):
    """The two orders of the FFT passes give the same box up to rounding
    (FP32), and BF16 storage differs by at most one bf16 step where the FP32
    values straddle a rounding boundary; with fixed amplitudes (the generic
    synthesiser) too.  The plane padding is never written."""
    import torch
    dx, seed = 2.19, 99
    print("two-buffer against in-place n=%d" % n, flush=True)
    for kw in (dict(), dict(fixed_amp=True)):
        a = gpu_box(L, n, dx, seed, 1.0, **dict(PK, **kw)).clone()
        b = gpu_box(L, n, dx, seed, 1.0, two_buffer=True, **dict(PK, **kw))
        e = (rel_rms(b[..., 0].cpu().numpy().astype(np.float64), a[..., 0].cpu().numpy().astype(np.float64)),
             rel_rms(b[..., 1].cpu().numpy().astype(np.float64), a[..., 1].cpu().numpy().astype(np.float64)))
        print("FP32 %s: rel rms %.2e %.2e" % (kw, e[0], e[1]), flush=True)
        assert max(e) < 1e-6
        del a, b
        torch.cuda.empty_cache()
    a = gpu_box(L, n, dx, seed, 1.0, storage=L.LYA_BF16, **PK).clone()
    b = gpu_box(L, n, dx, seed, 1.0, storage=L.LYA_BF16, two_buffer=True, **PK)
    fa, fb = bf16_to_f32(a), bf16_to_f32(b)
    diff = np.abs(fa - fb)
    # one bf16 step at the value's magnitude, plus what the FP32 values may
    # differ by (2e-5 of the field's RMS, tens of times their RMS difference),
    # which decides the rounding near zero
    rms = np.sqrt(np.mean(fa.astype(np.float64) ** 2, axis=(0, 1, 2)))
    step = np.maximum(np.abs(fa), np.abs(fb)) * 2.0 ** -7 + 2e-5 * rms
    frac = float(np.mean(diff > 0))
    print("BF16: fraction of cells that differ %.2e, largest excess %.2e" % (frac, float(np.max(diff - step))),
          flush=True)
    assert np.all(diff <= step) and frac < 1e-2
