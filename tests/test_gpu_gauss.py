"""GPU parity of lya_draw_skewers_gauss (the 7^3 Gaussian-kernel average of
section "Gaussian fields along lines of sight") against the FP64 oracle."""
import numpy as np
import pytest

import mockinputs
from oracle import fgpa, field, skewers
from tests.lyahelp import FBAR_RTOL, fbar_bin_err, gpu_box, gpu_skewers, oracle_table, rel_rms

pytestmark = pytest.mark.gpu
TOL = 1e-5
T32 = 2 ** 32


@pytest.fixture(scope="module")
def L():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_18996_amd import lyamock
    lyamock.load()
    return lyamock


@pytest.fixture(scope="module")
def tiny(L):
    cfg = mockinputs.config("tiny")
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    ref = field.make_box(n, seed, oracle_table(cfg["pk"], n, dx), ("delta", "zz"), f=cfg["f"])
    return cfg, ref, {s: gpu_box(L, n, dx, seed, cfg["f"], storage=s, **cfg["pk"]) for s in (0, 1)}


def edge_table(n, dx, S, seed, dpix=0.2):
    """Skewers in every direction starting near the box faces (the 7^3
    neighbourhoods wrap), some exactly through grid points and half-cell
    points (where the nearest grid point switches)."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(S, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    o = rng.uniform(-2.0, 2.0, (S, 3)) + rng.integers(0, 2, (S, 3)) * n
    o[:4] = [[0, 0, 0], [0.5, 0.5, 0.5], [n - 0.5, 3.0, n - 1.0], [1.0, n - 2.5, 0.5]]
    u[:4] = [[0, 0, 1], [1, 0, 0], [0, 1, 0], [0, 0, -1]]
    npix = rng.integers(1, 200, S).astype(np.int32)
    off = np.zeros(S, np.int64)
    off[1:] = np.cumsum(npix[:-1])
    # steps of a whole number of 2^-4 cells keep the half-cell points exact on the axis skewers
    step = np.round(u * (dpix / dx) * 16) / 16
    step[4:] = u[4:] * (dpix / dx)
    return dict(origin_fx=np.round(o * T32).astype(np.int64), step_fx=np.round(step * T32).astype(np.int64),
                npix=npix, offset=off, chi0=rng.uniform(3500.0, 4700.0, S), dchi=dpix, id_base=3,
                total=int(npix.sum()))


@pytest.mark.parametrize("which", ["table", "edges"])
def test_gauss_pipeline_matches_oracle(L, tiny, which):
    cfg, ref, gpu = tiny
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    sk = mockinputs.skewer_table(cfg) if which == "table" else edge_table(n, dx, 300, 5)
    print("gauss skewers (%s): %d skewers, %d pixels" % (which, len(sk["npix"]), sk["total"]), flush=True)
    edges = fgpa.chi_edges_for_z(cfg["z_edges"])
    out = gpu_skewers(L, gpu[0], n, dx, sk, seed, cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"], cfg["fgpa"], edges,
                      gauss=True)
    rd, re_ = skewers.draw_skewers(ref.real, ref.imag, sk, seed, cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"],
                                   interp=skewers.gauss7)
    rf, _ = fgpa.apply_fgpa(rd, re_, sk, cfg["fgpa"])
    e = dict(dens=rel_rms(out["dens"], rd), eta=rel_rms(out["eta"], re_), flux=rel_rms(out["flux"], rf))
    print("gauss rel rms", {k: "%.2e" % v for k, v in e.items()}, flush=True)
    assert all(v < TOL for v in e.values()), e
    fs, cnt = fgpa.mean_flux_bins(rf, fgpa.pixel_chi(sk), edges)
    np.testing.assert_array_equal(out["count"], cnt)
    err = fbar_bin_err(out["fsum"], fs, cnt)
    print("mean flux per bin: largest relative error %.2e" % err)
    assert err <= FBAR_RTOL, err


def test_gauss_smooths_relative_to_trilinear(L, tiny):
    # the kernel average has less variance than trilinear values (the paper's
    # window W^2 = exp(-dx^2 k^2) damps small scales); both against the oracle
    cfg, ref, gpu = tiny
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    sk = mockinputs.skewer_table(cfg)
    g = gpu_skewers(L, gpu[0], n, dx, sk, seed, 0.0, 1.5, 0.2, None, want=("dens",), gauss=True)
    t = gpu_skewers(L, gpu[0], n, dx, sk, seed, 0.0, 1.5, 0.2, None, want=("dens",))
    rg, _ = skewers.draw_skewers(ref.real, ref.imag, sk, seed, interp=skewers.gauss7)
    rt, _ = skewers.draw_skewers(ref.real, ref.imag, sk, seed)
    assert rel_rms(g["dens"], rg) < TOL and rel_rms(t["dens"], rt) < TOL
    assert np.var(rg) < 0.8 * np.var(rt)


def test_gauss_bf16_storage(L, tiny):
    cfg, ref, gpu = tiny
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    sk = edge_table(n, dx, 100, 9)
    out = gpu_skewers(L, gpu[1], n, dx, sk, seed, cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"], cfg["fgpa"],
                      storage=1, gauss=True)
    rd, re_ = skewers.draw_skewers(ref.real, ref.imag, sk, seed, cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"],
                                   interp=skewers.gauss7)
    rf, _ = fgpa.apply_fgpa(rd, re_, sk, cfg["fgpa"])
    e = dict(dens=rel_rms(out["dens"], rd), eta=rel_rms(out["eta"], re_), flux=rel_rms(out["flux"], rf))
    print("gauss bf16 rel rms", {k: "%.2e" % v for k, v in e.items()}, flush=True)
    assert all(v < 1e-2 for v in e.values()), e
