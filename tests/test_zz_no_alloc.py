"""The allocation-free entry point lya_draw_skewers_static (its workspace is
the library's static device array) against lya_draw_skewers with a caller
workspace, through the C-ABI: two calls in a row, the second on a smaller
input with fewer redshift bins, each bit-identical to the workspace call (the
same kernels on the same inputs), which the parity tests hold to the oracle."""
import numpy as np
import pytest

import mockinputs
from tests.lyahelp import gpu_box, skewer_tensors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_18996_amd import lyamock
    lyamock.load()
    return lyamock


def _run(L, torch, fn, box, fld, sk, cfg, edges, work=None):
    s, keep = skewer_tensors(L, sk)
    tot = int(sk["total"])
    d, e, f = (torch.full((tot,), float("nan"), dtype=torch.float32, device="cuda") for _ in range(3))
    ed = torch.from_numpy(np.asarray(edges, dtype=np.float64)).cuda()
    fs = torch.full((len(edges) - 1,), -1.0, dtype=torch.float64, device="cuda")
    cn = torch.full((len(edges) - 1,), -1, dtype=torch.int64, device="cuda")
    args = (box, fld, s, L.Ps1d(cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"], 0), cfg["seed"], L.Cosmo(cfg["omega_m"]),
            L.fgpa_struct(cfg["fgpa"]), d, e, f, L.zbins_struct(ed, fs, cn))
    if work is None:
        fn(*args)
    else:
        fn(*args, work)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (d, e, f, fs, cn)]


def test_static_scratch_entry_point_matches_the_workspace_call(L):
    import torch
    from oracle import fgpa
    cfg = mockinputs.config("tiny")
    n, dx = cfg["n"], cfg["dx"]
    box = L.box_struct(n, dx)
    view = gpu_box(L, n, dx, cfg["seed"], cfg["f"], **cfg["pk"])
    fld = torch.zeros((L.field_elems(box), 2), dtype=torch.float32, device="cuda")
    L.box_view(fld, n).copy_(view)
    work = torch.empty(L.workspace_size(L.LYA_OP_SKEWERS, box), dtype=torch.uint8, device="cuda")
    big = mockinputs.skewer_table(cfg)
    small = mockinputs.skewer_table(cfg, n_sk=37, seed=99)
    edges_big = fgpa.chi_edges_for_z(cfg["z_edges"])
    edges_small = edges_big[::3]
    print("static scratch: %d skewers (%d pixels) then %d skewers (%d pixels)" % (
        len(big["npix"]), big["total"], len(small["npix"]), small["total"]), flush=True)
    for sk, edges in ((big, edges_big), (small, edges_small)):
        got = _run(L, torch, L.draw_skewers_static, box, fld, sk, cfg, edges)
        ref = _run(L, torch, L.draw_skewers, box, fld, sk, cfg, edges, work)
        for name, g, r in zip(("dens", "eta", "flux", "fsum", "count"), got, ref):
            assert np.array_equal(g, r), name
        assert np.all(np.isfinite(got[2])) and int(got[4].sum()) > 0
