"""Shared helpers of the GPU parity tests: device buffers and calls through
the C-ABI binding, plus the oracle side on the same seeded inputs."""
import numpy as np

import mockinputs
from oracle import power

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None


def rel_rms(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    den = np.sqrt(np.sum(y ** 2))
    return float(np.sqrt(np.sum((x - y) ** 2)) / (den if den > 0 else 1.0))


# Mean flux per redshift bin: relative error at most 1e-6.  The kernels add
# round(F 2^32) as exact integers, so each pixel also carries at most half a
# quantum (2^-33) of rounding; that part is allowed on top.
FBAR_RTOL = 1e-6


def fbar_bin_err(gpu_fsum, fs, cnt):
    """Largest relative error of the per-bin flux sums beyond the fixed-point
    quantum (0 when every bin is within it; inf for a bin whose exact sum is 0
    and whose GPU sum is off by more than the quantum)."""
    g = np.asarray(gpu_fsum, dtype=np.float64)
    r = np.asarray(fs, dtype=np.float64)
    excess = np.maximum(np.abs(g - r) - np.asarray(cnt, dtype=np.float64) * 2.0 ** -33, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(excess > 0, excess / np.abs(r), 0.0)
    return float(np.max(rel)) if rel.size else 0.0


def oracle_table(cfg_pk, n, dx, smooth=0.0):
    pk = power.PowerSpectrum(**cfg_pk)
    return power.amplitude_table(pk, n, dx, smooth)


def gpu_box(L, n, dx, seed, f=1.0, with_eta=True, storage=0, comps=None, two_buffer=False, **pkkw):
    """Run lya_make_box (or lya_make_eta when comps is given) and return the
    device field tensor; two_buffer gives it the workspace of the two-buffer
    order of the FFT passes."""
    box = L.box_struct(n, dx, storage)
    pk = L.pk_struct(**pkkw)
    ws = L.workspace_size(L.LYA_OP_BOX_2BUF if two_buffer else L.LYA_OP_BOX, box)
    work = torch.empty(ws, dtype=torch.uint8, device="cuda")
    elems = L.field_elems(box)
    if storage == L.LYA_F32:
        field = torch.empty((elems, 2), dtype=torch.float32, device="cuda")
    else:
        field = torch.empty((elems,), dtype=torch.int32, device="cuda")
    if comps is None:
        L.make_box(box, pk, seed, f, with_eta, field, work)
    else:
        L.make_eta(box, pk, seed, f, comps[0], comps[1], field, work)
    torch.cuda.synchronize()
    return L.box_view(field, n)


def padded_box(L, arr):
    """Device box in the library layout (padded x planes) holding the host
    array arr [n, n, n, 2] float32."""
    n = arr.shape[0]
    box = L.box_struct(n, 1.0)
    field = torch.zeros((L.field_elems(box), 2), dtype=torch.float32, device="cuda")
    L.box_view(field, n).copy_(torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32)))
    return field


def bf16_to_f32(field_i32):
    """Unpack a BF16x2 box (int32 words) into float32 [..., 2] on the host."""
    w = field_i32.cpu().numpy().view(np.uint32)
    lo = (w << 16).view(np.float32)
    hi = (w & 0xFFFF0000).view(np.float32)
    return np.stack([lo, hi], axis=-1)


def skewer_tensors(L, sk):
    dev = "cuda"
    t = dict(origin_fx=torch.from_numpy(np.ascontiguousarray(sk["origin_fx"])).to(dev),
             step_fx=torch.from_numpy(np.ascontiguousarray(sk["step_fx"])).to(dev),
             npix=torch.from_numpy(np.ascontiguousarray(sk["npix"], dtype=np.int32)).to(dev),
             offset=torch.from_numpy(np.ascontiguousarray(sk["offset"], dtype=np.int64)).to(dev),
             chi0=torch.from_numpy(np.ascontiguousarray(sk["chi0"], dtype=np.float64)).to(dev))
    s = L.skewers_struct(len(sk["npix"]), t["origin_fx"], t["step_fx"], t["npix"], t["offset"], t["chi0"],
                         sk["dchi"], sk.get("id_base", 0))
    return s, t


def total_pixels(sk):
    npix = np.asarray(sk["npix"], dtype=np.int64)
    off = np.asarray(sk["offset"], dtype=np.int64)
    return int(np.max(off + npix)) if len(npix) else 0


def gpu_skewers(L, field, n, dx, sk, seed, ps_amp, ps_kcut, dpix, coef=None, chi_edges=None, omega_m=0.3147,
                storage=0, want=("dens", "eta", "flux"), ps_fixed=False, gauss=False):
    box = L.box_struct(n, dx, storage)
    s, keep = skewer_tensors(L, sk)
    tot = max(total_pixels(sk), 1)
    dens = torch.full((tot,), float("nan"), dtype=torch.float32, device="cuda") if "dens" in want else None
    eta = torch.full((tot,), float("nan"), dtype=torch.float32, device="cuda") if "eta" in want else None
    flux = torch.full((tot,), float("nan"), dtype=torch.float32, device="cuda") if ("flux" in want and coef is not None) else None
    zb = None
    fsum = cnt = edges = None
    if chi_edges is not None:
        edges = torch.from_numpy(np.asarray(chi_edges, dtype=np.float64)).cuda()
        fsum = torch.zeros(len(chi_edges) - 1, dtype=torch.float64, device="cuda")
        cnt = torch.zeros(len(chi_edges) - 1, dtype=torch.int64, device="cuda")
        zb = L.zbins_struct(edges, fsum, cnt)
    ws = L.workspace_size(L.LYA_OP_SKEWERS, box)
    work = torch.empty(ws, dtype=torch.uint8, device="cuda")
    ps = L.Ps1d(float(ps_amp), float(ps_kcut), float(dpix), int(bool(ps_fixed)))
    fg = L.fgpa_struct(coef) if coef is not None else None
    if isinstance(field, (list, tuple)):   # the four boxes of the wide-angle eta_par
        L.draw_skewers_wide(box, field, s, ps, seed, L.Cosmo(omega_m), fg, dens, eta, flux, zb, work)
    elif gauss:
        L.draw_skewers_gauss(box, field, s, ps, seed, L.Cosmo(omega_m), fg, dens, eta, flux, zb, work)
    else:
        L.draw_skewers(box, field, s, ps, seed, L.Cosmo(omega_m), fg, dens, eta, flux, zb, work)
    torch.cuda.synchronize()
    out = {}
    for k, v in (("dens", dens), ("eta", eta), ("flux", flux), ("fsum", fsum), ("count", cnt)):
        if v is not None:
            out[k] = v.cpu().numpy()
    return out


def gpu_apply_fgpa(L, sk, dens, eta, coef, chi_edges=None, omega_m=0.3147):
    s, keep = skewer_tensors(L, sk)
    d = torch.from_numpy(np.asarray(dens, dtype=np.float32)).cuda()
    e = torch.from_numpy(np.asarray(eta, dtype=np.float32)).cuda()
    flux = torch.full_like(d, float("nan"))
    zb = None
    fsum = cnt = None
    if chi_edges is not None:
        edges = torch.from_numpy(np.asarray(chi_edges, dtype=np.float64)).cuda()
        fsum = torch.zeros(len(chi_edges) - 1, dtype=torch.float64, device="cuda")
        cnt = torch.zeros(len(chi_edges) - 1, dtype=torch.int64, device="cuda")
        zb = L.zbins_struct(edges, fsum, cnt)
    work = torch.empty(L.workspace_size(L.LYA_OP_SKEWERS), dtype=torch.uint8, device="cuda")
    L.apply_fgpa(s, L.Cosmo(omega_m), d, e, L.fgpa_struct(coef), flux, zb, work)
    torch.cuda.synchronize()
    out = dict(flux=flux.cpu().numpy())
    if fsum is not None:
        out["fsum"] = fsum.cpu().numpy()
        out["count"] = cnt.cpu().numpy()
    return out
