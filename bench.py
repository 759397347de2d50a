"""Benchmark of the Lyman-alpha mock hot path on one MI355X.

One step = one pass of the whole hot path over the workload:
  lya_make_box   P(k) table + sigma8, Philox modes, inverse 3D FFT -> {delta, eta_par}
  lya_draw_skewers  ray-march + trilinear + delta_S + FGPA, per-redshift mean flux
Inputs (skewer table, pixel buffers) are resident in HBM before timing starts.

Prints one JSON line.  `value` is box cells per second of the whole step;
`box_cells_per_s` and `skewer_pixels_per_s` split it by stage (per-kernel HIP
events on the launch stream).  `roofline` reports the dominant kernel's
algorithmic bytes per launch over its mean launch time against 8 TB/s.
`cpu_baseline` times the FP64 oracle on the host on a bounded sample of the
same workload (same cells-to-pixels ratio), scaled to cells per second.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "box cells/s (GRF+FFT), skewer pixels/s (interp+FGPA), %HBM roofline, tune time"
HBM_PEAK_GBS = 8000.0

# HBM traffic of the plain copy kernel against rocprofv3 counters, and the
# counter-based traffic of the dominant kernel (see profiles/); None until taken
TRAFFIC = {}


def algorithmic_bytes(name, n, pixels, n_sk, voxel_bytes):
    cells = float(n) ** 3
    if name == "fft_z_gen":
        return 8.0 * cells                   # writes the complex64 box
    if name in ("fft_y", "fft_x"):
        return 16.0 * cells                  # reads and writes it
    if name == "skewers":
        return 12.0 * pixels + voxel_bytes + 44.0 * n_sk
    return None


def distinct_voxel_bytes(sk, n, sample=2000, seed=0):
    """8 bytes per distinct voxel a skewer's trilinear gathers touch, counted
    exactly on a sample of skewers and scaled to all of them."""
    rng = np.random.default_rng(seed)
    S = len(sk["npix"])
    idx = rng.choice(S, size=min(sample, S), replace=False)
    tot_vox = 0
    tot_pix = 0
    for q in idx:
        j = np.arange(int(sk["npix"][q]), dtype=np.int64)[:, None]
        pos = sk["origin_fx"][q][None, :] + j * sk["step_fx"][q][None, :]
        cell = (pos >> 32) % n
        corners = set()
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    lin = (((cell[:, 0] + a) % n) * n + (cell[:, 1] + b) % n) * n + (cell[:, 2] + c) % n
                    corners.update(lin.tolist())
        tot_vox += len(corners)
        tot_pix += len(j)
    per_pix = tot_vox / max(tot_pix, 1)
    return 8.0 * per_pix * float(np.sum(sk["npix"], dtype=np.int64)), per_pix


def cpu_baseline(cfg, pixels_per_cell, budget_n=256):
    """Time the oracle on a bounded sample of the workload: a budget_n^3 box and
    the same number of pixels per box cell as the full workload."""
    import mockinputs
    from oracle import fgpa, field, power, skewers
    cells = budget_n ** 3
    want_pix = pixels_per_cell * cells
    sk_full = mockinputs.skewer_table(dict(cfg, n=budget_n), n_sk=max(64, int(want_pix / 700)))
    # keep the workload's length mix, take just enough skewers
    cum = np.cumsum(sk_full["npix"].astype(np.int64))
    ns = int(np.searchsorted(cum, want_pix)) + 1
    sk = {k: (v[:ns] if isinstance(v, np.ndarray) else v) for k, v in sk_full.items()}
    pix = int(np.sum(sk["npix"], dtype=np.int64))
    t0 = time.perf_counter()
    tab = power.amplitude_table(power.PowerSpectrum(**cfg["pk"]), budget_n, cfg["dx"])
    box = field.make_box(budget_n, cfg["seed"], tab, ("delta", "zz"), f=cfg["f"])
    t1 = time.perf_counter()
    dens, eta = skewers.draw_skewers(box.real, box.imag, sk, cfg["seed"], cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"])
    F, _ = fgpa.apply_fgpa(dens, eta, sk, cfg["fgpa"])
    fgpa.mean_flux_bins(F, fgpa.pixel_chi(sk), fgpa.chi_edges_for_z(cfg["z_edges"]))
    t2 = time.perf_counter()
    return dict(value=cells / (t2 - t0), unit="box cells/s", cores=1, kind="oracle",
                sample="%d^3 box (%d cells) + %d skewers (%d pixels, the workload's pixels per cell) on the host; "
                       "box %.2f s, skewers+FGPA %.2f s; numpy/scipy single-threaded" % (
                           budget_n, cells, ns, pix, t1 - t0, t2 - t1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="big", choices=["tiny", "mid", "big", "precision", "emulator"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=192)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 4 GiB device copy first (reference for rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path is single-GPU (multi-GPU sharding is "
              "a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import mockinputs
    from oracle import fgpa as ofgpa
    from paper_2310_18996_amd import lyamock as L

    L.load()
    torch.cuda.set_device(0)
    cfg = mockinputs.config(args.config)
    n, dx, seed = cfg["n"], cfg["dx"], cfg["seed"]
    print("bench: config %s n=%d skewers=%d" % (args.config, n, cfg["n_sk"]), file=sys.stderr, flush=True)
    sk = mockinputs.skewer_table(cfg)
    pixels = sk["total"]
    n_sk = len(sk["npix"])
    box = L.box_struct(n, dx)
    pk = L.pk_struct(**cfg["pk"])
    field = torch.empty((L.field_elems(box), 2), dtype=torch.float32, device="cuda")
    bwork = torch.empty(L.workspace_size(L.LYA_OP_BOX, box), dtype=torch.uint8, device="cuda")
    swork = torch.empty(L.workspace_size(L.LYA_OP_SKEWERS, box), dtype=torch.uint8, device="cuda")
    dev = {k: torch.from_numpy(np.ascontiguousarray(sk[k])).cuda()
           for k in ("origin_fx", "step_fx", "npix", "offset", "chi0")}
    s = L.skewers_struct(n_sk, dev["origin_fx"], dev["step_fx"], dev["npix"], dev["offset"], dev["chi0"], sk["dchi"])
    dens = torch.empty(pixels, dtype=torch.float32, device="cuda")
    eta = torch.empty_like(dens)
    flux = torch.empty_like(dens)
    # redshift-bin edges in comoving distance: the library's own host-side
    # conversion is not exposed, the FP64 oracle's table of 23 numbers is used
    edges = torch.from_numpy(ofgpa.chi_edges_for_z(cfg["z_edges"])).cuda()
    fsum = torch.zeros(len(cfg["z_edges"]) - 1, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(len(cfg["z_edges"]) - 1, dtype=torch.int64, device="cuda")
    zb = L.zbins_struct(edges, fsum, cnt)
    ps = L.Ps1d(cfg["ps_amp"], cfg["ps_kcut"], cfg["dpix"], 0)
    cosmo = L.Cosmo(cfg["omega_m"])
    fg = L.fgpa_struct(cfg["fgpa"])
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        # a plain copy of known size: 4 GiB read, 4 GiB written
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        L.make_box(box, pk, seed, cfg["f"], True, field, bwork, stream)
        L.draw_skewers(box, field, s, ps, seed, cosmo, fg, dens, eta, flux, zb, swork, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)
    L.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = L.timing_read()
    L.timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    box_names = ("pk_sigma8", "pk_finalize", "pk_table", "fft_z_gen", "fft_y", "fft_x")
    sk_names = ("zchi_table", "twiddles", "skewer_reset", "skewers", "skewer_finalize")
    box_ms = sum(kt[k][0] for k in box_names if k in kt) / args.steps
    sk_ms = sum(kt[k][0] for k in sk_names if k in kt) / args.steps
    cells = float(n) ** 3
    vox_bytes, vox_per_pix = distinct_voxel_bytes(sk, n)
    dom = max(kt, key=lambda k: kt[k][0])
    avg_ms = kt[dom][0] / kt[dom][1]
    ab = algorithmic_bytes(dom, n, pixels, n_sk, vox_bytes)
    achieved = ab / (avg_ms * 1e-3) / 1e9 if ab else None
    roof = dict(kernel=dom, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(achieved / HBM_PEAK_GBS) if achieved else None, traffic=TRAFFIC.get(dom),
                algorithmic_bytes_per_launch=ab, mean_launch_ms=avg_ms)
    kernels = {k: dict(mean_ms=v[0] / v[1], launches=v[1]) for k, v in sorted(kt.items())}
    for k in kernels:
        b = algorithmic_bytes(k, n, pixels, n_sk, vox_bytes)
        if b:
            kernels[k]["algorithmic_GBps"] = b / (kernels[k]["mean_ms"] * 1e-3) / 1e9
    out = dict(metric=METRIC, value=cells / (ms_step * 1e-3), unit="box cells/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload="%s: %d^3 box at %.2f Mpc/h, %d skewers, %d pixels (%d-%d per skewer)" % (
                   args.config, n, dx, n_sk, pixels, int(sk["npix"].min()), int(sk["npix"].max())),
                   n=n, dx=dx, n_skewers=n_sk, pixels=pixels, seed=seed),
               box_cells_per_s=cells / (box_ms * 1e-3), box_ms=box_ms,
               skewer_pixels_per_s=pixels / (sk_ms * 1e-3), skewer_ms=sk_ms,
               distinct_voxels_per_pixel=vox_per_pix, roofline=roof, kernels=kernels)
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, pixels / cells, args.cpu_n)
        out["cpu_baseline"]["host_cpus"] = os.cpu_count()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
