"""ctypes binding of liblyamock.so (include/lyamock.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library.  Device buffers are torch tensors on the current HIP
device; the stream is torch's current stream unless one is given.  A missing
or unloadable library raises immediately: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblyamock.so")

LYA_OK, LYA_EINVAL, LYA_EWORKSPACE, LYA_EUNSUPPORTED, LYA_EHIP = 0, -1, -2, -3, -4
LYA_F32, LYA_BF16 = 0, 1
LYA_OP_BOX, LYA_OP_SKEWERS, LYA_OP_QUASARS, LYA_OP_BOX_2BUF = 0, 1, 2, 3
LYA_C_NONE, LYA_C_DELTA, LYA_C_XX, LYA_C_YY, LYA_C_ZZ, LYA_C_XY, LYA_C_XZ, LYA_C_YZ = -1, 0, 1, 2, 3, 4, 5, 6
LYA_C_VX, LYA_C_VY, LYA_C_VZ = 7, 8, 9
COMPONENTS = {"none": -1, "delta": 0, "xx": 1, "yy": 2, "zz": 3, "xy": 4, "xz": 5, "yz": 6, "vx": 7, "vy": 8,
              "vz": 9}

EXPORTS = ("lya_field_elems", "lya_plane_pitch", "lya_workspace_size", "lya_make_box", "lya_make_eta",
           "lya_make_box_pair", "lya_lognormal_workspace_size", "lya_lognormal_pk", "lya_box_moments",
           "lya_draw_quasars", "lya_quasar_skewers",
           "lya_draw_skewers", "lya_draw_skewers_static", "lya_draw_skewers_gauss", "lya_draw_skewers_wide", "lya_apply_fgpa",
           "lya_apply_fgpa_ds", "lya_tune_ps_workspace_size", "lya_tune_ps", "lya_tune_ps_last_error",
           "lya_emulator_labels_ps",
           "lya_p1d_workspace_size", "lya_p1d",
           "lya_tune_workspace_size",
           "lya_tune_params", "lya_emulator_labels", "lya_emulator_bytes", "lya_emulator_param_offset",
           "lya_emulator_param_count", "lya_emulator_init", "lya_emulator_train_workspace_size",
           "lya_emulator_set_scaling", "lya_emulator_loss_grad", "lya_emulator_train", "lya_emulator_predict",
           "lya_emulator_last_error", "lya_chi_of_z", "lya_get_tuning", "lya_set_tuning",
           "lya_autotune_fft", "lya_autotune_skewers", "lya_graph_begin", "lya_graph_end", "lya_graph_launch",
           "lya_graph_destroy", "lya_autotune_last_error", "lya_timing_enable", "lya_timing_collect", "lya_timing_get",
           "lya_last_error", "lya_version")


class LyaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lyamock error %d: %s" % (code, msg))
        self.code = code


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dx", ctypes.c_double), ("storage", ctypes.c_int32)]


class Pk(ctypes.Structure):
    _fields_ = [("sigma8", ctypes.c_double), ("ns", ctypes.c_double), ("gamma", ctypes.c_double),
                ("wig_amp", ctypes.c_double), ("wig_r", ctypes.c_double), ("wig_kd", ctypes.c_double),
                ("smooth", ctypes.c_double), ("fixed_amp", ctypes.c_int32), ("only_n2", ctypes.c_int32),
                ("k_tab", ctypes.c_void_p), ("p_tab", ctypes.c_void_p), ("n_tab", ctypes.c_int32)]


class Skewers(ctypes.Structure):
    _fields_ = [("n_sk", ctypes.c_int64), ("origin_fx", ctypes.c_void_p), ("step_fx", ctypes.c_void_p),
                ("npix", ctypes.c_void_p), ("offset", ctypes.c_void_p), ("chi0", ctypes.c_void_p),
                ("dchi", ctypes.c_double), ("id_base", ctypes.c_int64)]


class Ps1d(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("kcut", ctypes.c_double), ("dpix", ctypes.c_double),
                ("fixed_amp", ctypes.c_int32)]


class Fgpa(ctypes.Structure):
    _fields_ = [("coef", (ctypes.c_double * 3) * 3)]


class Cosmo(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double)]


class ZBins(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("chi_edges", ctypes.c_void_p), ("fsum", ctypes.c_void_p),
                ("count", ctypes.c_void_p)]


_lib = None


def load():
    """Load the in-tree library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblyamock.so not built at %s (run __graft_entry__.build())" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, VP = ctypes.POINTER, ctypes.c_void_p
    lib.lya_field_elems.restype = ctypes.c_size_t
    lib.lya_field_elems.argtypes = [P(Box)]
    lib.lya_plane_pitch.restype = ctypes.c_size_t
    lib.lya_plane_pitch.argtypes = [P(Box)]
    lib.lya_workspace_size.restype = ctypes.c_size_t
    lib.lya_workspace_size.argtypes = [ctypes.c_int, P(Box)]
    lib.lya_make_box.restype = ctypes.c_int
    lib.lya_make_box.argtypes = [P(Box), P(Pk), ctypes.c_uint64, ctypes.c_double, ctypes.c_int, VP, VP,
                                 ctypes.c_size_t, VP]
    lib.lya_make_eta.restype = ctypes.c_int
    lib.lya_make_eta.argtypes = [P(Box), P(Pk), ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 VP, VP, ctypes.c_size_t, VP]
    lib.lya_draw_skewers.restype = ctypes.c_int
    lib.lya_draw_skewers.argtypes = [P(Box), VP, P(Skewers), P(Ps1d), ctypes.c_uint64, P(Cosmo), P(Fgpa),
                                     VP, VP, VP, P(ZBins), VP, ctypes.c_size_t, VP]
    lib.lya_draw_skewers_static.restype = ctypes.c_int
    lib.lya_draw_skewers_static.argtypes = [P(Box), VP, P(Skewers), P(Ps1d), ctypes.c_uint64, P(Cosmo), P(Fgpa),
                                            VP, VP, VP, P(ZBins), VP]
    lib.lya_draw_skewers_gauss.restype = ctypes.c_int
    lib.lya_draw_skewers_gauss.argtypes = lib.lya_draw_skewers.argtypes
    lib.lya_draw_skewers_wide.restype = ctypes.c_int
    lib.lya_draw_skewers_wide.argtypes = [P(Box), P(VP), P(Skewers), P(Ps1d), ctypes.c_uint64, P(Cosmo),
                                          P(Fgpa), VP, VP, VP, P(ZBins), VP, ctypes.c_size_t, VP]
    lib.lya_apply_fgpa.restype = ctypes.c_int
    lib.lya_apply_fgpa.argtypes = [P(Skewers), P(Cosmo), VP, VP, P(Fgpa), VP, P(ZBins), VP, ctypes.c_size_t, VP]
    lib.lya_timing_enable.restype = ctypes.c_int
    lib.lya_timing_enable.argtypes = [ctypes.c_int]
    lib.lya_timing_collect.restype = ctypes.c_int
    lib.lya_timing_get.restype = ctypes.c_int
    lib.lya_timing_get.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
    lib.lya_last_error.restype = ctypes.c_char_p
    lib.lya_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error():
    return load().lya_last_error().decode()


def _check(rc):
    if rc != LYA_OK:
        raise LyaError(rc, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def box_struct(n, dx, storage=LYA_F32):
    return Box(int(n), float(dx), int(storage))


def pk_struct(sigma8=0.8, ns=0.96, gamma=0.21, wig_amp=0.05, wig_r=105.0, wig_kd=0.2, smooth=0.0,
              fixed_amp=False, only_n2=-1, k_tab=None, p_tab=None):
    """lya_pk; k_tab/p_tab: device float64 tensors of a tabulated P(k) (both or neither)."""
    if (k_tab is None) != (p_tab is None):
        raise ValueError("k_tab and p_tab go together")
    n_tab = 0 if k_tab is None else int(k_tab.numel())
    return Pk(sigma8, ns, gamma, wig_amp, wig_r, wig_kd, smooth, int(bool(fixed_amp)), int(only_n2),
              None if k_tab is None else k_tab.data_ptr(), None if p_tab is None else p_tab.data_ptr(), n_tab)


def field_elems(box):
    return int(load().lya_field_elems(ctypes.byref(box)))


def plane_pitch(box):
    return int(load().lya_plane_pitch(ctypes.byref(box)))


def box_view(field, n):
    """[n, n, n, ...] view (no copy) of a box tensor whose first dimension holds
    the field_elems elements; the plane padding is sliced away."""
    pitch = field.shape[0] // n
    return field.view(n, pitch, *field.shape[1:])[:, :n * n].unflatten(1, (n, n))


def workspace_size(op, box=None):
    return int(load().lya_workspace_size(int(op), ctypes.byref(box) if box is not None else None))


def make_box(box, pk, seed, f, with_eta, field, work, stream=None):
    """lya_make_box: field (n^3 x 2 float32, or n^3 int32 for BF16) on device."""
    _check(load().lya_make_box(ctypes.byref(box), ctypes.byref(pk), int(seed), float(f), int(bool(with_eta)),
                               _ptr(field), _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def make_eta(box, pk, seed, f, comp_a, comp_b, field, work, stream=None):
    """lya_make_eta: {comp_a, comp_b} of the same modes (component names as in COMPONENTS)."""
    ca = COMPONENTS[comp_a] if isinstance(comp_a, str) else int(comp_a)
    cb = COMPONENTS[comp_b] if isinstance(comp_b, str) else int(comp_b)
    _check(load().lya_make_eta(ctypes.byref(box), ctypes.byref(pk), int(seed), float(f), ca, cb, _ptr(field),
                               _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def skewers_struct(n_sk, origin_fx, step_fx, npix, offset, chi0, dchi, id_base=0):
    return Skewers(int(n_sk), _ptr(origin_fx), _ptr(step_fx), _ptr(npix), _ptr(offset), _ptr(chi0),
                   float(dchi), int(id_base))


def fgpa_struct(coef):
    fg = Fgpa()
    for p in range(3):
        for i in range(3):
            fg.coef[p][i] = float(coef[p][i])
    return fg


def zbins_struct(chi_edges, fsum, count):
    if chi_edges is None:
        return None
    return ZBins(int(chi_edges.numel() - 1), _ptr(chi_edges), _ptr(fsum), _ptr(count))


def draw_skewers(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zbins, work, stream=None):
    """lya_draw_skewers (see include/lyamock.h)."""
    _check(load().lya_draw_skewers(ctypes.byref(box), _ptr(field), ctypes.byref(sk),
                                   ctypes.byref(ps) if ps is not None else None, int(seed),
                                   ctypes.byref(cosmo) if cosmo is not None else None,
                                   ctypes.byref(fgpa) if fgpa is not None else None,
                                   _ptr(dens), _ptr(eta), _ptr(flux),
                                   ctypes.byref(zbins) if zbins is not None else None,
                                   _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def draw_skewers_static(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zbins, stream=None):
    """lya_draw_skewers_static: lya_draw_skewers without a workspace argument
    (the library's static device scratch; see include/lyamock.h)."""
    _check(load().lya_draw_skewers_static(ctypes.byref(box), _ptr(field), ctypes.byref(sk),
                                          ctypes.byref(ps) if ps is not None else None, int(seed),
                                          ctypes.byref(cosmo) if cosmo is not None else None,
                                          ctypes.byref(fgpa) if fgpa is not None else None,
                                          _ptr(dens), _ptr(eta), _ptr(flux),
                                          ctypes.byref(zbins) if zbins is not None else None, _stream(stream)))


def draw_skewers_gauss(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zbins, work, stream=None):
    """lya_draw_skewers_gauss (see include/lyamock.h): the 7^3 Gaussian-kernel
    average in place of trilinear interpolation."""
    _check(load().lya_draw_skewers_gauss(ctypes.byref(box), _ptr(field), ctypes.byref(sk),
                                         ctypes.byref(ps) if ps is not None else None, int(seed),
                                         ctypes.byref(cosmo) if cosmo is not None else None,
                                         ctypes.byref(fgpa) if fgpa is not None else None,
                                         _ptr(dens), _ptr(eta), _ptr(flux),
                                         ctypes.byref(zbins) if zbins is not None else None,
                                         _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def draw_skewers_wide(box, fields, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zbins, work, stream=None):
    """lya_draw_skewers_wide (see include/lyamock.h): fields = the four boxes
    {delta, eta_zz}, {eta_xx, eta_yy}, {eta_xy, eta_xz}, {eta_yz, 0}."""
    if len(fields) != 4:
        raise ValueError("fields must hold four boxes")
    arr = (ctypes.c_void_p * 4)(*[_ptr(f) for f in fields])
    _check(load().lya_draw_skewers_wide(ctypes.byref(box), arr, ctypes.byref(sk),
                                        ctypes.byref(ps) if ps is not None else None, int(seed),
                                        ctypes.byref(cosmo) if cosmo is not None else None,
                                        ctypes.byref(fgpa) if fgpa is not None else None,
                                        _ptr(dens), _ptr(eta), _ptr(flux),
                                        ctypes.byref(zbins) if zbins is not None else None,
                                        _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def apply_fgpa(sk, cosmo, dens, eta, fgpa, flux, zbins, work, stream=None):
    """lya_apply_fgpa (see include/lyamock.h)."""
    _check(load().lya_apply_fgpa(ctypes.byref(sk), ctypes.byref(cosmo) if cosmo is not None else None,
                                 _ptr(dens), _ptr(eta), ctypes.byref(fgpa) if fgpa is not None else None,
                                 _ptr(flux), ctypes.byref(zbins) if zbins is not None else None,
                                 _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def timing_enable(on=True):
    _check(load().lya_timing_enable(int(bool(on))))


def timing_read():
    """{kernel name: (total ms, launches)} of the launches recorded since
    timing_enable(True)."""
    lib = load()
    n = lib.lya_timing_collect()
    if n < 0:
        raise LyaError(n, "timing collection failed")
    out = {}
    buf = ctypes.create_string_buffer(64)
    for i in range(n):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib.lya_timing_get(i, buf, 64, ctypes.byref(ms), ctypes.byref(cnt)))
        out[buf.value.decode()] = (ms.value, cnt.value)
    return out


# ---------------------------------------------------------------- 1D power, tuning, emulator
class P1dSpec(ctypes.Structure):
    _fields_ = [("n_kbins", ctypes.c_int32), ("k_edges", ctypes.c_void_p), ("z_ref", ctypes.c_double),
                ("dpix", ctypes.c_double)]


TUNE_MAX_Z = 16
LYA_TUNE_PLAIN, LYA_TUNE_EMULATOR = 0, 1


class TuneSpec(ctypes.Structure):
    _fields_ = [("sk", ctypes.POINTER(Skewers)), ("dens", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("cosmo", Cosmo), ("n_zt", ctypes.c_int32),
                ("z_t", ctypes.c_double * TUNE_MAX_Z), ("c_t", ctypes.c_double * TUNE_MAX_Z),
                ("fbar_t", ctypes.c_double * TUNE_MAX_Z), ("p1d_t", ctypes.c_void_p), ("p1d", P1dSpec),
                ("a0", ctypes.c_double), ("b0", ctypes.c_double), ("sigma_rel", ctypes.c_double),
                ("xatol", ctypes.c_double), ("fatol", ctypes.c_double), ("max_evals", ctypes.c_int32),
                ("emulator", ctypes.c_void_p), ("emu_checks", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * TUNE_MAX_Z), ("b", ctypes.c_double * TUNE_MAX_Z),
                ("chi2", ctypes.c_double * TUNE_MAX_Z), ("fbar", ctypes.c_double * TUNE_MAX_Z),
                ("p1d", ctypes.c_double * (TUNE_MAX_Z * 64)), ("evals", ctypes.c_int32 * TUNE_MAX_Z),
                ("gpu_evals", ctypes.c_int32 * TUNE_MAX_Z),
                ("coef", (ctypes.c_double * 3) * 3), ("seconds", ctypes.c_double),
                ("fallback", ctypes.c_int32 * TUNE_MAX_Z)]


TUNE_PS_MAX_ITER = 16
TUNE_PS_MAX_OUTER = 8
TUNE_PS_RATIOS = 0
TUNE_PS_EMULATOR = 1
PS_UPDATE_PAPER = 0
PS_UPDATE_SECANT = 1


class PsTable(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("k_edges", ctypes.c_void_p), ("ratio", ctypes.c_void_p)]


class TunePsSpec(ctypes.Structure):
    _fields_ = [("sk", ctypes.POINTER(Skewers)), ("dens_l", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("n_pixels", ctypes.c_int64), ("cosmo", Cosmo), ("seed", ctypes.c_uint64), ("n_zt", ctypes.c_int32),
                ("z_t", ctypes.c_double * TUNE_MAX_Z), ("c_t", ctypes.c_double * TUNE_MAX_Z),
                ("fbar_t", ctypes.c_double * TUNE_MAX_Z), ("sigf_t", ctypes.c_double * TUNE_MAX_Z),
                ("p1d_t", ctypes.c_void_p), ("p1d", P1dSpec), ("ps_amp", ctypes.c_double),
                ("ps_kcut", ctypes.c_double), ("n_iter", ctypes.c_int32), ("n_outer", ctypes.c_int32),
                ("beff_t", ctypes.c_double * TUNE_MAX_Z), ("f", ctypes.c_double), ("beff_at_z", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("emu", ctypes.c_void_p * TUNE_MAX_Z), ("emu_checks", ctypes.c_int32),
                ("emu_refine", ctypes.c_int32), ("update", ctypes.c_int32)]


class TunePsResult(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * TUNE_MAX_Z), ("b", ctypes.c_double * TUNE_MAX_Z),
                ("s", ctypes.c_double * TUNE_MAX_Z), ("sigma2", ctypes.c_double * 3),
                ("ratio", ctypes.c_double * (TUNE_MAX_Z * 64)), ("p1d", ctypes.c_double * (TUNE_MAX_Z * 64)),
                ("fbar", ctypes.c_double * (TUNE_MAX_Z * TUNE_PS_MAX_ITER)),
                ("rms", ctypes.c_double * (TUNE_MAX_Z * TUNE_PS_MAX_ITER)), ("seconds", ctypes.c_double),
                ("beff", ctypes.c_double * (TUNE_MAX_Z * TUNE_PS_MAX_OUTER)),
                ("n_outer_done", ctypes.c_int32 * TUNE_MAX_Z), ("growth", ctypes.c_double * TUNE_MAX_Z),
                ("ps_fit", ctypes.c_double * (2 * TUNE_MAX_Z)), ("gpu_evals", ctypes.c_int32 * TUNE_MAX_Z),
                ("fallback", ctypes.c_int32 * TUNE_MAX_Z)]


FFT_VARIANTS = 16
SK_CHUNKS = (1, 2, 4, 8, 16, 32, 64)
SK_BLOCKS_PER_CU = (1, 2, 3, 4)
SK_UNROLL = (1, 2, 4)


class Tuning(ctypes.Structure):
    _fields_ = [("fft_y", ctypes.c_int32), ("fft_x", ctypes.c_int32), ("sk_chunk", ctypes.c_int32),
                ("sk_blocks_per_cu", ctypes.c_int32), ("sk_unroll", ctypes.c_int32)]


class QsoSpec(ctypes.Structure):
    _fields_ = [("n_box", ctypes.c_int32), ("box_a", ctypes.c_void_p), ("box_b", ctypes.c_void_p),
                ("z_box", ctypes.c_double * 3), ("var", ctypes.c_void_p * 3), ("xi5", ctypes.c_double),
                ("observer", ctypes.c_double * 3), ("n_nbar", ctypes.c_int32), ("nbar_z", ctypes.c_void_p),
                ("nbar", ctypes.c_void_p), ("seed", ctypes.c_uint64)]


def qso_spec(boxes, z_box, var_ptrs, observer, nbar_z, nbar, seed, xi5=0.0):
    """lya_qso_spec.  boxes: [box_a] or [box_a, box_b] device tensors; var_ptrs:
    device addresses (ints) of the variances; nbar_z, nbar: device float64.
    The spec holds references to the tensors it points to."""
    sp = QsoSpec()
    sp.n_box = len(z_box)
    sp.box_a = boxes[0].data_ptr()
    sp.box_b = boxes[1].data_ptr() if len(boxes) > 1 else None
    for i, z in enumerate(z_box):
        sp.z_box[i] = float(z)
        sp.var[i] = int(var_ptrs[i])
    sp.xi5 = float(xi5)
    for i in range(3):
        sp.observer[i] = float(observer[i])
    sp.n_nbar = int(nbar_z.numel())
    sp.nbar_z = nbar_z.data_ptr()
    sp.nbar = nbar.data_ptr()
    sp.seed = int(seed)
    sp._refs = (boxes, nbar_z, nbar)   # the device arrays must outlive the spec
    return sp


class QsoLosSpec(ctypes.Structure):
    _fields_ = [("n_q", ctypes.c_int64), ("pos_fx", ctypes.c_void_p), ("vel_xy", ctypes.c_void_p),
                ("vel_z", ctypes.c_void_p), ("observer", ctypes.c_double * 3), ("lam_lo", ctypes.c_double),
                ("lam_hi", ctypes.c_double), ("z_min", ctypes.c_double), ("dchi", ctypes.c_double)]


def _bind_more(lib):
    P, VP = ctypes.POINTER, ctypes.c_void_p
    lib.lya_p1d_workspace_size.restype = ctypes.c_size_t
    lib.lya_p1d_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.lya_p1d.restype = ctypes.c_int
    lib.lya_p1d.argtypes = [P(Skewers), P(Cosmo), VP, P(ZBins), P(P1dSpec), VP, VP, VP, ctypes.c_size_t, VP]
    lib.lya_tune_workspace_size.restype = ctypes.c_size_t
    lib.lya_tune_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.lya_tune_params.restype = ctypes.c_int
    lib.lya_tune_params.argtypes = [P(TuneSpec), P(TuneResult), ctypes.c_int, VP, ctypes.c_size_t, VP]
    lib.lya_emulator_labels.restype = ctypes.c_int
    lib.lya_emulator_labels.argtypes = [P(TuneSpec), VP, ctypes.c_int64, VP, VP, ctypes.c_size_t, VP]
    lib.lya_emulator_bytes.restype = ctypes.c_size_t
    lib.lya_emulator_bytes.argtypes = [ctypes.c_int32]
    lib.lya_emulator_param_offset.restype = ctypes.c_size_t
    lib.lya_emulator_param_count.restype = ctypes.c_size_t
    lib.lya_emulator_param_count.argtypes = [ctypes.c_int32]
    lib.lya_emulator_init.restype = ctypes.c_int
    lib.lya_emulator_init.argtypes = [VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P(ctypes.c_double),
                                      P(ctypes.c_double), ctypes.c_int32, VP]
    lib.lya_emulator_train_workspace_size.restype = ctypes.c_size_t
    lib.lya_emulator_train_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.lya_emulator_set_scaling.restype = ctypes.c_int
    lib.lya_emulator_set_scaling.argtypes = [VP, VP, ctypes.c_int64, VP]
    lib.lya_emulator_loss_grad.restype = ctypes.c_int
    lib.lya_emulator_loss_grad.argtypes = [VP, VP, VP, ctypes.c_int32, ctypes.c_int32, VP, VP, VP, ctypes.c_size_t,
                                           VP]
    lib.lya_emulator_train.restype = ctypes.c_int
    lib.lya_emulator_train.argtypes = [VP, VP, VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int32, VP, VP, ctypes.c_size_t, VP]
    lib.lya_emulator_predict.restype = ctypes.c_int
    lib.lya_emulator_predict.argtypes = [VP, VP, ctypes.c_int64, VP, VP]
    lib.lya_emulator_last_error.restype = ctypes.c_char_p
    lib.lya_chi_of_z.restype = ctypes.c_int
    lib.lya_get_tuning.restype = ctypes.c_int
    lib.lya_get_tuning.argtypes = [ctypes.c_int32, P(Tuning)]
    lib.lya_set_tuning.restype = ctypes.c_int
    lib.lya_set_tuning.argtypes = [ctypes.c_int32, P(Tuning)]
    lib.lya_autotune_fft.restype = ctypes.c_int
    lib.lya_autotune_fft.argtypes = [P(Box), VP, VP, ctypes.c_size_t, ctypes.c_int32, VP, P(Tuning), VP]
    lib.lya_autotune_skewers.restype = ctypes.c_int
    lib.lya_autotune_skewers.argtypes = [P(Box), VP, P(Skewers), P(Ps1d), ctypes.c_uint64, P(Cosmo), P(Fgpa), VP, VP,
                                         VP, P(ZBins), VP, ctypes.c_size_t, ctypes.c_int32, VP, P(Tuning), VP]
    lib.lya_graph_begin.restype = ctypes.c_int
    lib.lya_graph_begin.argtypes = [VP]
    lib.lya_graph_end.restype = ctypes.c_int
    lib.lya_graph_end.argtypes = [VP, P(VP)]
    lib.lya_graph_launch.restype = ctypes.c_int
    lib.lya_graph_launch.argtypes = [VP, VP]
    lib.lya_graph_destroy.restype = ctypes.c_int
    lib.lya_graph_destroy.argtypes = [VP]
    lib.lya_autotune_last_error.restype = ctypes.c_char_p
    lib.lya_chi_of_z.argtypes = [P(Cosmo), ctypes.c_int32, VP, VP]
    lib.lya_apply_fgpa_ds.restype = ctypes.c_int
    lib.lya_apply_fgpa_ds.argtypes = [P(Skewers), P(Cosmo), VP, VP, P(Ps1d), P(PsTable), ctypes.c_uint64, P(Fgpa),
                                      VP, P(ZBins), VP, ctypes.c_size_t, VP]
    lib.lya_tune_ps_workspace_size.restype = ctypes.c_size_t
    lib.lya_tune_ps_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    lib.lya_tune_ps.restype = ctypes.c_int
    lib.lya_tune_ps.argtypes = [P(TunePsSpec), P(TunePsResult), VP, ctypes.c_size_t, VP]
    lib.lya_tune_ps_last_error.restype = ctypes.c_char_p
    lib.lya_emulator_labels_ps.restype = ctypes.c_int
    lib.lya_emulator_labels_ps.argtypes = [P(TunePsSpec), ctypes.c_int32, VP, ctypes.c_int64, VP, VP, ctypes.c_size_t,
                                           VP]
    lib.lya_make_box_pair.restype = ctypes.c_int
    lib.lya_make_box_pair.argtypes = [P(Box), P(Pk), P(Pk), ctypes.c_uint64, VP, VP, ctypes.c_size_t, VP]
    lib.lya_lognormal_workspace_size.restype = ctypes.c_size_t
    lib.lya_lognormal_workspace_size.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32]
    lib.lya_lognormal_pk.restype = ctypes.c_int
    lib.lya_lognormal_pk.argtypes = [P(Pk), ctypes.c_double, ctypes.c_double, P(Cosmo), ctypes.c_double,
                                     ctypes.c_int32, ctypes.c_int32, VP, VP, VP, VP, ctypes.c_size_t, VP]
    lib.lya_box_moments.restype = ctypes.c_int
    lib.lya_box_moments.argtypes = [P(Box), VP, VP, VP, ctypes.c_size_t, VP]
    lib.lya_quasar_skewers.restype = ctypes.c_int
    lib.lya_quasar_skewers.argtypes = [P(Box), P(QsoLosSpec), P(Cosmo), VP, VP, VP, VP, VP, VP, VP, VP,
                                       ctypes.c_size_t, VP]
    lib.lya_draw_quasars.restype = ctypes.c_int
    lib.lya_draw_quasars.argtypes = [P(Box), P(QsoSpec), P(Cosmo), VP, ctypes.c_int64, VP, VP, ctypes.c_size_t, VP]


def _lib2():
    lib = load()
    if not getattr(lib, "_bound_more", False):
        _bind_more(lib)
        lib._bound_more = True
    return lib


def _echeck(rc):
    if rc != LYA_OK:
        raise LyaError(rc, _lib2().lya_emulator_last_error().decode())


def p1d_workspace_size(n_sk, n_kbins):
    return int(_lib2().lya_p1d_workspace_size(int(n_sk), int(n_kbins)))


def p1d(sk, cosmo, flux, fbar_zbins, spec, psum, pcount, work, stream=None):
    """lya_p1d (see include/lyamock.h)."""
    _check(_lib2().lya_p1d(ctypes.byref(sk), ctypes.byref(cosmo), _ptr(flux), ctypes.byref(fbar_zbins),
                           ctypes.byref(spec), _ptr(psum), _ptr(pcount), _ptr(work),
                           work.numel() * work.element_size(), _stream(stream)))


def apply_fgpa_ds(sk, cosmo, dens_l, eta, ps, table, seed, fgpa, flux, zbins, work, stream=None):
    """lya_apply_fgpa_ds (see include/lyamock.h); table: PsTable or None."""
    _check(_lib2().lya_apply_fgpa_ds(ctypes.byref(sk), ctypes.byref(cosmo), _ptr(dens_l), _ptr(eta),
                                     ctypes.byref(ps), ctypes.byref(table) if table is not None else None, int(seed),
                                     ctypes.byref(fgpa), _ptr(flux), ctypes.byref(zbins) if zbins is not None else None,
                                     _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def tune_ps_workspace_size(n_sk, n_pixels, n_kbins):
    return int(_lib2().lya_tune_ps_workspace_size(int(n_sk), int(n_pixels), int(n_kbins)))


def tune_ps(spec, work, stream=None):
    """lya_tune_ps: returns a TunePsResult."""
    res = TunePsResult()
    rc = _lib2().lya_tune_ps(ctypes.byref(spec), ctypes.byref(res), _ptr(work), work.numel() * work.element_size(),
                             _stream(stream))
    if rc != LYA_OK:
        raise LyaError(rc, _lib2().lya_tune_ps_last_error().decode())
    return res


def emulator_labels_ps(spec, zi, draws_host, y, work, stream=None):
    """lya_emulator_labels_ps: draws_host is a C-contiguous float64 numpy array [n, 4] of (a, b, amp, kcut)."""
    import numpy as np
    d = np.ascontiguousarray(draws_host, dtype=np.float64)
    rc = _lib2().lya_emulator_labels_ps(ctypes.byref(spec), int(zi), d.ctypes.data, int(d.shape[0]), _ptr(y),
                                        _ptr(work), work.numel() * work.element_size(), _stream(stream))
    if rc != LYA_OK:
        raise LyaError(rc, _lib2().lya_tune_ps_last_error().decode())


def tune_workspace_size(n_sk, n_kbins):
    return int(_lib2().lya_tune_workspace_size(int(n_sk), int(n_kbins)))


def tune_params(spec, mode, work, stream=None):
    """lya_tune_params: returns a TuneResult."""
    res = TuneResult()
    _check(_lib2().lya_tune_params(ctypes.byref(spec), ctypes.byref(res), int(mode), _ptr(work),
                                   work.numel() * work.element_size(), _stream(stream)))
    return res


def emulator_labels(spec, draws_host, y, work, stream=None):
    """lya_emulator_labels: draws_host is a C-contiguous float64 numpy array [n, 4]."""
    import numpy as np
    d = np.ascontiguousarray(draws_host, dtype=np.float64)
    _check(_lib2().lya_emulator_labels(ctypes.byref(spec), d.ctypes.data, int(d.shape[0]), _ptr(y), _ptr(work),
                                       work.numel() * work.element_size(), _stream(stream)))


def emulator_bytes(n_out):
    return int(_lib2().lya_emulator_bytes(int(n_out)))


def emulator_param_offset():
    return int(_lib2().lya_emulator_param_offset())


def emulator_param_count(n_out):
    return int(_lib2().lya_emulator_param_count(int(n_out)))


def emulator_init(emu, n_out, log_from, seed, in_lo, in_hi, log_inputs=0, stream=None):
    lo = (ctypes.c_double * 4)(*[float(v) for v in in_lo])
    hi = (ctypes.c_double * 4)(*[float(v) for v in in_hi])
    _echeck(_lib2().lya_emulator_init(_ptr(emu), int(n_out), int(log_from), int(seed), lo, hi, int(log_inputs),
                                      _stream(stream)))


def emulator_train_workspace_size(batch, n_out):
    return int(_lib2().lya_emulator_train_workspace_size(int(batch), int(n_out)))


def emulator_set_scaling(emu, y, n, stream=None):
    _echeck(_lib2().lya_emulator_set_scaling(_ptr(emu), _ptr(y), int(n), _stream(stream)))


def emulator_loss_grad(emu, x0, t, batch, use_bf16, grad, loss, work, stream=None):
    _echeck(_lib2().lya_emulator_loss_grad(_ptr(emu), _ptr(x0), _ptr(t), int(batch), int(bool(use_bf16)), _ptr(grad),
                                           _ptr(loss), _ptr(work), work.numel() * work.element_size(),
                                           _stream(stream)))


def emulator_train(emu, x, y, n, steps, batch, lr, use_bf16, loss_hist, work, stream=None):
    _echeck(_lib2().lya_emulator_train(_ptr(emu), _ptr(x), _ptr(y), int(n), int(steps), int(batch), float(lr),
                                       int(bool(use_bf16)), _ptr(loss_hist), _ptr(work),
                                       work.numel() * work.element_size(), _stream(stream)))


def emulator_predict(emu, x, n, y, stream=None):
    _echeck(_lib2().lya_emulator_predict(_ptr(emu), _ptr(x), int(n), _ptr(y), _stream(stream)))


def chi_of_z(z, omega_m=0.3147):
    """lya_chi_of_z on the host: comoving distance (Mpc/h) of redshifts z."""
    import numpy as np
    zz = np.ascontiguousarray(np.atleast_1d(z), dtype=np.float64)
    out = np.empty_like(zz)
    _check(_lib2().lya_chi_of_z(ctypes.byref(Cosmo(float(omega_m))), int(zz.size), zz.ctypes.data,
                                out.ctypes.data))
    return out


def tune_spec(sk, dens, eta, cosmo, z_t, c_t, fbar_t, p1d_t, k_edges, dpix, a0=0.3, b0=1.5, sigma_rel=0.002,
              xatol=1e-6, fatol=1e-8, max_evals=400, emulator=None, emu_checks=4):
    """Build a TuneSpec.  sk is a Skewers structure, dens/eta/k_edges/emulator
    device tensors, p1d_t a host array [n_zt][n_kbins].  Returns (spec, keep):
    keep holds the host arrays the spec points to and must outlive its use."""
    import numpy as np
    z_t = np.atleast_1d(np.asarray(z_t, dtype=np.float64))
    n = len(z_t)
    if n < 1 or n > TUNE_MAX_Z:
        raise ValueError("1..%d tuning redshifts" % TUNE_MAX_Z)
    nk = int(k_edges.numel()) - 1
    pt = np.ascontiguousarray(np.asarray(p1d_t, dtype=np.float64).reshape(n, nk))
    sp = TuneSpec()
    skp = ctypes.pointer(sk)
    sp.sk = skp
    sp.dens = dens.data_ptr()
    sp.eta = eta.data_ptr()
    sp.cosmo = cosmo
    sp.n_zt = n
    for i in range(n):
        sp.z_t[i] = float(z_t[i])
        sp.c_t[i] = float(np.atleast_1d(c_t)[i])
        sp.fbar_t[i] = float(np.atleast_1d(fbar_t)[i])
    sp.p1d_t = pt.ctypes.data
    sp.p1d = P1dSpec(nk, k_edges.data_ptr(), 0.0, float(dpix))
    sp.a0, sp.b0 = float(a0), float(b0)
    sp.sigma_rel = float(sigma_rel)
    sp.xatol, sp.fatol = float(xatol), float(fatol)
    sp.max_evals = int(max_evals)
    sp.emulator = None if emulator is None else emulator.data_ptr()
    sp.emu_checks = int(emu_checks)
    return sp, (skp, pt, sk)


def _acheck(rc):
    if rc != LYA_OK:
        raise LyaError(rc, _lib2().lya_autotune_last_error().decode())


def get_tuning(n):
    t = Tuning()
    _acheck(_lib2().lya_get_tuning(int(n), ctypes.byref(t)))
    return t


def set_tuning(n, t):
    _acheck(_lib2().lya_set_tuning(int(n), ctypes.byref(t)))


def autotune_fft(box, field, work, reps=3, stream=None):
    """lya_autotune_fft: returns (Tuning, ms[2][FFT_VARIANTS] as nested lists)."""
    ms = (ctypes.c_double * (2 * FFT_VARIANTS))()
    t = Tuning()
    _acheck(_lib2().lya_autotune_fft(ctypes.byref(box), _ptr(field), _ptr(work), work.numel() * work.element_size(),
                                     int(reps), ms, ctypes.byref(t), _stream(stream)))
    return t, [[ms[p * FFT_VARIANTS + v] for v in range(FFT_VARIANTS)] for p in range(2)]


def autotune_skewers(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zbins, work, reps=2, stream=None):
    """lya_autotune_skewers: returns (Tuning, ms[len(SK_CHUNKS)][len(SK_BLOCKS_PER_CU)][len(SK_UNROLL)])."""
    nc, nb, nu = len(SK_CHUNKS), len(SK_BLOCKS_PER_CU), len(SK_UNROLL)
    ms = (ctypes.c_double * (nc * nb * nu))()
    t = Tuning()
    _acheck(_lib2().lya_autotune_skewers(ctypes.byref(box), _ptr(field), ctypes.byref(sk), ctypes.byref(ps),
                                         int(seed), ctypes.byref(cosmo), ctypes.byref(fgpa) if fgpa else None,
                                         _ptr(dens), _ptr(eta), _ptr(flux),
                                         ctypes.byref(zbins) if zbins is not None else None, _ptr(work),
                                         work.numel() * work.element_size(), int(reps), ms, ctypes.byref(t),
                                         _stream(stream)))
    return t, [[[ms[(i * nb + j) * nu + k] for k in range(nu)] for j in range(nb)] for i in range(nc)]


class Graph:
    """A captured sequence of library calls (lya_graph_*): use as
    `with L.Graph(stream) as g: <library calls on stream>`, then g.launch()."""

    def __init__(self, stream=None):
        self.stream = stream
        self.handle = ctypes.c_void_p()

    def __enter__(self):
        _acheck(_lib2().lya_graph_begin(_stream(self.stream)))
        return self

    def __exit__(self, et, ev, tb):
        rc = _lib2().lya_graph_end(_stream(self.stream), ctypes.byref(self.handle))
        if et is None:
            _acheck(rc)
        return False

    def launch(self, stream=None):
        _acheck(_lib2().lya_graph_launch(self.handle, _stream(stream if stream is not None else self.stream)))

    def close(self):
        if self.handle:
            _acheck(_lib2().lya_graph_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_box_pair(box, pk_a, pk_b, seed, field, work, stream=None):
    """lya_make_box_pair: {delta_a, delta_b} of one set of modes, two spectra."""
    _check(_lib2().lya_make_box_pair(ctypes.byref(box), ctypes.byref(pk_a), ctypes.byref(pk_b), int(seed),
                                     _ptr(field), _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def lognormal_workspace_size(smooth, rmax, n_r):
    return int(_lib2().lya_lognormal_workspace_size(float(smooth), float(rmax), int(n_r)))


def lognormal_pk(pk, z_box, z_ref, cosmo, rmax, n_r, k, pq, xi, work, stream=None):
    """lya_lognormal_pk: P_q at k (device float64) into pq; xi_m at the r nodes into xi (or None)."""
    _check(_lib2().lya_lognormal_pk(ctypes.byref(pk), float(z_box), float(z_ref), ctypes.byref(cosmo), float(rmax),
                                    int(n_r), int(k.numel()), _ptr(k), _ptr(pq), _ptr(xi), _ptr(work),
                                    work.numel() * work.element_size(), _stream(stream)))


def box_moments(box, field, out, work, stream=None):
    """lya_box_moments: out (device float64 [4]) = mean/var of the real and imaginary parts."""
    _check(_lib2().lya_box_moments(ctypes.byref(box), _ptr(field), _ptr(out), _ptr(work),
                                   work.numel() * work.element_size(), _stream(stream)))


def draw_quasars(box, spec, cosmo, pos_fx, count, work, stream=None):
    """lya_draw_quasars: pos_fx (device int64 [cap, 3] or None), count (device int64 [1])."""
    cap = 0 if pos_fx is None else int(pos_fx.shape[0])
    _check(_lib2().lya_draw_quasars(ctypes.byref(box), ctypes.byref(spec), ctypes.byref(cosmo), _ptr(pos_fx), cap,
                                    _ptr(count), _ptr(work), work.numel() * work.element_size(), _stream(stream)))


def quasar_skewers(box, pos_fx, vel_xy, vel_z, observer, lam_lo, lam_hi, z_min, dchi, cosmo, work, stream=None):
    """lya_quasar_skewers: returns dict of device tensors z_q, origin_fx,
    step_fx, npix, offset, chi0 and the total pixel count (synchronises)."""
    import torch
    nq = 0 if pos_fx is None else int(pos_fx.shape[0])
    dev = pos_fx.device if pos_fx is not None else torch.device("cuda")
    out = dict(z_q=torch.empty(nq, dtype=torch.float64, device=dev),
               origin_fx=torch.empty((nq, 3), dtype=torch.int64, device=dev),
               step_fx=torch.empty((nq, 3), dtype=torch.int64, device=dev),
               npix=torch.empty(nq, dtype=torch.int32, device=dev),
               offset=torch.empty(nq, dtype=torch.int64, device=dev),
               chi0=torch.empty(nq, dtype=torch.float64, device=dev))
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    sp = QsoLosSpec(nq, None if pos_fx is None else pos_fx.data_ptr(),
                    None if vel_xy is None else vel_xy.data_ptr(), None if vel_z is None else vel_z.data_ptr(),
                    (ctypes.c_double * 3)(*[float(v) for v in observer]), float(lam_lo), float(lam_hi),
                    float(z_min), float(dchi))
    _check(_lib2().lya_quasar_skewers(ctypes.byref(box), ctypes.byref(sp), ctypes.byref(cosmo),
                                      *[_ptr(out[k]) for k in ("z_q", "origin_fx", "step_fx", "npix", "offset",
                                                               "chi0")],
                                      _ptr(total), _ptr(work), work.numel() * work.element_size(), _stream(stream)))
    out["total"] = int(total.item())
    return out
