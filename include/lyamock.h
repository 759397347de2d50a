/* lyamock: the data-parallel hot path of the Saclay Lyman-alpha mock method
 * (Etourneau, Le Goff, Rich et al., "Mock data sets for the eBOSS and DESI
 * Lyman-alpha forest surveys", arXiv 2310.18996) on AMD MI355X (gfx950).
 *
 * C-ABI.  Conventions for every entry point:
 *   - Struct arguments (lya_box, lya_pk, ...) are HOST pointers read during
 *     the call only.  Every array pointer (inside structs or as an argument)
 *     is a DEVICE pointer on the current HIP device, allocated and owned by
 *     the caller; the library never allocates, frees or retains them.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *     default stream).  No call synchronises the device.
 *   - Arguments are validated on the host before anything is enqueued.  On a
 *     non-zero return nothing was enqueued (LYA_EINVAL, LYA_EWORKSPACE,
 *     LYA_EUNSUPPORTED) or the state of the outputs is undefined (LYA_EHIP).
 *     lya_last_error() then returns a message (thread-local).
 *   - Real-space boxes are [x][y][z] with z fastest: grid point (i, j, k),
 *     at position (i, j, k) * dx, is element i * pitch + j * n + k, where
 *     pitch = lya_plane_pitch(box) = n^2 + 32 (each x plane is followed by 32
 *     unused elements, which keeps the x-direction FFT pass off a
 *     power-of-two stride).  A box holds lya_field_elems(box) = n * pitch
 *     elements.  Element type: LYA_F32 -> float2 {C_a, C_b} (8 bytes);
 *     LYA_BF16 -> two bfloat16 packed in a uint32, C_a in the low half (4 bytes).
 */
#ifndef LYAMOCK_H
#define LYAMOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LYA_OK = 0,
  LYA_EINVAL = -1,       /* bad argument (null pointer, size out of range) */
  LYA_EWORKSPACE = -2,   /* work_bytes smaller than lya_workspace_size() */
  LYA_EUNSUPPORTED = -3, /* valid but not implemented (e.g. n not a power of two) */
  LYA_EHIP = -4          /* a HIP runtime call or kernel launch failed */
} lya_status;

enum { LYA_F32 = 0, LYA_BF16 = 1 };

/* Field components (eq:deltaL, eq:eta, eq:velocity): delta, then
 * eta_pq = f k_p k_q / k^2 delta, then the velocity v_j = i f (aH)_0 k_j / k^2 delta
 * in km/s with (aH)_0 = 100 km/s per Mpc/h (the box's redshift is 0). */
enum { LYA_C_NONE = -1, LYA_C_DELTA = 0, LYA_C_XX = 1, LYA_C_YY = 2, LYA_C_ZZ = 3,
       LYA_C_XY = 4, LYA_C_XZ = 5, LYA_C_YZ = 6, LYA_C_VX = 7, LYA_C_VY = 8, LYA_C_VZ = 9 };

/* Workspace kinds for lya_workspace_size. */
enum { LYA_OP_BOX = 0, LYA_OP_SKEWERS = 1, LYA_OP_QUASARS = 2, LYA_OP_BOX_2BUF = 3 };

/* Periodic box (section "Mock generation"). */
typedef struct {
  int32_t n;        /* grid points per side: 32, 64, ..., 2048 */
  double dx;        /* voxel side in Mpc/h (> 0) */
  int32_t storage;  /* LYA_F32 or LYA_BF16 element type of the output box */
} lya_box;

/* Linear power spectrum (eq:deltaL).  Either the analytic stand-in for the
 * paper's CAMB P_m(k):
 *   P(k) = A k^ns T_BBKS(k/gamma)^2 (1 + wig_amp sin(k wig_r) exp(-(k/wig_kd)^2)),
 * A set so that sigma_8 = sigma8; or, when k_tab is not NULL, a table such as
 * CAMB's: ln P linear in ln k between the nodes (k_tab increasing, k_tab > 0,
 * p_tab > 0; device arrays of n_tab >= 2 doubles), the end intervals' power
 * laws continued outside, used as given (sigma8 and the shape parameters are
 * then ignored).  k in h/Mpc, P in (Mpc/h)^3. */
typedef struct {
  double sigma8, ns, gamma, wig_amp, wig_r, wig_kd;
  double smooth;     /* Gaussian window sigma in Mpc/h on the mode amplitude, 0 = off
                        (the paper's smoothing, Appendix B, W^2 = exp(-dx^2 k^2), is smooth = dx) */
  int32_t fixed_amp; /* 1: |W(k)| = 1 (fixed-amplitude test hook) */
  int32_t only_n2;   /* >= 0: keep only the modes with |n|^2 == only_n2 (test hook); -1: all */
  const double* k_tab;  /* NULL: analytic form */
  const double* p_tab;
  int32_t n_tab;
} lya_pk;

/* Quasar lines of sight.  Pixel j (0 <= j < npix[q]) of skewer q sits at the
 * fixed-point position origin_fx[q] + j * step_fx[q] (per axis, cell units
 * times 2^32, periodic modulo n cells) and at comoving distance
 * chi0[q] - j * dchi from the observer (each product and difference rounded
 * in FP64).  Its values live at index offset[q] + j of the flat pixel arrays. */
typedef struct {
  int64_t n_sk;              /* number of skewers (>= 0) */
  const int64_t* origin_fx;  /* device [n_sk][3] */
  const int64_t* step_fx;    /* device [n_sk][3] */
  const int32_t* npix;       /* device [n_sk], 0 <= npix <= 2048 (drawing delta_S on a longer
                                skewer is an input error: NaN in its outputs, none in the bins) */
  const int64_t* offset;     /* device [n_sk] */
  const double* chi0;        /* device [n_sk], Mpc/h */
  double dchi;               /* pixel length in Mpc/h (the paper: 0.2) */
  int64_t id_base;           /* quasar id of row 0: seeds its small-scale field;
                                0 <= id_base, n_sk + id_base <= 2^31 */
} lya_skewers;

/* Small-scale 1D spectrum of delta_S (section "Gaussian fields along lines of
 * sight"): P_s(k) = amp exp(-(k/kcut)^2), k in h/Mpc; amp = 0 disables delta_S. */
typedef struct {
  double amp, kcut;
  double dpix;        /* pixel length used for the 1D modes, Mpc/h */
  int32_t fixed_amp;  /* 1: |W| = 1 test hook */
} lya_ps1d;

/* FGPA parameters (eq:FGPA): a, b, c = sum_i coef[p][i] (1+z)^i, p = a, b, c. */
typedef struct {
  double coef[3][3];
} lya_fgpa;

/* Flat LCDM background for pixel redshifts (Table cosmoparams). */
typedef struct {
  double omega_m;
} lya_cosmo;

/* Mean-flux accumulation per redshift bin: a pixel is in bin b when
 * chi_edges[b] <= chi_j < chi_edges[b+1] (edges increasing).  fsum[b] = sum of F,
 * count[b] = number of pixels (outputs, device). */
typedef struct {
  int32_t n_bins;           /* 0..64 */
  const double* chi_edges;  /* device [n_bins + 1] */
  double* fsum;             /* device [n_bins] */
  int64_t* count;           /* device [n_bins] */
} lya_zbins;

/* Elements of a box (n * plane pitch) and the plane pitch; 0 for an invalid box. */
size_t lya_field_elems(const lya_box* box);
size_t lya_plane_pitch(const lya_box* box);

/* Bytes of device workspace a call needs.  op = LYA_OP_BOX for lya_make_box,
 * lya_make_eta and lya_make_box_pair (for LYA_BF16 storage this includes an
 * n^3 complex64 staging box); LYA_OP_BOX_2BUF for the same calls with one more
 * complex64 box of workspace, with which they run their FFT passes in the
 * two-buffer order (faster for large boxes; see lya_make_box);
 * LYA_OP_SKEWERS for lya_draw_skewers and
 * lya_apply_fgpa, LYA_OP_QUASARS for lya_box_moments, lya_draw_quasars and
 * lya_quasar_skewers.
 * Returns 0 for invalid arguments. */
size_t lya_workspace_size(int op, const lya_box* box);

/* Gaussian box and line-of-sight velocity gradient (section "Mock generation",
 * eq:deltaL, eq:eta).  Draws the k-space noise W(k) from Philox4x32-10 (key =
 * seed, stream 0), forms delta_hat = sqrt(P(k)/L^3) W and
 * eta_par_hat = f mu_z^2 delta_hat (line of sight = z axis), and writes the
 * real-space box {delta, eta_par} = inverse DFT (unnormalised, exp(+i k.x)).
 * field: device, n^3 cells of the box's storage type.  with_eta = 0 writes
 * eta_par = 0.  work: device, >= lya_workspace_size(LYA_OP_BOX, box) bytes.
 * The inverse DFT runs as three 1D passes.  With work_bytes >=
 * lya_workspace_size(LYA_OP_BOX_2BUF, box) the z pass writes its pencils
 * with x and y exchanged into the workspace's second box, the x pass reads
 * them there within planes and writes field transposed back, and the y pass
 * finishes in place: no pass reads across the x planes, and the box is the
 * same up to rounding (the x and y
 * transforms run in the other order).  With less workspace the passes run
 * z, y, x in place in field.  Either way the result for a given workspace
 * size is deterministic. */
int lya_make_box(const lya_box* box, const lya_pk* pk, uint64_t seed, double f, int with_eta,
                 void* field, void* work, size_t work_bytes, void* stream);

/* Any pair of components of the same modes (eq:eta: eta_pq = f k_p k_q/k^2
 * delta_hat; cross terms vanish on the Nyquist plane of p or q; eq:velocity:
 * v_j = i f (aH)_0 k_j/k^2 delta_hat, zero on the Nyquist plane of j): writes
 * {comp_a, comp_b} (comp_b may be LYA_C_NONE).  Same layout and workspace as
 * lya_make_box. */
int lya_make_eta(const lya_box* box, const lya_pk* pk, uint64_t seed, double f, int comp_a, int comp_b,
                 void* field, void* work, size_t work_bytes, void* stream);

/* Two Gaussian fields of the same modes with different spectra (section
 * "Quasar generation": the quasar-density field takes the original
 * delta_hat(k) with the amplitudes sqrt(P_q/V)): writes {delta_a, delta_b},
 * delta_a from pk_a in the real part and delta_b from pk_b in the imaginary
 * part, each exactly what lya_make_box with that spectrum and seed writes as
 * delta.  The test hooks fixed_amp and only_n2 of pk_a apply to both.  Same
 * layout and workspace as lya_make_box. */
int lya_make_box_pair(const lya_box* box, const lya_pk* pk_a, const lya_pk* pk_b, uint64_t seed, void* field,
                      void* work, size_t work_bytes, void* stream);

/* Ray-march every skewer through the box {delta, eta_par} (section "Gaussian
 * fields along lines of sight"): periodic trilinear interpolation at each
 * pixel, plus the small-scale field delta_S drawn from Philox (key = seed,
 * stream 1) when ps->amp > 0.  Writes dens = delta_L + delta_S and eta (either
 * may be NULL).  If fgpa is not NULL also applies eq:FGPA and writes flux (may
 * be NULL) and, if zb is not NULL, the per-bin mean-flux sums.  field: the box
 * written by lya_make_box with the same lya_box.  work: >= lya_workspace_size(
 * LYA_OP_SKEWERS, box) bytes. */
int lya_draw_skewers(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                     uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                     float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream);

/* Allocation-free variant of lya_draw_skewers, for callers that cannot
 * allocate device memory (code under HIP-graph capture, tight serving loops,
 * hosts that forbid hipMalloc): the same arguments, outputs and errors, without
 * work and work_bytes.  Its workspace (the redshift table, the twiddles, the
 * work-queue counter and the fixed-point sums of up to 64 bins, about 100 KB)
 * is a static 128 KiB device array that each GPU the library runs on holds
 * until the process ends; the first call on a device looks up its address.
 * Every call on one GPU uses that GPU's array and leaves its contents behind,
 * so calls that overlap on one GPU (other streams, other host threads) race;
 * each call clears the counters it needs with kernels (no memset nodes).
 * LYA_EWORKSPACE if the workspace would not fit the array (no valid input
 * needs more: n_bins <= 64). */
int lya_draw_skewers_static(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                            uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                            float* flux, const lya_zbins* zb, void* stream);

/* The paper's interpolation (section "Gaussian fields along lines of sight"):
 * as lya_draw_skewers, but delta_L and eta_par at a pixel are the Gaussian-
 * kernel average of the 7^3 voxels around it, standard deviation one voxel
 * side: with u the pixel position in cell units and c = floor(u + 1/2) its
 * nearest grid point (per axis), voxel c + o, o in [-3, 3]^3 (periodic),
 * weighs exp(-|c + o - u|^2 / 2), and the average divides by the sum of the
 * 343 weights.  Same arguments, outputs and errors as lya_draw_skewers. */
int lya_draw_skewers_gauss(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                           uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                           float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream);

/* Wide-angle line-of-sight velocity gradient (section "Mock generation": the
 * six boxes of eq:eta and eta_par = u_p u_q eta^pq).  As lya_draw_skewers, but
 * eta_par at each pixel is
 *   u_x^2 eta_xx + u_y^2 eta_yy + u_z^2 eta_zz
 *     + 2 (u_x u_y eta_xy + u_x u_z eta_xz + u_y u_z eta_yz),
 * u = step/|step| the skewer's own direction (a straight radial line keeps
 * one), formed at the eight corner voxels and interpolated trilinearly like
 * delta.  fields[4] (host array of device pointers), four boxes of the same
 * lya_box made from the same pk, seed and f:
 *   fields[0]  lya_make_box(with_eta = 1)           {delta, eta_zz}
 *   fields[1]  lya_make_eta(LYA_C_XX, LYA_C_YY)     {eta_xx, eta_yy}
 *   fields[2]  lya_make_eta(LYA_C_XY, LYA_C_XZ)     {eta_xy, eta_xz}
 *   fields[3]  lya_make_eta(LYA_C_YZ, LYA_C_NONE)   {eta_yz, 0}
 * Everything else (delta_S, FGPA, bins, outputs, workspace, errors) is as for
 * lya_draw_skewers; a NULL entry in fields is LYA_EINVAL. */
int lya_draw_skewers_wide(const lya_box* box, const void* const* fields, const lya_skewers* sk, const lya_ps1d* ps,
                          uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                          float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream);

/* FGPA on stored pre-FGPA pixels (eq:FGPA; the paper's post-production step):
 * flux = exp(-a(z) exp(b(z) (dens + c(z) eta))), z the redshift of chi_j.
 * Geometry fields of sk other than npix, offset, chi0 and dchi are unused.
 * flux may be NULL when only the per-bin sums are wanted. */
int lya_apply_fgpa(const lya_skewers* sk, const lya_cosmo* cosmo, const float* dens, const float* eta,
                   const lya_fgpa* fgpa, float* flux, const lya_zbins* zb, void* work, size_t work_bytes,
                   void* stream);

/* Post-production with a new small-scale spectrum (section "Adjusting mock
 * parameters": the spectra are drawn again with the current P_s): draws
 * delta_S for every skewer exactly as lya_draw_skewers does (Philox key seed,
 * stream 1, lengths up to 2048 pixels) with
 *   P_s(k) = ps->amp exp(-(k/ps->kcut)^2) r(k),
 * r(k) = tab->ratio[b] for tab->k_edges[b] <= k < tab->k_edges[b+1] (k in
 * h/Mpc; below the first edge the first ratio, from the last edge up the last
 * one; tab NULL: r = 1), adds it to dens_l (stored delta_L without delta_S)
 * and applies eq:FGPA as lya_apply_fgpa does.  tab->k_edges (n_bins + 1
 * doubles, increasing) and tab->ratio (n_bins floats) are device arrays. */
typedef struct {
  int32_t n_bins;          /* 1..64 */
  const double* k_edges;   /* device, h/Mpc */
  const float* ratio;      /* device */
} lya_ps_table;

int lya_apply_fgpa_ds(const lya_skewers* sk, const lya_cosmo* cosmo, const float* dens_l, const float* eta,
                      const lya_ps1d* ps, const lya_ps_table* tab, uint64_t seed, const lya_fgpa* fgpa, float* flux,
                      const lya_zbins* zb, void* work, size_t work_bytes, void* stream);

/* 1D flux power spectrum (the statistic the paper's tuning matches, section
 * "Adjusting mock parameters"; delta_F = F/Fbar - 1 of
 * equation::definition_delta).  Per skewer the first
 * N_P = min(2^floor(log2 npix), 2048) pixels (skewers with npix < 2 add
 * nothing); Fbar of a pixel = fsum/count of its distance bin in `fbar` (pixels
 * outside the bins take the nearest one; the sums are the output of
 * lya_draw_skewers / lya_apply_fgpa); velocity pixel
 * Dv = dpix 100 E(z_ref)/(1+z_ref) km/s for all skewers; P(k_m) = Dv |X_m|^2/N_P
 * for m = 1..N_P/2, k_m = 2 pi m/(N_P Dv) s/km, summed into bins
 * k_edges[b] <= k_m < k_edges[b+1].  Outputs (device): psum[b] (FP64 sum of P)
 * and pcount[b] (modes); mean = psum/pcount.  Deterministic: per-skewer sums
 * in a fixed order, then a fixed-order sum over skewers. */
typedef struct {
  int32_t n_kbins;         /* 1..64 */
  const double* k_edges;   /* device [n_kbins + 1], s/km, increasing */
  double z_ref;            /* redshift of the velocity units */
  double dpix;             /* pixel length, Mpc/h */
} lya_p1d_spec;

size_t lya_p1d_workspace_size(int64_t n_sk, int32_t n_kbins);
int lya_p1d(const lya_skewers* sk, const lya_cosmo* cosmo, const float* flux, const lya_zbins* fbar,
            const lya_p1d_spec* spec, double* psum, int64_t* pcount, void* work, size_t work_bytes, void* stream);

/* FGPA parameter tuning (section "Adjusting mock parameters").  At each tuning
 * redshift z_t, with c fixed to c_t, (a, b) are chosen to minimise
 *   chi^2 = ((Fbar - fbar_t)/(s fbar_t))^2 + sum_b ((P_b - P_t,b)/(s P_t,b))^2
 * (s = sigma_rel, bins with a non-finite target skipped), where Fbar and P_b
 * (mean P1D of bin b, velocity units at z_t, delta_F = F/Fbar - 1) are measured
 * on the stored pre-FGPA pixels under constant (a, b, c): the paper's reuse of
 * saved forests in post-production.  Search: Nelder-Mead in (ln a, ln b) from
 * (a0, b0), initial steps 0.3, stopping when all vertices lie within xatol
 * (coordinates) and fatol (chi^2) of the best or after max_evals evaluations.
 * Mode LYA_TUNE_PLAIN evaluates every Nelder-Mead point on the GPU.
 * LYA_TUNE_EMULATOR searches on the device against a model of the
 * statistics, the emulator's prediction (see lya_emulator_*) plus an offset
 * plus a linear correction in (ln a, ln b), by Levenberg-Marquardt on the
 * residuals above (Jacobian by forward differences of the model, h = 1e-3);
 * each search is followed by one GPU evaluation at its optimum, after which
 * the offset is set so that the model equals the GPU there and the linear
 * correction takes a Broyden update so that it also reproduces the previous
 * GPU evaluation; the next search starts there.  Points outside the
 * emulator's (a, b) input range are rejected.  It stops when a search moves
 * the point by at most max(10 xatol, 5e-4) from the previous GPU evaluation;
 * the result then holds the last GPU evaluation.  When no search has settled
 * after emu_checks GPU evaluations (an emulator trained poorly or used outside
 * its range; always when emu_checks is 1), the plain loop takes over from the
 * last point evaluated on the GPU and fallback[z_t] is set.  a(z), b(z), c(z)
 * are then least-squares quadratics in (1+z) (n_zt >= 3; the line through
 * two points, a constant for one).  Synchronous (reads back the
 * statistics of every evaluation); all GPU work runs on `stream`. */
#define LYA_TUNE_MAX_Z 16
enum { LYA_TUNE_PLAIN = 0, LYA_TUNE_EMULATOR = 1 };

typedef struct {
  const lya_skewers* sk;     /* table of the stored pixels (npix, offset, chi0, dchi used) */
  const float* dens;         /* device: delta_L + delta_S per pixel */
  const float* eta;          /* device: eta_par per pixel */
  lya_cosmo cosmo;
  int32_t n_zt;              /* 1..16 */
  double z_t[LYA_TUNE_MAX_Z], c_t[LYA_TUNE_MAX_Z], fbar_t[LYA_TUNE_MAX_Z];
  const double* p1d_t;       /* host [n_zt][p1d.n_kbins] target mean P1D (NaN: bin unused) */
  lya_p1d_spec p1d;          /* k bins (device edges) and dpix; z_ref is z_t */
  double a0, b0;             /* starting point */
  double sigma_rel;          /* relative error of each statistic (e.g. 0.002) */
  double xatol, fatol;
  int32_t max_evals;         /* per z_t */
  const void* emulator;      /* emulator state (device) for LYA_TUNE_EMULATOR, else NULL */
  int32_t emu_checks;        /* LYA_TUNE_EMULATOR: most GPU evaluations per z_t (<= 0: 1) */
} lya_tune_spec;

typedef struct {
  double a[LYA_TUNE_MAX_Z], b[LYA_TUNE_MAX_Z], chi2[LYA_TUNE_MAX_Z], fbar[LYA_TUNE_MAX_Z];
  double p1d[LYA_TUNE_MAX_Z * 64];   /* reached mean P1D, [z_t][bin] with row length 64 */
  int32_t evals[LYA_TUNE_MAX_Z];     /* search evaluations per z_t (GPU or emulator) */
  int32_t gpu_evals[LYA_TUNE_MAX_Z]; /* GPU evaluations per z_t, the final one included */
  double coef[3][3];                 /* a, b, c = sum_i coef[p][i] (1+z)^i */
  double seconds;                    /* wall time of the call */
  int32_t fallback[LYA_TUNE_MAX_Z];  /* LYA_TUNE_EMULATOR: 1 where the plain loop took over */
} lya_tune_result;

size_t lya_tune_workspace_size(int64_t n_sk, int32_t n_kbins);
int lya_tune_params(const lya_tune_spec* spec, lya_tune_result* res, int mode, void* work, size_t work_bytes,
                    void* stream);

/* Small-scale power iteration of the tuning (section "Adjusting mock
 * parameters").  dens_l and eta are stored pre-FGPA pixels WITHOUT delta_S.
 * Their moments sigma_L^2, sigma_eta^2 and cov(delta_L, eta_par) are measured
 * once (FP64).  At each z_t:
 *   1. a and s = b sigma_g solve Fbar(a, s) = fbar_t and sigma_F(a, s) =
 *      sigma_F,t for F = exp(-a exp(s x)), x a unit normal (host FP64);
 *      sigma_F,t = sigf_t[z] if positive, else fbar_t (sum_b P_t,b dk_b /
 *      pi)^(1/2) over the bins with a finite target;
 *   2. iteration n (n_iter of them): P_s^n(k) = ps_amp exp(-(k/ps_kcut)^2)
 *      r_n(bin of k), the P1D bins converted to h/Mpc at z_t (k = k_v 100
 *      E(z_t)/(1+z_t)), r_0 = 1; sigma_s^2 = (1/pi) int_0^{pi/dpix} P_s^n dk;
 *      b = s / (sigma_L^2 + sigma_s^2 + c_t^2 sigma_eta^2 + 2 c_t cov)^(1/2);
 *      delta_S redrawn with P_s^n (lya_apply_fgpa_ds, key seed), F under
 *      constant (a, b, c_t), Fbar = mean F and the P1D of F/Fbar - 1 at z_t
 *      (lya_p1d); then r_{n+1} = r_n P_t / P1D in every bin where both are
 *      finite and P1D > 0.
 * The result holds a, b and the ratios of the last iteration, its P1D, and
 * per iteration Fbar and the relative RMS P1D error over the bins with a
 * target.
 * The outer loop (n_outer >= 2; the paper adjusts a and b so that the bias
 * its correlation-function prediction implies meets the target while Fbar
 * stays, then iterates P_s again, five times): the prediction's flux bias is
 * b_F = E[dF/dg]/Fbar = -(a s/sigma_g) E[e^{s x} F]/Fbar (the first term of
 * the bivariate-Gaussian expansion of the flux correlation), beta = f c_t,
 * and the effective bias |b_F| (1 + 2 beta/3 + beta^2/5)^(1/2); each outer
 * step after the first takes sigma_g from the current ratios, solves (a, s)
 * for Fbar = fbar_t and the effective bias = beff_t[z], and runs the n_iter
 * iterations again from the current ratios.  With beff_at_z set, beff_t[z]
 * is a bias with respect to the matter field at z_t, as the paper's targets
 * (fits to measured correlations) are: the pixels come from a z = 0 box, so
 * the target becomes beff_t[z] G(z_t), G the linear growth of flat LCDM with
 * G(0) = 1.  A target the current sigma_g
 * cannot reach (at fixed Fbar the bias tends to phi(x_0)/(sigma_g Fbar) as s
 * grows) ends the outer loop early; n_outer_done[z] counts the steps run and
 * beff[z][o] is the effective bias with respect to the box after step o
 * (sigma_g of its last iteration).  fbar and rms then describe the last
 * step's iterations.
 *
 * Emulator mode (mode = LYA_TUNE_PS_EMULATOR; not in the paper): P_s keeps
 * the form ps_amp exp(-(k/ps_kcut)^2) with (amp, kcut) free, and each z_t
 * solves at once what the iterations above approach step by step: P1D(amp,
 * kcut) = P_t in least squares over the bins with a target, with (a, s) from
 * (fbar_t, sigma_F,t) (n_outer <= 1) or from (fbar_t, beff_t) at the sigma_g
 * of (amp, kcut) (n_outer >= 2), and b = s / sigma_g.  The search runs on
 * emu[z] (inputs (a, b, amp, kcut) at (c_t, z_t), outputs (Fbar, P_1..P_nk),
 * trained on lya_emulator_labels_ps) plus a correction: after each search one
 * GPU evaluation at its optimum sets the model's offset to the measured
 * statistics there and a Broyden update corrects its slope, as in
 * lya_tune_params.  It stops when a check moves (ln amp, ln kcut) by at most
 * 5e-4, or by at most 0.05 with the measured relative RMS P1D error changed
 * by at most 1e-3 of itself, or after emu_checks GPU evaluations; a z_t that
 * has not settled by then runs the plain iteration instead (fallback[z] = 1).  Results: a, b, s
 * and ps_fit[2 z .. 2 z + 1] = (amp, kcut) of the last check, p1d its P1D,
 * fbar[z][0] and rms[z][0] its mean flux and relative RMS P1D error, ratio
 * the fitted P_s over P_s^0 at each bin's centre (geometric mean of its
 * edges in h/Mpc), beff[z][0] the effective bias there, n_outer_done[z] = 1.
 * With emu_refine = n > 0, n iterations of the per-bin update (step 2 above)
 * follow the fit, with P_s^0 the fitted form and (a, s) those of the fit (b
 * from sigma_g at each iteration); fbar, rms and p1d then describe them,
 * ratio holds the per-bin factors on top of the fitted form, and beff[z][0]
 * the effective bias at the last iteration's sigma_g.
 * Per-bin update (both modes; update = LYA_PS_UPDATE_SECANT is not in the
 * paper): the paper's r_{n+1} = r_n P_t/P1D assumes a bin's P1D answers one
 * to one to its r, while with b sigma_g held it answers less.  The secant
 * update estimates each bin's response gamma = d ln P1D / d ln r from the
 * last two iterations of the run and steps r_{n+1} = r_n (P_t/P1D)^w with
 * w = 1/gamma clipped to [1, 3]; w = 1 at a run's first iteration and
 * where the secant is undefined (|d ln r| <= 1e-6 or gamma <= 0.05).  Each
 * outer step, and the refinement after an emulator fit, starts a new run.
 * gpu_evals[z] counts GPU evaluations of the statistics in both modes.
 * Synchronous; GPU work on `stream`; errors in lya_tune_ps_last_error(). */
#define LYA_TUNE_PS_MAX_ITER 16
#define LYA_TUNE_PS_MAX_OUTER 8
#define LYA_TUNE_PS_RATIOS 0
#define LYA_TUNE_PS_EMULATOR 1
#define LYA_PS_UPDATE_PAPER 0
#define LYA_PS_UPDATE_SECANT 1
typedef struct {
  const lya_skewers* sk;     /* npix, offset, chi0, dchi, id_base used */
  const float* dens_l;       /* device: delta_L per pixel (no delta_S) */
  const float* eta;          /* device: eta_par per pixel */
  int64_t n_pixels;          /* length of the pixel arrays (max offset + npix) */
  lya_cosmo cosmo;
  uint64_t seed;             /* Philox key of delta_S (stream 1) */
  int32_t n_zt;              /* 1..16 */
  double z_t[LYA_TUNE_MAX_Z], c_t[LYA_TUNE_MAX_Z], fbar_t[LYA_TUNE_MAX_Z], sigf_t[LYA_TUNE_MAX_Z];
  const double* p1d_t;       /* host [n_zt][p1d.n_kbins] target mean P1D (NaN: bin unused) */
  lya_p1d_spec p1d;          /* k bins (device edges, s/km) and dpix; z_ref is z_t */
  double ps_amp, ps_kcut;    /* P_s^0 */
  int32_t n_iter;            /* 1..16 (the paper uses 10) */
  int32_t n_outer;           /* 0 or 1: no outer loop; up to 8 (the paper uses 5) */
  double beff_t[LYA_TUNE_MAX_Z];  /* outer loop: target effective bias per z_t (> 0) */
  double f;                  /* outer loop: growth rate of the boxes' eta_par (beta = f c_t) */
  int32_t beff_at_z;         /* outer loop: 1 = beff_t is with respect to the matter field at z_t */
  int32_t mode;              /* LYA_TUNE_PS_RATIOS (the paper's iteration) or LYA_TUNE_PS_EMULATOR */
  const void* emu[LYA_TUNE_MAX_Z];  /* emulator mode: device emulator per z_t, 1 + n_kbins outputs */
  int32_t emu_checks;        /* emulator mode: GPU evaluations per z_t, 1..16 */
  int32_t emu_refine;        /* emulator mode: per-bin iterations after the fit, 0..16 */
  int32_t update;            /* per-bin update: LYA_PS_UPDATE_PAPER (0) or LYA_PS_UPDATE_SECANT */
} lya_tune_ps_spec;

typedef struct {
  double a[LYA_TUNE_MAX_Z], b[LYA_TUNE_MAX_Z], s[LYA_TUNE_MAX_Z];
  double sigma2[3];                                    /* sigma_L^2, sigma_eta^2, cov */
  double ratio[LYA_TUNE_MAX_Z * 64];                   /* r of the last iteration, [z_t][bin] */
  double p1d[LYA_TUNE_MAX_Z * 64];                     /* its mean P1D, [z_t][bin] */
  double fbar[LYA_TUNE_MAX_Z * LYA_TUNE_PS_MAX_ITER];  /* [z_t][iteration] */
  double rms[LYA_TUNE_MAX_Z * LYA_TUNE_PS_MAX_ITER];   /* [z_t][iteration] */
  double seconds;
  double beff[LYA_TUNE_MAX_Z * LYA_TUNE_PS_MAX_OUTER]; /* [z_t][outer step] */
  int32_t n_outer_done[LYA_TUNE_MAX_Z];
  double growth[LYA_TUNE_MAX_Z];                       /* G(z_t) if beff_at_z, else 1 */
  double ps_fit[2 * LYA_TUNE_MAX_Z];                   /* emulator mode: (amp, kcut) per z_t */
  int32_t gpu_evals[LYA_TUNE_MAX_Z];                   /* GPU evaluations of the statistics per z_t */
  int32_t fallback[LYA_TUNE_MAX_Z];                    /* emulator mode: 1 where the plain iteration ran */
} lya_tune_ps_result;

size_t lya_tune_ps_workspace_size(int64_t n_sk, int64_t n_pixels, int32_t n_kbins);
int lya_tune_ps(const lya_tune_ps_spec* spec, lya_tune_ps_result* res, void* work, size_t work_bytes, void* stream);
const char* lya_tune_ps_last_error(void);

/* Training labels for the emulator of lya_tune_ps's emulator mode at tuning
 * redshift z_t[zi]: for each host draw (a, b, amp, kcut) (draws[4 i + 0..3],
 * FP64), delta_S is drawn on every skewer with P_s(k) = amp exp(-(k/kcut)^2)
 * (Philox stream 1, key spec->seed, as lya_apply_fgpa_ds draws it) and added
 * to dens_l; F = exp(-a exp(b (delta_L + delta_S + c_t eta))) with c_t =
 * c_t[zi]; y[i][0] = the mean flux of all pixels and y[i][1 + b] the mean
 * P1D of k bin b (lya_p1d's estimator with one redshift bin, velocity units
 * at z_t[zi]) on the device (n_out = 1 + n_kbins).  Skewers must have at
 * most 2048 pixels (else the label is NaN).  Uses the lya_tune_ps workspace;
 * asynchronous; errors in lya_tune_ps_last_error(). */
int lya_emulator_labels_ps(const lya_tune_ps_spec* spec, int32_t zi, const double* draws, int64_t n, float* y,
                           void* work, size_t work_bytes, void* stream);

/* Tuning emulator (not in the paper: a surrogate for the evaluations of the
 * tuning loop above).  A multilayer perceptron 4 -> 256 -> 256 -> 256 -> n_out
 * with exact GELU hidden layers (x Phi(x)) and a linear output maps
 * (a, b, c, z) to (Fbar, P_1, ..., P_nk), the statistics lya_tune_params
 * matches.  Row-vector convention h = gelu(x W + b), W stored [in][out]
 * row-major, parameters in the order W1 b1 W2 b2 W3 b3 W4 b4 (FP32).
 * Inputs are scaled to [-1, 1] by the ranges given at init (optionally in
 * ln x); outputs are standardised per column with statistics taken from the
 * training labels (natural log first for columns >= log_from).  Training: mean squared error
 * over batch and unmasked columns, Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected); the matrix products run on the matrix cores in bfloat16
 * with FP32 accumulation (use_bf16 = 1) or in plain FP32.
 *
 * The emulator state is one device buffer of lya_emulator_bytes(n_out) bytes
 * owned by the caller: a header, then the parameters at byte offset
 * lya_emulator_param_offset(), then the two Adam moment arrays.  Errors of
 * these calls are reported by lya_emulator_last_error(). */
size_t lya_emulator_bytes(int32_t n_out);          /* 0 unless 1 <= n_out <= 64 */
size_t lya_emulator_param_offset(void);
size_t lya_emulator_param_count(int32_t n_out);    /* 0 unless 1 <= n_out <= 64 */

/* Writes the header (input ranges in_lo < in_hi per input; bit i of
 * log_inputs (0..15) makes input i enter as ln x, which needs in_lo > 0; each
 * input is mapped affinely onto [-1, 1] over its range; identity output
 * scaling, step 0) and He-normal weights (std sqrt(2/fan_in), Philox stream 3
 * of `seed`), zero biases and zero moments.  Asynchronous on `stream` after a
 * header upload that synchronises the stream. */
int lya_emulator_init(void* emu, int32_t n_out, int32_t log_from, uint64_t seed, const double in_lo[4],
                      const double in_hi[4], int32_t log_inputs, void* stream);

/* Output standardisation from labels y (device, [n][n_out] row-major): per
 * column FP64 mean and standard deviation (of ln y for columns >= log_from); a
 * column with any non-finite value is masked out of the loss. */
int lya_emulator_set_scaling(void* emu, const float* y, int64_t n, void* stream);

/* Workspace of one training batch (activations, gradients): bytes. */
size_t lya_emulator_train_workspace_size(int32_t batch, int32_t n_out);

/* Loss and gradient of one batch of already standardised inputs x0
 * ([batch][4]) and targets t ([batch][n_out]) (device): grad receives
 * lya_emulator_param_count(n_out) floats in parameter order, loss (may be
 * NULL) one float.  Parameters are not changed. */
int lya_emulator_loss_grad(const void* emu, const float* x0, const float* t, int32_t batch, int32_t use_bf16,
                           float* grad, float* loss, void* work, size_t work_bytes, void* stream);

/* `steps` Adam steps with learning rate lr on the rows of x ([n][4], raw
 * inputs) and y ([n][n_out], raw labels) (device); step s (counted from the
 * emulator's own step counter) takes rows (s batch + i) mod n.  loss_hist
 * (device, may be NULL) receives each step's loss.  Synchronises the stream at
 * the end. */
int lya_emulator_train(void* emu, const float* x, const float* y, int64_t n, int32_t steps, int32_t batch,
                       double lr, int32_t use_bf16, float* loss_hist, void* work, size_t work_bytes, void* stream);

/* FP32 prediction of raw outputs (exp applied for columns >= log_from) for n
 * raw inputs x ([n][4]) into y ([n][n_out]) (device).  Asynchronous. */
int lya_emulator_predict(const void* emu, const float* x, int64_t n, float* y, void* stream);

/* Training labels for the emulator: for each host draw (a, b, c, z)
 * (draws[4 i + 0..3], FP64) the statistics lya_tune_params evaluates at those
 * constant parameters with velocity units at z, written to y[i][0] (Fbar) and
 * y[i][1 + b] (mean P1D of k bin b) on the device (n_out = 1 + n_kbins).
 * Uses the tuning workspace (lya_tune_workspace_size); errors are reported by
 * lya_last_error(). */
int lya_emulator_labels(const lya_tune_spec* spec, const double* draws, int64_t n, float* y, void* work,
                        size_t work_bytes, void* stream);

const char* lya_emulator_last_error(void);

/* Lognormal quasar field (section "Quasar generation", Appendix A).
 *
 * lya_lognormal_pk: the quasar-density spectrum
 *   P_q(k) = 4 pi int_0^rmax G(r) r^2 sin(kr)/(kr) dr,  G = ln(1 + b_0^2 xi_m(r)),
 * xi_m(r) = 1/(2 pi^2) int P(k) exp(-k^2 s^2) k^2 sin(kr)/(kr) dk the
 * correlation function of the matter spectrum pk smoothed by s = pk->smooth
 * (> 0; the box's own window, so P_q needs no further smoothing), and
 * b_0 = b_q(z_box) G(z_ref) (1 + z_ref)/(1 + z_box), b_q(z) = 3.7 ((1+z)/3.33)^1.7,
 * G the linear growth of flat LCDM with G(0) = 1: the growth between boxes is
 * taken as 1/(1+z), which the appendix's a(z) presumes.  z_ref: the middle box
 * of three, or the only box.  Quadrature, FP64: xi_m by composite Simpson on
 * [0, 12/s] with spacing <= 0.1/rmax; P_q by composite Simpson on the n_r
 * (odd) nodes r_i = i rmax/(n_r - 1).  k: device [n_k] (h/Mpc, k = 0 gives
 * the limit); pq: device [n_k], values below 1e-12 of the largest raised to
 * that floor (so the result serves as lya_pk's p_tab); xi: device [n_r] or
 * NULL, xi_m at r_i.  work >= lya_lognormal_workspace_size(pk->smooth, rmax,
 * n_r) bytes (0: invalid arguments). */
size_t lya_lognormal_workspace_size(double smooth, double rmax, int32_t n_r);
int lya_lognormal_pk(const lya_pk* pk, double z_box, double z_ref, const lya_cosmo* cosmo, double rmax, int32_t n_r,
                     int32_t n_k, const double* k, double* pq, double* xi, void* work, size_t work_bytes,
                     void* stream);

/* Mean and variance over the n^3 grid points of both parts of an LYA_F32
 * box: out (device [4]) = {mean re, var re, mean im, var im}, FP64 sums.
 * work >= lya_workspace_size(LYA_OP_QUASARS, box). */
int lya_box_moments(const lya_box* box, const void* field, double* out, void* work, size_t work_bytes,
                    void* stream);

typedef struct {
  int32_t n_box;          /* 1 or 3 */
  const void* box_a;      /* LYA_F32 box: delta_q of box 1 in the real part; with three boxes
                             delta_q of box 2 in the imaginary part (lya_make_box_pair) */
  const void* box_b;      /* three boxes: LYA_F32 box with delta_q of box 3 in the real part */
  double z_box[3];        /* box redshifts, increasing (the paper: 1.9, 2.75, 3.6) */
  const double* var[3];   /* device scalars: the variance of each delta_q (lya_box_moments:
                             out + 1 for a real part, out + 3 for an imaginary part) */
  double xi5;             /* three boxes: xi_m(5 Mpc/h) of the smoothed matter spectrum */
  double observer[3];     /* Mpc/h, in the frame where grid point m sits at m dx */
  int32_t n_nbar;         /* 2..256 */
  const double* nbar_z;   /* device [n_nbar], increasing */
  const double* nbar;     /* device [n_nbar]: comoving quasar density, (h/Mpc)^3 */
  uint64_t seed;
} lya_qso_spec;

/* Draws quasars voxel by voxel: grid point m (at x = m dx, z its redshift at
 * comoving distance |x - observer|) is selected with probability
 *   p = nbar(z) dx^3 sum_i c_i(z) exp(a_i delta_i(m) - a_i^2 var_i / 2), clipped to [0, 1],
 * a_i = b_q(z)(1 + z_i)/(b_q(z_i)(1 + z)), nbar linear between its nodes and 0
 * outside them; one box: c_1 = 1; three boxes: p = w p_12 + (1 - w) p_23 with
 * p_12 the linear interpolation in z of boxes 1 and 2, p_23 the linear
 * extrapolation of boxes 2 and 3, and w in [0, 1] such that
 * w xi_12 + (1 - w) xi_23 = (b_q(z) G_q(z))^2 xi5 at r = 5 Mpc/h, where
 * xi_i = (1 + b_0i^2 xi5)^(a_i^2) - 1, G_q(z) = G(z_2)(1 + z_2)/(1 + z) and
 * b_0i = b_q(z_i) G_q(z_i), as lya_lognormal_pk takes them with z_ref = z_2
 * (Appendix A); w = 1/2 where xi_12 = xi_23.  Random numbers:
 * Philox4x32-10, key = seed; the decision of voxel m (linear index
 * (m_x n + m_y) n + m_z) takes word m & 3 of counter (m >> 2, 0, 2, 0) as
 * u = ((w >> 9) + 1/2) 2^-23 and selects when u < p; the selected voxel's
 * position takes words 0-2 of counter (m, 0, 4, 0): per axis
 * (m_axis << 32) - 2^31 + word, cell units times 2^32 (uniform in
 * [m - 1/2, m + 1/2)).  Outputs: *count (device) = number selected; pos_fx
 * (device [cap][3]) holds min(count, cap) positions in an unspecified order
 * (a count above cap asks for a larger buffer).  Every grid point must lie
 * within 10000 Mpc/h of the observer.  work >= lya_workspace_size(
 * LYA_OP_QUASARS, box). */
int lya_draw_quasars(const lya_box* box, const lya_qso_spec* spec, const lya_cosmo* cosmo, int64_t* pos_fx,
                     int64_t cap, int64_t* count, void* work, size_t work_bytes, void* stream);

typedef struct {
  int64_t n_q;            /* quasars */
  const int64_t* pos_fx;  /* device [n_q][3]: positions, cell units times 2^32 (lya_draw_quasars) */
  const void* vel_xy;     /* LYA_F32 box {v_x, v_y}: lya_make_eta(LYA_C_VX, LYA_C_VY) with f = 1, or NULL */
  const void* vel_z;      /* LYA_F32 box {v_z, 0}: lya_make_eta(LYA_C_VZ, LYA_C_NONE) with f = 1, or NULL */
  double observer[3];     /* Mpc/h, as in lya_qso_spec */
  double lam_lo, lam_hi;  /* rest-frame forest window over the Lya wavelength (e.g. 1040/1215.67, 1200/1215.67) */
  double z_min;           /* lowest pixel redshift */
  double dchi;            /* pixel length, Mpc/h (the paper: 0.2) */
} lya_qso_los_spec;

/* The catalogue and its skewer table (section "Quasar generation": the
 * quasar velocity of eq:velocity; section "Gaussian fields along lines of
 * sight": pixels along the line to the observer).  Quasar q at
 * x = pos_fx[q] 2^-32 dx has chi = |x - O| and z_c = z(chi) (Newton on the
 * Simpson chi(z) below, FP64); with velocity
 * boxes, v_par = v(x) . (x - O)/chi (periodic trilinear, FP64 weights) times
 * G(z_c) f(z_c) E(z_c)/(1 + z_c) (the boxes are at z = 0 with f = 1; G and
 * f = dln G/dln a of flat LCDM), and z_q = z_c + (1 + z_c) v_par / c (without
 * velocity boxes z_q = z_c).  Its row of the skewer table (lya_skewers, with
 * dchi): the forest from z_hi = (1 + z_q) lam_hi - 1 towards the observer
 * down to z_lo = max((1 + z_q) lam_lo - 1, z_min); chi0 = chi(z_hi) (FP64
 * Simpson, 1024 intervals); npix = floor((chi(z_hi) - chi(z_lo))/dchi), at
 * most 2048, 0 when z_hi <= z_lo; origin_fx = (O + u chi0)/dx and step_fx =
 * -u dchi/dx in cell units times 2^32, rounded to nearest, u = (x - O)/chi;
 * offset = exclusive prefix sum of npix, *total (device) = the sum.
 * Outputs: device arrays of n_q rows (origin_fx, step_fx: [n_q][3]).
 * work >= lya_workspace_size(LYA_OP_QUASARS, box). */
int lya_quasar_skewers(const lya_box* box, const lya_qso_los_spec* spec, const lya_cosmo* cosmo, double* z_q,
                       int64_t* origin_fx, int64_t* step_fx, int32_t* npix, int64_t* offset, double* chi0,
                       int64_t* total, void* work, size_t work_bytes, void* stream);

/* Launch-shape tuning (the batching and autotuning row of the hot path).
 * Per box size n the library keeps:
 *   fft_y, fft_x      variant of the strided FFT passes, 0..LYA_FFT_VARIANTS-1:
 *                     0/1 one tile of the full pencil count per block, tile
 *                     order 0/1; 2/3 half the pencils per tile (half the LDS,
 *                     two blocks per CU), order 0/1; 4/5 half tiles in the
 *                     persistent software-pipelined kernel (next tile's loads
 *                     issued before the current tile's FFT), order 0/1; 6/7
 *                     full tiles with half the elements per thread (twice the
 *                     waves), order 0/1; 8/9 those in the pipelined kernel;
 *                     10/11 full tiles with tile order 2 (plain block order) /
 *                     3 (outer index fastest within an XCD); 12/13 full tiles
 *                     in the pipelined kernel, order 0/1; 14/15 as 8/9 with
 *                     the next tile's loads issued in parts, one before each
 *                     FFT stage.  All variants give bit-identical boxes.
 *                     Boxes below 1024 have variants 0 and 1 only.
 *                     Defaults: y 8, x 15 from 1024 up, y 0, x 1 below.
 *   sk_chunk          skewers taken per pull from the skewer work queue (default 4);
 *   sk_blocks_per_cu  persistent skewer blocks per CU, 1..4 (default 4);
 *   sk_unroll         pixels per lane whose gathers are issued together, 1, 2 or 4
 *                     (default 1).
 * The table is process-wide and applies to every later call for that n. */
#define LYA_FFT_VARIANTS 16
typedef struct {
  int32_t fft_y, fft_x, sk_chunk, sk_blocks_per_cu, sk_unroll;
} lya_tuning;

int lya_get_tuning(int32_t n, lya_tuning* t);
int lya_set_tuning(int32_t n, const lya_tuning* t);

/* Times both strided FFT passes in every variant on `field` (an FP32 box of
 * size box->n, whose contents are overwritten), `reps` runs each after one
 * untimed run, with HIP events on `stream`; stores the fastest variant of
 * each pass in the table.  ms (may be NULL) receives the mean milliseconds,
 * [pass][variant] with 2 x LYA_FFT_VARIANTS entries (-1 for variants not
 * available at this n).  A variant replaces the current one only if it is at
 * least 2% faster.  work: at least 8 n bytes (twiddles).  Synchronous. */
int lya_autotune_fft(const lya_box* box, void* field, void* work, size_t work_bytes, int32_t reps, double* ms,
                     lya_tuning* out, void* stream);

/* Times lya_draw_skewers (same arguments; outputs overwritten) for skewer
 * chunks {1, 2, 4, 8, 16, 32, 64} x blocks per CU {1, 2, 3, 4} x unroll
 * {1, 2, 4}, `reps` runs each; stores the fastest in the table for box->n.
 * ms (may be NULL) receives 7 x 4 x 3 mean milliseconds, [chunk][blocks][unroll].
 * Synchronous. */
int lya_autotune_skewers(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                         uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                         float* flux, const lya_zbins* zb, void* work, size_t work_bytes, int32_t reps, double* ms,
                         lya_tuning* out, void* stream);

/* HIP-graph capture of a sequence of library calls on one stream:
 * lya_graph_begin(stream), then the calls (lya_make_box, lya_make_eta,
 * lya_draw_skewers, lya_draw_skewers_gauss, lya_draw_skewers_wide,
 * lya_apply_fgpa, lya_p1d: none of
 * them synchronises the host or records memset nodes; kernel timing must be
 * off), then
 * lya_graph_end(stream, &g) instantiates the graph; lya_graph_launch replays
 * it with the same pointers and arguments; lya_graph_destroy frees it (host
 * memory only). */
typedef struct lya_graph_s* lya_graph;
int lya_graph_begin(void* stream);
int lya_graph_end(void* stream, lya_graph* out);
int lya_graph_launch(lya_graph g, void* stream);
int lya_graph_destroy(lya_graph g);

/* Last error message of the tuning and graph calls (thread-local). */
const char* lya_autotune_last_error(void);

/* Kernel timing for benchmarks.  lya_timing_enable(1) clears the records and
 * brackets every kernel the library launches afterwards with two HIP events on
 * the launch stream; lya_timing_enable(0) clears and stops.
 * lya_timing_collect() waits for the recorded events and returns the number of
 * distinct kernel names (or LYA_EHIP); lya_timing_get(i, ...) returns the i-th
 * name, its summed elapsed milliseconds and its number of launches. */
int lya_timing_enable(int on);
int lya_timing_collect(void);
int lya_timing_get(int i, char* name, int name_len, double* total_ms, int64_t* launches);

/* Comoving distance chi(z) = (c/H0) int_0^z dz'/E(z') in Mpc/h, E^2 =
 * Omega_m (1+z)^3 + 1 - Omega_m (the flat background of the mocks, section
 * "Mock generation"), for n host redshifts in [0, 1100] into host chi; FP64 Simpson
 * rule with 4096 intervals.  Host-only (no GPU call): converts redshift-bin
 * edges into the distance edges lya_zbins takes. */
int lya_chi_of_z(const lya_cosmo* cosmo, int32_t n, const double* z, double* chi);

/* Last error message of the calling thread ("" if none). */
const char* lya_last_error(void);

/* Library version string. */
const char* lya_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LYAMOCK_H */
