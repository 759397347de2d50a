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

/* Field components (eq:deltaL and eq:eta): delta, then eta_pq = f k_p k_q / k^2 delta. */
enum { LYA_C_NONE = -1, LYA_C_DELTA = 0, LYA_C_XX = 1, LYA_C_YY = 2, LYA_C_ZZ = 3,
       LYA_C_XY = 4, LYA_C_XZ = 5, LYA_C_YZ = 6 };

/* Workspace kinds for lya_workspace_size. */
enum { LYA_OP_BOX = 0, LYA_OP_SKEWERS = 1 };

/* Periodic box (section "Mock generation"). */
typedef struct {
  int32_t n;        /* grid points per side: 32, 64, ..., 2048 */
  double dx;        /* voxel side in Mpc/h (> 0) */
  int32_t storage;  /* LYA_F32 or LYA_BF16 element type of the output box */
} lya_box;

/* Linear power spectrum, stand-in for the paper's CAMB P_m(k) (eq:deltaL):
 *   P(k) = A k^ns T_BBKS(k/gamma)^2 (1 + wig_amp sin(k wig_r) exp(-(k/wig_kd)^2)),
 * A set so that sigma_8 = sigma8.  k in h/Mpc, P in (Mpc/h)^3. */
typedef struct {
  double sigma8, ns, gamma, wig_amp, wig_r, wig_kd;
  double smooth;     /* Gaussian window sigma in Mpc/h on the mode amplitude, 0 = off
                        (the paper's smoothing, Appendix B, W^2 = exp(-dx^2 k^2), is smooth = dx) */
  int32_t fixed_amp; /* 1: |W(k)| = 1 (fixed-amplitude test hook) */
  int32_t only_n2;   /* >= 0: keep only the modes with |n|^2 == only_n2 (test hook); -1: all */
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
  const int32_t* npix;       /* device [n_sk], 0 <= npix <= 2048 */
  const int64_t* offset;     /* device [n_sk] */
  const double* chi0;        /* device [n_sk], Mpc/h */
  double dchi;               /* pixel length in Mpc/h (the paper: 0.2) */
  int64_t id_base;           /* quasar id of row 0: seeds its small-scale field */
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

/* Bytes of device workspace a call needs.  op = LYA_OP_BOX for lya_make_box and
 * lya_make_eta (for LYA_BF16 storage this includes an n^3 complex64 staging box),
 * LYA_OP_SKEWERS for lya_draw_skewers and lya_apply_fgpa.  Returns 0 for
 * invalid arguments. */
size_t lya_workspace_size(int op, const lya_box* box);

/* Gaussian box and line-of-sight velocity gradient (section "Mock generation",
 * eq:deltaL, eq:eta).  Draws the k-space noise W(k) from Philox4x32-10 (key =
 * seed, stream 0), forms delta_hat = sqrt(P(k)/L^3) W and
 * eta_par_hat = f mu_z^2 delta_hat (line of sight = z axis), and writes the
 * real-space box {delta, eta_par} = inverse DFT (unnormalised, exp(+i k.x)).
 * field: device, n^3 cells of the box's storage type.  with_eta = 0 writes
 * eta_par = 0.  work: device, >= lya_workspace_size(LYA_OP_BOX, box) bytes. */
int lya_make_box(const lya_box* box, const lya_pk* pk, uint64_t seed, double f, int with_eta,
                 void* field, void* work, size_t work_bytes, void* stream);

/* Any pair of components of the same modes (eq:eta: eta_pq = f k_p k_q/k^2
 * delta_hat; cross terms vanish on the Nyquist plane of p or q): writes
 * {comp_a, comp_b} (comp_b may be LYA_C_NONE).  Same layout and workspace as
 * lya_make_box. */
int lya_make_eta(const lya_box* box, const lya_pk* pk, uint64_t seed, double f, int comp_a, int comp_b,
                 void* field, void* work, size_t work_bytes, void* stream);

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

/* FGPA on stored pre-FGPA pixels (eq:FGPA; the paper's post-production step):
 * flux = exp(-a(z) exp(b(z) (dens + c(z) eta))), z the redshift of chi_j.
 * Geometry fields of sk other than npix, offset, chi0 and dchi are unused.
 * flux may be NULL when only the per-bin sums are wanted. */
int lya_apply_fgpa(const lya_skewers* sk, const lya_cosmo* cosmo, const float* dens, const float* eta,
                   const lya_fgpa* fgpa, float* flux, const lya_zbins* zb, void* work, size_t work_bytes,
                   void* stream);

/* Kernel timing for benchmarks.  lya_timing_enable(1) clears the records and
 * brackets every kernel the library launches afterwards with two HIP events on
 * the launch stream; lya_timing_enable(0) clears and stops.
 * lya_timing_collect() waits for the recorded events and returns the number of
 * distinct kernel names (or LYA_EHIP); lya_timing_get(i, ...) returns the i-th
 * name, its summed elapsed milliseconds and its number of launches. */
int lya_timing_enable(int on);
int lya_timing_collect(void);
int lya_timing_get(int i, char* name, int name_len, double* total_ms, int64_t* launches);

/* Last error message of the calling thread ("" if none). */
const char* lya_last_error(void);

/* Library version string. */
const char* lya_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LYAMOCK_H */
