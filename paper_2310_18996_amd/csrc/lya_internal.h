// Internal declarations of the lyamock HIP library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lya_device.h"

namespace lya {

constexpr double kCOverH0 = 2997.92458;  // Mpc/h
constexpr int kSigmaBlocks = 64;          // partial sums of the sigma8 integral
constexpr double kZTabH = 0.5;            // Mpc/h spacing of the z(chi) table
constexpr int kZTabN = 20001;             // covers chi in [0, 10000] Mpc/h
constexpr int kMaxZBins = 64;
constexpr int kTw2048 = 2048;             // twiddles for the small-scale 1D FFTs
constexpr float kFgpaX0 = 3.5f;           // centre (in 1+z) of the FGPA quadratics

struct PkParams {
  double sigma8, ns, gamma, wig_amp, wig_r, wig_kd, smooth;
  // tabulated P(k) (device, n_tab >= 2, k increasing): used instead of the
  // analytic form when k_tab is not null
  const double* k_tab;
  const double* p_tab;
  int n_tab;
};

inline int amp_table_entries(int n) { return 3 * (n / 2) * (n / 2) + 1; }

// Box layout: element (x, y, z) at x * plane_pitch(n) + y * n + z.  The x
// planes are padded by kPlanePad elements: without it the x-direction FFT pass
// walks memory with a stride of a large power of two and its requests pile up
// on few HBM channels.
constexpr int kPlanePad = 32;
__host__ __device__ constexpr size_t plane_pitch(int n) {
  return static_cast<size_t>(n) * static_cast<size_t>(n) + kPlanePad;
}
__host__ __device__ constexpr size_t box_elems(int n) { return static_cast<size_t>(n) * plane_pitch(n); }

// Workspace carve-up of lya_make_box / lya_make_eta.
struct TableWork {
  double* partial;  // kSigmaBlocks
  double* amp;      // 1
  float2* tw;       // n twiddles exp(+2 pi i k/n)
  float* table;     // amp_table_entries(n)
};

// What the first FFT pass synthesises for each mode.
struct GenParams {
  const float* table;
  const float* table_b;  // non-null: component b takes its own amplitudes (two spectra, one set of modes)
  uint64_t seed;
  float f;
  int comp_a, comp_b;  // 0 delta, 1 xx, 2 yy, 3 zz, 4 xy, 5 xz, 6 yz, 7-9 v_x, v_y, v_z; -1 none
  int fixed_amp;
  int only_n2;
  float vscale;        // velocities: f 100 L / (2 pi), km/s
  float2* dst;         // the transposing pass of the two-buffer order writes here
  const uint32_t* order;  // paired tiles of the synthesising pass in this order (null: the mirrored order)
};

// Optional event timing around each launch (see lya_timing_enable).
void timer_begin(const char* name, hipStream_t st);
void timer_end(hipStream_t st);
#define LYA_TIMED(name, st, ...)     \
  do {                               \
    ::lya::timer_begin(name, st);    \
    __VA_ARGS__;                     \
    ::lya::timer_end(st);            \
  } while (0)

// Compute units of the current device (cached per device).
int device_cus();
// Linear growth of flat LCDM with G(0) = 1 (host, FP64).
double growth_lcdm(double z, double om);

hipError_t launch_pk_table(const PkParams& p, int n, double dx, TableWork& w, hipStream_t st);
hipError_t launch_zchi_table(double omega_m, float* ztab, hipStream_t st);
// Simpson-weighted integrand of xi_m (k_j = j h, j = 0..m): sigma8
// normalisation first for the analytic form (partial: kSigmaBlocks, amp: 1).
hipError_t launch_xi_weights(const PkParams& p, double s, double h, int m, double* partial, double* amp,
                             double* f, hipStream_t st);
hipError_t launch_twiddles(float2* tw, int ntw, hipStream_t st);
// second: a complex64 box buffer of the same size (workspace) for the
// two-buffer order, or null for the in-place order.  zorder: zorder_words(n)
// words of workspace for the synthesising pass's tile order (boxes from
// kZOrderMinN up; null or below: the mirrored order).
constexpr int kZOrderMinN = 2048;
size_t zorder_words(int n);
hipError_t launch_box_fft(int n, const GenParams& g, const float2* tw, float2* field, uint32_t* field_bf16,
                          float2* second, uint32_t* zorder, hipStream_t st);
// Strided-pass variants (0..kFftVariants-1) per box size and pass (0 = y, 1 = x).
constexpr int kFftVariants = 16;
int fft_variant(int n, int pass);
int set_fft_variant(int n, int pass, int v);
hipError_t launch_fft_strided_pass(int n, int pass, int variant, const float2* tw, float2* field, hipStream_t st);
// Skewer-kernel launch shape per box size (autotuned): skewers per queue pull,
// persistent blocks per CU, pixels per lane per gather step.
int sk_chunk(int n);
int sk_blocks_per_cu(int n);
int sk_unroll(int n);
void set_sk_shape(int n, int chunk, int bpc, int unroll);

// Skewer stage.
struct SkewerArgs {
  // geometry
  int64_t n_sk;
  const int64_t* origin_fx;
  const int64_t* step_fx;
  const int32_t* npix;
  const int64_t* offset;
  const double* chi0;
  double dchi;
  int64_t id_base;
  // field
  int n;
  const float2* field;         // FP32 {delta, eta} or null
  const uint32_t* field_bf16;  // BF16 {delta, eta} or null
  // wide-angle eta_par (all null: eta_par is the box's second component): the
  // boxes {eta_xx, eta_yy}, {eta_xy, eta_xz}, {eta_yz, 0} in the box's storage
  const float2* wide[3];
  const uint32_t* wide_bf16[3];
  bool is_wide;
  // the 7^3 Gaussian-kernel average in place of trilinear interpolation
  bool is_gauss;
  // delta_S added to stored pixels in apply mode, and a tabulated factor of
  // P_s per k bin (ps_ratio null: 1): bin b holds ps_edges_k[b] <= k <
  // ps_edges_k[b+1] (h/Mpc), the ends clamped
  bool ds_in_apply;
  int ps_nb;
  const double* ps_edges_k;
  const float* ps_ratio;
  // small-scale field
  double ps_amp, ps_kcut, dpix;
  int ps_fixed_amp;
  uint64_t seed;
  // FGPA (valid when do_flux): a, b, c as quadratics in t = (1+z) - kFgpaX0,
  // converted on the host in FP64 from the powers of (1+z)
  int do_flux;
  float cf[3][3];
  // pre-FGPA inputs for apply_fgpa (gather skipped when non-null)
  const float* in_dens;
  const float* in_eta;
  // outputs (each may be null)
  float* dens;
  float* eta;
  float* flux;
  // redshift bins
  int n_bins;
  const double* chi_edges;
  unsigned long long* bin_sum;  // workspace, fixed point F * 2^32
  unsigned long long* bin_cnt;
  double* out_fsum;
  int64_t* out_count;
  // tables and scheduling
  const float* ztab;
  const float2* tw2048;
  unsigned int* queue;
  int chunk;
  int blocks_per_cu;  // persistent blocks per CU (<= 0: 4)
  int unroll;         // pixels per lane per step: 1, 2 or 4 (other values: 2)
};

hipError_t launch_skewers(const SkewerArgs& a, hipStream_t st);

// 1D flux power spectrum.
constexpr int kMaxKBins = 64;
struct P1dArgs {
  int64_t n_sk;
  const int32_t* npix;
  const int64_t* offset;
  const double* chi0;
  double dchi;
  const float* flux;         // or null: F from dens/eta under constant (fa, fb, fc)
  const float* dens;
  const float* eta;
  float fa, fb, fc;
  int n_fbins;               // mean-flux bins in comoving distance
  const double* chi_edges;   // [n_fbins + 1]
  const double* fsum;        // [n_fbins]
  const int64_t* fcount;     // [n_fbins]
  int n_kbins;
  const double* k_edges;     // [n_kbins + 1], s/km
  double dv;                 // velocity pixel, km/s
  double* part_sum;          // workspace [n_kbins][n_sk]
  int* part_cnt;             // workspace [n_kbins][n_sk]
  const float2* tw2048;
  unsigned int* queue;
  int chunk;
};
hipError_t launch_p1d(const P1dArgs& a, double* psum, int64_t* pcount, hipStream_t st);

// Batched tuning statistics (Fbar and binned P1D) of stored pixels for up to
// kTuneEvalMaxG constant-parameter draws in one pass.
constexpr int kTuneEvalMaxG = 8;
struct TuneEvalArgs {
  int64_t n_sk;
  const int32_t* npix;
  const int64_t* offset;
  const float* dens;
  const float* eta;
  int G;                          // draws in this launch
  float draw[kTuneEvalMaxG][3];   // a, b, c of each draw
  double dv[kTuneEvalMaxG];       // velocity pixel (km/s) at each draw's z
  int nk;
  const double* k_edges;          // device [nk + 1]
  double* fs;                     // workspace [G][n_sk]: sum of F per skewer
  double* ps;                     // workspace [G][nk][n_sk]: sum |X_m|^2 / N_P
  int* pc;                        // workspace [G][nk][n_sk]: modes
  const float2* tw2048;
  unsigned int* queue;
  int chunk;
  // delta_S redrawn per draw (with_ds): P_s(k) = ds_amp[g] exp(-(k/ds_kcut[g])^2)
  // on every skewer (Philox key seed, line id_base + q, pixel length dpix),
  // added to dens before the FGPA; skewers above 2048 pixels then give NaN
  int with_ds;
  double ds_amp[kTuneEvalMaxG], ds_kcut[kTuneEvalMaxG];
  double dpix;
  uint64_t seed;
  int64_t id_base;
  // what the shared delta_S synthesis reads besides: no P_s table, random phases
  int ps_nb;
  const double* ps_edges_k;
  const float* ps_ratio;
  int ps_fixed_amp;
};
// sums/counts: [G][nk + 1] (bins, then flux and pixels); rows (FP64) and rows32
// (FP32, may be NULL): [G][1 + nk] = Fbar, P_1..P_nk.
hipError_t launch_tune_eval(const TuneEvalArgs& a, double* sums, int64_t* counts, double* rows, float* rows32,
                            hipStream_t st);

// Tuning statistics with delta_S redrawn per draw (lya_tune.hip), for the
// small-scale power tuning: stored pixels without delta_S and their table,
// device k edges (s/km), Philox key of delta_S.  The workspace w is laid out
// as the tuning workspace of (n_sk, nk): tune_workspace_bytes bytes.
struct DsSource {
  int64_t n_sk, id_base;
  const int32_t* npix;
  const int64_t* offset;
  const float* dens;
  const float* eta;
  const double* k_edges;
  int nk;
  double dpix, omega_m;
  uint64_t seed;
};
struct DsDraw {
  double a, b, c, z, amp, kcut;   // FGPA (a, b, c) at redshift z; P_s = amp exp(-(k/kcut)^2)
};
size_t tune_workspace_bytes(int64_t n_sk, int nk);
hipError_t tune_eval_prepare(char* w, hipStream_t st);           // twiddles into w
char* tune_eval_scratch(char* w, int64_t n_sk, int nk);          // the emulator search's output slot in w
// G <= kTuneEvalMaxG draws: rows [G][1 + nk] = Fbar, P_1..P_nk into rows_host
// (then synchronises the stream) and/or into rows32 (device FP32).
hipError_t tune_eval_ds(const DsSource& src, char* w, const DsDraw* d, int G, double* rows_host, float* rows32,
                        hipStream_t st);

// Lognormal quasar field (lya_qso.hip).
struct LognormalArgs {
  double smooth;   // Gaussian smoothing length of the matter spectrum, Mpc/h
  double h;        // k spacing of the xi quadrature; nodes j = 0..m (m even)
  int m;
  double dr;       // r spacing; nodes i = 0..n_r-1 (n_r odd)
  int n_r;
  double b2;       // b_0^2
  int n_k;
  const double* k;   // device [n_k]
  double* pq;        // device [n_k]
  double* xi;        // device [n_r]
  double* f;         // workspace [m + 1]
  double* g;         // workspace [n_r]
  double* partial;   // workspace [kSigmaBlocks]
  double* amp;       // workspace [1]
};
hipError_t launch_lognormal(const PkParams& p, const LognormalArgs& a, hipStream_t st);

constexpr int kQsoMomBlocks = 1024;
// box: FP32 {re, im} box; part: workspace [kQsoMomBlocks][4]; out: device [4]
// = {mean re, var re, mean im, var im}.
hipError_t launch_box_moments(const float2* box, int n, double* part, double* out, hipStream_t st);

constexpr int kQsoMaxNbar = 256;
struct QsoCoef {
  int nb;
  double z[3];
  double b2[3];
  double g_ref, z_ref;
  double xi5;
};
struct QsoDrawArgs {
  int n, log2n;
  size_t pitch;
  int nb;
  const float2* box_a;    // delta_1 (re) and, for three boxes, delta_2 (im)
  const float2* box_b;    // delta_3 (re)
  const double* var[3];   // device scalars
  float dx, oz, dx3;
  double dx_d, o[3];
  float l2z[3];           // log2(1 + z_i)
  const float4* tab;      // {z, c_1, c_2, c_3} per kZTabH of comoving distance
  int n_nbar;
  const double* nbar_z;
  const double* nbar;
  uint64_t seed;
  int64_t* pos;
  int64_t cap;
  unsigned long long* count;
};
hipError_t launch_qso_draw(const QsoCoef& c, const QsoDrawArgs& a, const float* ztab, float4* tab, hipStream_t st);

struct QsoLosArgs {
  int64_t n_q;
  const int64_t* pos;     // [n_q][3] fixed point
  const float2* vxy;      // {v_x, v_y} box or null (no velocities)
  const float2* vz;       // {v_z, .} box
  int n;
  size_t pitch;
  double dx, o[3], om;
  double r_lo, r_hi, z_min, dchi;
  const float* ztab;      // z at chi = i kZTabH
  const float* vtab;      // G f E / (1 + z) at the same nodes
  double* z_q;
  int64_t* origin;
  int64_t* step;
  int32_t* npix;
  int64_t* offset;
  double* chi0;
  int64_t* total;
};
// Fills ztab_w and vtab_w (kZTabN floats each), then the catalogue.
hipError_t launch_qso_los(const QsoLosArgs& a, float* ztab_w, float* vtab_w, hipStream_t st);

// Tuning (lya_tune.hip) and the emulator used by it (lya_mlp.hip).
size_t emulator_eval_bytes();
// Device-side Nelder-Mead over th = (ln a, ln b) on the model
// emulator(th) + off + jac (th - xk) (statistics: Fbar, then the P1D bins);
// x holds the start on entry and the optimum on return, pred the raw emulator
// prediction [1 + nk] there (synchronous).
struct EmuSearchSpec {
  double fbar_t, c, z, step, xatol, fatol, sigma;
  int nk, max_evals;
  const double* pk_t;   // [nk]
  const double* off;    // [1 + nk]
  const double* jac;    // [1 + nk][2]
  double xk[2];
  // small-scale power mode: x = (ln amp, ln kcut) of P_s; emulator inputs
  // (a, b, amp, kcut) with sigma_g^2 = sig0 + sigma_s^2(amp, kcut; dpix),
  // (ln a, ln s) = lin[0..1] + lin[2..3] (ln sigma_g - lin[4]), b = s / sigma_g
  int ps = 0;
  double sig0 = 0.0, dpix = 0.0, lin[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
};
hipError_t emulator_search(const void* emu, const EmuSearchSpec& sp, double x[2], double* fbest, int* nev,
                           double* pred, char* scratch, hipStream_t st);

}  // namespace lya
