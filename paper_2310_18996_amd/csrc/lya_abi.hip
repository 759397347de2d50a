// C-ABI of the lyamock library: argument checks, workspace carve-up and
// launch sequencing.  All compute happens in the kernels of k_tables.hip,
// k_fft.hip and k_skewers.hip.
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/lyamock.h"
#include "lya_internal.h"

constexpr size_t kStaticScratchBytes = size_t(1) << 17;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace lya {

// Linear growth of flat LCDM normalised to G(0) = 1: D(a) proportional to
// E(a) int_0^a da' / (a' E(a'))^3, with a' = t^2 (a smooth integrand near 0)
// and composite Simpson over t in [0, sqrt(a)], 4096 intervals, FP64.
double growth_lcdm(double z, double om) {
  auto d = [om](double a) {
    constexpr int kN = 4096;
    const double tmax = sqrt(a), h = tmax / kN;
    double acc = 0.0;
    for (int i = 1; i <= kN; ++i) {
      const double t = h * i, ap = t * t;
      const double ae2 = om / ap + (1.0 - om) * ap * ap;  // (a E)^2
      acc += (i == kN ? 1.0 : (i & 1 ? 4.0 : 2.0)) * 2.0 * t / (ae2 * sqrt(ae2));
    }
    return sqrt(om / (a * a * a) + 1.0 - om) * acc * h / 3.0;
  };
  return d(1.0 / (1.0 + z)) / d(1.0);
}

}  // namespace lya

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, const char* a = "") {
  snprintf(g_err, sizeof(g_err), fmt, a);
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
  return LYA_EHIP;
}

bool pow2_in_range(int n) { return n >= 32 && n <= 2048 && (n & (n - 1)) == 0; }

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct BoxCarve {
  size_t partial, amp, tw, table, table_b, zorder, staging, second, total;
};

// two_buffer: room for a second complex64 box after the staging box (the
// two-buffer order of the FFT passes)
BoxCarve carve_box(const lya_box* b, bool two_buffer = false) {
  BoxCarve c{};
  size_t o = 0;
  c.partial = o; o += align256(sizeof(double) * lya::kSigmaBlocks);
  c.amp = o;     o += align256(sizeof(double));
  c.tw = o;      o += align256(sizeof(float2) * b->n);
  c.table = o;   o += align256(sizeof(float) * lya::amp_table_entries(b->n));
  c.table_b = o; o += align256(sizeof(float) * lya::amp_table_entries(b->n));
  c.zorder = o;  o += align256(sizeof(uint32_t) * lya::zorder_words(b->n));
  c.staging = o;
  if (b->storage == LYA_BF16) o += align256(sizeof(float2) * lya::box_elems(b->n));
  c.second = o;
  if (two_buffer) o += align256(sizeof(float2) * lya::box_elems(b->n));
  c.total = o;
  return c;
}

struct SkCarve {
  size_t ztab, tw, queue, bsum, bcnt, total;
};

SkCarve carve_sk() {
  SkCarve c{};
  size_t o = 0;
  c.ztab = o;  o += align256(sizeof(float) * lya::kZTabN);
  c.tw = o;    o += align256(sizeof(float2) * lya::kTw2048);
  c.queue = o; o += 256;
  c.bsum = o;  o += align256(sizeof(unsigned long long) * lya::kMaxZBins);
  c.bcnt = o;  o += align256(sizeof(unsigned long long) * lya::kMaxZBins);
  c.total = o;
  return c;
}

// Workspace of lya_draw_skewers_static: the file-scope device array
// `scratch` (below), one copy in every GPU the library runs on, held until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy (on the host it only stands in for the symbol): the address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (LYA_OK) or an error code.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LYA_EUNSUPPORTED, "device index above 63%s");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LYA_OK;
}

struct QsoCarve {
  size_t ztab, tab, vtab, part, total;
};

QsoCarve carve_qso() {
  QsoCarve c{};
  size_t o = 0;
  c.ztab = o; o += align256(sizeof(float) * lya::kZTabN);
  c.tab = o;  o += align256(sizeof(float4) * lya::kZTabN);
  c.vtab = o; o += align256(sizeof(float) * lya::kZTabN);
  c.part = o; o += align256(sizeof(double) * 4 * lya::kQsoMomBlocks);
  c.total = o;
  return c;
}

// xi quadrature of lya_lognormal_pk: Simpson on [0, 12/s] with spacing at
// most 0.1/rmax (a tenth of a radian per node at the largest r), m even.
constexpr int64_t kMaxXiNodes = int64_t(1) << 26;
int64_t xi_nodes(double smooth, double rmax) {
  const double kmax = 12.0 / smooth;
  const double h = fmin(0.1 / rmax, kmax / 64.0);
  const double m = 2.0 * ceil(kmax / (2.0 * h));
  return m > static_cast<double>(kMaxXiNodes) ? -1 : static_cast<int64_t>(m);
}

struct LnCarve {
  size_t partial, amp, f, xi, g, total;
};

LnCarve carve_lognormal(int64_t m, int32_t n_r) {
  LnCarve c{};
  size_t o = 0;
  c.partial = o; o += align256(sizeof(double) * lya::kSigmaBlocks);
  c.amp = o;     o += align256(sizeof(double));
  c.f = o;       o += align256(sizeof(double) * static_cast<size_t>(m + 1));
  c.xi = o;      o += align256(sizeof(double) * static_cast<size_t>(n_r));
  c.g = o;       o += align256(sizeof(double) * static_cast<size_t>(n_r));
  c.total = o;
  return c;
}

double bias_qso(double z) { return 3.7 * pow((1.0 + z) / 3.33, 1.7); }

// b_0^2 of the quasar box at z_box: (b_q(z_box) G(z_ref) (1 + z_ref)/(1 + z_box))^2.
double qso_b2(double z_box, double z_ref, double g_ref) {
  const double b = bias_qso(z_box) * g_ref * (1.0 + z_ref) / (1.0 + z_box);
  return b * b;
}

int check_box(const lya_box* box) {
  if (!box) return fail(LYA_EINVAL, "box is NULL%s");
  if (box->n < 32 || box->n > 2048) return fail(LYA_EINVAL, "box n must be in [32, 2048]%s");
  if (!pow2_in_range(box->n)) return fail(LYA_EUNSUPPORTED, "box n must be a power of two%s");
  if (!(box->dx > 0.0)) return fail(LYA_EINVAL, "box dx must be > 0%s");
  if (box->storage != LYA_F32 && box->storage != LYA_BF16) return fail(LYA_EINVAL, "unknown storage type%s");
  return LYA_OK;
}

int check_pk(const lya_pk* pk) {
  if (!pk) return fail(LYA_EINVAL, "pk is NULL%s");
  if (pk->k_tab) {
    if (!pk->p_tab || pk->n_tab < 2 || pk->smooth < 0.0)
      return fail(LYA_EINVAL, "tabulated P(k) needs p_tab and n_tab >= 2%s");
  } else if (!(pk->sigma8 > 0.0) || !(pk->gamma > 0.0) || !(pk->wig_kd > 0.0) || pk->smooth < 0.0) {
    return fail(LYA_EINVAL, "invalid power-spectrum parameters%s");
  }
  return LYA_OK;
}

lya::PkParams pk_params(const lya_pk* pk) {
  return lya::PkParams{pk->sigma8, pk->ns, pk->gamma, pk->wig_amp, pk->wig_r, pk->wig_kd, pk->smooth,
                       pk->k_tab, pk->p_tab, pk->n_tab};
}

// Components (ca, cb) of the modes of pk; with pk_b, component b takes the
// amplitudes of pk_b instead.
int make_pair(const lya_box* box, const lya_pk* pk, const lya_pk* pk_b, uint64_t seed, double f, int ca, int cb,
              void* field, void* work, size_t work_bytes, void* stream) {
  int rc = check_box(box);
  if (rc) return rc;
  if ((rc = check_pk(pk))) return rc;
  if (pk_b && (rc = check_pk(pk_b))) return rc;
  if (!field) return fail(LYA_EINVAL, "field is NULL%s");
  if (!work) return fail(LYA_EINVAL, "work is NULL%s");
  if (ca < LYA_C_DELTA || ca > LYA_C_VZ || cb < LYA_C_NONE || cb > LYA_C_VZ)
    return fail(LYA_EINVAL, "unknown field component%s");
  const BoxCarve c = carve_box(box);
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small for the box%s");
  const bool two_buffer = work_bytes >= carve_box(box, true).total;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(work);
  lya::TableWork tw{reinterpret_cast<double*>(w + c.partial), reinterpret_cast<double*>(w + c.amp),
                    reinterpret_cast<float2*>(w + c.tw), reinterpret_cast<float*>(w + c.table)};
  hipError_t e = lya::launch_pk_table(pk_params(pk), box->n, box->dx, tw, st);
  if (e != hipSuccess) return hip_fail(e, "power-spectrum table");
  const float* table_b = nullptr;
  if (pk_b) {
    lya::TableWork twb = tw;
    twb.table = reinterpret_cast<float*>(w + c.table_b);
    e = lya::launch_pk_table(pk_params(pk_b), box->n, box->dx, twb, st);
    if (e != hipSuccess) return hip_fail(e, "second power-spectrum table");
    table_b = twb.table;
  }
  const double vscale = f * 100.0 * box->n * box->dx / (2.0 * M_PI);
  lya::GenParams g{tw.table, table_b, seed, static_cast<float>(f), ca, cb, pk->fixed_amp ? 1 : 0, pk->only_n2,
                   static_cast<float>(vscale)};
  float2* f32 = box->storage == LYA_F32 ? static_cast<float2*>(field) : reinterpret_cast<float2*>(w + c.staging);
  uint32_t* b16 = box->storage == LYA_BF16 ? static_cast<uint32_t*>(field) : nullptr;
  uint32_t* zorder = lya::zorder_words(box->n) ? reinterpret_cast<uint32_t*>(w + c.zorder) : nullptr;
  e = lya::launch_box_fft(box->n, g, tw.tw, f32, b16, two_buffer ? reinterpret_cast<float2*>(w + c.second) : nullptr,
                          zorder, st);
  if (e != hipSuccess) return hip_fail(e, "box FFT");
  return LYA_OK;
}

int check_skewers(const lya_skewers* sk, bool need_geometry) {
  if (!sk) return fail(LYA_EINVAL, "skewers is NULL%s");
  if (sk->n_sk < 0) return fail(LYA_EINVAL, "n_sk < 0%s");
  if (sk->id_base < 0) return fail(LYA_EINVAL, "id_base < 0%s");
  // quasar ids id_base + q stay below 2^31: the small-scale field's Philox
  // counter is (id << 33) + mode, and the skewer work queue counts chunks in 32 bits
  if (sk->n_sk > (int64_t(1) << 31) - sk->id_base) return fail(LYA_EINVAL, "n_sk + id_base above 2^31%s");
  if (sk->n_sk == 0) return LYA_OK;
  if (!sk->npix || !sk->offset || !sk->chi0) return fail(LYA_EINVAL, "skewer arrays are NULL%s");
  if (need_geometry && (!sk->origin_fx || !sk->step_fx)) return fail(LYA_EINVAL, "skewer geometry is NULL%s");
  if (!(sk->dchi >= 0.0)) return fail(LYA_EINVAL, "dchi must be >= 0%s");
  return LYA_OK;
}

int check_zbins(const lya_zbins* zb) {
  if (!zb) return LYA_OK;
  if (zb->n_bins < 0 || zb->n_bins > lya::kMaxZBins) return fail(LYA_EINVAL, "n_bins must be in [0, 64]%s");
  if (zb->n_bins > 0 && (!zb->chi_edges || (!zb->fsum && !zb->count)))
    return fail(LYA_EINVAL, "redshift-bin arrays are NULL%s");
  return LYA_OK;
}

// a, b, c = c0 + c1 x + c2 x^2 in x = 1+z are re-centred at x0 (FP64) so that
// the device evaluates d0 + d1 t + d2 t^2, t = x - x0, in FP32 without the
// cancellation between large powers of x.
void fill_fgpa(lya::SkewerArgs& a, const lya_fgpa* fg) {
  a.do_flux = fg ? 1 : 0;
  const double x0 = lya::kFgpaX0;
  for (int p = 0; p < 3; ++p) {
    const double c0 = fg ? fg->coef[p][0] : 0.0, c1 = fg ? fg->coef[p][1] : 0.0, c2 = fg ? fg->coef[p][2] : 0.0;
    a.cf[p][0] = static_cast<float>(c0 + x0 * (c1 + x0 * c2));
    a.cf[p][1] = static_cast<float>(c1 + 2.0 * x0 * c2);
    a.cf[p][2] = static_cast<float>(c2);
  }
}

int run_skewers(lya::SkewerArgs& a, const lya_cosmo* cosmo, const lya_zbins* zb, void* work, size_t work_bytes,
                void* stream) {
  const SkCarve c = carve_sk();
  if (!work) return fail(LYA_EINVAL, "work is NULL%s");
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small for the skewers%s");
  if (a.do_flux && !cosmo) return fail(LYA_EINVAL, "cosmo is NULL%s");
  if (cosmo && !(cosmo->omega_m >= 0.0 && cosmo->omega_m <= 1.0)) return fail(LYA_EINVAL, "omega_m out of [0,1]%s");
  char* w = static_cast<char*>(work);
  a.ztab = reinterpret_cast<float*>(w + c.ztab);
  a.tw2048 = reinterpret_cast<float2*>(w + c.tw);
  a.queue = reinterpret_cast<unsigned int*>(w + c.queue);
  a.bin_sum = reinterpret_cast<unsigned long long*>(w + c.bsum);
  a.bin_cnt = reinterpret_cast<unsigned long long*>(w + c.bcnt);
  a.n_bins = zb ? zb->n_bins : 0;
  a.chi_edges = zb ? zb->chi_edges : nullptr;
  a.out_fsum = zb ? zb->fsum : nullptr;
  a.out_count = zb ? zb->count : nullptr;
  // launch shape from the autotuned table of the box size (defaults for stored pixels)
  a.chunk = (a.field || a.field_bf16) ? lya::sk_chunk(a.n) : 8;
  a.blocks_per_cu = (a.field || a.field_bf16) ? lya::sk_blocks_per_cu(a.n) : 4;
  a.unroll = (a.field || a.field_bf16) ? lya::sk_unroll(a.n) : 2;
  if (a.n_sk == 0) {
    if (a.n_bins > 0 && a.do_flux) {
      // still produce zero sums
    } else {
      return LYA_OK;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (a.do_flux) {
    e = lya::launch_zchi_table(cosmo->omega_m, const_cast<float*>(a.ztab), st);
    if (e != hipSuccess) return hip_fail(e, "redshift table");
  }
  if (a.field || a.field_bf16 || a.ds_in_apply) {
    e = lya::launch_twiddles(const_cast<float2*>(a.tw2048), lya::kTw2048, st);
    if (e != hipSuccess) return hip_fail(e, "twiddles");
  }
  e = lya::launch_skewers(a, st);
  if (e != hipSuccess) return hip_fail(e, "skewer kernel");
  return LYA_OK;
}

struct PdCarve {
  size_t sum, cnt, tw, queue, total;
};

PdCarve carve_p1d(int64_t n_sk, int nk) {
  PdCarve c{};
  size_t o = 0;
  c.sum = o;   o += align256(sizeof(double) * static_cast<size_t>(n_sk) * nk);
  c.cnt = o;   o += align256(sizeof(int) * static_cast<size_t>(n_sk) * nk);
  c.tw = o;    o += align256(sizeof(float2) * lya::kTw2048);
  c.queue = o; o += 256;
  c.total = o;
  return c;
}

// velocity pixel in km/s: dpix 100 E(z)/(1+z), E^2 = Om (1+z)^3 + 1 - Om
double velocity_pixel(double dpix, double z, double om) {
  const double x = 1.0 + z;
  return dpix * (100.0 * sqrt(om * (x * x * x) + (1.0 - om)) / x);
}

}  // namespace

namespace lya {
size_t tune_workspace_bytes(int64_t n_sk, int nk);
int tune_params(const lya_tune_spec* spec, lya_tune_result* res, int mode, void* work, size_t work_bytes,
                hipStream_t st, char* err, size_t errlen);
int emulator_labels(const lya_tune_spec* spec, const double* draws, int64_t n, float* y, void* work,
                    size_t work_bytes, hipStream_t st, char* err, size_t errlen);
}  // namespace lya

namespace {
int check_tune_spec(const lya_tune_spec* spec) {
  if (!spec) return fail(LYA_EINVAL, "spec is NULL%s");
  int rc = check_skewers(spec->sk, false);
  if (rc) return rc;
  if (spec->sk->n_sk > 0 && (!spec->dens || !spec->eta)) return fail(LYA_EINVAL, "stored pixels are NULL%s");
  if (!(spec->cosmo.omega_m >= 0.0 && spec->cosmo.omega_m <= 1.0)) return fail(LYA_EINVAL, "omega_m out of [0,1]%s");
  if (spec->p1d.n_kbins < 1 || spec->p1d.n_kbins > lya::kMaxKBins || !spec->p1d.k_edges || !(spec->p1d.dpix > 0.0))
    return fail(LYA_EINVAL, "invalid p1d spec%s");
  return LYA_OK;
}
}  // namespace

extern "C" {

size_t lya_tune_workspace_size(int64_t n_sk, int32_t n_kbins) {
  if (n_sk < 0 || n_kbins < 1 || n_kbins > lya::kMaxKBins) return 0;
  return lya::tune_workspace_bytes(n_sk, n_kbins);
}

int lya_tune_params(const lya_tune_spec* spec, lya_tune_result* res, int mode, void* work, size_t work_bytes,
                    void* stream) {
  g_err[0] = 0;
  int rc = check_tune_spec(spec);
  if (rc) return rc;
  if (!res || !work) return fail(LYA_EINVAL, "result or work is NULL%s");
  if (spec->n_zt < 1 || spec->n_zt > LYA_TUNE_MAX_Z || !spec->p1d_t) return fail(LYA_EINVAL, "invalid tuning redshifts%s");
  if (!(spec->a0 > 0.0) || !(spec->b0 > 0.0) || !(spec->sigma_rel > 0.0) || spec->max_evals < 4)
    return fail(LYA_EINVAL, "invalid start point, sigma_rel or max_evals%s");
  if (mode != LYA_TUNE_PLAIN && mode != LYA_TUNE_EMULATOR) return fail(LYA_EINVAL, "unknown tuning mode%s");
  if (mode == LYA_TUNE_EMULATOR && !spec->emulator) return fail(LYA_EINVAL, "emulator is NULL%s");
  return lya::tune_params(spec, res, mode, work, work_bytes, static_cast<hipStream_t>(stream), g_err, sizeof(g_err));
}

int lya_emulator_labels(const lya_tune_spec* spec, const double* draws, int64_t n, float* y, void* work,
                        size_t work_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_tune_spec(spec);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!draws || !y)) || !work) return fail(LYA_EINVAL, "invalid label arguments%s");
  return lya::emulator_labels(spec, draws, n, y, work, work_bytes, static_cast<hipStream_t>(stream), g_err,
                              sizeof(g_err));
}

size_t lya_p1d_workspace_size(int64_t n_sk, int32_t n_kbins) {
  if (n_sk < 0 || n_kbins < 1 || n_kbins > lya::kMaxKBins) return 0;
  return carve_p1d(n_sk, n_kbins).total;
}

int lya_p1d(const lya_skewers* sk, const lya_cosmo* cosmo, const float* flux, const lya_zbins* fbar,
            const lya_p1d_spec* spec, double* psum, int64_t* pcount, void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_skewers(sk, false);
  if (rc) return rc;
  if (!cosmo || !(cosmo->omega_m >= 0.0 && cosmo->omega_m <= 1.0)) return fail(LYA_EINVAL, "invalid cosmo%s");
  if (!spec || spec->n_kbins < 1 || spec->n_kbins > lya::kMaxKBins || !spec->k_edges)
    return fail(LYA_EINVAL, "invalid p1d spec (1..64 k bins and their edges)%s");
  if (!(spec->dpix > 0.0) || !(spec->z_ref > -1.0)) return fail(LYA_EINVAL, "invalid dpix or z_ref%s");
  if (!fbar || fbar->n_bins < 1 || fbar->n_bins > lya::kMaxZBins || !fbar->chi_edges || !fbar->fsum || !fbar->count)
    return fail(LYA_EINVAL, "mean-flux bins (1..64 with sums and counts) are required%s");
  if (sk->n_sk > 0 && !flux) return fail(LYA_EINVAL, "flux is NULL%s");
  if (!psum && !pcount) return fail(LYA_EINVAL, "no output%s");
  const PdCarve c = carve_p1d(sk->n_sk, spec->n_kbins);
  if (!work) return fail(LYA_EINVAL, "work is NULL%s");
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small for the 1D power%s");
  char* w = static_cast<char*>(work);
  lya::P1dArgs a{};
  a.n_sk = sk->n_sk;
  a.npix = sk->npix;
  a.offset = sk->offset;
  a.chi0 = sk->chi0;
  a.dchi = sk->dchi;
  a.flux = flux;
  a.n_fbins = fbar->n_bins;
  a.chi_edges = fbar->chi_edges;
  a.fsum = fbar->fsum;
  a.fcount = fbar->count;
  a.n_kbins = spec->n_kbins;
  a.k_edges = spec->k_edges;
  a.dv = velocity_pixel(spec->dpix, spec->z_ref, cosmo->omega_m);
  a.part_sum = reinterpret_cast<double*>(w + c.sum);
  a.part_cnt = reinterpret_cast<int*>(w + c.cnt);
  a.tw2048 = reinterpret_cast<float2*>(w + c.tw);
  a.queue = reinterpret_cast<unsigned int*>(w + c.queue);
  a.chunk = 4;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = lya::launch_twiddles(const_cast<float2*>(a.tw2048), lya::kTw2048, st);
  if (e != hipSuccess) return hip_fail(e, "twiddles");
  e = lya::launch_p1d(a, psum, pcount, st);
  if (e != hipSuccess) return hip_fail(e, "1D power kernel");
  return LYA_OK;
}

int lya_chi_of_z(const lya_cosmo* cosmo, int32_t n, const double* z, double* chi) {
  g_err[0] = 0;
  if (!cosmo || !(cosmo->omega_m >= 0.0 && cosmo->omega_m <= 1.0)) return fail(LYA_EINVAL, "invalid cosmo%s");
  if (n < 0 || (n > 0 && (!z || !chi))) return fail(LYA_EINVAL, "invalid redshift arrays%s");
  const double om = cosmo->omega_m;
  for (int32_t i = 0; i < n; ++i) {
    if (!(z[i] >= 0.0 && z[i] <= 1100.0)) return fail(LYA_EINVAL, "redshift outside [0, 1100]%s");
    // composite Simpson rule over [0, z] with 4096 intervals, FP64
    constexpr int kN = 4096;
    const double h = z[i] / kN;
    double acc = 0.0;
    for (int k = 0; k <= kN; ++k) {
      const double x = 1.0 + k * h;
      const double inv_e = 1.0 / sqrt(om * (x * x * x) + (1.0 - om));
      acc += (k == 0 || k == kN ? 1.0 : (k & 1 ? 4.0 : 2.0)) * inv_e;
    }
    chi[i] = lya::kCOverH0 * acc * h / 3.0;
  }
  return LYA_OK;
}

const char* lya_last_error(void) { return g_err; }

const char* lya_version(void) { return "lyamock 0.1 gfx950"; }

size_t lya_field_elems(const lya_box* box) {
  if (!box || !pow2_in_range(box->n)) return 0;
  return lya::box_elems(box->n);
}

size_t lya_plane_pitch(const lya_box* box) {
  if (!box || !pow2_in_range(box->n)) return 0;
  return lya::plane_pitch(box->n);
}

size_t lya_workspace_size(int op, const lya_box* box) {
  if (op == LYA_OP_BOX || op == LYA_OP_BOX_2BUF) {
    if (!box || !pow2_in_range(box->n) || (box->storage != LYA_F32 && box->storage != LYA_BF16)) return 0;
    return carve_box(box, op == LYA_OP_BOX_2BUF).total;
  }
  if (op == LYA_OP_SKEWERS) return carve_sk().total;
  if (op == LYA_OP_QUASARS) return carve_qso().total;
  return 0;
}

int lya_make_box(const lya_box* box, const lya_pk* pk, uint64_t seed, double f, int with_eta, void* field,
                 void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  return make_pair(box, pk, nullptr, seed, f, LYA_C_DELTA, with_eta ? LYA_C_ZZ : LYA_C_NONE, field, work,
                   work_bytes, stream);
}

int lya_make_eta(const lya_box* box, const lya_pk* pk, uint64_t seed, double f, int comp_a, int comp_b,
                 void* field, void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  return make_pair(box, pk, nullptr, seed, f, comp_a, comp_b, field, work, work_bytes, stream);
}

int lya_make_box_pair(const lya_box* box, const lya_pk* pk_a, const lya_pk* pk_b, uint64_t seed, void* field,
                      void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  if (!pk_b) return fail(LYA_EINVAL, "pk_b is NULL%s");
  return make_pair(box, pk_a, pk_b, seed, 1.0, LYA_C_DELTA, LYA_C_DELTA, field, work, work_bytes, stream);
}

static int draw_skewers_impl(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                             uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                             float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream,
                             bool gauss) {
  g_err[0] = 0;
  int rc = check_box(box);
  if (rc) return rc;
  if (!field) return fail(LYA_EINVAL, "field is NULL%s");
  if ((rc = check_skewers(sk, true))) return rc;
  if ((rc = check_zbins(zb))) return rc;
  if (ps && ps->amp > 0.0 && (!(ps->kcut > 0.0) || !(ps->dpix > 0.0)))
    return fail(LYA_EINVAL, "invalid small-scale spectrum%s");
  lya::SkewerArgs a{};
  a.n_sk = sk->n_sk;
  a.origin_fx = sk->origin_fx;
  a.step_fx = sk->step_fx;
  a.npix = sk->npix;
  a.offset = sk->offset;
  a.chi0 = sk->chi0;
  a.dchi = sk->dchi;
  a.id_base = sk->id_base;
  a.n = box->n;
  a.field = box->storage == LYA_F32 ? static_cast<const float2*>(field) : nullptr;
  a.field_bf16 = box->storage == LYA_BF16 ? static_cast<const uint32_t*>(field) : nullptr;
  a.ps_amp = ps ? ps->amp : 0.0;
  a.ps_kcut = ps ? ps->kcut : 1.0;
  a.dpix = ps ? ps->dpix : 1.0;
  a.ps_fixed_amp = ps ? ps->fixed_amp : 0;
  a.seed = seed;
  fill_fgpa(a, fgpa);
  a.dens = dens;
  a.eta = eta;
  a.flux = fgpa ? flux : nullptr;
  a.is_gauss = gauss;
  return run_skewers(a, cosmo, fgpa ? zb : nullptr, work, work_bytes, stream);
}

int lya_draw_skewers(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                     uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                     float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream) {
  return draw_skewers_impl(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zb, work, work_bytes, stream,
                           false);
}

int lya_draw_skewers_static(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                            uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                            float* flux, const lya_zbins* zb, void* stream) {
  g_err[0] = 0;
  const size_t need = carve_sk().total;
  if (need > kStaticScratchBytes)
    return fail(LYA_EWORKSPACE, "the skewer workspace exceeds the static scratch array%s");
  if (zb && zb->n_bins > lya::kMaxZBins) return fail(LYA_EINVAL, "n_bins must be in [0, 64]%s");
  void* work = nullptr;
  const int rc = scratch_address(&work);
  if (rc) return rc;
  return draw_skewers_impl(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zb, work, kStaticScratchBytes,
                           stream, false);
}

int lya_draw_skewers_gauss(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                           uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                           float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream) {
  return draw_skewers_impl(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zb, work, work_bytes, stream,
                           true);
}

int lya_draw_skewers_wide(const lya_box* box, const void* const* fields, const lya_skewers* sk, const lya_ps1d* ps,
                          uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                          float* flux, const lya_zbins* zb, void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_box(box);
  if (rc) return rc;
  if (!fields || !fields[0] || !fields[1] || !fields[2] || !fields[3])
    return fail(LYA_EINVAL, "fields must hold four non-NULL boxes%s");
  if ((rc = check_skewers(sk, true))) return rc;
  if ((rc = check_zbins(zb))) return rc;
  if (ps && ps->amp > 0.0 && (!(ps->kcut > 0.0) || !(ps->dpix > 0.0)))
    return fail(LYA_EINVAL, "invalid small-scale spectrum%s");
  lya::SkewerArgs a{};
  a.n_sk = sk->n_sk;
  a.origin_fx = sk->origin_fx;
  a.step_fx = sk->step_fx;
  a.npix = sk->npix;
  a.offset = sk->offset;
  a.chi0 = sk->chi0;
  a.dchi = sk->dchi;
  a.id_base = sk->id_base;
  a.n = box->n;
  const bool f32 = box->storage == LYA_F32;
  a.field = f32 ? static_cast<const float2*>(fields[0]) : nullptr;
  a.field_bf16 = f32 ? nullptr : static_cast<const uint32_t*>(fields[0]);
  for (int k = 0; k < 3; ++k) {
    a.wide[k] = f32 ? static_cast<const float2*>(fields[k + 1]) : nullptr;
    a.wide_bf16[k] = f32 ? nullptr : static_cast<const uint32_t*>(fields[k + 1]);
  }
  a.is_wide = true;
  a.ps_amp = ps ? ps->amp : 0.0;
  a.ps_kcut = ps ? ps->kcut : 1.0;
  a.dpix = ps ? ps->dpix : 1.0;
  a.ps_fixed_amp = ps ? ps->fixed_amp : 0;
  a.seed = seed;
  fill_fgpa(a, fgpa);
  a.dens = dens;
  a.eta = eta;
  a.flux = fgpa ? flux : nullptr;
  return run_skewers(a, cosmo, fgpa ? zb : nullptr, work, work_bytes, stream);
}

int lya_apply_fgpa_ds(const lya_skewers* sk, const lya_cosmo* cosmo, const float* dens_l, const float* eta,
                      const lya_ps1d* ps, const lya_ps_table* tab, uint64_t seed, const lya_fgpa* fgpa, float* flux,
                      const lya_zbins* zb, void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_skewers(sk, false);
  if (rc) return rc;
  if ((rc = check_zbins(zb))) return rc;
  if (!fgpa) return fail(LYA_EINVAL, "fgpa is NULL%s");
  if (sk->n_sk > 0 && (!dens_l || !eta)) return fail(LYA_EINVAL, "dens_l/eta are NULL%s");
  if (!ps || !(ps->amp >= 0.0) || !(ps->kcut > 0.0) || !(ps->dpix > 0.0))
    return fail(LYA_EINVAL, "invalid small-scale spectrum%s");
  if (tab && (tab->n_bins < 1 || tab->n_bins > lya::kMaxKBins || !tab->k_edges || !tab->ratio))
    return fail(LYA_EINVAL, "invalid P_s table (1..64 bins with edges and ratios)%s");
  lya::SkewerArgs a{};
  a.n_sk = sk->n_sk;
  a.npix = sk->npix;
  a.offset = sk->offset;
  a.chi0 = sk->chi0;
  a.dchi = sk->dchi;
  a.id_base = sk->id_base;
  a.n = 32;
  a.in_dens = dens_l;
  a.in_eta = eta;
  a.ds_in_apply = true;
  a.ps_amp = ps->amp;
  a.ps_kcut = ps->kcut;
  a.dpix = ps->dpix;
  a.ps_fixed_amp = ps->fixed_amp;
  a.seed = seed;
  if (tab) {
    a.ps_nb = tab->n_bins;
    a.ps_edges_k = tab->k_edges;
    a.ps_ratio = tab->ratio;
  }
  fill_fgpa(a, fgpa);
  a.flux = flux;
  return run_skewers(a, cosmo, zb, work, work_bytes, stream);
}

int lya_apply_fgpa(const lya_skewers* sk, const lya_cosmo* cosmo, const float* dens, const float* eta,
                   const lya_fgpa* fgpa, float* flux, const lya_zbins* zb, void* work, size_t work_bytes,
                   void* stream) {
  g_err[0] = 0;
  int rc = check_skewers(sk, false);
  if (rc) return rc;
  if ((rc = check_zbins(zb))) return rc;
  if (!fgpa) return fail(LYA_EINVAL, "fgpa is NULL%s");
  if (sk->n_sk > 0 && (!dens || !eta)) return fail(LYA_EINVAL, "dens/eta are NULL%s");
  lya::SkewerArgs a{};
  a.n_sk = sk->n_sk;
  a.npix = sk->npix;
  a.offset = sk->offset;
  a.chi0 = sk->chi0;
  a.dchi = sk->dchi;
  a.id_base = sk->id_base;
  a.n = 32;
  a.in_dens = dens;
  a.in_eta = eta;
  fill_fgpa(a, fgpa);
  a.flux = flux;
  return run_skewers(a, cosmo, zb, work, work_bytes, stream);
}

size_t lya_lognormal_workspace_size(double smooth, double rmax, int32_t n_r) {
  if (!(smooth > 0.0) || !(rmax > 0.0) || n_r < 3 || n_r > (1 << 22) || !(n_r & 1)) return 0;
  const int64_t m = xi_nodes(smooth, rmax);
  return m < 0 ? 0 : carve_lognormal(m, n_r).total;
}

int lya_lognormal_pk(const lya_pk* pk, double z_box, double z_ref, const lya_cosmo* cosmo, double rmax, int32_t n_r,
                     int32_t n_k, const double* k, double* pq, double* xi, void* work, size_t work_bytes,
                     void* stream) {
  g_err[0] = 0;
  int rc = check_pk(pk);
  if (rc) return rc;
  if (!(pk->smooth > 0.0)) return fail(LYA_EINVAL, "the matter spectrum needs smooth > 0%s");
  if (!cosmo || !(cosmo->omega_m > 0.0 && cosmo->omega_m <= 1.0)) return fail(LYA_EINVAL, "invalid cosmo%s");
  if (!(z_box > -1.0 && z_box < 20.0) || !(z_ref > -1.0 && z_ref < 20.0))
    return fail(LYA_EINVAL, "redshifts must lie in (-1, 20)%s");
  if (!(rmax > 0.0) || n_r < 3 || n_r > (1 << 22) || !(n_r & 1))
    return fail(LYA_EINVAL, "need rmax > 0 and an odd n_r in [3, 2^22]%s");
  if (n_k < 0 || n_k > (1 << 20) || (n_k > 0 && (!k || !pq))) return fail(LYA_EINVAL, "invalid k/pq arrays%s");
  if (!work) return fail(LYA_EINVAL, "work is NULL%s");
  const int64_t m = xi_nodes(pk->smooth, rmax);
  if (m < 0) return fail(LYA_EUNSUPPORTED, "rmax / smooth too large for the xi quadrature%s");
  const LnCarve c = carve_lognormal(m, n_r);
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small for the lognormal spectrum%s");
  char* w = static_cast<char*>(work);
  lya::LognormalArgs a{};
  a.smooth = pk->smooth;
  a.m = static_cast<int>(m);
  a.h = (12.0 / pk->smooth) / static_cast<double>(m);
  a.n_r = n_r;
  a.dr = rmax / (n_r - 1);
  a.b2 = qso_b2(z_box, z_ref, lya::growth_lcdm(z_ref, cosmo->omega_m));
  a.n_k = n_k;
  a.k = k;
  a.pq = pq;
  a.xi = xi ? xi : reinterpret_cast<double*>(w + c.xi);
  a.f = reinterpret_cast<double*>(w + c.f);
  a.g = reinterpret_cast<double*>(w + c.g);
  a.partial = reinterpret_cast<double*>(w + c.partial);
  a.amp = reinterpret_cast<double*>(w + c.amp);
  hipError_t e = lya::launch_lognormal(pk_params(pk), a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lognormal spectrum");
  return LYA_OK;
}

int lya_box_moments(const lya_box* box, const void* field, double* out, void* work, size_t work_bytes,
                    void* stream) {
  g_err[0] = 0;
  int rc = check_box(box);
  if (rc) return rc;
  if (box->storage != LYA_F32) return fail(LYA_EUNSUPPORTED, "box moments need LYA_F32 storage%s");
  if (!field || !out || !work) return fail(LYA_EINVAL, "field/out/work is NULL%s");
  const QsoCarve c = carve_qso();
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small%s");
  hipError_t e = lya::launch_box_moments(static_cast<const float2*>(field), box->n,
                                         reinterpret_cast<double*>(static_cast<char*>(work) + c.part), out,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "box moments");
  return LYA_OK;
}

int lya_draw_quasars(const lya_box* box, const lya_qso_spec* spec, const lya_cosmo* cosmo, int64_t* pos_fx,
                     int64_t cap, int64_t* count, void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_box(box);
  if (rc) return rc;
  if (box->storage != LYA_F32) return fail(LYA_EUNSUPPORTED, "the quasar draw needs LYA_F32 boxes%s");
  if (!spec) return fail(LYA_EINVAL, "spec is NULL%s");
  if (!cosmo || !(cosmo->omega_m > 0.0 && cosmo->omega_m <= 1.0)) return fail(LYA_EINVAL, "invalid cosmo%s");
  const int nb = spec->n_box;
  if (nb != 1 && nb != 3) return fail(LYA_EINVAL, "n_box must be 1 or 3%s");
  if (!spec->box_a || (nb == 3 && !spec->box_b)) return fail(LYA_EINVAL, "quasar boxes are NULL%s");
  for (int i = 0; i < nb; ++i) {
    if (!spec->var[i]) return fail(LYA_EINVAL, "variance pointer is NULL%s");
    if (!(spec->z_box[i] > -1.0 && spec->z_box[i] < 20.0)) return fail(LYA_EINVAL, "box redshift out of range%s");
  }
  if (nb == 3 && !(spec->z_box[0] < spec->z_box[1] && spec->z_box[1] < spec->z_box[2]))
    return fail(LYA_EINVAL, "box redshifts must increase%s");
  if (nb == 3 && !(spec->xi5 > 0.0)) return fail(LYA_EINVAL, "xi5 must be > 0%s");
  if (spec->n_nbar < 2 || spec->n_nbar > lya::kQsoMaxNbar || !spec->nbar_z || !spec->nbar)
    return fail(LYA_EINVAL, "nbar table needs 2..256 nodes%s");
  if (cap < 0 || (cap > 0 && !pos_fx) || !count) return fail(LYA_EINVAL, "invalid output arrays%s");
  if (!work) return fail(LYA_EINVAL, "work is NULL%s");
  const QsoCarve c = carve_qso();
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small%s");
  // every grid point must lie inside the distance table
  const double span = (box->n - 1) * box->dx;
  double far = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double o = spec->observer[ax];
    if (!(fabs(o) < 1e6)) return fail(LYA_EINVAL, "observer out of range%s");
    const double d = fmax(fabs(o), fabs(span - o));
    far += d * d;
  }
  if (!(sqrt(far) < (lya::kZTabN - 2) * lya::kZTabH))
    return fail(LYA_EUNSUPPORTED, "box reaches beyond 10000 Mpc/h from the observer%s");

  char* w = static_cast<char*>(work);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* ztab = reinterpret_cast<float*>(w + c.ztab);
  hipError_t e = lya::launch_zchi_table(cosmo->omega_m, ztab, st);
  if (e != hipSuccess) return hip_fail(e, "redshift table");
  const double z_ref = nb == 3 ? spec->z_box[1] : spec->z_box[0];
  lya::QsoCoef cf{};
  cf.nb = nb;
  cf.z_ref = z_ref;
  cf.g_ref = lya::growth_lcdm(z_ref, cosmo->omega_m);
  cf.xi5 = spec->xi5;
  lya::QsoDrawArgs a{};
  a.n = box->n;
  while ((1 << a.log2n) < box->n) ++a.log2n;
  a.pitch = lya::plane_pitch(box->n);
  a.nb = nb;
  a.box_a = static_cast<const float2*>(spec->box_a);
  a.box_b = nb == 3 ? static_cast<const float2*>(spec->box_b) : nullptr;
  for (int i = 0; i < nb; ++i) {
    cf.z[i] = spec->z_box[i];
    cf.b2[i] = qso_b2(spec->z_box[i], z_ref, cf.g_ref);
    a.var[i] = spec->var[i];
    a.l2z[i] = static_cast<float>(log2(1.0 + spec->z_box[i]));
  }
  a.dx = static_cast<float>(box->dx);
  a.dx_d = box->dx;
  a.dx3 = static_cast<float>(box->dx * box->dx * box->dx);
  for (int ax = 0; ax < 3; ++ax) a.o[ax] = spec->observer[ax];
  a.oz = static_cast<float>(spec->observer[2]);
  a.tab = reinterpret_cast<const float4*>(w + c.tab);
  a.n_nbar = spec->n_nbar;
  a.nbar_z = spec->nbar_z;
  a.nbar = spec->nbar;
  a.seed = spec->seed;
  a.pos = pos_fx;
  a.cap = cap;
  a.count = reinterpret_cast<unsigned long long*>(count);
  e = lya::launch_qso_draw(cf, a, ztab, reinterpret_cast<float4*>(w + c.tab), st);
  if (e != hipSuccess) return hip_fail(e, "quasar draw");
  return LYA_OK;
}

int lya_quasar_skewers(const lya_box* box, const lya_qso_los_spec* spec, const lya_cosmo* cosmo, double* z_q,
                       int64_t* origin_fx, int64_t* step_fx, int32_t* npix, int64_t* offset, double* chi0,
                       int64_t* total, void* work, size_t work_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_box(box);
  if (rc) return rc;
  if (!spec) return fail(LYA_EINVAL, "spec is NULL%s");
  if (!cosmo || !(cosmo->omega_m > 0.0 && cosmo->omega_m <= 1.0)) return fail(LYA_EINVAL, "invalid cosmo%s");
  if (spec->n_q < 0 || spec->n_q > (int64_t(1) << 36)) return fail(LYA_EINVAL, "n_q out of range%s");
  if (spec->n_q > 0 && (!spec->pos_fx || !z_q || !origin_fx || !step_fx || !npix || !offset || !chi0))
    return fail(LYA_EINVAL, "catalogue arrays are NULL%s");
  if (!total || !work) return fail(LYA_EINVAL, "total/work is NULL%s");
  if ((spec->vel_xy == nullptr) != (spec->vel_z == nullptr))
    return fail(LYA_EINVAL, "give both velocity boxes or neither%s");
  if (spec->vel_xy && box->storage != LYA_F32) return fail(LYA_EUNSUPPORTED, "velocity boxes need LYA_F32%s");
  if (!(spec->lam_lo > 0.0 && spec->lam_lo < spec->lam_hi) || !(spec->dchi > 0.0) || !(spec->z_min >= 0.0))
    return fail(LYA_EINVAL, "need 0 < lam_lo < lam_hi, dchi > 0, z_min >= 0%s");
  for (int ax = 0; ax < 3; ++ax)
    if (!(fabs(spec->observer[ax]) < 1e6)) return fail(LYA_EINVAL, "observer out of range%s");
  const QsoCarve c = carve_qso();
  if (work_bytes < c.total) return fail(LYA_EWORKSPACE, "workspace too small%s");
  char* w = static_cast<char*>(work);
  lya::QsoLosArgs a{};
  a.n_q = spec->n_q;
  a.pos = spec->pos_fx;
  a.vxy = static_cast<const float2*>(spec->vel_xy);
  a.vz = static_cast<const float2*>(spec->vel_z);
  a.n = box->n;
  a.pitch = lya::plane_pitch(box->n);
  a.dx = box->dx;
  for (int ax = 0; ax < 3; ++ax) a.o[ax] = spec->observer[ax];
  a.om = cosmo->omega_m;
  a.r_lo = spec->lam_lo;
  a.r_hi = spec->lam_hi;
  a.z_min = spec->z_min;
  a.dchi = spec->dchi;
  a.ztab = reinterpret_cast<const float*>(w + c.ztab);
  a.vtab = reinterpret_cast<const float*>(w + c.vtab);
  a.z_q = z_q;
  a.origin = origin_fx;
  a.step = step_fx;
  a.npix = npix;
  a.offset = offset;
  a.chi0 = chi0;
  a.total = total;
  hipError_t e = lya::launch_qso_los(a, reinterpret_cast<float*>(w + c.ztab), reinterpret_cast<float*>(w + c.vtab),
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "quasar lines of sight");
  return LYA_OK;
}

}  // extern "C"
