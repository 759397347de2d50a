// Small-scale power iteration of the tuning (section "Adjusting mock
// parameters"): at each tuning redshift, a and s = b sigma_g from the target
// mean flux and flux dispersion of a Gaussian g, sigma_g from the moments of
// the stored pixels and the current P_s, then repeatedly: delta_S redrawn
// with P_s (lya_apply_fgpa_ds), Fbar and P1D measured (lya_p1d), and P_s
// multiplied per k bin by P_target / P1D.  The outer loop re-solves (a, s)
// for Fbar and the target effective bias of the correlation-function
// prediction, then runs the iteration again.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "../../include/lyamock.h"
#include "lya_internal.h"

namespace lya {
namespace {

constexpr int kMomBlocks = 1024;
constexpr int kMomNT = 256;

// Per block, over skewers blockIdx.x, blockIdx.x + gridDim.x, ...: FP64 sums
// of d, e, d^2, e^2, d e; fixed order within the block.
__global__ void __launch_bounds__(kMomNT) k_moments(int64_t n_sk, const int32_t* __restrict__ npix,
                                                    const int64_t* __restrict__ offset, const float* __restrict__ d,
                                                    const float* __restrict__ e, double* __restrict__ part) {
  __shared__ double s[5][kMomNT];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t q = blockIdx.x; q < n_sk; q += gridDim.x) {
    const int np = npix[q];
    const int64_t off = offset[q];
    for (int j = threadIdx.x; j < np; j += kMomNT) {
      const double x = d[off + j], y = e[off + j];
      acc[0] += x;
      acc[1] += y;
      acc[2] += x * x;
      acc[3] += y * y;
      acc[4] += x * y;
    }
  }
  for (int k = 0; k < 5; ++k) s[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = kMomNT / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w)
      for (int k = 0; k < 5; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) part[threadIdx.x * kMomBlocks + blockIdx.x] = s[threadIdx.x][0];
}

// out[k] = sum over blocks of part[k][.], fixed tree order (one block per k).
__global__ void __launch_bounds__(kMomBlocks) k_moments_reduce(const double* __restrict__ part, double* out) {
  __shared__ double s[kMomBlocks];
  s[threadIdx.x] = part[blockIdx.x * kMomBlocks + threadIdx.x];
  __syncthreads();
  for (int w = kMomBlocks / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

size_t al(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct PsCarve {
  size_t sk, p1d, flux, ratio, edges, zb, psum, pcnt, part, mom, te, total;
};

PsCarve carve_ps(int64_t n_sk, int64_t n_pix, int nk) {
  PsCarve c{};
  size_t o = 0;
  c.sk = o;
  o += al(lya_workspace_size(LYA_OP_SKEWERS, nullptr));
  c.p1d = o;
  o += al(lya_p1d_workspace_size(n_sk, nk));
  c.flux = o;
  o += al(sizeof(float) * static_cast<size_t>(n_pix > 0 ? n_pix : 1));
  c.ratio = o;
  o += al(sizeof(float) * kMaxKBins);
  c.edges = o;
  o += al(sizeof(double) * (kMaxKBins + 1));
  c.zb = o;  // chi edges [2], fsum [1], count [1]
  o += al(4 * sizeof(double));
  c.psum = o;
  o += al(sizeof(double) * kMaxKBins);
  c.pcnt = o;
  o += al(sizeof(int64_t) * kMaxKBins);
  c.part = o;
  o += al(sizeof(double) * 5 * kMomBlocks);
  c.mom = o;
  o += al(sizeof(double) * 5);
  c.te = o;  // the batched evaluation with delta_S (emulator mode and its labels)
  o += al(tune_workspace_bytes(n_sk, nk));
  c.total = o;
  return c;
}

// F = exp(-a exp(s x)), x a unit normal: mean and dispersion, and
// E[e^{s x} F] (the flux bias), by the trapezoid rule on [-12, 12].  The
// integrands are analytic in a strip about the real axis, so the rule
// converges geometrically in 1/h: 960 intervals (h = 0.025) agree with
// 96,000 to 1e-14 relative for 1e-4 <= a <= 3 and s <= 10.
void gauss_flux(double a, double s, double* f1, double* sf, double* mb = nullptr) {
  const int n = 960;
  const double h = 24.0 / n;
  double m1 = 0.0, m2 = 0.0, m3 = 0.0;
  for (int i = 0; i <= n; ++i) {
    const double x = -12.0 + i * h;
    const double w = (i == 0 || i == n ? 0.5 : 1.0) * exp(-0.5 * x * x);
    const double e = exp(s * x);
    const double F = exp(-a * e);
    m1 += w * F;
    m2 += w * F * F;
    m3 += w * exp(s * x - a * e);
  }
  const double norm = h / sqrt(2.0 * M_PI);
  m1 *= norm;
  m2 *= norm;
  *f1 = m1;
  *sf = sqrt(m2 - m1 * m1 > 0.0 ? m2 - m1 * m1 : 0.0);
  if (mb) *mb = m3 * norm;
}

// Effective bias of the correlation-function prediction: |b_F| (1 + 2 beta/3
// + beta^2/5)^(1/2), b_F = E[dF/dg] / Fbar = -(a s / sigma_g) E[e^{s x} F] / Fbar.
double effective_bias(double a, double s, double sigma_g, double beta, double* fbar) {
  double f1, sf, mb;
  gauss_flux(a, s, &f1, &sf, &mb);
  if (fbar) *fbar = f1;
  return (a * s / sigma_g) * mb / f1 * sqrt(1.0 + 2.0 * beta / 3.0 + beta * beta / 5.0);
}

// Damped Newton in t = (ln a, ln s) on two residuals; true when both end
// below 1e-9.
template <typename R>
bool newton2(R resid, double* a, double* s) {
  double t[2] = {log(*a), log(*s)};
  double r[2];
  if (!resid(t, r)) return false;
  for (int it = 0; it < 200; ++it) {
    const double nr = fabs(r[0]) + fabs(r[1]);
    if (nr < 1e-13) break;
    double J[2][2];
    for (int k = 0; k < 2; ++k) {
      double up[2] = {t[0], t[1]}, dn[2] = {t[0], t[1]}, rp[2], rm[2];
      up[k] += 1e-6;
      dn[k] -= 1e-6;
      if (!resid(up, rp) || !resid(dn, rm)) return false;
      J[0][k] = (rp[0] - rm[0]) / 2e-6;
      J[1][k] = (rp[1] - rm[1]) / 2e-6;
    }
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!(fabs(det) > 1e-300)) return false;
    const double d0 = -(J[1][1] * r[0] - J[0][1] * r[1]) / det;
    const double d1 = -(-J[1][0] * r[0] + J[0][0] * r[1]) / det;
    double lam = 1.0;
    bool moved = false;
    for (int ls = 0; ls < 40; ++ls, lam *= 0.5) {
      double u[2] = {t[0] + lam * d0, t[1] + lam * d1}, ru[2];
      if (resid(u, ru) && fabs(ru[0]) + fabs(ru[1]) < nr) {
        t[0] = u[0];
        t[1] = u[1];
        r[0] = ru[0];
        r[1] = ru[1];
        moved = true;
        break;
      }
    }
    if (!moved) break;
  }
  if (!(fabs(r[0]) + fabs(r[1]) < 1e-9)) return false;
  *a = exp(t[0]);
  *s = exp(t[1]);
  return true;
}

// (a, s) with gauss_flux = (fbar_t, sigf_t), from (0.3, 0.5).
bool fit_a_s(double fbar_t, double sigf_t, double* a, double* s) {
  *a = 0.3;
  *s = 0.5;
  return newton2(
      [&](const double* u, double* r) {
        double f1, sf;
        gauss_flux(exp(u[0]), exp(u[1]), &f1, &sf);
        if (!(f1 > 0.0) || !(sf > 0.0)) return false;
        r[0] = log(f1 / fbar_t);
        r[1] = log(sf / sigf_t);
        return true;
      },
      a, s);
}

// (a, s) with Fbar = fbar_t and the effective bias = beff_t at sigma_g, from
// the given (a, s); false when no solution is found (a target beyond the
// bias the step limit allows).
bool fit_a_s_bias(double fbar_t, double beff_t, double sigma_g, double beta, double* a, double* s) {
  return newton2(
      [&](const double* u, double* r) {
        double f1;
        const double be = effective_bias(exp(u[0]), exp(u[1]), sigma_g, beta, &f1);
        if (!(f1 > 0.0) || !(be > 0.0) || !isfinite(be)) return false;
        r[0] = log(f1 / fbar_t);
        r[1] = log(be / beff_t);
        return true;
      },
      a, s);
}

// d(ln a, ln s)/d ln sigma_g along the solutions of fit_a_s_bias at (a, s):
// the effective bias goes as 1/sigma_g, so with J the Jacobian of (ln Fbar,
// ln b_eff) in (ln a, ln s) the slope is J^-1 (0, 1) (implicit functions).
bool bias_slope(double a, double s, double sigma_g, double beta, double* dla, double* dls) {
  double J[2][2];
  const double h = 1e-5;
  for (int k = 0; k < 2; ++k) {
    double r[2][2];
    for (int sg = 0; sg < 2; ++sg) {
      const double d = sg ? -h : h;
      const double aa = k == 0 ? a * exp(d) : a, sa = k == 1 ? s * exp(d) : s;
      double f1;
      const double be = effective_bias(aa, sa, sigma_g, beta, &f1);
      if (!(f1 > 0.0) || !(be > 0.0)) return false;
      r[sg][0] = log(f1);
      r[sg][1] = log(be);
    }
    J[0][k] = (r[0][0] - r[1][0]) / (2.0 * h);
    J[1][k] = (r[0][1] - r[1][1]) / (2.0 * h);
  }
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  if (!(fabs(det) > 1e-300)) return false;
  *dla = -J[0][1] / det;
  *dls = J[0][0] / det;
  return true;
}

// sigma_s^2 of P_s = amp exp(-(k/kcut)^2) on a line of pixel length dpix:
// (1/pi) int_0^{pi/dpix} P_s dk = amp kcut erf(pi/(dpix kcut)) / (2 sqrt(pi))
double sigma_s2_gauss(double amp, double kcut, double dpix) {
  return amp * kcut * erf(M_PI / (dpix * kcut)) / (2.0 * sqrt(M_PI));
}

// (1/pi) int_0^{pi/dpix} amp exp(-(k/kcut)^2) r(k) dk, r piecewise constant
// on the edges (h/Mpc), clamped at both ends.
double sigma_s2(double amp, double kcut, const double* ratio, const double* edges, int nk, double dpix) {
  const double kmax = M_PI / dpix;
  auto prim = [&](double k) { return amp * kcut * sqrt(M_PI) * 0.5 * erf(k / kcut); };
  double tot = 0.0, lo = 0.0;
  for (int p = 0; p <= nk + 1; ++p) {
    double hi = p <= nk ? edges[p] : kmax;
    hi = hi < 0.0 ? 0.0 : (hi > kmax ? kmax : hi);
    const double r = p == 0 ? ratio[0] : (p <= nk ? ratio[p - 1] : ratio[nk - 1]);
    if (hi > lo) tot += r * (prim(hi) - prim(lo));
    if (hi > lo) lo = hi;
  }
  return tot / M_PI;
}

}  // namespace
}  // namespace lya

namespace {
thread_local char g_perr[256] = "";
int pfail(int code, const char* msg) {
  snprintf(g_perr, sizeof(g_perr), "%s", msg);
  return code;
}
int phip(hipError_t e, const char* where) {
  snprintf(g_perr, sizeof(g_perr), "%s: %s", where, hipGetErrorString(e));
  return LYA_EHIP;
}
}  // namespace

extern "C" {

const char* lya_tune_ps_last_error(void) { return g_perr; }

size_t lya_tune_ps_workspace_size(int64_t n_sk, int64_t n_pixels, int32_t n_kbins) {
  if (n_sk < 0 || n_pixels < 0 || n_kbins < 1 || n_kbins > lya::kMaxKBins) return 0;
  return lya::carve_ps(n_sk, n_pixels, n_kbins).total;
}

int lya_tune_ps(const lya_tune_ps_spec* spec, lya_tune_ps_result* res, void* work, size_t work_bytes,
                void* stream) {
  using namespace lya;
  g_perr[0] = 0;
  const auto t_start = std::chrono::steady_clock::now();
  if (!spec || !res || !spec->sk) return pfail(LYA_EINVAL, "spec, result or skewers is NULL");
  const lya_skewers* sk = spec->sk;
  const int nk = spec->p1d.n_kbins;
  if (spec->n_zt < 1 || spec->n_zt > LYA_TUNE_MAX_Z) return pfail(LYA_EINVAL, "n_zt must be in [1, 16]");
  if (nk < 1 || nk > kMaxKBins || !spec->p1d.k_edges || !spec->p1d_t)
    return pfail(LYA_EINVAL, "P1D bins (1..64 with edges) and targets are required");
  if (spec->n_iter < 1 || spec->n_iter > LYA_TUNE_PS_MAX_ITER) return pfail(LYA_EINVAL, "n_iter must be in [1, 16]");
  if (spec->n_outer < 0 || spec->n_outer > LYA_TUNE_PS_MAX_OUTER) return pfail(LYA_EINVAL, "n_outer must be in [0, 8]");
  if (spec->mode != LYA_TUNE_PS_RATIOS && spec->mode != LYA_TUNE_PS_EMULATOR)
    return pfail(LYA_EINVAL, "mode must be LYA_TUNE_PS_RATIOS or LYA_TUNE_PS_EMULATOR");
  const bool emu_mode = spec->mode == LYA_TUNE_PS_EMULATOR;
  if (spec->update != LYA_PS_UPDATE_PAPER && spec->update != LYA_PS_UPDATE_SECANT)
    return pfail(LYA_EINVAL, "update must be LYA_PS_UPDATE_PAPER or LYA_PS_UPDATE_SECANT");
  const bool secant = spec->update == LYA_PS_UPDATE_SECANT;
  if (emu_mode) {
    if (spec->emu_checks < 1 || spec->emu_checks > 16) return pfail(LYA_EINVAL, "emu_checks must be in [1, 16]");
    if (spec->emu_refine < 0 || spec->emu_refine > LYA_TUNE_PS_MAX_ITER)
      return pfail(LYA_EINVAL, "emu_refine must be in [0, 16]");
    for (int z = 0; z < spec->n_zt; ++z)
      if (!spec->emu[z]) return pfail(LYA_EINVAL, "emulator mode needs an emulator at every z_t");
  }
  const int n_outer = spec->n_outer < 1 ? 1 : spec->n_outer;
  if (n_outer > 1) {
    if (!(spec->f > 0.0)) return pfail(LYA_EINVAL, "the outer loop needs f > 0");
    for (int z = 0; z < spec->n_zt; ++z)
      if (!(spec->beff_t[z] > 0.0)) return pfail(LYA_EINVAL, "the outer loop needs beff_t > 0 at every z_t");
  }
  if (!(spec->ps_amp > 0.0) || !(spec->ps_kcut > 0.0) || !(spec->p1d.dpix > 0.0))
    return pfail(LYA_EINVAL, "P_s^0 amplitude, cut-off and dpix must be positive");
  if (sk->n_sk < 1 || !sk->npix || !sk->offset || !sk->chi0 || !spec->dens_l || !spec->eta)
    return pfail(LYA_EINVAL, "stored pixels and their skewer table are required");
  if (!(spec->cosmo.omega_m >= 0.0 && spec->cosmo.omega_m <= 1.0)) return pfail(LYA_EINVAL, "omega_m out of [0,1]");
  if (!work) return pfail(LYA_EINVAL, "work is NULL");
  const PsCarve c = carve_ps(sk->n_sk, spec->n_pixels, nk);
  if (spec->n_pixels < 1 || work_bytes < c.total) return pfail(LYA_EWORKSPACE, "workspace too small (or n_pixels < 1)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(work);
  float* flux = reinterpret_cast<float*>(w + c.flux);
  float* d_ratio = reinterpret_cast<float*>(w + c.ratio);
  double* d_edges = reinterpret_cast<double*>(w + c.edges);
  double* d_zb = reinterpret_cast<double*>(w + c.zb);
  double* d_psum = reinterpret_cast<double*>(w + c.psum);
  int64_t* d_pcnt = reinterpret_cast<int64_t*>(w + c.pcnt);
  double* d_part = reinterpret_cast<double*>(w + c.part);
  double* d_mom = reinterpret_cast<double*>(w + c.mom);
  memset(res, 0, sizeof(*res));

  hipError_t e;
  if (emu_mode) {  // each emulator must predict (Fbar, P_1..P_nk)
    for (int z = 0; z < spec->n_zt; ++z) {
      int32_t n_out = 0;
      if ((e = hipMemcpyAsync(&n_out, spec->emu[z], sizeof(n_out), hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return phip(e, "reading an emulator header");
      if (n_out != 1 + nk) return pfail(LYA_EINVAL, "an emulator's outputs are not 1 + n_kbins");
    }
    if ((e = tune_eval_prepare(w + c.te, st)) != hipSuccess) return phip(e, "evaluation set-up");
  }

  // moments of the stored pixels
  hipLaunchKernelGGL(k_moments, dim3(kMomBlocks), dim3(kMomNT), 0, st, sk->n_sk, sk->npix, sk->offset, spec->dens_l,
                     spec->eta, d_part);
  hipLaunchKernelGGL(k_moments_reduce, dim3(5), dim3(kMomBlocks), 0, st, d_part, d_mom);
  e = hipGetLastError();
  if (e != hipSuccess) return phip(e, "moments");
  double mom[5];
  std::vector<int32_t> npix(sk->n_sk);
  if ((e = hipMemcpyAsync(mom, d_mom, sizeof(mom), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(npix.data(), sk->npix, sizeof(int32_t) * sk->n_sk, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return phip(e, "moments read-back");
  double n_tot = 0.0;
  for (int32_t v : npix) n_tot += v;
  if (!(n_tot > 0.0)) return pfail(LYA_EINVAL, "no stored pixels");
  const double ml = mom[0] / n_tot, me = mom[1] / n_tot;
  const double sl2 = mom[2] / n_tot - ml * ml, se2 = mom[3] / n_tot - me * me, cov = mom[4] / n_tot - ml * me;
  res->sigma2[0] = sl2;
  res->sigma2[1] = se2;
  res->sigma2[2] = cov;

  std::vector<double> kv(nk + 1);
  if ((e = hipMemcpyAsync(kv.data(), spec->p1d.k_edges, sizeof(double) * (nk + 1), hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return phip(e, "k edges read-back");
  const double zb_edges[2] = {-1e30, 1e30};
  lya_zbins zb{1, d_zb, d_zb + 2, reinterpret_cast<int64_t*>(d_zb + 3)};
  lya_ps_table tab{nk, d_edges, d_ratio};
  const double dpix = spec->p1d.dpix;

  for (int z = 0; z < spec->n_zt; ++z) {
    const double zt = spec->z_t[z], ct = spec->c_t[z], ft = spec->fbar_t[z];
    const double* pt = spec->p1d_t + static_cast<size_t>(z) * nk;
    if (!(ft > 0.0 && ft < 1.0)) return pfail(LYA_EINVAL, "target mean flux must lie in (0, 1)");
    double sigf = spec->sigf_t[z];
    if (!(sigf > 0.0)) {
      double v = 0.0;
      for (int b = 0; b < nk; ++b)
        if (isfinite(pt[b])) v += pt[b] * (kv[b + 1] - kv[b]);
      sigf = ft * sqrt(v / M_PI);
    }
    double a0 = 0.0, s0 = 0.0;
    if (!(sigf > 0.0) || !fit_a_s(ft, sigf, &a0, &s0))
      return pfail(LYA_EINVAL, "no (a, b sigma_g) reaches the target mean flux and dispersion");
    const double opz = 1.0 + zt;
    const double E = sqrt(spec->cosmo.omega_m * opz * opz * opz + 1.0 - spec->cosmo.omega_m);
    const double dvdchi = 100.0 * E / opz;
    std::vector<double> ek(nk + 1);
    for (int b = 0; b <= nk; ++b) ek[b] = kv[b] * dvdchi;
    const double beta = spec->f * ct;
    // the bias target with respect to the z = 0 box the pixels come from
    res->growth[z] = spec->beff_at_z ? growth_lcdm(zt, spec->cosmo.omega_m) : 1.0;
    const double beff_box = spec->beff_t[z] * res->growth[z];
    const double sig0 = sl2 + ct * ct * se2 + 2.0 * ct * cov;  // sigma_g^2 without delta_S
    auto rel_rms = [&](const double* p) {
      double se = 0.0;
      int ne = 0;
      for (int b = 0; b < nk; ++b)
        if (isfinite(pt[b]) && isfinite(p[b]) && pt[b] != 0.0) {
          se += (p[b] / pt[b] - 1.0) * (p[b] / pt[b] - 1.0);
          ++ne;
        }
      return ne ? sqrt(se / ne) : NAN;
    };

    // ---- the paper's iteration: P_s = psA exp(-(k/psK)^2) r(bin of k), r
    // multiplied per k bin by P_target / P1D, n_it iterations per outer step
    // from (a, s); outer steps after the first re-solve (a, s) for Fbar and
    // the target effective bias at the sigma_g of the current ratios
    auto run_plain = [&](double psA, double psK, double a, double s, int n_out, int n_it, bool outer_fit) -> int {
      std::vector<double> ratio(nk, 1.0);
      std::vector<float> ratio32(nk);
      std::vector<double> psum(nk);
      std::vector<int64_t> pcnt(nk);
      const lya_ps1d psl{psA, psK, dpix, 0};
      double fbar = 0.0, b_used = 0.0;
      int done = 0;
      // the secant update's previous iteration of this run, per bin (NaN: none)
      std::vector<double> prev_r(nk), prev_p(nk);
      for (int o = 0; o < n_out; ++o) {
        std::fill(prev_p.begin(), prev_p.end(), NAN);
        if (o > 0 && outer_fit) {
          const double ss2 = sigma_s2(psA, psK, ratio.data(), ek.data(), nk, dpix);
          const double sg2 = sig0 + ss2;
          double a2 = a, s2 = s;
          if (!(sg2 > 0.0) || !fit_a_s_bias(ft, beff_box, sqrt(sg2), beta, &a2, &s2)) break;
          a = a2;
          s = s2;
        }
        for (int it = 0; it < n_it; ++it) {
          const double ss2 = sigma_s2(psA, psK, ratio.data(), ek.data(), nk, dpix);
          const double sg2 = sig0 + ss2;
          if (!(sg2 > 0.0)) return pfail(LYA_EINVAL, "sigma_g^2 is not positive");
          b_used = s / sqrt(sg2);
          for (int b = 0; b < nk; ++b) ratio32[b] = static_cast<float>(ratio[b]);
          if ((e = hipMemcpyAsync(d_ratio, ratio32.data(), sizeof(float) * nk, hipMemcpyHostToDevice, st)) !=
                  hipSuccess ||
              (e = hipMemcpyAsync(d_edges, ek.data(), sizeof(double) * (nk + 1), hipMemcpyHostToDevice, st)) !=
                  hipSuccess ||
              (e = hipMemcpyAsync(d_zb, zb_edges, sizeof(zb_edges), hipMemcpyHostToDevice, st)) != hipSuccess)
            return phip(e, "table upload");
          lya_fgpa fg{};
          fg.coef[0][0] = a;
          fg.coef[1][0] = b_used;
          fg.coef[2][0] = ct;
          int rc = lya_apply_fgpa_ds(sk, &spec->cosmo, spec->dens_l, spec->eta, &psl, &tab, spec->seed, &fg, flux,
                                     &zb, w + c.sk, c.p1d - c.sk, stream);
          if (rc != LYA_OK) {
            snprintf(g_perr, sizeof(g_perr), "lya_apply_fgpa_ds: %s", lya_last_error());
            return rc;
          }
          lya_p1d_spec pspec = spec->p1d;
          pspec.z_ref = zt;
          rc = lya_p1d(sk, &spec->cosmo, flux, &zb, &pspec, d_psum, d_pcnt, w + c.p1d, c.flux - c.p1d, stream);
          if (rc != LYA_OK) {
            snprintf(g_perr, sizeof(g_perr), "lya_p1d: %s", lya_last_error());
            return rc;
          }
          double zsum[2];
          if ((e = hipMemcpyAsync(zsum, d_zb + 2, sizeof(zsum), hipMemcpyDeviceToHost, st)) != hipSuccess ||
              (e = hipMemcpyAsync(psum.data(), d_psum, sizeof(double) * nk, hipMemcpyDeviceToHost, st)) !=
                  hipSuccess ||
              (e = hipMemcpyAsync(pcnt.data(), d_pcnt, sizeof(int64_t) * nk, hipMemcpyDeviceToHost, st)) !=
                  hipSuccess ||
              (e = hipStreamSynchronize(st)) != hipSuccess)
            return phip(e, "statistics read-back");
          ++res->gpu_evals[z];
          int64_t count;
          memcpy(&count, &zsum[1], sizeof(count));
          fbar = count > 0 ? zsum[0] / static_cast<double>(count) : NAN;
          for (int b = 0; b < nk; ++b) {
            res->p1d[z * 64 + b] = pcnt[b] > 0 ? psum[b] / static_cast<double>(pcnt[b]) : NAN;
            res->ratio[z * 64 + b] = ratio[b];
          }
          res->fbar[z * LYA_TUNE_PS_MAX_ITER + it] = fbar;
          res->rms[z * LYA_TUNE_PS_MAX_ITER + it] = rel_rms(res->p1d + z * 64);
          // P_s^{n+1} = P_s^n (P_target / P1D)^w in every bin with both
          // values: w = 1 (the paper's rule), or with the secant update w =
          // 1/gamma clipped to [1, 3], gamma = d ln P1D / d ln r from the last
          // two iterations of this run (w = 1 where it is undefined)
          for (int b = 0; b < nk; ++b) {
            const double p = res->p1d[z * 64 + b];
            const double r = ratio[b];
            if (isfinite(pt[b]) && isfinite(p) && p > 0.0) {
              double w = 1.0;
              if (secant && isfinite(prev_p[b]) && prev_p[b] > 0.0) {
                const double dr = log(r) - log(prev_r[b]);
                if (fabs(dr) > 1e-6) {
                  const double gam = (log(p) - log(prev_p[b])) / dr;
                  if (gam > 0.05) w = fmin(fmax(1.0 / gam, 1.0), 3.0);
                }
              }
              ratio[b] = w == 1.0 ? r * (pt[b] / p) : r * pow(pt[b] / p, w);
            }
            prev_r[b] = r;
            prev_p[b] = p;
          }
        }
        res->beff[z * LYA_TUNE_PS_MAX_OUTER + o] = effective_bias(a, s, s / b_used, beta, nullptr);
        done = o + 1;
      }
      res->n_outer_done[z] = done;
      res->a[z] = a;
      res->b[z] = b_used;
      res->s[z] = s;
      return LYA_OK;
    };

    // ---- emulator mode: (amp, kcut) of P_s by a corrected emulator search
    bool plain = !emu_mode;
    if (emu_mode) {
      const bool outer = n_outer > 1;
      const int checks = spec->emu_checks;
      const double xtol = 5e-4;
      double th[2] = {log(spec->ps_amp), log(spec->ps_kcut)};
      double off[kMaxKBins + 1] = {0.0}, jac[2 * (kMaxKBins + 1)] = {0.0}, dprev[kMaxKBins + 1] = {0.0};
      double xk[2] = {th[0], th[1]};
      double a = a0, s = s0, step = 0.3;
      bool converged = false, ok = true;
      double rms_prev = HUGE_VAL;
      int gpu_ev = 0;
      double rows[kMaxKBins + 1];
      // (a, s) and their slope in ln sigma_g at the sigma_g of th
      auto solve_as = [&](const double* t, double* la, double* ls, double* dla, double* dls, double* lsg) {
        const double sg = sqrt(sig0 + sigma_s2_gauss(exp(t[0]), exp(t[1]), dpix));
        if (!(sg > 0.0)) return false;
        *lsg = log(sg);
        if (outer) {
          if (!fit_a_s_bias(ft, beff_box, sg, beta, &a, &s) || !bias_slope(a, s, sg, beta, dla, dls)) return false;
        } else {
          *dla = *dls = 0.0;
        }
        *la = log(a);
        *ls = log(s);
        return true;
      };
      double lin[5];
      ok = solve_as(th, &lin[0], &lin[1], &lin[2], &lin[3], &lin[4]);
      for (int it = 0; ok && it < checks; ++it) {
        EmuSearchSpec ss{ft, ct, zt, step, 0.01 * xtol, HUGE_VAL, 0.002, nk, 600, pt, off, jac, {xk[0], xk[1]}};
        ss.ps = 1;
        ss.sig0 = sig0;
        ss.dpix = dpix;
        for (int i = 0; i < 5; ++i) ss.lin[i] = lin[i];
        double x[2] = {th[0], th[1]}, fbest = 0.0, pe[kMaxKBins + 1];
        int n1 = 0;
        if ((e = emulator_search(spec->emu[z], ss, x, &fbest, &n1, pe, tune_eval_scratch(w + c.te, sk->n_sk, nk),
                                 st)) != hipSuccess)
          return phip(e, "emulator search");
        // the exact (a, s) at the new point, then one GPU evaluation there
        if (!solve_as(x, &lin[0], &lin[1], &lin[2], &lin[3], &lin[4])) {
          ok = false;
          break;
        }
        DsSource src{sk->n_sk, sk->id_base, sk->npix, sk->offset, spec->dens_l, spec->eta, spec->p1d.k_edges, nk,
                     dpix, spec->cosmo.omega_m, spec->seed};
        DsDraw dd{a, s / exp(lin[4]), ct, zt, exp(x[0]), exp(x[1])};
        if ((e = tune_eval_ds(src, w + c.te, &dd, 1, rows, nullptr, st)) != hipSuccess) return phip(e, "evaluation");
        ++gpu_ev;
        double d[kMaxKBins + 1];
        for (int j = 0; j <= nk; ++j) d[j] = rows[j] - pe[j];
        const double dx0 = xk[0] - x[0], dx1 = xk[1] - x[1], dxx = dx0 * dx0 + dx1 * dx1;
        if (it > 0 && dxx > 1e-24) {
          for (int j = 0; j <= nk; ++j) {
            if (!isfinite(d[j]) || !isfinite(dprev[j])) {
              jac[2 * j] = jac[2 * j + 1] = 0.0;
              continue;
            }
            const double r = (dprev[j] - d[j]) - (jac[2 * j] * dx0 + jac[2 * j + 1] * dx1);
            jac[2 * j] += r * dx0 / dxx;
            jac[2 * j + 1] += r * dx1 / dxx;
          }
        }
        const double moved = fmax(fabs(dx0), fabs(dx1));
        for (int j = 0; j <= nk; ++j) off[j] = dprev[j] = d[j];
        xk[0] = th[0] = x[0];
        xk[1] = th[1] = x[1];
        step = 0.05;
        // settled: the point no longer moves, or it moves a little along a
        // valley (amp and kcut trade against each other through sigma_s)
        // without changing the measured P1D error
        const double rms_now = rel_rms(rows + 1);
        if (it > 0 && (moved <= xtol || (moved <= 0.05 && fabs(rms_now - rms_prev) <= 1e-3 * rms_now))) {
          converged = true;
          break;
        }
        rms_prev = rms_now;
      }
      res->gpu_evals[z] = gpu_ev;
      if (ok && converged) {
        const double sg = exp(lin[4]), amp = exp(th[0]), kc = exp(th[1]);
        res->a[z] = a;
        res->b[z] = s / sg;
        res->s[z] = s;
        res->ps_fit[2 * z] = amp;
        res->ps_fit[2 * z + 1] = kc;
        for (int b = 0; b < nk; ++b) {
          res->p1d[z * 64 + b] = rows[1 + b];
          const double kc_b = sqrt(ek[b] * ek[b + 1]);
          res->ratio[z * 64 + b] =
              (amp * exp(-(kc_b / kc) * (kc_b / kc))) / (spec->ps_amp * exp(-(kc_b / spec->ps_kcut) * (kc_b / spec->ps_kcut)));
        }
        res->fbar[z * LYA_TUNE_PS_MAX_ITER] = rows[0];
        res->rms[z * LYA_TUNE_PS_MAX_ITER] = rel_rms(rows + 1);
        res->beff[z * LYA_TUNE_PS_MAX_OUTER] = effective_bias(a, s, sg, beta, nullptr);
        res->n_outer_done[z] = 1;
        // the paper's per-bin update on top of the fitted form, at the fit's (a, s)
        if (spec->emu_refine > 0)
          if (int rc = run_plain(amp, kc, a, s, 1, spec->emu_refine, false)) return rc;
        continue;
      }
      // not settled within emu_checks GPU evaluations (or no (a, s) for the
      // targets along the way): the plain iteration runs instead
      res->fallback[z] = 1;
      plain = true;
    }
    if (!plain) continue;
    if (int rc = run_plain(spec->ps_amp, spec->ps_kcut, a0, s0, n_outer, spec->n_iter, true)) return rc;
  }
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return LYA_OK;
}

int lya_emulator_labels_ps(const lya_tune_ps_spec* spec, int32_t zi, const double* draws, int64_t n, float* y,
                           void* work, size_t work_bytes, void* stream) {
  using namespace lya;
  g_perr[0] = 0;
  if (!spec || !spec->sk || !draws || !y || !work || n < 0) return pfail(LYA_EINVAL, "NULL argument or n < 0");
  const lya_skewers* sk = spec->sk;
  const int nk = spec->p1d.n_kbins;
  if (zi < 0 || zi >= spec->n_zt || spec->n_zt > LYA_TUNE_MAX_Z) return pfail(LYA_EINVAL, "zi outside the z_t list");
  if (nk < 1 || nk > kMaxKBins || !spec->p1d.k_edges) return pfail(LYA_EINVAL, "P1D bins (1..64 with edges) required");
  if (!(spec->p1d.dpix > 0.0)) return pfail(LYA_EINVAL, "dpix must be positive");
  if (sk->n_sk < 1 || !sk->npix || !sk->offset || !spec->dens_l || !spec->eta)
    return pfail(LYA_EINVAL, "stored pixels and their skewer table are required");
  if (!(spec->cosmo.omega_m >= 0.0 && spec->cosmo.omega_m <= 1.0)) return pfail(LYA_EINVAL, "omega_m out of [0,1]");
  for (int64_t i = 0; i < n; ++i)
    if (!(draws[4 * i + 2] > 0.0) || !(draws[4 * i + 3] > 0.0))
      return pfail(LYA_EINVAL, "P_s amplitude and cut-off of every draw must be positive");
  const PsCarve c = carve_ps(sk->n_sk, spec->n_pixels, nk);
  if (work_bytes < c.total) return pfail(LYA_EWORKSPACE, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(work) + c.te;
  hipError_t e = tune_eval_prepare(w, st);
  const DsSource src{sk->n_sk, sk->id_base, sk->npix, sk->offset, spec->dens_l, spec->eta, spec->p1d.k_edges, nk,
                     spec->p1d.dpix, spec->cosmo.omega_m, spec->seed};
  for (int64_t i0 = 0; i0 < n && e == hipSuccess; i0 += kTuneEvalMaxG) {
    const int G = static_cast<int>(n - i0 < kTuneEvalMaxG ? n - i0 : kTuneEvalMaxG);
    DsDraw dd[kTuneEvalMaxG];
    for (int g = 0; g < G; ++g) {
      const double* d = draws + 4 * (i0 + g);
      dd[g] = DsDraw{d[0], d[1], spec->c_t[zi], spec->z_t[zi], d[2], d[3]};
    }
    e = tune_eval_ds(src, w, dd, G, nullptr, y + i0 * (1 + nk), st);
  }
  if (e != hipSuccess) return phip(e, "label evaluation");
  return LYA_OK;
}

}  // extern "C"
