// FGPA parameter tuning (section "Adjusting mock parameters"): host-side FP64
// Nelder-Mead over (ln a, ln b) at each tuning redshift z_t with c fixed,
// driving GPU evaluations (k_tune_eval.hip) of the mean flux and the 1D power
// of the stored pre-FGPA pixels under constant (a, b, c) (the paper's
// post-production reuse of saved forests), then least-squares quadratics in
// (1+z).  The emulator
// mode runs the same search on the MLP's predictions, checks the optimum on the
// GPU and corrects the prediction by the measured defect before searching
// again (a few GPU evaluations per redshift instead of one per search step).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>

#include "../../include/lyamock.h"
#include "lya_internal.h"
#include "lya_nm.h"

namespace lya {

namespace {

size_t al256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct TuneCarve {
  size_t tw, queue, fs, ps, pc, sums, counts, rows, emu, total;
};

// workspace of the batched evaluation: per-skewer partials for up to
// kTuneEvalMaxG draws, the reductions, the statistics rows
TuneCarve carve_tune(int64_t n_sk, int nk) {
  TuneCarve c{};
  const size_t G = kTuneEvalMaxG, S = static_cast<size_t>(n_sk > 0 ? n_sk : 1);
  size_t o = 0;
  c.tw = o;     o += al256(sizeof(float2) * kTw2048);
  c.queue = o;  o += 256;
  c.fs = o;     o += al256(sizeof(double) * G * S);
  c.ps = o;     o += al256(sizeof(double) * G * nk * S);
  c.pc = o;     o += al256(sizeof(int) * G * nk * S);
  c.sums = o;   o += al256(sizeof(double) * G * (nk + 1));
  c.counts = o; o += al256(sizeof(int64_t) * G * (nk + 1));
  c.rows = o;   o += al256(sizeof(double) * G * (nk + 1));
  c.emu = o;    o += al256(emulator_eval_bytes());
  c.total = o;
  return c;
}

TuneEvalArgs eval_args(const lya_tune_spec* spec, char* w, const TuneCarve& c) {
  TuneEvalArgs a{};
  const lya_skewers* sk = spec->sk;
  a.n_sk = sk->n_sk;
  a.npix = sk->npix;
  a.offset = sk->offset;
  a.dens = spec->dens;
  a.eta = spec->eta;
  a.nk = spec->p1d.n_kbins;
  a.k_edges = spec->p1d.k_edges;
  a.fs = reinterpret_cast<double*>(w + c.fs);
  a.ps = reinterpret_cast<double*>(w + c.ps);
  a.pc = reinterpret_cast<int*>(w + c.pc);
  a.tw2048 = reinterpret_cast<const float2*>(w + c.tw);
  a.queue = reinterpret_cast<unsigned int*>(w + c.queue);
  a.chunk = 4;
  return a;
}

// velocity pixel in km/s at redshift z: dpix 100 E(z)/(1+z)
double velocity_pixel_at(const lya_tune_spec* spec, double z) {
  const double x = 1.0 + z, om = spec->cosmo.omega_m;
  return spec->p1d.dpix * (100.0 * sqrt(om * (x * x * x) + (1.0 - om)) / x);
}

struct Evaluator {
  const lya_tune_spec* spec;
  char* w;
  TuneCarve c;
  hipStream_t st;
  int nk;

  // Mean flux and mean P1D per bin of the stored pixels under constant (a, b, c).
  hipError_t eval(double a, double b, double cc, double z, double* fbar, double* pk) {
    TuneEvalArgs ea = eval_args(spec, w, c);
    ea.G = 1;
    ea.draw[0][0] = static_cast<float>(a);
    ea.draw[0][1] = static_cast<float>(b);
    ea.draw[0][2] = static_cast<float>(cc);
    ea.dv[0] = velocity_pixel_at(spec, z);
    hipError_t e = launch_tune_eval(ea, reinterpret_cast<double*>(w + c.sums), reinterpret_cast<int64_t*>(w + c.counts),
                                    reinterpret_cast<double*>(w + c.rows), nullptr, st);
    if (e != hipSuccess) return e;
    double h[kMaxKBins + 1];
    if ((e = hipMemcpyAsync(h, w + c.rows, sizeof(double) * (nk + 1), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *fbar = h[0];
    for (int i = 0; i < nk; ++i) pk[i] = h[1 + i];
    return hipSuccess;
  }
};

// least squares y = p0 + p1 x + p2 x^2 through (x_i, y_i), normal equations in FP64
void quad_fit(const double* x, const double* y, int n, double out[3]) {
  double A[3][4] = {{0}};
  for (int i = 0; i < n; ++i) {
    const double p[3] = {1.0, x[i], x[i] * x[i]};
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) A[r][k] += p[r] * p[k];
      A[r][3] += p[r] * y[i];
    }
  }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r) if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    for (int k = 0; k < 4; ++k) { const double t = A[col][k]; A[col][k] = A[piv][k]; A[piv][k] = t; }
    if (A[col][col] == 0.0) { out[0] = out[1] = out[2] = NAN; return; }
    for (int r = 0; r < 3; ++r) {
      if (r == col) continue;
      const double fct = A[r][col] / A[col][col];
      for (int k = col; k < 4; ++k) A[r][k] -= fct * A[col][k];
    }
  }
  for (int r = 0; r < 3; ++r) out[r] = A[r][3] / A[r][r];
}


}  // namespace

size_t tune_workspace_bytes(int64_t n_sk, int nk) { return carve_tune(n_sk, nk).total; }

hipError_t tune_eval_prepare(char* w, hipStream_t st) {
  return launch_twiddles(reinterpret_cast<float2*>(w + carve_tune(1, 1).tw), kTw2048, st);
}

char* tune_eval_scratch(char* w, int64_t n_sk, int nk) { return w + carve_tune(n_sk, nk).emu; }

hipError_t tune_eval_ds(const DsSource& src, char* w, const DsDraw* d, int G, double* rows_host, float* rows32,
                        hipStream_t st) {
  const TuneCarve c = carve_tune(src.n_sk, src.nk);
  TuneEvalArgs a{};
  a.n_sk = src.n_sk;
  a.npix = src.npix;
  a.offset = src.offset;
  a.dens = src.dens;
  a.eta = src.eta;
  a.nk = src.nk;
  a.k_edges = src.k_edges;
  a.fs = reinterpret_cast<double*>(w + c.fs);
  a.ps = reinterpret_cast<double*>(w + c.ps);
  a.pc = reinterpret_cast<int*>(w + c.pc);
  a.tw2048 = reinterpret_cast<const float2*>(w + c.tw);
  a.queue = reinterpret_cast<unsigned int*>(w + c.queue);
  a.chunk = 4;
  a.with_ds = 1;
  a.dpix = src.dpix;
  a.seed = src.seed;
  a.id_base = src.id_base;
  a.G = G;
  for (int g = 0; g < G; ++g) {
    a.draw[g][0] = static_cast<float>(d[g].a);
    a.draw[g][1] = static_cast<float>(d[g].b);
    a.draw[g][2] = static_cast<float>(d[g].c);
    a.ds_amp[g] = d[g].amp;
    a.ds_kcut[g] = d[g].kcut;
    const double x = 1.0 + d[g].z, om = src.omega_m;
    a.dv[g] = src.dpix * (100.0 * sqrt(om * (x * x * x) + (1.0 - om)) / x);
  }
  double* rows = reinterpret_cast<double*>(w + c.rows);
  hipError_t e = launch_tune_eval(a, reinterpret_cast<double*>(w + c.sums), reinterpret_cast<int64_t*>(w + c.counts),
                                  rows, rows32, st);
  if (e != hipSuccess || !rows_host) return e;
  if ((e = hipMemcpyAsync(rows_host, rows, sizeof(double) * G * (src.nk + 1), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return e;
  return hipStreamSynchronize(st);
}

// Emulator training labels: for each host draw (a, b, c, z) the mean flux and
// mean P1D per bin (velocity units at z) of the stored pixels, written to
// y[i][0] and y[i][1 + b] on the device, kTuneEvalMaxG draws per pass over
// the pixels; no host synchronisation per draw.
int emulator_labels(const lya_tune_spec* spec, const double* draws, int64_t n, float* y, void* work, size_t work_bytes,
                    hipStream_t st, char* err, size_t errlen) {
  const int nk = spec->p1d.n_kbins;
  const TuneCarve c = carve_tune(spec->sk->n_sk, nk);
  if (work_bytes < c.total) {
    snprintf(err, errlen, "workspace too small for labels");
    return LYA_EWORKSPACE;
  }
  char* w = static_cast<char*>(work);
  hipError_t e = launch_twiddles(reinterpret_cast<float2*>(w + c.tw), kTw2048, st);
  for (int64_t i0 = 0; i0 < n && e == hipSuccess; i0 += kTuneEvalMaxG) {
    TuneEvalArgs ea = eval_args(spec, w, c);
    ea.G = static_cast<int>(n - i0 < kTuneEvalMaxG ? n - i0 : kTuneEvalMaxG);
    for (int g = 0; g < ea.G; ++g) {
      const double* d = draws + 4 * (i0 + g);
      ea.draw[g][0] = static_cast<float>(d[0]);
      ea.draw[g][1] = static_cast<float>(d[1]);
      ea.draw[g][2] = static_cast<float>(d[2]);
      ea.dv[g] = velocity_pixel_at(spec, d[3]);
    }
    e = launch_tune_eval(ea, reinterpret_cast<double*>(w + c.sums), reinterpret_cast<int64_t*>(w + c.counts),
                         nullptr, y + i0 * (1 + nk), st);
  }
  if (e != hipSuccess) {
    snprintf(err, errlen, "label evaluation: %s", hipGetErrorString(e));
    return LYA_EHIP;
  }
  return LYA_OK;
}

int tune_params(const lya_tune_spec* spec, lya_tune_result* res, int mode, void* work, size_t work_bytes,
                hipStream_t st, char* err, size_t errlen) {
  const auto t0 = std::chrono::steady_clock::now();
  const int nk = spec->p1d.n_kbins;
  const TuneCarve c = carve_tune(spec->sk->n_sk, nk);
  if (work_bytes < c.total) {
    snprintf(err, errlen, "workspace too small for tuning");
    return LYA_EWORKSPACE;
  }
  char* w = static_cast<char*>(work);
  Evaluator ev{spec, w, c, st, nk};
  hipError_t e;
  if ((e = launch_twiddles(reinterpret_cast<float2*>(w + c.tw), kTw2048, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    snprintf(err, errlen, "tuning set-up: %s", hipGetErrorString(e));
    return LYA_EHIP;
  }
  if (mode == LYA_TUNE_EMULATOR) {  // the emulator must predict (Fbar, P_1..P_nk)
    int32_t n_out = 0;
    if ((e = hipMemcpyAsync(&n_out, spec->emulator, sizeof(n_out), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      snprintf(err, errlen, "reading the emulator header: %s", hipGetErrorString(e));
      return LYA_EHIP;
    }
    if (n_out != 1 + nk) {
      snprintf(err, errlen, "emulator has %d outputs, tuning needs 1 + n_kbins = %d", n_out, 1 + nk);
      return LYA_EINVAL;
    }
  }
  memset(res, 0, sizeof(*res));
  for (int zi = 0; zi < spec->n_zt; ++zi) {
    const double z = spec->z_t[zi], cc = spec->c_t[zi], fbt = spec->fbar_t[zi];
    const double* pkt = spec->p1d_t + static_cast<size_t>(zi) * nk;
    bool failed = false;
    hipError_t last = hipSuccess;
    double pk[kMaxKBins];
    auto plain = [&](const double* t) -> double {
      double fb;
      last = ev.eval(exp(t[0]), exp(t[1]), cc, z, &fb, pk);
      if (last != hipSuccess) { failed = true; return HUGE_VAL; }
      return tune_chi2(fb, pk, fbt, pkt, nk, spec->sigma_rel);
    };
    double x[2] = {log(spec->a0), log(spec->b0)};
    double fbest = 0.0, fb = 0.0;
    int nev = 0, gpu_ev = 0;
    bool fallback = false;
    if (mode == LYA_TUNE_EMULATOR) {
      // Search on the model emulator + offset + slope correction (device
      // Levenberg-Marquardt), check the optimum on the GPU, then (i) move the
      // model onto the measured statistics there (offset = GPU - emulator) and
      // (ii) correct its slope along the last step by a Broyden update, so that
      // the model also reproduces the previous check; search again from the
      // new point.  Stops when a check moves the point by at most
      // max(10 xatol, 5e-4) or after emu_checks GPU evaluations.
      const int checks = spec->emu_checks > 0 ? spec->emu_checks : 1;
      const int ns = 1 + nk;
      const double xtol = fmax(10.0 * spec->xatol, 5e-4);
      double off[kMaxKBins + 1] = {0.0}, jac[2 * (kMaxKBins + 1)] = {0.0}, dprev[kMaxKBins + 1];
      double xk[2] = {x[0], x[1]};
      double step = 0.3;
      bool converged = false;
      for (int it = 0; it < checks; ++it) {
        int n1 = 0;
        // the search stops on position alone, a hundred times finer than the check tolerance
        EmuSearchSpec ss{fbt, cc, z, step, 0.01 * xtol, HUGE_VAL, spec->sigma_rel, nk, 3 * spec->max_evals, pkt,
                         off, jac, {xk[0], xk[1]}};
        double pe[kMaxKBins + 1];
        if ((last = emulator_search(spec->emulator, ss, x, &fbest, &n1, pe, reinterpret_cast<char*>(w + c.emu),
                                    st)) != hipSuccess) {
          failed = true;
          break;
        }
        nev += n1;
        if ((last = ev.eval(exp(x[0]), exp(x[1]), cc, z, &fb, pk)) != hipSuccess) {
          failed = true;
          break;
        }
        ++gpu_ev;
        double d[kMaxKBins + 1];
        d[0] = fb - pe[0];
        for (int i = 0; i < nk; ++i) d[1 + i] = pk[i] - pe[1 + i];
        const double s0 = xk[0] - x[0], s1 = xk[1] - x[1], s2 = s0 * s0 + s1 * s1;
        if (it > 0 && s2 > 1e-24) {
          for (int j = 0; j < ns; ++j) {
            if (!isfinite(d[j]) || !isfinite(dprev[j])) {
              jac[2 * j] = jac[2 * j + 1] = 0.0;
              continue;
            }
            const double r = (dprev[j] - d[j]) - (jac[2 * j] * s0 + jac[2 * j + 1] * s1);
            jac[2 * j] += r * s0 / s2;
            jac[2 * j + 1] += r * s1 / s2;
          }
        }
        const double moved = fmax(fabs(s0), fabs(s1));
        for (int j = 0; j < ns; ++j) off[j] = dprev[j] = d[j];
        xk[0] = x[0];
        xk[1] = x[1];
        if (it > 0 && moved <= xtol) {
          converged = true;
          break;
        }
        step = 0.05;
      }
      // a search that has not settled after emu_checks GPU evaluations (an
      // emulator trained poorly or used outside its range) hands over to the
      // plain loop, which starts from the last point checked on the GPU
      fallback = !failed && !converged;
    }
    if (mode != LYA_TUNE_EMULATOR || fallback) {
      Nm2 nm;
      nm.init(x, 0.3, spec->xatol, spec->fatol, spec->max_evals);
      double p[2];
      while (!failed && nm.ask(p)) nm.tell(plain(p));
      int n_nm = 0;
      nm.result(x, &fbest, &n_nm);
      nev += n_nm;
      gpu_ev += n_nm;
    }
    if (failed) {
      snprintf(err, errlen, "tuning evaluation at z=%g: %s", z, hipGetErrorString(last));
      return LYA_EHIP;
    }
    if (mode != LYA_TUNE_EMULATOR || fallback) {
      // statistics actually reached (one GPU evaluation)
      if ((e = ev.eval(exp(x[0]), exp(x[1]), cc, z, &fb, pk)) != hipSuccess) {
        snprintf(err, errlen, "tuning evaluation: %s", hipGetErrorString(e));
        return LYA_EHIP;
      }
      ++gpu_ev;
    }
    res->a[zi] = exp(x[0]);
    res->b[zi] = exp(x[1]);
    res->fbar[zi] = fb;
    res->chi2[zi] = tune_chi2(fb, pk, fbt, pkt, nk, spec->sigma_rel);
    res->evals[zi] = nev;
    res->gpu_evals[zi] = gpu_ev;
    res->fallback[zi] = fallback ? 1 : 0;
    for (int i = 0; i < nk; ++i) res->p1d[zi * kMaxKBins + i] = pk[i];
  }
  double xs[16], ys[3][16];
  for (int zi = 0; zi < spec->n_zt; ++zi) {
    xs[zi] = 1.0 + spec->z_t[zi];
    ys[0][zi] = res->a[zi];
    ys[1][zi] = res->b[zi];
    ys[2][zi] = spec->c_t[zi];
  }
  for (int p = 0; p < 3; ++p) {
    if (spec->n_zt >= 3) {
      quad_fit(xs, ys[p], spec->n_zt, res->coef[p]);
    } else if (spec->n_zt == 2) {  // the line through both points
      res->coef[p][1] = (ys[p][1] - ys[p][0]) / (xs[1] - xs[0]);
      res->coef[p][0] = ys[p][0] - res->coef[p][1] * xs[0];
      res->coef[p][2] = 0.0;
    } else {
      res->coef[p][0] = ys[p][0];
      res->coef[p][1] = res->coef[p][2] = 0.0;
    }
  }
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return LYA_OK;
}

}  // namespace lya
