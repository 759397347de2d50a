// Two-dimensional Nelder-Mead minimiser shared by the host tuning loop and
// the device-side emulator search (every thread of the searching block runs
// the same steps on the same values, so the control flow is uniform).
#pragma once

#include <math.h>

namespace lya {

// Nelder-Mead (reflection 1, expansion 2, contraction 1/2, shrink 1/2), 2D;
// stops when every vertex is within xatol of the best one in each coordinate
// and within fatol in value, or after max_evals evaluations.
template <typename F>
__host__ __device__ int nelder_mead2(F&& f, double x[2], double step, double xatol, double fatol, int max_evals, double* fbest,
                 int* nev, bool* failed) {
  double s[3][2] = {{x[0], x[1]}, {x[0] + step, x[1]}, {x[0], x[1] + step}};
  double fv[3];
  int n = 0;
  for (int i = 0; i < 3; ++i) {
    fv[i] = f(s[i]);
    ++n;
    if (*failed) return n;
  }
  while (n < max_evals) {
    // order
    for (int i = 0; i < 2; ++i)
      for (int j = i + 1; j < 3; ++j)
        if (fv[j] < fv[i]) {
          double t = fv[i]; fv[i] = fv[j]; fv[j] = t;
          for (int d = 0; d < 2; ++d) { t = s[i][d]; s[i][d] = s[j][d]; s[j][d] = t; }
        }
    double dx = 0.0, df = 0.0;
    for (int i = 1; i < 3; ++i) {
      for (int d = 0; d < 2; ++d) dx = fmax(dx, fabs(s[i][d] - s[0][d]));
      df = fmax(df, fabs(fv[i] - fv[0]));
    }
    if (dx <= xatol && df <= fatol) break;
    const double cx[2] = {0.5 * (s[0][0] + s[1][0]), 0.5 * (s[0][1] + s[1][1])};
    double xr[2] = {2.0 * cx[0] - s[2][0], 2.0 * cx[1] - s[2][1]};
    const double fr = f(xr);
    ++n;
    if (*failed) return n;
    if (fr < fv[0]) {
      double xe[2] = {3.0 * cx[0] - 2.0 * s[2][0], 3.0 * cx[1] - 2.0 * s[2][1]};
      const double fe = f(xe);
      ++n;
      if (*failed) return n;
      if (fe < fr) { s[2][0] = xe[0]; s[2][1] = xe[1]; fv[2] = fe; }
      else { s[2][0] = xr[0]; s[2][1] = xr[1]; fv[2] = fr; }
    } else if (fr < fv[1]) {
      s[2][0] = xr[0]; s[2][1] = xr[1]; fv[2] = fr;
    } else {
      const bool outside = fr < fv[2];
      double xc[2];
      if (outside) { xc[0] = 1.5 * cx[0] - 0.5 * s[2][0]; xc[1] = 1.5 * cx[1] - 0.5 * s[2][1]; }
      else { xc[0] = 0.5 * (cx[0] + s[2][0]); xc[1] = 0.5 * (cx[1] + s[2][1]); }
      const double fc = f(xc);
      ++n;
      if (*failed) return n;
      if (fc < (outside ? fr : fv[2])) {
        s[2][0] = xc[0]; s[2][1] = xc[1]; fv[2] = fc;
      } else {
        for (int i = 1; i < 3; ++i) {
          for (int d = 0; d < 2; ++d) s[i][d] = s[0][d] + 0.5 * (s[i][d] - s[0][d]);
          fv[i] = f(s[i]);
          ++n;
          if (*failed) return n;
        }
      }
    }
  }
  int best = 0;
  for (int i = 1; i < 3; ++i) if (fv[i] < fv[best]) best = i;
  x[0] = s[best][0];
  x[1] = s[best][1];
  *fbest = fv[best];
  *nev = n;
  return n;
}

// Tuning objective: squared relative misfit of the mean flux and of every P1D
// bin whose target and value are finite, each in units of s.
__host__ __device__ inline double tune_chi2(double fbar, const double* pk, double fbar_t, const double* pk_t, int nk, double s) {
  double r = (fbar - fbar_t) / (s * fbar_t);
  r *= r;
  for (int i = 0; i < nk; ++i) {
    if (!isfinite(pk_t[i]) || !isfinite(pk[i])) continue;
    const double d = (pk[i] - pk_t[i]) / (s * pk_t[i]);
    r += d * d;
  }
  return r;
}

}  // namespace lya
