// Two-dimensional Nelder-Mead minimiser and tuning objective shared by the
// host tuning loop and the device-side emulator search (every thread of the
// searching block runs the same steps on the same values, so the control flow
// is uniform).
#pragma once

#include <math.h>

namespace lya {

// Nelder-Mead in two dimensions (reflection 1, expansion 2, contraction 1/2,
// shrink 1/2) written as a reverse-communication state machine: ask() gives
// the next point to evaluate (false once finished), tell() takes its value.
// The initial simplex is x, x + step e1, x + step e2.  It stops when every
// vertex lies within xatol of the best one in each coordinate and within
// fatol in value, or once max_evals values have been told.  One evaluation
// site keeps a device caller's code small.
struct Nm2 {
  enum { kInit, kTop, kReflect, kExpand, kContract, kShrink, kDone };
  double s[3][2], fv[3], cx[2], xr[2], xe[2], xc[2], fr;
  double xatol, fatol;
  int phase, i, n, max_evals;
  bool outside;

  __host__ __device__ void init(const double x[2], double step, double xat, double fat, int maxev) {
    s[0][0] = x[0]; s[0][1] = x[1];
    s[1][0] = x[0] + step; s[1][1] = x[1];
    s[2][0] = x[0]; s[2][1] = x[1] + step;
    xatol = xat;
    fatol = fat;
    max_evals = maxev;
    phase = kInit;
    i = 0;
    n = 0;
    outside = false;
    fr = 0.0;
  }

  __host__ __device__ bool ask(double p[2]) {
    switch (phase) {
      case kInit:
      case kShrink:
        p[0] = s[i][0]; p[1] = s[i][1];
        return true;
      case kTop: {
        if (n >= max_evals) { phase = kDone; return false; }
        for (int a = 0; a < 2; ++a)  // order the vertices by value
          for (int b = a + 1; b < 3; ++b)
            if (fv[b] < fv[a]) {
              double t = fv[a]; fv[a] = fv[b]; fv[b] = t;
              for (int d = 0; d < 2; ++d) { t = s[a][d]; s[a][d] = s[b][d]; s[b][d] = t; }
            }
        double dx = 0.0, df = 0.0;
        for (int a = 1; a < 3; ++a) {
          for (int d = 0; d < 2; ++d) dx = fmax(dx, fabs(s[a][d] - s[0][d]));
          df = fmax(df, fabs(fv[a] - fv[0]));
        }
        if (dx <= xatol && df <= fatol) { phase = kDone; return false; }
        for (int d = 0; d < 2; ++d) {
          cx[d] = 0.5 * (s[0][d] + s[1][d]);
          xr[d] = 2.0 * cx[d] - s[2][d];
        }
        phase = kReflect;
        p[0] = xr[0]; p[1] = xr[1];
        return true;
      }
      case kExpand:
        p[0] = xe[0]; p[1] = xe[1];
        return true;
      case kContract:
        p[0] = xc[0]; p[1] = xc[1];
        return true;
      default:
        return false;
    }
  }

  __host__ __device__ void tell(double f) {
    ++n;
    switch (phase) {
      case kInit:
        fv[i] = f;
        if (++i == 3) phase = kTop;
        break;
      case kReflect:
        fr = f;
        if (fr < fv[0]) {
          for (int d = 0; d < 2; ++d) xe[d] = 3.0 * cx[d] - 2.0 * s[2][d];
          phase = kExpand;
        } else if (fr < fv[1]) {
          s[2][0] = xr[0]; s[2][1] = xr[1]; fv[2] = fr;
          phase = kTop;
        } else {
          outside = fr < fv[2];
          for (int d = 0; d < 2; ++d) xc[d] = outside ? 1.5 * cx[d] - 0.5 * s[2][d] : 0.5 * (cx[d] + s[2][d]);
          phase = kContract;
        }
        break;
      case kExpand:
        if (f < fr) { s[2][0] = xe[0]; s[2][1] = xe[1]; fv[2] = f; }
        else { s[2][0] = xr[0]; s[2][1] = xr[1]; fv[2] = fr; }
        phase = kTop;
        break;
      case kContract:
        if (f < (outside ? fr : fv[2])) {
          s[2][0] = xc[0]; s[2][1] = xc[1]; fv[2] = f;
          phase = kTop;
        } else {  // shrink towards the best vertex, then evaluate both moved ones
          for (int a = 1; a < 3; ++a)
            for (int d = 0; d < 2; ++d) s[a][d] = s[0][d] + 0.5 * (s[a][d] - s[0][d]);
          i = 1;
          phase = kShrink;
        }
        break;
      case kShrink:
        fv[i] = f;
        if (++i == 3) phase = kTop;
        break;
      default:
        break;
    }
  }

  // best vertex seen in the final simplex, its value, and the number of values told
  __host__ __device__ void result(double x[2], double* fbest, int* nev) const {
    int b = 0;
    const int nv = (phase == kInit) ? i : 3;
    for (int a = 1; a < nv; ++a)
      if (fv[a] < fv[b]) b = a;
    x[0] = s[b][0];
    x[1] = s[b][1];
    *fbest = nv > 0 ? fv[b] : HUGE_VAL;
    *nev = n;
  }
};

// Tuning objective: squared relative misfit of the mean flux and of every P1D
// bin whose target and value are finite, each in units of s.
__host__ __device__ inline double chi2_term(double v, double t, double s) {
  if (!isfinite(v) || !isfinite(t)) return 0.0;
  const double d = (v - t) / (s * t);
  return d * d;
}

__host__ __device__ inline double tune_chi2(double fbar, const double* pk, double fbar_t, const double* pk_t, int nk,
                                            double s) {
  double r = (fbar - fbar_t) / (s * fbar_t);
  r *= r;
  for (int i = 0; i < nk; ++i) r += chi2_term(pk[i], pk_t[i], s);
  return r;
}

}  // namespace lya
