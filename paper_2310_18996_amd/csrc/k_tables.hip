// FP64 tables for the hot path (gfx950): the power-spectrum amplitude per
// integer n^2, the sigma8 normalisation, FFT twiddles, and z(chi) for pixel
// redshifts.  FP64 on the GPU is confined to these small tables.
//
// P(k) (stand-in for the paper's CAMB spectrum, eq:deltaL):
//   P = A k^ns T_BBKS(k/Gamma)^2 (1 + w sin(k r_w) exp(-(k/k_d)^2)),
//   T_BBKS(q) = ln(1+2.34q)/(2.34q) [1+3.89q+(16.1q)^2+(5.46q)^3+(6.71q)^4]^(-1/4)
//   (Bardeen, Bond, Kaiser & Szalay 1986);
//   A from sigma8: sigma_8^2 = 1/(2 pi^2) int k^3 P W_TH(8k)^2 dln k with the
//   sphere window W_TH(x) = 3 (sin x - x cos x)/x^3, composite Simpson in
//   ln k over [1e-5, 1e3] h/Mpc with 2^16+1 nodes.
// A tabulated P(k) (the paper's CAMB table) replaces the analytic form and its
// sigma8 normalisation when given.
// Amplitude per mode (eq:deltaL with unit-variance complex noise):
//   s(n^2) = sqrt(P(2 pi |n| / L) / L^3) * exp(-k^2 smooth^2 / 2), s(0) = 0.
// Pixel redshift (section "FGPA": unperturbed cosmological redshift), flat
// LCDM with E(z)^2 = Om (1+z)^3 + 1 - Om (Table cosmoparams), c/H0 in Mpc/h.
#include "lya_internal.h"

namespace lya {

__device__ __forceinline__ double t_bbks(double q) {
  const double x = 2.34 * q;
  const double lead = x > 0.0 ? log1p(x) / x : 1.0;
  const double a = 16.1 * q, b = 5.46 * q, c = 6.71 * q;
  const double poly = 1.0 + 3.89 * q + a * a + b * b * b + (c * c) * (c * c);
  return lead * pow(poly, -0.25);
}

__device__ __forceinline__ double pk_shape(double k, const PkParams& p) {
  const double t = t_bbks(k / p.gamma);
  const double kd = k / p.wig_kd;
  const double wig = 1.0 + p.wig_amp * sin(k * p.wig_r) * exp(-kd * kd);
  return pow(k, p.ns) * t * t * wig;
}

__device__ __forceinline__ double w_tophat(double x) {
  if (fabs(x) < 1e-2) {
    const double x2 = x * x;
    return 1.0 - x2 / 10.0 + x2 * x2 / 280.0;
  }
  return 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
}

constexpr int kSimpsonNodes = 65537;
constexpr double kLnkMin = -11.512925464970229;  // ln 1e-5
constexpr double kLnkMax = 6.907755278982137;    // ln 1e3

__global__ void __launch_bounds__(256) k_sigma8_partial(PkParams p, double* partial) {
  __shared__ double red[256];
  const double h = (kLnkMax - kLnkMin) / (kSimpsonNodes - 1);
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < kSimpsonNodes; i += gridDim.x * 256) {
    const double lnk = kLnkMin + h * i;
    const double k = exp(lnk);
    const double w = w_tophat(8.0 * k);
    const double wt = (i == 0 || i == kSimpsonNodes - 1) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
    acc += wt * k * k * k * pk_shape(k, p) * w * w;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block: amplitude A into amp[0]; all threads: twiddles exp(+2 pi i k / ntw).
__global__ void __launch_bounds__(256) k_pk_finalize(PkParams p, const double* partial, int npartial, double* amp,
                                                     float2* tw, int ntw) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < npartial; ++i) s += partial[i];
    const double h = (kLnkMax - kLnkMin) / (kSimpsonNodes - 1);
    const double sig2 = h / 3.0 * s / (2.0 * M_PI * M_PI);
    amp[0] = p.sigma8 * p.sigma8 / sig2;
  }
  for (int k = threadIdx.x; k < ntw; k += 256) {
    double sn, cs;
    sincospi(2.0 * k / ntw, &sn, &cs);
    tw[k] = make_float2(static_cast<float>(cs), static_cast<float>(sn));
  }
}

// Tabulated P(k): ln P linear in ln k between the nodes; below the first and
// above the last node the end intervals' power laws continue.
__device__ __forceinline__ double pk_tabulated(double k, const PkParams& p) {
  const double* kt = p.k_tab;
  const int n = p.n_tab;
  int i;   // interval [kt[i], kt[i+1]]
  if (k <= kt[0]) {
    i = 0;
  } else if (k >= kt[n - 1]) {
    i = n - 2;
  } else {
    int lo = 0, hi = n - 1;   // kt[lo] <= k < kt[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (kt[mid] <= k) lo = mid; else hi = mid;
    }
    i = lo;
  }
  const double x0 = log(kt[i]), x1 = log(kt[i + 1]);
  const double y0 = log(p.p_tab[i]), y1 = log(p.p_tab[i + 1]);
  return exp(y0 + (y1 - y0) * (log(k) - x0) / (x1 - x0));
}

__global__ void __launch_bounds__(256) k_amp_table(const double* amp, PkParams p, double L, int nentries, float* table) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nentries) return;
  if (e == 0) {
    table[0] = 0.0f;
    return;
  }
  const double k = 2.0 * M_PI * sqrt(static_cast<double>(e)) / L;
  const double P = p.k_tab ? pk_tabulated(k, p) : amp[0] * pk_shape(k, p);
  double s = sqrt(P / (L * L * L));
  if (p.smooth > 0.0) s *= exp(-0.5 * (k * p.smooth) * (k * p.smooth));
  table[e] = static_cast<float>(s);
}

// Integrand of the matter correlation function of the smoothed spectrum
// (section "Quasar generation"): xi(r) = 1/(2 pi^2 r) int_0^kmax P(k)
// exp(-k^2 s^2) k sin(k r) dk, composite Simpson on k_j = j h, j = 0..m
// (m even).  f_j holds the Simpson weight times P(k_j) exp(-k_j^2 s^2) k_j;
// k = 0 carries nothing.
__global__ void __launch_bounds__(256) k_xi_weights(const double* amp, PkParams p, double s, double h, int m,
                                                    double* f) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j > m) return;
  if (j == 0) {
    f[0] = 0.0;
    return;
  }
  const double k = h * j;
  const double P = p.k_tab ? pk_tabulated(k, p) : amp[0] * pk_shape(k, p);
  const double w = (j == m) ? 1.0 : ((j & 1) ? 4.0 : 2.0);
  f[j] = w * h / 3.0 * P * exp(-(k * s) * (k * s)) * k;
}

// ---- pixel redshift table: z at chi = i * h_chi, i = 0..n-1 ----
__device__ __forceinline__ double inv_e(double z, double om) {
  const double zp = 1.0 + z;
  return 1.0 / sqrt(om * zp * zp * zp + (1.0 - om));
}

__device__ double chi_of_z(double z, double om) {
  // composite Simpson, 128 intervals on [0, z]: relative error ~1e-9 for z < 5
  constexpr int m = 128;
  const double h = z / m;
  double s = inv_e(0.0, om) + inv_e(z, om);
  for (int i = 1; i < m; ++i) s += ((i & 1) ? 4.0 : 2.0) * inv_e(h * i, om);
  return kCOverH0 * h / 3.0 * s;
}

__global__ void __launch_bounds__(256) k_zchi_table(double om, double h_chi, int n, float* ztab) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double chi = h_chi * i;
  double z = chi / kCOverH0;
  for (int it = 0; it < 20; ++it) {
    const double dz = (chi_of_z(z, om) - chi) * sqrt(om * (1 + z) * (1 + z) * (1 + z) + 1 - om) / kCOverH0;
    z -= dz;
    if (fabs(dz) < 1e-11) break;
  }
  ztab[i] = static_cast<float>(z);
}

// ---- launchers ----
hipError_t launch_pk_table(const PkParams& p, int n, double dx, TableWork& w, hipStream_t st) {
  const double L = n * dx;
  LYA_TIMED("pk_sigma8", st, hipLaunchKernelGGL(k_sigma8_partial, dim3(kSigmaBlocks), dim3(256), 0, st, p, w.partial));
  LYA_TIMED("pk_finalize", st,
            hipLaunchKernelGGL(k_pk_finalize, dim3(1), dim3(256), 0, st, p, w.partial, kSigmaBlocks, w.amp, w.tw, n));
  const int ne = amp_table_entries(n);
  LYA_TIMED("pk_table", st,
            hipLaunchKernelGGL(k_amp_table, dim3((ne + 255) / 256), dim3(256), 0, st, w.amp, p, L, ne, w.table));
  return hipGetLastError();
}

hipError_t launch_xi_weights(const PkParams& p, double s, double h, int m, double* partial, double* amp,
                             double* f, hipStream_t st) {
  if (!p.k_tab) {
    LYA_TIMED("pk_sigma8", st, hipLaunchKernelGGL(k_sigma8_partial, dim3(kSigmaBlocks), dim3(256), 0, st, p, partial));
    LYA_TIMED("pk_finalize", st,
              hipLaunchKernelGGL(k_pk_finalize, dim3(1), dim3(256), 0, st, p, partial, kSigmaBlocks, amp,
                                 static_cast<float2*>(nullptr), 0));
  }
  LYA_TIMED("xi_weights", st,
            hipLaunchKernelGGL(k_xi_weights, dim3((m + 256) / 256), dim3(256), 0, st, amp, p, s, h, m, f));
  return hipGetLastError();
}

hipError_t launch_zchi_table(double omega_m, float* ztab, hipStream_t st) {
  LYA_TIMED("zchi_table", st,
            hipLaunchKernelGGL(k_zchi_table, dim3((kZTabN + 255) / 256), dim3(256), 0, st, omega_m, kZTabH, kZTabN, ztab));
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_twiddles(float2* tw, int ntw) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < ntw; k += gridDim.x * 256) {
    double sn, cs;
    sincospi(2.0 * k / ntw, &sn, &cs);
    tw[k] = make_float2(static_cast<float>(cs), static_cast<float>(sn));
  }
}

hipError_t launch_twiddles(float2* tw, int ntw, hipStream_t st) {
  LYA_TIMED("twiddles", st, hipLaunchKernelGGL(k_twiddles, dim3((ntw + 255) / 256), dim3(256), 0, st, tw, ntw));
  return hipGetLastError();
}

}  // namespace lya
