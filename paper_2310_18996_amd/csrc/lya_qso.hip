// Lognormal quasar field (gfx950), section "Quasar generation" and Appendix A:
//   * xi_m(r) of the smoothed matter spectrum and the lognormal spectrum
//     P_q(k) = FT of ln(1 + b_0^2 xi_m), both in FP64;
//   * the variance of a box (a reduction over the grid);
//   * per comoving distance: z and the three-box coefficients c_i(z);
//   * the draw: every voxel is selected with probability
//     p = nbar(z) dx^3 sum_i c_i(z) exp(a_i(z) delta_i - a_i(z)^2 var_i / 2),
//     a_i(z) = b_q(z) (1 + z_i) / (b_q(z_i) (1 + z)) = ((1 + z)/(1 + z_i))^0.7
//     for b_q proportional to (1 + z)^1.7, and a selected voxel gets a
//     uniform position inside it;
//   * the catalogue: each quasar's redshift with its line-of-sight velocity
//     (eq:velocity) and its line of sight as a skewer-table row.
#include <algorithm>

#include "lya_internal.h"

namespace lya {

namespace {

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ double block_sum256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return threadIdx.x == 0 ? red[0] + red[1] + red[2] + red[3] : 0.0;
}

// Nodes a thread takes between exact sines: the rest come from rotating by
// the angle of 256 nodes (rounding grows by about an ulp per rotation).
constexpr int kRotSteps = 32;

}  // namespace

// xi_m at r_b = b dr (one block per r): sum_j f_j sin(k_j r) / (2 pi^2 r),
// f from launch_xi_weights; r = 0 takes the limit sum_j f_j k_j / (2 pi^2).
__global__ void __launch_bounds__(256) k_xi_r(const double* __restrict__ f, int m, double h, double dr,
                                              double* __restrict__ xi) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const double r = dr * b;
  double acc = 0.0;
  if (b == 0) {
    for (int j = threadIdx.x; j <= m; j += 256) acc += f[j] * (h * j);
  } else {
    double sd, cd;
    sincos(256.0 * h * r, &sd, &cd);
    for (int j0 = threadIdx.x; j0 <= m; j0 += 256 * kRotSteps) {
      double sn, cs;
      sincos(h * j0 * r, &sn, &cs);
      const int jend = min(j0 + 256 * kRotSteps, m + 1);
      for (int j = j0; j < jend; j += 256) {
        acc += f[j] * sn;
        const double t = sn * cd + cs * sd;
        cs = cs * cd - sn * sd;
        sn = t;
      }
    }
  }
  const double tot = block_sum256(acc, red);
  if (threadIdx.x == 0) xi[b] = (b == 0 ? tot : tot / r) / (2.0 * M_PI * M_PI);
}

// g_i = Simpson weight (dr/3) ln(1 + b2 xi_i) r_i on r_i = i dr (n_r odd).
__global__ void __launch_bounds__(256) k_lognormal_g(const double* __restrict__ xi, int n_r, double dr, double b2,
                                                     double* __restrict__ g) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_r) return;
  const double w = (i == 0 || i == n_r - 1) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
  g[i] = w * dr / 3.0 * log1p(b2 * xi[i]) * (dr * i);
}

// P_q(k) = 4 pi / k sum_i g_i sin(k r_i), one block per k; k = 0: 4 pi sum g_i r_i.
__global__ void __launch_bounds__(256) k_lognormal_pq(const double* __restrict__ g, int n_r, double dr,
                                                      const double* __restrict__ kv, double* __restrict__ pq) {
  __shared__ double red[4];
  const double k = kv[blockIdx.x];
  double acc = 0.0;
  if (k <= 0.0) {
    for (int i = threadIdx.x; i < n_r; i += 256) acc += g[i] * (dr * i);
  } else {
    double sd, cd;
    sincos(256.0 * dr * k, &sd, &cd);
    for (int i0 = threadIdx.x; i0 < n_r; i0 += 256 * kRotSteps) {
      double sn, cs;
      sincos(dr * i0 * k, &sn, &cs);
      const int iend = min(i0 + 256 * kRotSteps, n_r);
      for (int i = i0; i < iend; i += 256) {
        acc += g[i] * sn;
        const double t = sn * cd + cs * sd;
        cs = cs * cd - sn * sd;
        sn = t;
      }
    }
  }
  const double tot = block_sum256(acc, red);
  if (threadIdx.x == 0) pq[blockIdx.x] = 4.0 * M_PI * (k <= 0.0 ? tot : tot / k);
}

// Values below 1e-12 of the largest are raised to that floor (one block), so
// that the result can serve as a tabulated spectrum (ln P interpolation).
__global__ void __launch_bounds__(256) k_lognormal_floor(double* pq, int n_k) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int i = threadIdx.x; i < n_k; i += 256) mx = fmax(mx, pq[i]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  const double fl = 1e-12 * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  if (fl <= 0.0) return;
  for (int i = threadIdx.x; i < n_k; i += 256) pq[i] = fmax(pq[i], fl);
}

hipError_t launch_lognormal(const PkParams& p, const LognormalArgs& a, hipStream_t st) {
  hipError_t e = launch_xi_weights(p, a.smooth, a.h, a.m, a.partial, a.amp, a.f, st);
  if (e != hipSuccess) return e;
  LYA_TIMED("xi_r", st, hipLaunchKernelGGL(k_xi_r, dim3(a.n_r), dim3(256), 0, st, a.f, a.m, a.h, a.dr, a.xi));
  LYA_TIMED("lognormal_g", st,
            hipLaunchKernelGGL(k_lognormal_g, dim3((a.n_r + 255) / 256), dim3(256), 0, st, a.xi, a.n_r, a.dr, a.b2,
                               a.g));
  if (a.n_k > 0) {
    LYA_TIMED("lognormal_pq", st,
              hipLaunchKernelGGL(k_lognormal_pq, dim3(a.n_k), dim3(256), 0, st, a.g, a.n_r, a.dr, a.k, a.pq));
    LYA_TIMED("lognormal_floor", st, hipLaunchKernelGGL(k_lognormal_floor, dim3(1), dim3(256), 0, st, a.pq, a.n_k));
  }
  return hipGetLastError();
}

// ---- box moments ----
// Per block: sums of re, re^2, im, im^2 over rows (x, y) of the box.
__global__ void __launch_bounds__(256) k_box_moments(const float2* __restrict__ box, int n, size_t pitch,
                                                     double* __restrict__ part) {
  __shared__ double red[4];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t rows = static_cast<int64_t>(n) * n;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    // two cells per 16-byte load (rows start 16-byte aligned: n and the
    // plane pitch are multiples of 4)
    const float4* q = reinterpret_cast<const float4*>(box + static_cast<size_t>(row / n) * pitch +
                                                      static_cast<size_t>(row % n) * n);
#pragma unroll 2
    for (int i = threadIdx.x; i < n / 2; i += 256) {
      const float4 v = q[i];
      s[0] += static_cast<double>(v.x) + v.z;
      s[1] += static_cast<double>(v.x) * v.x + static_cast<double>(v.z) * v.z;
      s[2] += static_cast<double>(v.y) + v.w;
      s[3] += static_cast<double>(v.y) * v.y + static_cast<double>(v.w) * v.w;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double t = block_sum256(s[c], red);
    if (threadIdx.x == 0) part[blockIdx.x * 4 + c] = t;
    __syncthreads();
  }
}

// out = {mean re, var re, mean im, var im} over the n^3 grid points.
__global__ void __launch_bounds__(256) k_box_moments_final(const double* __restrict__ part, int nblocks,
                                                           double inv_count, double* __restrict__ out) {
  __shared__ double red[4];
  double t[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += part[b * 4 + c];
    t[c] = block_sum256(s, red);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m0 = t[0] * inv_count, m1 = t[2] * inv_count;
    out[0] = m0;
    out[1] = t[1] * inv_count - m0 * m0;
    out[2] = m1;
    out[3] = t[3] * inv_count - m1 * m1;
  }
}

hipError_t launch_box_moments(const float2* box, int n, double* part, double* out, hipStream_t st) {
  LYA_TIMED("box_moments", st,
            hipLaunchKernelGGL(k_box_moments, dim3(kQsoMomBlocks), dim3(256), 0, st, box, n, plane_pitch(n), part));
  const double inv = 1.0 / (static_cast<double>(n) * n * n);
  LYA_TIMED("box_moments_final", st,
            hipLaunchKernelGGL(k_box_moments_final, dim3(1), dim3(256), 0, st, part, kQsoMomBlocks, inv, out));
  return hipGetLastError();
}

// ---- per-distance table: {z, c_1, c_2, c_3} at chi = i kZTabH ----
__device__ __forceinline__ double bias_qso(double z) { return 3.7 * pow((1.0 + z) / 3.33, 1.7); }

__global__ void __launch_bounds__(256) k_qso_coef(const float* __restrict__ ztab, QsoCoef c, float4* __restrict__ tab) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kZTabN) return;
  const double z = ztab[i];
  double cf[3] = {1.0, 0.0, 0.0};
  if (c.nb == 3) {
    double xi[3];
    for (int j = 0; j < 3; ++j) {
      const double al = pow((1.0 + z) / (1.0 + c.z[j]), 0.7);
      xi[j] = pow(1.0 + c.b2[j] * c.xi5, al * al) - 1.0;
    }
    const double gq = c.g_ref * (1.0 + c.z_ref) / (1.0 + z);
    const double bz = bias_qso(z) * gq;
    const double xi_mod = bz * bz * c.xi5;
    const double t12 = (z - c.z[0]) / (c.z[1] - c.z[0]);
    const double t23 = (z - c.z[1]) / (c.z[2] - c.z[1]);
    const double xi12 = (1.0 - t12) * xi[0] + t12 * xi[1];
    const double xi23 = (1.0 - t23) * xi[1] + t23 * xi[2];
    const double den = xi12 - xi23;
    const double w = fabs(den) <= 1e-12 * fabs(xi[1]) ? 0.5 : fmin(fmax((xi_mod - xi23) / den, 0.0), 1.0);
    cf[0] = w * (1.0 - t12);
    cf[1] = w * t12 + (1.0 - w) * (1.0 - t23);
    cf[2] = (1.0 - w) * t23;
  }
  tab[i] = make_float4(static_cast<float>(z), static_cast<float>(cf[0]), static_cast<float>(cf[1]),
                       static_cast<float>(cf[2]));
}

// ---- the draw ----
// One thread per VPT consecutive voxels along z (one Philox call gives the
// decision uniforms of four).  Selected voxels are appended with one atomic per
// wave; a slot at or beyond cap is counted but not written.
// The transcendentals run on the hardware units (v_sqrt_f32, v_log_f32,
// v_exp_f32: about 1 ulp each); the exponent's own rounding, |x| 2^-24 for
// |x| up to about 10, dominates the error of p (a few 1e-7 relative).
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kQsoVpt = 8;      // voxels per thread (consecutive along z)
constexpr int kQsoBlock = 256;  // threads per block (512: 59 ms against 54.5 at 2048^3)

template <int NB, int VPT>
__global__ void __launch_bounds__(kQsoBlock) k_qso_draw(QsoDrawArgs a) {
  static_assert(VPT % 4 == 0, "whole Philox calls per thread");
  __shared__ float snz[kQsoMaxNbar], snb[kQsoMaxNbar];
  const int n = a.n;
  // thread t of block b takes voxels v0 .. v0 + VPT - 1 along z, v0 = VPT (kQsoBlock b + t)
  const uint64_t g = static_cast<uint64_t>(blockIdx.x) * kQsoBlock + threadIdx.x;
  const uint64_t v0 = g * VPT;
  // n is a power of two: shifts and masks instead of 64-bit divisions
  const uint64_t row = v0 >> a.log2n;
  const int iz0 = static_cast<int>(v0 & static_cast<uint64_t>(n - 1));
  const int ix = static_cast<int>(row >> a.log2n), iy = static_cast<int>(row & static_cast<uint64_t>(n - 1));
  const size_t e0 = static_cast<size_t>(ix) * a.pitch + static_cast<size_t>(iy) * n + iz0;

  // the field loads first, so that their latency overlaps the block's
  // set-up (nbar into LDS, the variances) and the Philox rounds
  float d[NB][VPT];
#pragma unroll
  for (int h = 0; h < VPT / 2; ++h) {
    const float4 v = *reinterpret_cast<const float4*>(a.box_a + e0 + 2 * h);
    d[0][2 * h] = v.x;
    d[0][2 * h + 1] = v.z;
    if (NB == 3) {
      const float4 w = *reinterpret_cast<const float4*>(a.box_b + e0 + 2 * h);
      d[1 % NB][2 * h] = v.y;
      d[1 % NB][2 * h + 1] = v.w;
      d[2 % NB][2 * h] = w.x;
      d[2 % NB][2 * h + 1] = w.z;
    }
  }
  for (int i = threadIdx.x; i < a.n_nbar; i += kQsoBlock) {
    snz[i] = static_cast<float>(a.nbar_z[i]);
    snb[i] = static_cast<float>(a.nbar[i]);
  }
  float hv[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) hv[i] = 0.5f * static_cast<float>(*a.var[i]);
  // distance, z and the three-box coefficients of the voxels (table loads
  // issued before the barrier as well)
  const float rx = static_cast<float>(ix * a.dx_d - a.o[0]);
  const float ry = static_cast<float>(iy * a.dx_d - a.o[1]);
  const float r2xy = rx * rx + ry * ry;
  float zv[VPT], cfv[VPT][3];
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    const float rz = static_cast<float>(iz0 + e) * a.dx - a.oz;
    const float chi = __builtin_amdgcn_sqrtf(r2xy + rz * rz);
    const float t = chi * (1.0f / static_cast<float>(kZTabH));
    const int i0 = min(static_cast<int>(t), kZTabN - 2);
    const float fr = t - static_cast<float>(i0);
    const float4 c0 = a.tab[i0], c1 = a.tab[i0 + 1];
    zv[e] = c0.x + fr * (c1.x - c0.x);
    cfv[e][0] = c0.y + fr * (c1.y - c0.y);
    cfv[e][1] = c0.z + fr * (c1.z - c0.z);
    cfv[e][2] = c0.w + fr * (c1.w - c0.w);
  }
  // decision words: voxel m takes word m & 3 of the call for counter m >> 2
  uint32_t words[VPT];
#pragma unroll
  for (int c = 0; c < VPT / 4; ++c) {
    const uint64_t ctr = (v0 >> 2) + c;
    const uint4 wd = philox10_x3(make_uint4(static_cast<uint32_t>(ctr), static_cast<uint32_t>(ctr >> 32), 2u, 0u),
                                 static_cast<uint32_t>(a.seed), static_cast<uint32_t>(a.seed >> 32));
    words[4 * c] = wd.x;
    words[4 * c + 1] = wd.y;
    words[4 * c + 2] = wd.z;
    words[4 * c + 3] = wd.w;
  }
  __syncthreads();
  // the largest density, raised by a margin over the rounding of the
  // interpolation between two nodes
  float nb_top = 0.0f;
  for (int i = static_cast<int>(threadIdx.x & 63); i < a.n_nbar; i += 64) nb_top = fmaxf(nb_top, snb[i]);
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) nb_top = fmaxf(nb_top, __shfl_xor(nb_top, w));  // over the wave
  nb_top *= 1.0f + 1.0e-6f;

  bool sel[VPT];
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    const float z = zv[e];
    const float lz = __log2f(1.0f + z);
    float acc;
    if (NB == 1) {
      const float al = __builtin_amdgcn_exp2f(0.7f * (lz - a.l2z[0]));
      acc = __builtin_amdgcn_exp2f(kLog2e * (al * d[0][e] - al * al * hv[0]));
    } else {
      acc = 0.0f;
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const float al = __builtin_amdgcn_exp2f(0.7f * (lz - a.l2z[i]));
        acc += cfv[e][i] * __builtin_amdgcn_exp2f(kLog2e * (al * d[i][e] - al * al * hv[i]));
      }
    }
    // p <= nb_top dx^3 acc (rounding is monotone): most voxels are rejected
    // on that bound before nbar(z) is looked up
    const float u = u01(words[e]);
    sel[e] = false;
    if (u < fminf(nb_top * a.dx3 * acc, 1.0f)) {
      // nbar(z): linear between the nodes, zero outside
      float nb = 0.0f;
      if (z >= snz[0] && z <= snz[a.n_nbar - 1]) {
        int lo = 0, hi = a.n_nbar - 1;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (snz[mid] <= z) lo = mid; else hi = mid;
        }
        const float span = snz[hi] - snz[lo];
        nb = span > 0.0f ? snb[lo] + (snb[hi] - snb[lo]) * ((z - snz[lo]) / span) : snb[lo];
      }
      sel[e] = u < fminf(nb * a.dx3 * acc, 1.0f);
    }
  }

  uint64_t b[VPT];
  int tot = 0;
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    b[e] = __ballot(sel[e]);
    tot += __popcll(b[e]);
  }
  if (tot == 0) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(a.count, static_cast<unsigned long long>(tot));
  const uint32_t blo = __shfl(static_cast<uint32_t>(base), 0, 64);
  const uint32_t bhi = __shfl(static_cast<uint32_t>(base >> 32), 0, 64);
  base = (static_cast<unsigned long long>(bhi) << 32) | blo;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  unsigned long long before = 0;
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    if (sel[e]) {
      const unsigned long long slot = base + before + __popcll(b[e] & below);
      if (slot < static_cast<unsigned long long>(a.cap)) {
        const uint64_t m = v0 + e;
        const uint4 pw = philox10_x3(make_uint4(static_cast<uint32_t>(m), static_cast<uint32_t>(m >> 32), 4u, 0u),
                                     static_cast<uint32_t>(a.seed), static_cast<uint32_t>(a.seed >> 32));
        int64_t* o = a.pos + 3 * slot;
        o[0] = (static_cast<int64_t>(ix) << 32) - (int64_t(1) << 31) + pw.x;
        o[1] = (static_cast<int64_t>(iy) << 32) - (int64_t(1) << 31) + pw.y;
        o[2] = (static_cast<int64_t>(iz0 + e) << 32) - (int64_t(1) << 31) + pw.z;
      }
    }
    before += __popcll(b[e]);
  }
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

hipError_t launch_qso_draw(const QsoCoef& c, const QsoDrawArgs& a, const float* ztab, float4* tab, hipStream_t st) {
  LYA_TIMED("qso_coef", st,
            hipLaunchKernelGGL(k_qso_coef, dim3((kZTabN + 255) / 256), dim3(256), 0, st, ztab, c, tab));
  LYA_TIMED("qso_zero", st, hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, a.count));
  // kQsoBlock threads x kQsoVpt voxels per block: n^3 / (kQsoBlock kQsoVpt) blocks, a
  // whole number for every supported n (n >= 32), so every wave is full, as
  // the wave-wide ballots need
  const uint64_t blocks = static_cast<uint64_t>(a.n) * a.n * a.n / (kQsoBlock * kQsoVpt);
  if (a.nb == 3) {
    LYA_TIMED("qso_draw", st, hipLaunchKernelGGL((k_qso_draw<3, kQsoVpt>), dim3(static_cast<unsigned>(blocks)),
                                                 dim3(kQsoBlock), 0, st, a));
  } else {
    LYA_TIMED("qso_draw", st, hipLaunchKernelGGL((k_qso_draw<1, kQsoVpt>), dim3(static_cast<unsigned>(blocks)),
                                                 dim3(kQsoBlock), 0, st, a));
  }
  return hipGetLastError();
}

// ---- catalogue: redshift-space quasar redshifts and their lines of sight ----
// Flat LCDM in FP64.  I(a) = int_0^a da' / (a' E(a'))^3 by composite Simpson
// in t = sqrt(a') (a smooth integrand near 0), 512 intervals.
__device__ double growth_integral(double a, double om) {
  constexpr int kN = 512;
  const double tmax = sqrt(a), h = tmax / kN;
  double acc = 0.0;
  for (int i = 1; i <= kN; ++i) {
    const double t = h * i, ap = t * t;
    const double ae2 = om / ap + (1.0 - om) * ap * ap;  // (a E)^2
    acc += (i == kN ? 1.0 : (i & 1 ? 4.0 : 2.0)) * 2.0 * t / (ae2 * sqrt(ae2));
  }
  return acc * h / 3.0;
}

// chi(z) = c/H0 int_0^z dz' / E(z'), composite Simpson with 1024 intervals.
__device__ double chi_of_z_fine(double z, double om) {
  constexpr int kN = 1024;
  const double h = z / kN;
  double acc = 0.0;
  for (int i = 0; i <= kN; ++i) {
    const double x = 1.0 + h * i;
    acc += (i == 0 || i == kN ? 1.0 : (i & 1 ? 4.0 : 2.0)) / sqrt(om * x * x * x + (1.0 - om));
  }
  return kCOverH0 * acc * h / 3.0;
}

// Velocity factor G(z) f(z) E(z) / (1 + z) at chi = i kZTabH (z from ztab):
// the velocity boxes (z = 0, f = 1) to redshift z.  f = dln D / dln a =
// -3 Om / (2 a^3 E^2) + a / (I (a E)^3) for D = E I.
__global__ void __launch_bounds__(256) k_qso_vtab(const float* __restrict__ ztab, double om, float* __restrict__ vtab) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kZTabN) return;
  const double z = ztab[i];
  const double a = 1.0 / (1.0 + z);
  const double e2 = om / (a * a * a) + 1.0 - om;
  const double I = growth_integral(a, om), I1 = growth_integral(1.0, om);
  const double g = sqrt(e2) * I / I1;
  const double ae2 = a * a * e2;
  const double f = -1.5 * om / (a * a * a * e2) + a / (I * ae2 * sqrt(ae2));
  vtab[i] = static_cast<float>(g * f * sqrt(e2) / (1.0 + z));
}

__device__ __forceinline__ double lerp_tab(const float* tab, double chi) {
  const double t = chi / kZTabH;
  const int i0 = min(static_cast<int>(t), kZTabN - 2);
  const double fr = t - i0;
  return tab[i0] + fr * (static_cast<double>(tab[i0 + 1]) - tab[i0]);
}

// One thread per quasar.
__global__ void __launch_bounds__(256) k_qso_los(QsoLosArgs a) {
  constexpr double kTwo32 = 4294967296.0;
  constexpr double kCKms = 299792.458;
  for (int64_t q = blockIdx.x * 256ll + threadIdx.x; q < a.n_q; q += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t p[3] = {a.pos[3 * q], a.pos[3 * q + 1], a.pos[3 * q + 2]};
    double d[3], chi2 = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
      d[ax] = static_cast<double>(p[ax]) / kTwo32 * a.dx - a.o[ax];
      chi2 += d[ax] * d[ax];
    }
    const double chi = sqrt(chi2);
    double u[3] = {d[0] / chi, d[1] / chi, d[2] / chi};
    // z(chi): the table's value refined by Newton steps on chi(z) (FP64)
    double zc = lerp_tab(a.ztab, chi);
    for (int it = 0; it < 3; ++it) {
      const double x = 1.0 + zc;
      zc -= (chi_of_z_fine(zc, a.om) - chi) * sqrt(a.om * x * x * x + 1.0 - a.om) / kCOverH0;
    }
    double vpar = 0.0;
    if (a.vxy) {
      // periodic trilinear of {v_x, v_y} and v_z at the quasar
      int c0[3], c1[3];
      double w1[3];
      for (int ax = 0; ax < 3; ++ax) {
        const int64_t cell = p[ax] >> 32;
        c0[ax] = static_cast<int>(((cell % a.n) + a.n) % a.n);
        c1[ax] = c0[ax] + 1 == a.n ? 0 : c0[ax] + 1;
        w1[ax] = static_cast<double>(p[ax] & 0xffffffffll) / kTwo32;
      }
      double v[3] = {0.0, 0.0, 0.0};
      for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy)
          for (int cz = 0; cz < 2; ++cz) {
            const double w = (cx ? w1[0] : 1.0 - w1[0]) * (cy ? w1[1] : 1.0 - w1[1]) * (cz ? w1[2] : 1.0 - w1[2]);
            const size_t e = static_cast<size_t>(cx ? c1[0] : c0[0]) * a.pitch +
                             static_cast<size_t>(cy ? c1[1] : c0[1]) * a.n + (cz ? c1[2] : c0[2]);
            const float2 xy = a.vxy[e];
            v[0] += w * xy.x;
            v[1] += w * xy.y;
            v[2] += w * a.vz[e].x;
          }
      vpar = (v[0] * u[0] + v[1] * u[1] + v[2] * u[2]) * lerp_tab(a.vtab, chi);
    }
    const double zq = zc + (1.0 + zc) * vpar / kCKms;
    const double z_hi = (1.0 + zq) * a.r_hi - 1.0;
    const double z_lo = fmax((1.0 + zq) * a.r_lo - 1.0, a.z_min);
    const double c_hi = chi_of_z_fine(z_hi, a.om);
    int np = 0;
    if (z_hi > z_lo) np = static_cast<int>(fmin(floor((c_hi - chi_of_z_fine(z_lo, a.om)) / a.dchi), 2048.0));
    a.z_q[q] = zq;
    a.chi0[q] = c_hi;
    a.npix[q] = np;
    for (int ax = 0; ax < 3; ++ax) {
      a.origin[3 * q + ax] = llrint((a.o[ax] + u[ax] * c_hi) / a.dx * kTwo32);
      a.step[3 * q + ax] = llrint(-u[ax] * a.dchi / a.dx * kTwo32);
    }
  }
}

// Exclusive prefix sum of npix into offset, and the total (one block).
__global__ void __launch_bounds__(1024) k_qso_offsets(const int32_t* __restrict__ npix, int64_t n_q,
                                                      int64_t* __restrict__ offset, int64_t* __restrict__ total) {
  __shared__ int wsum[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long run = 0;
  for (int64_t base = 0; base < n_q; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int v = i < n_q ? npix[i] : 0;
    int x = v;  // inclusive scan in the wave (a chunk sums to at most 2^21)
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int before = 0, chunk = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wv) before += wsum[k];
      chunk += wsum[k];
    }
    if (i < n_q) offset[i] = run + before + x - v;
    run += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = run;
}

hipError_t launch_qso_los(const QsoLosArgs& a, float* ztab_w, float* vtab_w, hipStream_t st) {
  hipError_t e = launch_zchi_table(a.om, ztab_w, st);
  if (e != hipSuccess) return e;
  LYA_TIMED("qso_vtab", st, hipLaunchKernelGGL(k_qso_vtab, dim3((kZTabN + 255) / 256), dim3(256), 0, st, ztab_w,
                                               a.om, vtab_w));
  if (a.n_q > 0) {
    const int64_t blocks = std::min<int64_t>((a.n_q + 255) / 256, static_cast<int64_t>(device_cus()) * 16);
    LYA_TIMED("qso_los", st, hipLaunchKernelGGL(k_qso_los, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a));
  }
  LYA_TIMED("qso_offsets", st,
            hipLaunchKernelGGL(k_qso_offsets, dim3(1), dim3(1024), 0, st, a.npix, a.n_q, a.offset, a.total));
  return hipGetLastError();
}

}  // namespace lya
