// Lines of sight, small-scale field and FGPA (gfx950).
//
// For every quasar line of sight (section "Gaussian fields along lines of
// sight" and eq:gfield, eq:FGPA):
//   * pixel j sits at the int64 fixed-point position origin + j*step (cell
//     units x 2^32); delta_L and eta_par come from periodic trilinear
//     interpolation of the packed {delta, eta} box;
//   * delta_S: Philox normals (stream 1, counter (q<<33)+m) on modes
//     m = 0..N_S/2 of a length N_S = next_pow2(n_q) line, scaled by
//     sqrt(P_s(k_m)/(N_S dpix)), P_s = amp exp(-(k/kcut)^2), inverse FFT in LDS;
//   * g = delta_L + delta_S + c(z) eta_par, F = exp(-a(z) exp(b(z) g)), with
//     a, b, c quadratics in (1+z) and z the unperturbed redshift of
//     chi_j = chi0 - j*dchi (section "FGPA");
//   * per redshift bin, the sum of F and the pixel count, accumulated as
//     exact 64-bit integers of round(F 2^32), so the result does not depend on
//     the order in which work is scheduled.
// One persistent launch: blocks pull chunks of skewers from an atomic queue.
#include "lya_internal.h"

namespace lya {

constexpr int kSkNT = 256;

__global__ void __launch_bounds__(256) k_skewer_reset(unsigned int* queue, unsigned long long* bsum,
                                                      unsigned long long* bcnt) {
  const int t = threadIdx.x;
  if (t == 0) queue[0] = 0u;
  if (t < kMaxZBins) {
    bsum[t] = 0ull;
    bcnt[t] = 0ull;
  }
}

__global__ void __launch_bounds__(256) k_skewer_finalize(int n_bins, const unsigned long long* bsum,
                                                         const unsigned long long* bcnt, double* fsum,
                                                         int64_t* cnt) {
  const int t = threadIdx.x;
  if (t < n_bins) {
    if (fsum) fsum[t] = static_cast<double>(bsum[t]) * 2.3283064365386963e-10;  // 2^-32
    if (cnt) cnt[t] = static_cast<int64_t>(bcnt[t]);
  }
}

__device__ __forceinline__ float2 ld_field(const SkewerArgs& a, size_t i) {
  if (a.field) return a.field[i];
  return unpack_bf16x2(a.field_bf16[i]);
}

// delta_S of skewer (qid, npix) into one of the two LDS buffers; returns it.
__device__ float2* small_scale(const SkewerArgs& a, int64_t qid, int npix, float2 (*buf)[2048]) {
  int ns = 1;
  while (ns < npix) ns <<= 1;
  const int tid = threadIdx.x;
  const float amp_scale = static_cast<float>(a.ps_amp / (ns * a.dpix));
  const float dk = static_cast<float>(2.0 * M_PI / (ns * a.dpix));
  const float ikc = static_cast<float>(1.0 / a.ps_kcut);
  for (int m = tid; m <= ns / 2; m += kSkNT) {
    float2 y = make_float2(0.0f, 0.0f);
    if (m > 0) {
      const float k = dk * m;
      const float kk = k * ikc;
      const float amp = sqrtf(amp_scale * expf(-kk * kk));
      const float2 z = normal_pair(a.seed, 1u, (static_cast<uint64_t>(qid) << 33) + static_cast<uint64_t>(m));
      float2 w = (m == ns / 2) ? make_float2(z.x, 0.0f) : make_float2(z.x * kSqrtHalf, z.y * kSqrtHalf);
      if (a.ps_fixed_amp) {
        const float r = rsqrtf(w.x * w.x + w.y * w.y);
        w.x *= r;
        w.y *= r;
      }
      y = make_float2(amp * w.x, amp * w.y);
    }
    buf[0][m] = y;
    if (m > 0 && m < ns / 2) buf[0][ns - m] = make_float2(y.x, -y.y);
  }
  __syncthreads();
  int src = 0;
  for (int s = 1; s < ns;) {
    const int R = (ns / s >= 4) ? 4 : 2;
    const int nb = ns / R;
    const float2* in = buf[src];
    float2* out = buf[src ^ 1];
    for (int j = tid; j < nb; j += kSkNT) {
      const int k = j % s;
      float2 v[4];
      for (int r = 0; r < R; ++r) v[r] = in[j + r * nb];
      if (s > 1) {
        const int step = kTw2048 / (s * R);
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], a.tw2048[r * k * step]);
      }
      if (R == 4) {
        dft4(v[0], v[1], v[2], v[3]);
      } else {
        dft2(v[0], v[1]);
      }
      const int base = (j / s) * s * R + k;
      for (int r = 0; r < R; ++r) out[base + r * s] = v[r];
    }
    __syncthreads();
    src ^= 1;
    s *= R;
  }
  return buf[src];
}

__device__ __forceinline__ float trilerp(float tx, float ty, float tz, float c000, float c001, float c010, float c011,
                                         float c100, float c101, float c110, float c111) {
  const float c00 = c000 + tz * (c001 - c000);
  const float c01 = c010 + tz * (c011 - c010);
  const float c10 = c100 + tz * (c101 - c100);
  const float c11 = c110 + tz * (c111 - c110);
  const float c0 = c00 + ty * (c01 - c00);
  const float c1 = c10 + ty * (c11 - c10);
  return c0 + tx * (c1 - c0);
}

__global__ void __launch_bounds__(kSkNT) k_skewers(SkewerArgs a) {
  __shared__ float2 sbuf[2][2048];
  __shared__ unsigned long long s_sum[kMaxZBins], s_cnt[kMaxZBins];
  __shared__ double s_edges[kMaxZBins + 1];
  __shared__ int s_chunk;
  const int tid = threadIdx.x;
  for (int b = tid; b < kMaxZBins; b += kSkNT) {
    s_sum[b] = 0ull;
    s_cnt[b] = 0ull;
  }
  if (a.n_bins > 0 && a.chi_edges)
    for (int b = tid; b <= a.n_bins; b += kSkNT) s_edges[b] = a.chi_edges[b];
  const int N = a.n;
  const size_t NN = plane_pitch(N);
  const bool gather = a.in_dens == nullptr;
  const bool want_bins = a.n_bins > 0 && a.do_flux;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_chunk = static_cast<int>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int64_t q0 = static_cast<int64_t>(s_chunk) * a.chunk;
    if (q0 >= a.n_sk) break;
    const int64_t q1 = q0 + a.chunk < a.n_sk ? q0 + a.chunk : a.n_sk;
    for (int64_t q = q0; q < q1; ++q) {
      const int np = a.npix[q];
      const int64_t off = a.offset[q];
      const float2* ds = nullptr;
      // delta_S needs next_pow2(npix) <= 2048 (the LDS line); longer skewers get none
      if (gather && a.ps_amp > 0.0 && np <= 2048) ds = small_scale(a, a.id_base + q, np, sbuf);
      int64_t ox = 0, oy = 0, oz = 0, sx = 0, sy = 0, sz = 0;
      if (gather) {
        ox = a.origin_fx[3 * q];
        oy = a.origin_fx[3 * q + 1];
        oz = a.origin_fx[3 * q + 2];
        sx = a.step_fx[3 * q];
        sy = a.step_fx[3 * q + 1];
        sz = a.step_fx[3 * q + 2];
      }
      const double chi0 = a.chi0[q];
      for (int j = tid; j < np; j += kSkNT) {
        float d, e;
        if (gather) {
          const int64_t px = ox + j * sx, py = oy + j * sy, pz = oz + j * sz;
          const int ix = static_cast<int>((px >> 32) & (N - 1));
          const int iy = static_cast<int>((py >> 32) & (N - 1));
          const int iz = static_cast<int>((pz >> 32) & (N - 1));
          const int jx = (ix + 1) & (N - 1), jy = (iy + 1) & (N - 1), jz = (iz + 1) & (N - 1);
          const float tx = static_cast<float>(static_cast<uint32_t>(px)) * 2.3283064365386963e-10f;
          const float ty = static_cast<float>(static_cast<uint32_t>(py)) * 2.3283064365386963e-10f;
          const float tz = static_cast<float>(static_cast<uint32_t>(pz)) * 2.3283064365386963e-10f;
          const size_t r00 = ix * NN + static_cast<size_t>(iy) * N;
          const size_t r01 = ix * NN + static_cast<size_t>(jy) * N;
          const size_t r10 = jx * NN + static_cast<size_t>(iy) * N;
          const size_t r11 = jx * NN + static_cast<size_t>(jy) * N;
          const float2 c000 = ld_field(a, r00 + iz), c001 = ld_field(a, r00 + jz);
          const float2 c010 = ld_field(a, r01 + iz), c011 = ld_field(a, r01 + jz);
          const float2 c100 = ld_field(a, r10 + iz), c101 = ld_field(a, r10 + jz);
          const float2 c110 = ld_field(a, r11 + iz), c111 = ld_field(a, r11 + jz);
          d = trilerp(tx, ty, tz, c000.x, c001.x, c010.x, c011.x, c100.x, c101.x, c110.x, c111.x);
          e = trilerp(tx, ty, tz, c000.y, c001.y, c010.y, c011.y, c100.y, c101.y, c110.y, c111.y);
          if (ds) d += ds[j].x;
          if (a.dens) a.dens[off + j] = d;
          if (a.eta) a.eta[off + j] = e;
        } else {
          d = a.in_dens[off + j];
          e = a.in_eta[off + j];
        }
        if (a.do_flux) {
          const double chi = __dsub_rn(chi0, __dmul_rn(static_cast<double>(j), a.dchi));
          const double u = chi * (1.0 / kZTabH);
          int iu = static_cast<int>(u);
          iu = iu < 0 ? 0 : (iu > kZTabN - 2 ? kZTabN - 2 : iu);
          const float t = static_cast<float>(u - iu);
          const float zt0 = a.ztab[iu], zt1 = a.ztab[iu + 1];
          const double x = 1.0 + static_cast<double>(zt0 + t * (zt1 - zt0));
          const float ca = static_cast<float>(a.coef[0][0] + x * (a.coef[0][1] + x * a.coef[0][2]));
          const float cb = static_cast<float>(a.coef[1][0] + x * (a.coef[1][1] + x * a.coef[1][2]));
          const float cc = static_cast<float>(a.coef[2][0] + x * (a.coef[2][1] + x * a.coef[2][2]));
          const float F = expf(-ca * expf(cb * (d + cc * e)));
          if (a.flux) a.flux[off + j] = F;
          if (want_bins && chi >= s_edges[0] && chi < s_edges[a.n_bins]) {
            int lo = 0, hi = a.n_bins;  // edges[lo] <= chi < edges[hi]
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (chi >= s_edges[mid]) lo = mid; else hi = mid;
            }
            atomicAdd(&s_sum[lo], static_cast<unsigned long long>(__float2ull_rn(F * 4294967296.0f)));
            atomicAdd(&s_cnt[lo], 1ull);
          }
        }
      }
      __syncthreads();  // the small-scale buffers are reused by the next skewer
    }
  }
  if (want_bins) {
    __syncthreads();
    for (int b = tid; b < a.n_bins; b += kSkNT) {
      if (s_cnt[b]) {
        atomicAdd(&a.bin_sum[b], s_sum[b]);
        atomicAdd(&a.bin_cnt[b], s_cnt[b]);
      }
    }
  }
}

static int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

hipError_t launch_skewers(const SkewerArgs& a, hipStream_t st) {
  LYA_TIMED("skewer_reset", st,
            hipLaunchKernelGGL(k_skewer_reset, dim3(1), dim3(256), 0, st, a.queue, a.bin_sum, a.bin_cnt));
  const int64_t nchunks = (a.n_sk + a.chunk - 1) / a.chunk;
  int64_t blocks = static_cast<int64_t>(device_cus()) * 4;
  if (blocks > nchunks) blocks = nchunks;
  if (blocks < 1) blocks = 1;
  LYA_TIMED(a.in_dens ? "apply_fgpa" : "skewers", st,
            hipLaunchKernelGGL(k_skewers, dim3(static_cast<unsigned>(blocks)), dim3(kSkNT), 0, st, a));
  if (a.n_bins > 0 && a.do_flux)
    LYA_TIMED("skewer_finalize", st,
              hipLaunchKernelGGL(k_skewer_finalize, dim3(1), dim3(256), 0, st, a.n_bins, a.bin_sum, a.bin_cnt,
                                 a.out_fsum, a.out_count));
  return hipGetLastError();
}

}  // namespace lya
