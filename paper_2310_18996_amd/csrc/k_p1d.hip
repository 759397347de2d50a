// 1D flux power spectrum (gfx950).
//
// delta_F = F / Fbar - 1 (equation::definition_delta) on the first
// N_P = min(2^floor(log2 n_q), 2048) pixels of every skewer, Fbar taken per distance bin
// from given sums; periodogram P(k_m) = Dv |X_m|^2 / N_P for m = 1..N_P/2 with
// k_m = 2 pi m / (N_P Dv) (Dv one FP64 constant, the pixel at the reference
// redshift); the modes of each skewer are summed per k bin in FP64 in a fixed
// order and written per skewer, then a second kernel sums the skewers per bin
// in a fixed order (so the result does not depend on scheduling).
//
// The real DFT of length N_P is one complex FFT of length M = N_P/2 on
// z_n = d(2n) + i d(2n+1); with Z its transform (sign +, whose modulus equals
// the forward one's for real input) the full-length coefficient is
// X_m = (Z_m + conj Z_{M-m})/2 + w^m (Z_m - conj Z_{M-m})/(2i), w = exp(2 pi i/N_P).
#include "lya_internal.h"
#include "lya_wavefft.h"

namespace lya {

constexpr int kPdWaves = 4;
constexpr int kPdNT = 64 * kPdWaves;

__global__ void __launch_bounds__(64) k_p1d_reset(unsigned int* queue) {
  if (threadIdx.x == 0) queue[0] = 0u;
}

__global__ void __launch_bounds__(kPdNT) k_p1d(P1dArgs a) {
  __shared__ float2 sbuf[kPdWaves][kHalfBuf];
  __shared__ float spw[kPdWaves][kHalfMax + 1];
  __shared__ int sjb[kPdWaves][kMaxZBins + 1];
  __shared__ int smlo[kPdWaves][kMaxKBins + 1];
  __shared__ float sfm[kMaxZBins];
  __shared__ float2 stw[kTw2048];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  load_twiddles(stw, a.tw2048, tid, kPdNT);
  for (int b = tid; b < a.n_fbins; b += kPdNT) {
    const double c = static_cast<double>(a.fcount[b]);
    sfm[b] = c > 0.0 ? static_cast<float>(a.fsum[b] / c) : 1.0f;
  }
  __syncthreads();
  float2* buf = sbuf[wv];
  float* pw = spw[wv];
  int* jb = sjb[wv];
  int* mlo = smlo[wv];
  const int nk = a.n_kbins;
  for (;;) {
    int c = 0;
    if (lane == 0) c = static_cast<int>(atomicAdd(a.queue, 1u));
    c = __builtin_amdgcn_readfirstlane(__shfl(c, 0));
    const int64_t q0 = static_cast<int64_t>(static_cast<uint32_t>(c)) * a.chunk;  // pulls stay below 2^32
    if (q0 >= a.n_sk) break;
    const int64_t q1 = q0 + a.chunk < a.n_sk ? q0 + a.chunk : a.n_sk;
    for (int64_t q = q0; q < q1; ++q) {
      const int np = a.npix[q];
      // per-skewer partial sums, bin-major: [b][q]
      double* psum = a.part_sum + q;
      int* pcnt = a.part_cnt + q;
      const int64_t ld = a.n_sk;
      if (np < 2) {
        for (int b = lane; b < nk; b += 64) {
          psum[b * ld] = 0.0;
          pcnt[b * ld] = 0;
        }
        continue;
      }
      const int n_p = 1 << (31 - __clz(np < 2 * kHalfMax ? np : 2 * kHalfMax));
      const int M = n_p / 2;
      const int64_t off = a.offset[q];
      const double chi0 = a.chi0[q];
      bin_bounds(a.chi_edges, a.n_fbins, chi0, a.dchi, n_p, jb, lane);
      wave_sync();
      for (int n = lane; n < M; n += 64) {
        float d[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int j = 2 * n + e;
          // number of edges with jb > j: pixel j lies in bin cnt-1 (clamped)
          int lo = 0, hi = a.n_fbins + 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (jb[mid] > j) lo = mid + 1; else hi = mid;
          }
          int b = lo - 1;
          b = b < 0 ? 0 : (b > a.n_fbins - 1 ? a.n_fbins - 1 : b);
          const float F = a.flux ? a.flux[off + j]
                                 : __expf(-a.fa * __expf(a.fb * (a.dens[off + j] + a.fc * a.eta[off + j])));
          d[e] = F / sfm[b] - 1.0f;
        }
        buf[pidx(n)] = make_float2(d[0], d[1]);
      }
      wave_sync();
      wave_ifft(buf, M, stw, lane);
      const int twstep = kTw2048 / n_p;
      const float scale = static_cast<float>(a.dv / n_p);
      for (int m = lane + 1; m <= M; m += 64) {
        const float2 zm = buf[pidx(m == M ? 0 : m)];
        const float2 zc = buf[pidx(M - m)];
        const float2 E = make_float2(0.5f * (zm.x + zc.x), 0.5f * (zm.y - zc.y));
        const float2 O = make_float2(0.5f * (zm.y + zc.y), -0.5f * (zm.x - zc.x));
        const float2 X = cadd(E, cmul(stw[m * twstep], O));
        pw[m] = scale * (X.x * X.x + X.y * X.y);
      }
      // first mode of each k bin: smallest m >= 1 with k_m >= edge (M+1 if none)
      const double kf = 2.0 * M_PI / (n_p * a.dv);
      for (int b = lane; b <= nk; b += 64) {
        const double e = a.k_edges[b];
        double m0 = ceil(e / kf);
        m0 = m0 < 1.0 ? 1.0 : (m0 > M + 1.0 ? M + 1.0 : m0);
        int m = static_cast<int>(m0);
        while (m <= M && (2.0 * M_PI * m) / (n_p * a.dv) < e) ++m;
        while (m > 1 && (2.0 * M_PI * (m - 1)) / (n_p * a.dv) >= e) --m;
        mlo[b] = m;
      }
      wave_sync();
      for (int b = lane; b < nk; b += 64) {
        double s = 0.0;
        for (int m = mlo[b]; m < mlo[b + 1]; ++m) s += pw[m];
        psum[b * ld] = s;
        pcnt[b * ld] = mlo[b + 1] - mlo[b];
      }
      wave_sync();
    }
  }
}

// per k bin: sum over skewers in a fixed order (strided partial sums over the
// bin's contiguous row, then a fixed tree), FP64 sum and int64 count
__global__ void __launch_bounds__(256) k_p1d_reduce(int64_t n_sk, int nk, const double* __restrict__ part_sum,
                                                   const int* __restrict__ part_cnt, double* psum, int64_t* pcount) {
  __shared__ double ss[256];
  __shared__ long long sc[256];
  const int b = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  long long c = 0;
  const double* ps = part_sum + static_cast<int64_t>(b) * n_sk;
  const int* pc = part_cnt + static_cast<int64_t>(b) * n_sk;
  for (int64_t q = t; q < n_sk; q += 256) {
    s += ps[q];
    c += pc[q];
  }
  ss[t] = s;
  sc[t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      ss[t] += ss[t + w];
      sc[t] += sc[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (psum) psum[b] = ss[0];
    if (pcount) pcount[b] = sc[0];
  }
}

hipError_t launch_p1d(const P1dArgs& a, double* psum, int64_t* pcount, hipStream_t st) {
  LYA_TIMED("p1d_reset", st, hipLaunchKernelGGL(k_p1d_reset, dim3(1), dim3(64), 0, st, a.queue));
  const int64_t nchunks = (a.n_sk + a.chunk - 1) / a.chunk;
  int64_t blocks = static_cast<int64_t>(device_cus()) * 3;
  if (blocks * kPdWaves > nchunks) blocks = (nchunks + kPdWaves - 1) / kPdWaves;
  if (blocks < 1) blocks = 1;
  if (a.n_sk > 0) LYA_TIMED("p1d", st, hipLaunchKernelGGL(k_p1d, dim3(static_cast<unsigned>(blocks)), dim3(kPdNT), 0, st, a));
  LYA_TIMED("p1d_reduce", st,
            hipLaunchKernelGGL(k_p1d_reduce, dim3(a.n_kbins), dim3(256), 0, st, a.n_sk, a.n_kbins, a.part_sum,
                               a.part_cnt, psum, pcount));
  return hipGetLastError();
}

}  // namespace lya
