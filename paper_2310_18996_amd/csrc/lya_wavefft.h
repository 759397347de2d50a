// Per-line helpers shared by the skewer and 1D-power kernels: pixel distances,
// distance-bin boundaries, and a wavefront-level FFT in LDS (one wavefront owns
// a line of up to kHalfMax complex values in its slice of LDS and transforms it
// in place, without block barriers).
#pragma once

#include "lya_internal.h"

namespace lya {

constexpr int kHalfMax = 1024;                        // complex length <= 1024
constexpr int kHalfBuf = kHalfMax + kHalfMax / 16;    // one padding slot per 16

__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Comoving distance of pixel j: chi0 - (j * dchi), each operation rounded in
// FP64 (no fused multiply-add), as the C-ABI defines it.
__device__ __forceinline__ double pixel_chi(double chi0, int j, double dchi) {
  return __dsub_rn(chi0, __dmul_rn(static_cast<double>(j), dchi));
}

// jb[b] = first pixel j in [0, np] with chi_j < edges[b], for b = 0..n_bins
// (chi_j decreases with j), so pixel j lies in distance bin b exactly when
// jb[b+1] <= j < jb[b].  Lanes split the edges; exact FP64 comparisons.
__device__ __forceinline__ void bin_bounds(const double* __restrict__ edges, int n_bins, double chi0, double dchi,
                                           int np, int* jb, int lane) {
  for (int b = lane; b <= n_bins; b += 64) {
    const double e = edges[b];
    double j0 = dchi > 0.0 ? ceil((chi0 - e) / dchi) : 0.0;
    j0 = j0 < 0.0 ? 0.0 : (j0 > np ? np : j0);
    int j = static_cast<int>(j0);
    while (j < np && pixel_chi(chi0, j, dchi) >= e) ++j;
    while (j > 0 && pixel_chi(chi0, j - 1, dchi) < e) --j;
    jb[b] = j;
  }
}

// The block's copy of the twiddle table tw2048 in LDS (read by every stage of
// every wavefront FFT; global reads would put an L2 round trip in each stage).
__device__ __forceinline__ void load_twiddles(float2* stw, const float2* __restrict__ tw2048, int tid, int nt) {
  for (int i = tid; i < kTw2048; i += nt) stw[i] = tw2048[i];
}

// Unnormalised inverse DFT (exp(+2 pi i k n / M)) of buf[pidx(0..M-1)], M a
// power of two <= kHalfMax, by an in-place Stockham radix-4/2 FFT: every stage
// first reads all of the lane's inputs, then writes (the wave runs in lockstep).
// tw2048[k] = exp(2 pi i k / 2048).
__device__ __forceinline__ void wave_ifft(float2* buf, int M, const float2* tw2048, int lane) {
  for (int s = 1; s < M;) {
    const int R = (M / s >= 4) ? 4 : 2;
    const int nb = M / R;
    float2 v[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = lane + 64 * t;
      if (j < nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r < R) v[t][r] = buf[pidx(j + r * nb)];
      }
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = lane + 64 * t;
      if (j < nb) {
        const int k = j % s;
        if (s > 1) {
          const int step = kTw2048 / (s * R);
#pragma unroll
          for (int r = 1; r < 4; ++r)
            if (r < R) v[t][r] = cmul(v[t][r], tw2048[r * k * step]);
        }
        if (R == 4) {
          dft4(v[t][0], v[t][1], v[t][2], v[t][3]);
        } else {
          dft2(v[t][0], v[t][1]);
        }
        const int base = (j / s) * s * R + k;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r < R) buf[pidx(base + r * s)] = v[t][r];
      }
    }
    wave_sync();
    s *= R;
  }
}

// One radix-R stage of the in-place Stockham FFT wave_ifft8: s = product of the
// radices before it; every lane first reads all of its inputs, then writes.
template <int R>
__device__ __forceinline__ void wave_stage(float2* buf, int M, int s, const float2* tw2048, int lane) {
  constexpr int TMAX = kHalfMax / R / 64 > 0 ? kHalfMax / R / 64 : 1;  // butterflies per lane at M = kHalfMax
  const int nb = M / R;
  float2 v[TMAX][R];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    const int j = lane + 64 * t;
    if (j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[pidx(j + r * nb)];
    }
  }
  wave_sync();
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    const int j = lane + 64 * t;
    if (j < nb) {
      const int k = j % s;
      if (s > 1) {
        const int step = kTw2048 / (s * R);
#pragma unroll
        for (int r = 1; r < R; ++r) v[t][r] = cmul(v[t][r], tw2048[r * k * step]);
      }
      dft<R>(v[t]);
      const int base = (j / s) * s * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx(base + r * s)] = v[t][r];
    }
  }
  wave_sync();
}

// The same inverse DFT as wave_ifft by radix-8 stages (with radix-16 ones
// where they save a stage, then one radix-4 or radix-2 stage for what
// remains): fewer passes through LDS, more registers.
__device__ __forceinline__ void wave_ifft8(float2* buf, int M, const float2* tw2048, int lane) {
  const int lg = 31 - __clz(M);
  int s = 1;
  // radix-16 stages where they save a stage: 16 x 8^k for lg = 1 mod 3,
  // 16 x 16 x 8^k for lg = 2 mod 3 from 256 up
  const int n16 = (lg % 3 == 1 && lg >= 4) ? 1 : (lg % 3 == 2 && lg >= 8) ? 2 : 0;
  for (int i = 0; i < n16; ++i, s *= 16) wave_stage<16>(buf, M, s, tw2048, lane);
  for (; M / s >= 8; s *= 8) wave_stage<8>(buf, M, s, tw2048, lane);
  if (M / s == 4) wave_stage<4>(buf, M, s, tw2048, lane);
  else if (M / s == 2) wave_stage<2>(buf, M, s, tw2048, lane);
}


// ---- the small-scale field delta_S along one line (section "Gaussian fields
// along lines of sight"), shared by the skewer and tuning-evaluation kernels:
// Philox normals (stream 1, counter (qid << 33) + m) on the modes m = 1 ..
// ns/2 of a line of ns pixels, scaled by sqrt(P_s(k_m) / (ns dpix)), the DC
// mode zero, and one half-length complex inverse FFT.

// Mode Y_m of the small-scale spectrum (0 < m <= ns/2) from its normal pair z.
template <class A>
__device__ __forceinline__ float2 ps_mode(const A& a, int m, int ns, float amp_scale, float dk2, float2 z) {
  const float kk = static_cast<float>(m) * static_cast<float>(m) * dk2;   // (k/kcut)^2
  float ratio = 1.0f;
  if (a.ps_ratio) {
    // the mode's k bin (FP64, so the bin decision matches a double-precision
    // reference): the largest b with edge_b <= k, clamped to the table
    const double k = (2.0 * M_PI / (static_cast<double>(ns) * a.dpix)) * m;
    const double* e = a.ps_edges_k;
    int b = 0;
    if (k >= e[a.ps_nb]) {
      b = a.ps_nb - 1;
    } else if (k >= e[0]) {
      int lo = 0, hi = a.ps_nb;   // e[lo] <= k < e[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (e[mid] <= k) lo = mid; else hi = mid;
      }
      b = lo;
    }
    ratio = a.ps_ratio[b];
  }
  const float amp = __builtin_amdgcn_sqrtf(amp_scale * __expf(-kk) * ratio);
  float2 w = (m == ns / 2) ? make_float2(z.x, 0.0f) : make_float2(z.x * kSqrtHalf, z.y * kSqrtHalf);
  if (a.ps_fixed_amp) {
    const float r = rsqrtf(w.x * w.x + w.y * w.y);
    w.x *= r;
    w.y *= r;
  }
  return make_float2(amp * w.x, amp * w.y);
}

// delta_S of one skewer by one wavefront into buf (pixel 2n in .x and pixel
// 2n+1 in .y of element pidx(n)); ns = next_pow2(npix) >= 2.  P_s(k) =
// amp exp(-(k/kcut)^2), times the ratio of k's bin when a.ps_ratio is set.
// A supplies the Philox key (seed), the pixel length (dpix), the optional
// table (ps_nb, ps_edges_k, ps_ratio) and the fixed-amplitude switch
// (ps_fixed_amp).  R8: the radix-8 FFT (fewer LDS passes); otherwise the
// radix-4 one, for callers that cannot spare its registers.
template <class A, bool R8 = true>
__device__ void small_scale_wave(const A& a, double amp, double kcut, uint64_t qid, int ns, float2* buf,
                                 const float2* tw, int lane) {
  const int M = ns / 2;
  const float amp_scale = static_cast<float>(amp / (ns * a.dpix));
  const double dk = 2.0 * M_PI / (ns * a.dpix) / kcut;
  const float dk2 = static_cast<float>(dk * dk);
  const int twstep = kTw2048 / ns;  // w^k = exp(2 pi i k / ns)
  // the modes Y_1 .. Y_M into buf (Y_M in slot 0: the DC mode is zero).  Mode
  // m is linear index (qid << 33) + m of stream 1, so the modes 2i and 2i + 1
  // share one Philox call (counter = linear index >> 1, words 0-1 and 2-3).
  for (int i = lane; i <= M / 2; i += 64) {
    const uint64_t ctr = ((qid << 33) + 2 * static_cast<uint64_t>(i)) >> 1;
    const uint4 wd = philox10_x3(make_uint4(static_cast<uint32_t>(ctr), static_cast<uint32_t>(ctr >> 32), 1u, 0u),
                                 static_cast<uint32_t>(a.seed), static_cast<uint32_t>(a.seed >> 32));
    const int m0 = 2 * i, m1 = 2 * i + 1;
    if (m0 >= 1 && m0 <= M) buf[pidx(m0 == M ? 0 : m0)] = ps_mode(a, m0, ns, amp_scale, dk2, box_muller(wd.x, wd.y));
    if (m1 <= M) buf[pidx(m1 == M ? 0 : m1)] = ps_mode(a, m1, ns, amp_scale, dk2, box_muller(wd.z, wd.w));
  }
  wave_sync();
  // Z_k = (Y_k + Y_{k+M}) + i (Y_k - Y_{k+M}) w^k with Y_{k+M} = conj(Y_{M-k});
  // a lane reads both of its slots k and M - k before writing them
  for (int k = lane; k <= M / 2; k += 64) {
    if (k == 0) {
      const float2 yM = buf[pidx(0)];  // real Nyquist mode
      buf[pidx(0)] = make_float2(yM.x, -yM.x);
      continue;
    }
    const float2 yk = buf[pidx(k)];
    const float2 ymk = buf[pidx(M - k)];
    {
      const float2 s = make_float2(yk.x + ymk.x, yk.y - ymk.y);   // Y_k + conj(Y_{M-k})
      const float2 d = make_float2(yk.x - ymk.x, yk.y + ymk.y);   // Y_k - conj(Y_{M-k})
      const float2 t = cmul(d, tw[k * twstep]);
      buf[pidx(k)] = make_float2(s.x - t.y, s.y + t.x);
    }
    if (M - k != k) {
      const float2 s = make_float2(ymk.x + yk.x, ymk.y - yk.y);
      const float2 d = make_float2(ymk.x - yk.x, ymk.y + yk.y);
      const float2 t = cmul(d, tw[(M - k) * twstep]);
      buf[pidx(M - k)] = make_float2(s.x - t.y, s.y + t.x);
    }
  }
  wave_sync();
  if constexpr (R8) wave_ifft8(buf, M, tw, lane);
  else wave_ifft(buf, M, tw, lane);
}

}  // namespace lya
