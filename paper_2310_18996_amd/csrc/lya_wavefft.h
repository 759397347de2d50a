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


}  // namespace lya
