// Batched evaluation of the tuning statistics (gfx950): for G parameter draws
// (a, b, c) held constant over every stored pixel (the paper's reuse of saved
// forests, section "Adjusting mock parameters"), the mean flux of all pixels
// and the binned P1D of delta_F = F/Fbar - 1 with velocity units of the draw.
// Optionally each draw also carries a small-scale spectrum P_s, and delta_S is
// drawn again per draw and skewer (the P_s iteration's redraw) and added to
// the stored delta_L before the FGPA.
//
// One pass over the pixels for all G draws: a wavefront owns a skewer, holds
// its first 2048 (dens, eta) pixels in registers and, per draw, forms F, adds
// it to the skewer's sum and transforms the first N_P pixels in its LDS slice.
// For m >= 1 the DFT of F/Fbar - 1 is the DFT of F divided by Fbar (the
// constant only enters m = 0), so the periodogram is taken of F itself and
// divided by Fbar^2 once Fbar, a sum over all skewers, is known:
//   P_b = Dv sum_{q, m in b} |X_m(F_q)|^2 / N_P,q / (Fbar^2 count_b).
// Per-skewer partial sums are written in fixed order and reduced over skewers
// in a fixed tree, so the result does not depend on scheduling.
#include "lya_internal.h"
#include "lya_wavefft.h"

namespace lya {

constexpr int kTeWaves = 4;
constexpr int kTeNT = 64 * kTeWaves;
constexpr int kTeReg = 32;  // pixels per lane kept in registers (2048 per wave)

__global__ void __launch_bounds__(64) k_te_reset(unsigned int* queue) {
  if (threadIdx.x == 0) queue[0] = 0u;
}

// DS: delta_S redrawn per draw (a separate instantiation, so that the plain
// evaluation keeps its register budget).
template <bool DS>
__global__ void __launch_bounds__(kTeNT, 2) k_tune_eval(TuneEvalArgs a) {
  __shared__ float2 sbuf[kTeWaves][kHalfBuf];
  __shared__ float spw[kTeWaves][kHalfMax + 1];
  __shared__ int smlo[kTeWaves][kMaxKBins + 1];
  __shared__ float2 stw[kTw2048];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  load_twiddles(stw, a.tw2048, threadIdx.x, kTeNT);
  __syncthreads();
  float2* buf = sbuf[wv];
  float* bf = reinterpret_cast<float*>(buf);
  float* pw = spw[wv];
  int* mlo = smlo[wv];
  const int nk = a.nk;
  const int64_t ld = a.n_sk;
  for (;;) {
    int c = 0;
    if (lane == 0) c = static_cast<int>(atomicAdd(a.queue, 1u));
    c = __builtin_amdgcn_readfirstlane(__shfl(c, 0));
    const int64_t q0 = static_cast<int64_t>(static_cast<uint32_t>(c)) * a.chunk;  // pulls stay below 2^32
    if (q0 >= a.n_sk) break;
    const int64_t q1 = q0 + a.chunk < a.n_sk ? q0 + a.chunk : a.n_sk;
    for (int64_t q = q0; q < q1; ++q) {
      const int np = a.npix[q];
      const int64_t off = a.offset[q];
      const int n_p = np >= 2 ? 1 << (31 - __clz(np < 2 * kHalfMax ? np : 2 * kHalfMax)) : 0;
      const int M = n_p / 2;
      float d[kTeReg], e[kTeReg];
#pragma unroll
      for (int i = 0; i < kTeReg; ++i) {
        const int j = lane + 64 * i;
        d[i] = j < np ? a.dens[off + j] : 0.0f;
        e[i] = j < np ? a.eta[off + j] : 0.0f;
      }
      int ns = 1;
      while (ns < np) ns <<= 1;
      const bool with_ds = DS && ns >= 2;
      for (int g = 0; g < a.G; ++g) {
        const float ca = a.draw[g][0], cb = a.draw[g][1], cc = a.draw[g][2];
        double* ps = a.ps + static_cast<int64_t>(g) * nk * ld + q;
        int* pc = a.pc + static_cast<int64_t>(g) * nk * ld + q;
        if (with_ds && ns > 2 * kHalfMax) {
          // delta_S exists on lines of at most 2048 pixels: an input error,
          // which makes this draw's mean flux (and so its P1D) NaN
          if (lane == 0) a.fs[g * ld + q] = __builtin_nan("");
          for (int b = lane; b < nk; b += 64) {
            ps[b * ld] = 0.0;
            pc[b * ld] = 0;
          }
          continue;
        }
        if (with_ds) {
          // delta_S into the LDS line; each lane then reads and overwrites
          // only its own pixels' slots (pixel j at bf[2 pidx(j/2) + j%2])
          // (the radix-4 FFT: this kernel keeps 64 pixel registers live)
          small_scale_wave<TuneEvalArgs, false>(a, a.ds_amp[g], a.ds_kcut[g], static_cast<uint64_t>(a.id_base + q),
                                                ns, buf, stw, lane);
        }
        double fsum = 0.0;
#pragma unroll
        for (int i = 0; i < kTeReg; ++i) {
          const int j = lane + 64 * i;
          if (j < np) {
            const int slot = 2 * pidx(j >> 1) + (j & 1);
            const float delta = with_ds ? d[i] + bf[slot] : d[i];
            const float F = __expf(-ca * __expf(cb * (delta + cc * e[i])));
            fsum += F;
            if (j < n_p) bf[slot] = F;
          }
        }
        for (int j = 64 * kTeReg + lane; j < np; j += 64)  // pixels beyond the register window (no delta_S here)
          fsum += __expf(-ca * __expf(cb * (a.dens[off + j] + cc * a.eta[off + j])));
#pragma unroll
        for (int w = 32; w >= 1; w >>= 1) fsum += __shfl_xor(fsum, w);
        if (lane == 0) a.fs[g * ld + q] = fsum;
        if (M == 0) {
          for (int b = lane; b < nk; b += 64) {
            ps[b * ld] = 0.0;
            pc[b * ld] = 0;
          }
          continue;
        }
        wave_sync();
        wave_ifft(buf, M, stw, lane);
        const int twstep = kTw2048 / n_p;
        for (int m = lane + 1; m <= M; m += 64) {
          const float2 zm = buf[pidx(m == M ? 0 : m)];
          const float2 zc = buf[pidx(M - m)];
          const float2 E = make_float2(0.5f * (zm.x + zc.x), 0.5f * (zm.y - zc.y));
          const float2 O = make_float2(0.5f * (zm.y + zc.y), -0.5f * (zm.x - zc.x));
          const float2 X = cadd(E, cmul(stw[m * twstep], O));
          pw[m] = X.x * X.x + X.y * X.y;
        }
        // first mode of each k bin: smallest m >= 1 with k_m >= edge (M+1 if none)
        const double dv = a.dv[g];
        const double kf = 2.0 * M_PI / (n_p * dv);
        for (int b = lane; b <= nk; b += 64) {
          const double ed = a.k_edges[b];
          double m0 = ceil(ed / kf);
          m0 = m0 < 1.0 ? 1.0 : (m0 > M + 1.0 ? M + 1.0 : m0);
          int m = static_cast<int>(m0);
          while (m <= M && (2.0 * M_PI * m) / (n_p * dv) < ed) ++m;
          while (m > 1 && (2.0 * M_PI * (m - 1)) / (n_p * dv) >= ed) --m;
          mlo[b] = m;
        }
        wave_sync();
        const double inv_np = 1.0 / n_p;
        for (int b = lane; b < nk; b += 64) {
          double s = 0.0;
          for (int m = mlo[b]; m < mlo[b + 1]; ++m) s += pw[m];
          ps[b * ld] = s * inv_np;
          pc[b * ld] = mlo[b + 1] - mlo[b];
        }
        wave_sync();
      }
    }
  }
}

// Per draw g (blockIdx.y): blockIdx.x < nk sums bin blockIdx.x over the
// skewers, blockIdx.x == nk sums the flux and the pixel count; fixed order.
__global__ void __launch_bounds__(256) k_te_reduce(TuneEvalArgs a, double* sums, int64_t* counts) {
  __shared__ double ss[256];
  __shared__ long long sc[256];
  const int b = blockIdx.x, g = blockIdx.y, t = threadIdx.x, nk = a.nk;
  const int64_t ld = a.n_sk;
  double s = 0.0;
  long long c = 0;
  if (b < nk) {
    const double* ps = a.ps + (static_cast<int64_t>(g) * nk + b) * ld;
    const int* pc = a.pc + (static_cast<int64_t>(g) * nk + b) * ld;
    for (int64_t q = t; q < ld; q += 256) {
      s += ps[q];
      c += pc[q];
    }
  } else {
    const double* fs = a.fs + static_cast<int64_t>(g) * ld;
    for (int64_t q = t; q < ld; q += 256) {
      s += fs[q];
      c += a.npix[q];
    }
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
    sums[g * (nk + 1) + b] = ss[0];
    counts[g * (nk + 1) + b] = sc[0];
  }
}

// Statistics per draw: Fbar, then P_b (NaN for an empty bin); FP64 rows and,
// when rows32 is given, FP32 rows (emulator labels).
__global__ void __launch_bounds__(64) k_te_stats(TuneEvalArgs a, const double* __restrict__ sums,
                                                 const int64_t* __restrict__ counts, double* rows, float* rows32) {
  const int g = blockIdx.x, t = threadIdx.x, nk = a.nk;
  const double* dv = a.dv;
  const double* s = sums + g * (nk + 1);
  const int64_t* c = counts + g * (nk + 1);
  const double fbar = c[nk] > 0 ? s[nk] / static_cast<double>(c[nk]) : NAN;
  for (int b = t; b <= nk; b += 64) {
    double v;
    if (b == 0) {
      v = fbar;
    } else {
      const int k = b - 1;
      v = c[k] > 0 ? dv[g] * s[k] / (fbar * fbar * static_cast<double>(c[k])) : NAN;
    }
    if (rows) rows[g * (nk + 1) + b] = v;
    if (rows32) rows32[g * (nk + 1) + b] = static_cast<float>(v);
  }
}

hipError_t launch_tune_eval(const TuneEvalArgs& a, double* sums, int64_t* counts, double* rows, float* rows32,
                            hipStream_t st) {
  if (a.G < 1 || a.G > kTuneEvalMaxG || a.nk < 1 || a.nk > kMaxKBins) return hipErrorInvalidValue;
  LYA_TIMED("tune_eval_reset", st, hipLaunchKernelGGL(k_te_reset, dim3(1), dim3(64), 0, st, a.queue));
  const int64_t nchunks = (a.n_sk + a.chunk - 1) / a.chunk;
  int64_t blocks = static_cast<int64_t>(device_cus()) * 3;
  if (blocks * kTeWaves > nchunks) blocks = (nchunks + kTeWaves - 1) / kTeWaves;
  if (blocks < 1) blocks = 1;
  const dim3 grid(static_cast<unsigned>(blocks));
  if (a.n_sk > 0 && a.with_ds)
    LYA_TIMED("tune_eval_ds", st, hipLaunchKernelGGL(k_tune_eval<true>, grid, dim3(kTeNT), 0, st, a));
  else if (a.n_sk > 0)
    LYA_TIMED("tune_eval", st, hipLaunchKernelGGL(k_tune_eval<false>, grid, dim3(kTeNT), 0, st, a));
  LYA_TIMED("tune_eval_reduce", st,
            hipLaunchKernelGGL(k_te_reduce, dim3(a.nk + 1, a.G), dim3(256), 0, st, a, sums, counts));
  LYA_TIMED("tune_eval_stats", st,
            hipLaunchKernelGGL(k_te_stats, dim3(a.G), dim3(64), 0, st, a, sums, counts, rows, rows32));
  return hipGetLastError();
}

}  // namespace lya
