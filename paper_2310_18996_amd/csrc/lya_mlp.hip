// Tuning emulator: a 4 -> 256 -> 256 -> 256 -> n_out MLP (GELU hidden layers,
// linear output) mapping FGPA parameters and redshift (a, b, c, z) to the
// statistics the tuning loop matches (mean flux and ln P1D per k bin).
// Training: MSE on standardised inputs and outputs, Adam (Kingma & Ba 2014),
// FP32 master weights; the matrix products run on MFMA in bfloat16 with FP32
// accumulation (v_mfma_f32_16x16x16_bf16), or in plain FP32 for checks.
// Row-vector convention: h = gelu(x W + b), W stored [in][out] row-major.
// GELU is the exact form x Phi(x) = x erfc(-x / sqrt 2) / 2.
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/lyamock.h"
#include "lya_internal.h"
#include "lya_nm.h"

namespace lya {

constexpr int kIn = 4, kHid = 256, kMaxOut = 64;

struct EmuHeader {
  int32_t n_out;
  int32_t step;    // Adam steps taken
  int32_t log_from;
  int32_t in_log;  // bit i: input i enters as ln x
  float in_lo[4], in_hi[4];
  float in_mul[4], in_add[4];  // scaled input = in_mul (x or ln x) + in_add, in [-1, 1] over the range
  float out_mean[kMaxOut], out_std[kMaxOut], out_mask[kMaxOut];
};

__device__ __forceinline__ float scale_input(const EmuHeader* __restrict__ h, int i, float x) {
  const float v = ((h->in_log >> i) & 1) ? logf(x) : x;
  return fmaf(h->in_mul[i], v, h->in_add[i]);
}
constexpr size_t kHeaderBytes = 2048;
static_assert(sizeof(EmuHeader) <= kHeaderBytes, "header");

__host__ __device__ inline size_t n_params(int n_out) {
  return static_cast<size_t>(kIn) * kHid + kHid + 2 * (static_cast<size_t>(kHid) * kHid + kHid) +
         static_cast<size_t>(kHid) * n_out + n_out;
}

struct Offs {
  size_t W[4], b[4];
};
__host__ __device__ inline Offs param_offsets(int n_out) {
  Offs o;
  size_t p = 0;
  const int fin[4] = {kIn, kHid, kHid, kHid};
  const int fout[4] = {kHid, kHid, kHid, n_out};
  for (int l = 0; l < 4; ++l) {
    o.W[l] = p;
    p += static_cast<size_t>(fin[l]) * fout[l];
    o.b[l] = p;
    p += fout[l];
  }
  return o;
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * erfcf(-x * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * erfcf(-x * 0.70710678118654752f) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---------------------------------------------------------------- init
__global__ void __launch_bounds__(256) k_emu_init(float* params, float* m, float* v, int n_out, uint64_t seed) {
  const Offs o = param_offsets(n_out);
  const size_t np = n_params(n_out);
  const int fin[4] = {kIn, kHid, kHid, kHid};
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < np; i += static_cast<size_t>(gridDim.x) * 256) {
    int l = 3;
    while (l > 0 && i < o.W[l]) --l;
    float val = 0.0f;
    if (i < o.b[l]) {  // weight of layer l: He normal, std sqrt(2 / fan_in)
      const float2 z = normal_pair(seed, 3u, static_cast<uint64_t>(i) << 1);
      val = z.x * sqrtf(2.0f / fin[l]);
    }
    params[i] = val;
    m[i] = 0.0f;
    v[i] = 0.0f;
  }
}

// per output column: mean and std over the labels (ln for columns >= log_from),
// mask 0 if any label is not finite; one block per column, fixed-order FP64 sums
__global__ void __launch_bounds__(256) k_emu_stats(const float* __restrict__ y, int64_t n, int n_out, int log_from,
                                                   EmuHeader* h) {
  __shared__ double s1[256], s2[256];
  __shared__ int sbad[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double a = 0.0, b = 0.0;
  int bad = 0;
  for (int64_t i = t; i < n; i += 256) {
    float v = y[i * n_out + c];
    if (c >= log_from) v = logf(v);
    if (!isfinite(v)) {
      bad = 1;
      continue;
    }
    a += v;
    b += static_cast<double>(v) * v;
  }
  s1[t] = a;
  s2[t] = b;
  sbad[t] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      s1[t] += s1[t + w];
      s2[t] += s2[t + w];
      sbad[t] |= sbad[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double mean = s1[0] / static_cast<double>(n);
    const double var = s2[0] / static_cast<double>(n) - mean * mean;
    h->out_mean[c] = static_cast<float>(mean);
    h->out_std[c] = static_cast<float>(var > 1e-30 ? sqrt(var) : 1.0);
    h->out_mask[c] = sbad[0] ? 0.0f : 1.0f;
  }
}

// training batch of step s: rows (s B + i) mod n, standardised
__global__ void __launch_bounds__(256) k_emu_gather(const float* __restrict__ x, const float* __restrict__ y, int64_t n,
                                                    int64_t s, int B, const EmuHeader* __restrict__ h, float* x0,
                                                    float* tgt) {
  const int n_out = h->n_out;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < B * (kIn + n_out); k += gridDim.x * 256) {
    const int i = k / (kIn + n_out), c = k % (kIn + n_out);
    const int64_t r = (s * B + i) % n;
    if (c < kIn) {
      x0[i * kIn + c] = scale_input(h, c, x[r * kIn + c]);
    } else {
      const int o = c - kIn;
      float v = y[r * n_out + o];
      if (o >= h->log_from) v = logf(v);
      v = (v - h->out_mean[o]) / h->out_std[o];
      tgt[i * n_out + o] = (h->out_mask[o] > 0.0f && isfinite(v)) ? v : 0.0f;
    }
  }
}

// ---------------------------------------------------------------- GEMM
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

// C = op(A) op(B) with epilogue.  op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k],
// op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n].  EPI_BIAS_GELU also writes the
// pre-activation to aux; EPI_GELU_GRAD multiplies by gelu'(aux).
__device__ __forceinline__ float epilogue(int epi, float acc, int m, int n, const float* bias, float* aux, int ldaux,
                                          float& out_aux) {
  (void)out_aux;
  if (epi == EPI_BIAS) return acc + bias[n];
  if (epi == EPI_BIAS_GELU) {
    const float zv = acc + bias[n];
    aux[static_cast<size_t>(m) * ldaux + n] = zv;
    return gelu(zv);
  }
  if (epi == EPI_GELU_GRAD) return acc * gelu_grad(aux[static_cast<size_t>(m) * ldaux + n]);
  return acc;
}

// FP32 reference product: one output per thread
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_f32(int M, int N, int K, const float* __restrict__ A, int lda,
                                                  const float* __restrict__ B, int ldb, float* C, int ldc,
                                                  const float* bias, int epi, float* aux, int ldaux) {
  const int64_t id = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (id >= static_cast<int64_t>(M) * N) return;
  const int m = static_cast<int>(id / N), n = static_cast<int>(id % N);
  float acc = 0.0f;
  for (int k = 0; k < K; ++k) {
    const float a = TA ? A[static_cast<size_t>(k) * lda + m] : A[static_cast<size_t>(m) * lda + k];
    const float b = TB ? B[static_cast<size_t>(n) * ldb + k] : B[static_cast<size_t>(k) * ldb + n];
    acc = fmaf(a, b, acc);
  }
  float dummy;
  C[static_cast<size_t>(m) * ldc + n] = epilogue(epi, acc, m, n, bias, aux, ldaux, dummy);
}

// FP32 product for few outputs and a long inner dimension (the first
// layer's weight gradient): sixteen outputs per block, sixteen threads per
// output each summing every sixteenth k in order, then a fixed tree
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_f32_ks(int M, int N, int K, const float* __restrict__ A, int lda,
                                                     const float* __restrict__ B, int ldb, float* C, int ldc,
                                                     const float* bias, int epi, float* aux, int ldaux) {
  __shared__ float sp[16][17];
  const int oi = threadIdx.x & 15, j = threadIdx.x >> 4;
  const int64_t id = static_cast<int64_t>(blockIdx.x) * 16 + oi;
  const bool valid = id < static_cast<int64_t>(M) * N;
  const int m = valid ? static_cast<int>(id / N) : 0, n = valid ? static_cast<int>(id % N) : 0;
  float acc = 0.0f;
  if (valid)
    for (int k = j; k < K; k += 16) {
      const float a = TA ? A[static_cast<size_t>(k) * lda + m] : A[static_cast<size_t>(m) * lda + k];
      const float b = TB ? B[static_cast<size_t>(n) * ldb + k] : B[static_cast<size_t>(k) * ldb + n];
      acc = fmaf(a, b, acc);
    }
  sp[j][oi] = acc;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (j < w) sp[j][oi] += sp[j + w][oi];
    __syncthreads();
  }
  if (j == 0 && valid) {
    float dummy;
    C[static_cast<size_t>(m) * ldc + n] = epilogue(epi, sp[0][oi], m, n, bias, aux, ldaux, dummy);
  }
}

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}

// 64x64 output tile per block of 4 waves (2x2, 32x32 each = 2x2 MFMA 16x16
// tiles); K in tiles of 64 staged through LDS in bfloat16, the next tile's
// global loads issued before the current tile's MFMAs.  MFMA 16x16x16 operand
// layout: lane l supplies A rows (l % 16), k = 4 (l / 16) .. +3, and B columns
// (l % 16), k = 4 (l / 16) .. +3; result element r of lane l is row
// 4 (l / 16) + r, column l % 16.
constexpr int kGemmBK = 64;

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb, float* C, int ldc,
                                                   const float* bias, int epi, float* aux, int ldaux) {
  __shared__ unsigned short As[64][kGemmBK + 8];
  __shared__ unsigned short Bs[kGemmBK][64 + 8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  v4f32 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f32{0.f, 0.f, 0.f, 0.f};
  // element e of this thread in a 64 x 64 tile: consecutive threads read
  // consecutive addresses of the operand's own layout
  auto a_coord = [&](int e, int& mm, int& kk) {
    const int idx = tid + 256 * e;
    mm = TA ? idx % 64 : idx / 64;
    kk = TA ? idx / 64 : idx % 64;
  };
  auto b_coord = [&](int e, int& kk, int& nn) {
    const int idx = tid + 256 * e;
    kk = TB ? idx % 64 : idx / 64;
    nn = TB ? idx / 64 : idx % 64;
  };
  float ra[16], rb[16];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      int mm, kk;
      a_coord(e, mm, kk);
      const int m = m0 + mm, k = k0 + kk;
      ra[e] = (m < M && k < K) ? (TA ? A[static_cast<size_t>(k) * lda + m] : A[static_cast<size_t>(m) * lda + k])
                               : 0.0f;
      int kb, nn;
      b_coord(e, kb, nn);
      const int kg = k0 + kb, n = n0 + nn;
      rb[e] = (n < N && kg < K) ? (TB ? B[static_cast<size_t>(n) * ldb + kg] : B[static_cast<size_t>(kg) * ldb + n])
                                : 0.0f;
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += kGemmBK) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      int mm, kk, kb, nn;
      a_coord(e, mm, kk);
      b_coord(e, kb, nn);
      As[mm][kk] = to_bf16(ra[e]);
      Bs[kb][nn] = to_bf16(rb[e]);
    }
    __syncthreads();
    if (k0 + kGemmBK < K) gload(k0 + kGemmBK);
#pragma unroll
    for (int ks = 0; ks < kGemmBK; ks += 16) {
      const int kb = ks + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        v4i16 af;
        const int r = wm + 16 * i + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) af[q] = static_cast<short>(As[r][kb + q]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          v4i16 bfr;
          const int cidx = wn + 16 * j + (lane & 15);
#pragma unroll
          for (int q = 0; q < 4; ++q) bfr[q] = static_cast<short>(Bs[kb + q][cidx]);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bfr, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m < M && n < N) {
          float dummy;
          C[static_cast<size_t>(m) * ldc + n] = epilogue(epi, acc[i][j][r], m, n, bias, aux, ldaux, dummy);
        }
      }
}

template <bool TA, bool TB>
hipError_t gemm(bool bf16, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                const float* bias, int epi, float* aux, int ldaux, hipStream_t st) {
  if (bf16) {
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB>), dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, st, M, N, K, A, lda,
                       B, ldb, C, ldc, bias, epi, aux, ldaux);
  } else {
    const int64_t tot = static_cast<int64_t>(M) * N;
    if (tot <= 65536 && K >= 64) {
      hipLaunchKernelGGL((k_gemm_f32_ks<TA, TB>), dim3(static_cast<unsigned>((tot + 15) / 16)), dim3(256), 0, st, M,
                         N, K, A, lda, B, ldb, C, ldc, bias, epi, aux, ldaux);
    } else {
      hipLaunchKernelGGL((k_gemm_f32<TA, TB>), dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, st, M,
                         N, K, A, lda, B, ldb, C, ldc, bias, epi, aux, ldaux);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- loss, bias grads, Adam
// dY = 2 (Y - T) mask / (B n_eff), one element per thread; per-block FP64
// partial sums of the squared misfit, then k_emu_loss sums the partials in a
// fixed order (loss = sum / (B n_eff))
__device__ __forceinline__ float emu_neff(const EmuHeader* __restrict__ h) {
  float neff = 0.0f;
  for (int o = 0; o < h->n_out; ++o) neff += h->out_mask[o];
  return neff > 0.0f ? neff : 1.0f;
}

__global__ void __launch_bounds__(256) k_emu_dloss(const float* __restrict__ y, const float* __restrict__ t, int B,
                                                   const EmuHeader* __restrict__ h, float* dy, double* lpart) {
  __shared__ double sl[256];
  const int n_out = h->n_out;
  const float scale = 2.0f / (static_cast<float>(B) * emu_neff(h));
  const int k = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (k < B * n_out) {
    const float d = (y[k] - t[k]) * h->out_mask[k % n_out];
    dy[k] = scale * d;
    l = static_cast<double>(d) * d;
  }
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sl[threadIdx.x] += sl[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = sl[0];
}

__global__ void __launch_bounds__(256) k_emu_loss(const double* __restrict__ lpart, int nparts, int B,
                                                  const EmuHeader* __restrict__ h, float* loss) {
  __shared__ double sl[256];
  double l = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) l += lpart[i];
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sl[threadIdx.x] += sl[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = static_cast<float>(sl[0] / (static_cast<double>(B) * emu_neff(h)));
}

// db[n] = sum over rows of d[m][n]: 64 columns per block, sixteen row groups
// (rows g, g + 16, ...) summed in order, then the groups in a fixed tree
__global__ void __launch_bounds__(1024) k_colsum(const float* __restrict__ d, int M, int N, float* db) {
  __shared__ float sp[16][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.0f;
  if (n < N)
    for (int m = g; m < M; m += 16) s += d[static_cast<size_t>(m) * N + n];
  sp[g][c] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (g < w) sp[g][c] += sp[g + w][c];
    __syncthreads();
  }
  if (g == 0 && n < N) db[n] = sp[0][c];
}

__global__ void __launch_bounds__(256) k_adam(float* p, float* m, float* v, const float* __restrict__ g, size_t np,
                                              float lr, float b1, float b2, float eps, float bc1, float bc2) {
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < np; i += static_cast<size_t>(gridDim.x) * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// ---------------------------------------------------------------- small-batch FP32 forward (prediction)
// one block per group of up to 8 samples: each thread owns one hidden unit;
// outputs are un-standardised (exp for columns >= log_from)
__global__ void __launch_bounds__(256) k_emu_predict(const EmuHeader* __restrict__ h, const float* __restrict__ params,
                                                     const float* __restrict__ x, int64_t n, float* y) {
  __shared__ float hs[2][8][kHid];
  const int n_out = h->n_out;
  const Offs o = param_offsets(n_out);
  const int t = threadIdx.x;
  const int64_t s0 = static_cast<int64_t>(blockIdx.x) * 8;
  const int ns = n - s0 < 8 ? static_cast<int>(n - s0) : 8;
  float acc[8];
  // layer 1
  for (int s = 0; s < ns; ++s) {
    float a = params[o.b[0] + t];
    for (int i = 0; i < kIn; ++i) {
      const float u = scale_input(h, i, x[(s0 + s) * kIn + i]);
      a = fmaf(u, params[o.W[0] + i * kHid + t], a);
    }
    hs[0][s][t] = gelu(a);
  }
  __syncthreads();
  int cur = 0;
  for (int l = 1; l < 3; ++l) {
    for (int s = 0; s < ns; ++s) acc[s] = params[o.b[l] + t];
    for (int k = 0; k < kHid; ++k) {
      const float w = params[o.W[l] + static_cast<size_t>(k) * kHid + t];
      for (int s = 0; s < ns; ++s) acc[s] = fmaf(hs[cur][s][k], w, acc[s]);
    }
    for (int s = 0; s < ns; ++s) hs[cur ^ 1][s][t] = gelu(acc[s]);
    __syncthreads();
    cur ^= 1;
  }
  if (t < n_out) {
    for (int s = 0; s < ns; ++s) acc[s] = params[o.b[3] + t];
    for (int k = 0; k < kHid; ++k) {
      const float w = params[o.W[3] + static_cast<size_t>(k) * n_out + t];
      for (int s = 0; s < ns; ++s) acc[s] = fmaf(hs[cur][s][k], w, acc[s]);
    }
    for (int s = 0; s < ns; ++s) {
      float v = acc[s] * h->out_std[t] + h->out_mean[t];
      if (t >= h->log_from) v = expf(v);
      y[(s0 + s) * n_out + t] = v;
    }
  }
}

// ---------------------------------------------------------------- host side
struct TrainBufs {
  float *x0, *tgt, *z[3], *hh[3], *y, *dy, *dz[3], *grad, *loss;
  double* lpart;  // per-block loss partials
  size_t total;
};

static size_t al(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

static TrainBufs carve_train(char* w, int B, int n_out) {
  TrainBufs t{};
  size_t o = 0;
  auto take = [&](size_t nfloat) {
    float* p = w ? reinterpret_cast<float*>(w + o) : nullptr;
    o += al(nfloat * sizeof(float));
    return p;
  };
  t.x0 = take(static_cast<size_t>(B) * kIn);
  t.tgt = take(static_cast<size_t>(B) * n_out);
  for (int l = 0; l < 3; ++l) {
    t.z[l] = take(static_cast<size_t>(B) * kHid);
    t.hh[l] = take(static_cast<size_t>(B) * kHid);
    t.dz[l] = take(static_cast<size_t>(B) * kHid);
  }
  t.y = take(static_cast<size_t>(B) * n_out);
  t.dy = take(static_cast<size_t>(B) * n_out);
  t.grad = take(n_params(n_out));
  t.loss = take(1);
  t.lpart = reinterpret_cast<double*>(take(2 * ((static_cast<size_t>(B) * n_out + 255) / 256)));
  t.total = o;
  return t;
}

// Forward and backward of one batch (x0, tgt already standardised); gradients
// into t.grad, loss into t.loss.
static hipError_t emu_fwd_bwd(const EmuHeader* h_dev, const float* params, int n_out, int B, bool bf16,
                              const TrainBufs& t, hipStream_t st) {
  const Offs o = param_offsets(n_out);
  hipError_t e;
  // forward
  if ((e = gemm<false, false>(false, B, kHid, kIn, t.x0, kIn, params + o.W[0], kHid, t.hh[0], kHid, params + o.b[0],
                              EPI_BIAS_GELU, t.z[0], kHid, st)) != hipSuccess) return e;
  for (int l = 1; l < 3; ++l)
    if ((e = gemm<false, false>(bf16, B, kHid, kHid, t.hh[l - 1], kHid, params + o.W[l], kHid, t.hh[l], kHid,
                                params + o.b[l], EPI_BIAS_GELU, t.z[l], kHid, st)) != hipSuccess) return e;
  if ((e = gemm<false, false>(bf16, B, n_out, kHid, t.hh[2], kHid, params + o.W[3], n_out, t.y, n_out,
                              params + o.b[3], EPI_BIAS, nullptr, 0, st)) != hipSuccess) return e;
  {
    const int nparts = (B * n_out + 255) / 256;
    hipLaunchKernelGGL(k_emu_dloss, dim3(nparts), dim3(256), 0, st, t.y, t.tgt, B, h_dev, t.dy, t.lpart);
    hipLaunchKernelGGL(k_emu_loss, dim3(1), dim3(256), 0, st, t.lpart, nparts, B, h_dev, t.loss);
  }
  // backward: output layer
  if ((e = gemm<true, false>(bf16, kHid, n_out, B, t.hh[2], kHid, t.dy, n_out, t.grad + o.W[3], n_out, nullptr,
                             EPI_STORE, nullptr, 0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((n_out + 63) / 64), dim3(1024), 0, st, t.dy, B, n_out, t.grad + o.b[3]);
  // dZ3 = (dY W4^T) * gelu'(Z3)
  if ((e = gemm<false, true>(bf16, B, kHid, n_out, t.dy, n_out, params + o.W[3], n_out, t.dz[2], kHid, nullptr,
                             EPI_GELU_GRAD, t.z[2], kHid, st)) != hipSuccess) return e;
  for (int l = 2; l >= 1; --l) {
    if ((e = gemm<true, false>(bf16, kHid, kHid, B, t.hh[l - 1], kHid, t.dz[l], kHid, t.grad + o.W[l], kHid, nullptr,
                               EPI_STORE, nullptr, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(kHid / 64), dim3(1024), 0, st, t.dz[l], B, kHid, t.grad + o.b[l]);
    if ((e = gemm<false, true>(bf16, B, kHid, kHid, t.dz[l], kHid, params + o.W[l], kHid, t.dz[l - 1], kHid, nullptr,
                               EPI_GELU_GRAD, t.z[l - 1], kHid, st)) != hipSuccess) return e;
  }
  if ((e = gemm<true, false>(false, kIn, kHid, B, t.x0, kIn, t.dz[0], kHid, t.grad + o.W[0], kHid, nullptr,
                             EPI_STORE, nullptr, 0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3(kHid / 64), dim3(1024), 0, st, t.dz[0], B, kHid, t.grad + o.b[0]);
  return hipGetLastError();
}

size_t emulator_bytes(int n_out) { return kHeaderBytes + 3 * al(n_params(n_out) * sizeof(float)); }
static float* emu_params(void* emu) { return reinterpret_cast<float*>(static_cast<char*>(emu) + kHeaderBytes); }
static const float* emu_params(const void* emu) {
  return reinterpret_cast<const float*>(static_cast<const char*>(emu) + kHeaderBytes);
}

size_t emulator_eval_bytes() { return 1024; }

// ---------------------------------------------------------------- device-side tuning search
constexpr int kSearchNT = 1024;
constexpr int kLmS = 3;  // samples per batched forward pass: a point and two difference steps

struct SearchArgs {
  const EmuHeader* h;
  const float* params;
  double fbar_t, c, z, x0[2], xk[2], step, xatol, fatol, sigma;
  int nk, max_evals;
  // small-scale power mode (ps = 1): th = (ln amp, ln kcut) of P_s, emulator
  // inputs (a, b, amp, kcut) with sigma_g^2 = sig0 + sigma_s^2(amp, kcut; dpix),
  // (ln a, ln s) = lin[0..1] + lin[2..3] (ln sigma_g - lin[4]) and b = s / sigma_g
  int ps;
  double sig0, dpix, lin[5];
  double pk_t[kMaxOut];
  double off[kMaxOut];       // model offset per statistic (Fbar first)
  double jac[kMaxOut][2];    // model slope per statistic in (ln a, ln b) about xk
  double* out;               // x[2], best objective, evaluations, raw prediction [1 + nk] at x
};

// Forward passes of ns <= kLmS inputs by a block of kSearchNT threads sharing
// every weight load (hidden layers: float4 loads of four units, sixteen
// threads per unit group; output layer: sixteen threads per column); raw
// outputs (exp for columns >= log_from) into outv[s].
__device__ void forward_batch(const EmuHeader* __restrict__ h, const float* __restrict__ params, const Offs& o,
                              const float (*xin)[4], int ns, float (*hs)[kLmS][kHid], float* part,
                              float (*outv)[kMaxOut]) {
  const int t = threadIdx.x, n_out = h->n_out;
  if (t < kHid) {
    const float b0 = params[o.b[0] + t];
    for (int s = 0; s < ns; ++s) {
      float a = b0;
#pragma unroll
      for (int i = 0; i < kIn; ++i) a = fmaf(scale_input(h, i, xin[s][i]), params[o.W[0] + i * kHid + t], a);
      hs[0][s][t] = gelu(a);
    }
  }
  __syncthreads();
  int cur = 0;
  // hidden layers: thread = four consecutive units (one float4 weight load per
  // k) x a sixteenth of the inner sum; the sixteen partial sums are added in
  // a fixed order
  const int ug = t & 63, kg = t >> 6;
  for (int l = 1; l < 3; ++l) {
    float acc[kLmS][4] = {};
    const float4* W = reinterpret_cast<const float4*>(params + o.W[l]) + ug;
#pragma unroll 8
    for (int k = 16 * kg; k < 16 * kg + 16; ++k) {
      const float4 w = W[static_cast<size_t>(k) * (kHid / 4)];
#pragma unroll
      for (int s = 0; s < kLmS; ++s) {
        if (s < ns) {
          const float hv = hs[cur][s][k];
          acc[s][0] = fmaf(hv, w.x, acc[s][0]);
          acc[s][1] = fmaf(hv, w.y, acc[s][1]);
          acc[s][2] = fmaf(hv, w.z, acc[s][2]);
          acc[s][3] = fmaf(hv, w.w, acc[s][3]);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kLmS; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) part[(kg * kLmS + s) * kHid + 4 * ug + j] = acc[s][j];
    __syncthreads();
    if (t < kHid) {
      const float bl = params[o.b[l] + t];
      for (int s = 0; s < ns; ++s) {
        float v = 0.0f;
        for (int i = 0; i < 16; ++i) v += part[(i * kLmS + s) * kHid + t];
        hs[cur ^ 1][s][t] = gelu(bl + v);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  const int oc = t & 63, r = t >> 6;  // column, sixteenth of the sum
  float acc[kLmS] = {0.0f, 0.0f, 0.0f};
  if (oc < n_out) {
    const float* W = params + o.W[3] + oc;
#pragma unroll
    for (int k = 16 * r; k < 16 * r + 16; ++k) {
      const float w = W[static_cast<size_t>(k) * n_out];
#pragma unroll
      for (int s = 0; s < kLmS; ++s)
        if (s < ns) acc[s] = fmaf(hs[cur][s][k], w, acc[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < kLmS; ++s) part[(r * kLmS + s) * 64 + oc] = acc[s];
  __syncthreads();
  if (t < n_out) {
    for (int s = 0; s < ns; ++s) {
      float v = 0.0f;
      for (int i = 0; i < 16; ++i) v += part[(i * kLmS + s) * 64 + t];
      v = (params[o.b[3] + t] + v) * h->out_std[t] + h->out_mean[t];
      if (t >= h->log_from) v = expf(v);
      outv[s][t] = v;
    }
  }
  __syncthreads();
}

// Levenberg-Marquardt over th = (ln a, ln b) on the residuals of the model
//   stat(th) = emulator(th) + off + jac (th - xk),
//   r_0 = (stat_0 - Fbar_t)/(s Fbar_t), r_{1+b} = (stat_{1+b} - P_t,b)/(s P_t,b)
// (0 where the target or the value is not finite; chi^2 = sum r^2), entirely
// on the device in one block.  In the small-scale power mode th = (ln amp,
// ln kcut) of P_s instead, a and b follow from th (SearchArgs), and only the
// P1D residuals count (Fbar is fixed by a and b sigma_g).  Each iteration runs one batched forward pass at
// the trial point and its two forward-difference steps (h = 1e-3), so the
// Jacobian of an accepted point comes with it.  Wave 0 forms the residuals
// (one statistic per lane) and the 2x2 normal equations (fixed-order shuffle
// sums); lane 0 steps the search and broadcasts through LDS.  Trial points
// outside the emulator's (a, b) input range are rejected like uphill steps.
// Stops when an accepted step is below xatol in both coordinates, when the
// damping exceeds 1e10, or after max_evals forward samples.
__global__ void __launch_bounds__(kSearchNT) k_emu_search(SearchArgs a) {
  __shared__ float hs[2][kLmS][kHid];
  __shared__ float part[16 * kLmS * kHid];
  __shared__ float outv[kLmS][kMaxOut];
  __shared__ double strial[2];
  __shared__ int sstate;  // 0 evaluate strial, 1 done
  const Offs o = param_offsets(a.h->n_out);
  const int nk = a.nk, t = threadIdx.x;
  // the emulator's input ranges in logarithms; a non-positive lower limit
  // leaves that side open
  auto lnlim = [](float v) { return v > 0.0f ? log(static_cast<double>(v)) : -HUGE_VAL; };
  double lo[4], hi[4];
  for (int i = 0; i < 4; ++i) {
    lo[i] = lnlim(a.h->in_lo[i]);
    hi[i] = log(static_cast<double>(a.h->in_hi[i]));
  }
  constexpr double kH = 1e-3;
  // emulator inputs at th: (a, b, c, z), or (a, b, amp, kcut) in the
  // small-scale power mode, with (ln a, ln b) returned for the range check
  auto inputs = [&](double p0, double p1, float* x, double* lab) {
    if (!a.ps) {
      x[0] = static_cast<float>(exp(p0));
      x[1] = static_cast<float>(exp(p1));
      x[2] = static_cast<float>(a.c);
      x[3] = static_cast<float>(a.z);
      lab[0] = p0;
      lab[1] = p1;
      return;
    }
    const double amp = exp(p0), kc = exp(p1);
    const double ss2 = amp * kc * erf(M_PI / (a.dpix * kc)) / (2.0 * sqrt(M_PI));
    const double lsg = 0.5 * log(a.sig0 + ss2);
    lab[0] = a.lin[0] + a.lin[2] * (lsg - a.lin[4]);
    lab[1] = a.lin[1] + a.lin[3] * (lsg - a.lin[4]) - lsg;
    x[0] = static_cast<float>(exp(lab[0]));
    x[1] = static_cast<float>(exp(lab[1]));
    x[2] = static_cast<float>(amp);
    x[3] = static_cast<float>(kc);
  };
  // lane-0 state
  double th[2] = {a.x0[0], a.x0[1]}, chi2 = HUGE_VAL, lam = 1e-3, A00 = 0, A01 = 0, A11 = 0, g0 = 0, g1 = 0;
  bool have = false;
  int nev = 0;
  if (t == 0) {
    strial[0] = th[0];
    strial[1] = th[1];
    sstate = 0;
  }
  __syncthreads();
  const int max_iter = a.max_evals / kLmS + 1;
  for (int it = 0; it < max_iter + 1; ++it) {
    const double p0 = strial[0], p1 = strial[1];
    const int state = sstate;
    float xin[kLmS][4];
    double lab[2], lab1[2];
    inputs(p0, p1, xin[0], lab);
    inputs(p0 + kH, p1, xin[1], lab1);
    inputs(p0, p1 + kH, xin[2], lab1);
    forward_batch(a.h, a.params, o, xin, state ? 1 : kLmS, hs, part, outv);
    if (state) break;  // the last pass: the raw prediction at the optimum
    if (t < 64) {
      double r = 0.0, j0 = 0.0, j1 = 0.0;
      const int i = t;
      if (i <= nk && !(a.ps && i == 0)) {
        const double tgt = i == 0 ? a.fbar_t : a.pk_t[i - 1];
        const double inv = 1.0 / (a.sigma * tgt);
        const double d0 = p0 - a.xk[0], d1 = p1 - a.xk[1];
        const double lin = a.off[i] + a.jac[i][0] * d0 + a.jac[i][1] * d1;
        const double m = static_cast<double>(outv[0][i]) + lin;
        const double ma = static_cast<double>(outv[1][i]) + lin + a.jac[i][0] * kH;
        const double mb = static_cast<double>(outv[2][i]) + lin + a.jac[i][1] * kH;
        if (isfinite(tgt) && isfinite(m) && isfinite(ma) && isfinite(mb)) {
          r = (m - tgt) * inv;
          j0 = (ma - m) * inv / kH;
          j1 = (mb - m) * inv / kH;
        }
      }
      double c2 = r * r, s00 = j0 * j0, s01 = j0 * j1, s11 = j1 * j1, q0 = j0 * r, q1 = j1 * r;
#pragma unroll
      for (int w = 32; w >= 1; w >>= 1) {
        c2 += __shfl_xor(c2, w);
        s00 += __shfl_xor(s00, w);
        s01 += __shfl_xor(s01, w);
        s11 += __shfl_xor(s11, w);
        q0 += __shfl_xor(q0, w);
        q1 += __shfl_xor(q1, w);
      }
      if (t == 0) {
        nev += kLmS;
        bool inside = lab[0] >= lo[0] && lab[0] <= hi[0] && lab[1] >= lo[1] && lab[1] <= hi[1];
        if (a.ps) inside = inside && p0 >= lo[2] && p0 <= hi[2] && p1 >= lo[3] && p1 <= hi[3];
        bool done = false;
        if (inside && c2 < chi2) {  // accept the point (and its Jacobian)
          const double step = have ? fmax(fabs(p0 - th[0]), fabs(p1 - th[1])) : HUGE_VAL;
          th[0] = p0;
          th[1] = p1;
          chi2 = c2;
          A00 = s00;
          A01 = s01;
          A11 = s11;
          g0 = q0;
          g1 = q1;
          lam = fmax(lam / 3.0, 1e-12);
          have = true;
          if (step <= a.xatol) done = true;
        } else {
          lam *= 4.0;
          if (lam > 1e10) done = true;
        }
        if (!have) done = true;  // the start itself is unusable
        if (nev + kLmS > a.max_evals) done = true;
        double n0 = th[0], n1 = th[1];
        if (!done) {  // (A + lam diag A) delta = -g
          const double m00 = A00 * (1.0 + lam) + 1e-300, m11 = A11 * (1.0 + lam) + 1e-300, m01 = A01;
          const double det = m00 * m11 - m01 * m01;
          if (!(det > 0.0) || !isfinite(det)) {
            done = true;
          } else {
            n0 = th[0] + (-g0 * m11 + g1 * m01) / det;
            n1 = th[1] + (-g1 * m00 + g0 * m01) / det;
          }
        }
        strial[0] = done ? th[0] : n0;
        strial[1] = done ? th[1] : n1;
        sstate = done ? 1 : 0;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    a.out[0] = th[0];
    a.out[1] = th[1];
    a.out[2] = chi2;
    a.out[3] = static_cast<double>(nev);
  }
  if (t <= nk) a.out[4 + t] = static_cast<double>(outv[0][t]);
}

hipError_t emulator_search(const void* emu, const EmuSearchSpec& sp, double x[2], double* fbest, int* nev,
                           double* pred, char* scratch, hipStream_t st) {
  if (!emu || sp.nk < 0 || sp.nk + 1 > kMaxOut) return hipErrorInvalidValue;
  SearchArgs a{};
  a.h = static_cast<const EmuHeader*>(emu);
  a.params = emu_params(emu);
  a.fbar_t = sp.fbar_t;
  a.c = sp.c;
  a.z = sp.z;
  a.x0[0] = x[0];
  a.x0[1] = x[1];
  a.xk[0] = sp.xk[0];
  a.xk[1] = sp.xk[1];
  a.step = sp.step;
  a.xatol = sp.xatol;
  a.fatol = sp.fatol;
  a.sigma = sp.sigma;
  a.nk = sp.nk;
  a.max_evals = sp.max_evals;
  a.ps = sp.ps;
  a.sig0 = sp.sig0;
  a.dpix = sp.dpix;
  for (int i = 0; i < 5; ++i) a.lin[i] = sp.lin[i];
  for (int i = 0; i <= sp.nk; ++i) {
    if (i < sp.nk) a.pk_t[i] = sp.pk_t[i];
    a.off[i] = sp.off[i];
    a.jac[i][0] = sp.jac[2 * i];
    a.jac[i][1] = sp.jac[2 * i + 1];
  }
  a.out = reinterpret_cast<double*>(scratch);
  hipLaunchKernelGGL(k_emu_search, dim3(1), dim3(kSearchNT), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double hout[4 + kMaxOut];
  if ((e = hipMemcpyAsync(hout, a.out, sizeof(double) * (5 + sp.nk), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  x[0] = hout[0];
  x[1] = hout[1];
  *fbest = hout[2];
  *nev = static_cast<int>(hout[3]);
  for (int i = 0; i <= sp.nk; ++i) pred[i] = hout[4 + i];
  return hipSuccess;
}

}  // namespace lya

// ---------------------------------------------------------------- C-ABI
namespace {
thread_local char g_emu_err[256] = "";
int efail(int code, const char* msg) {
  snprintf(g_emu_err, sizeof(g_emu_err), "%s", msg);
  return code;
}
}  // namespace

extern "C" {

const char* lya_emulator_last_error(void) { return g_emu_err; }

size_t lya_emulator_bytes(int32_t n_out) {
  if (n_out < 1 || n_out > lya::kMaxOut) return 0;
  return lya::emulator_bytes(n_out);
}

size_t lya_emulator_param_offset(void) { return lya::kHeaderBytes; }
size_t lya_emulator_param_count(int32_t n_out) {
  return (n_out < 1 || n_out > lya::kMaxOut) ? 0 : lya::n_params(n_out);
}

int lya_emulator_init(void* emu, int32_t n_out, int32_t log_from, uint64_t seed, const double in_lo[4],
                      const double in_hi[4], int32_t log_inputs, void* stream) {
  if (!emu || n_out < 1 || n_out > lya::kMaxOut || !in_lo || !in_hi || log_from < 0 || log_inputs < 0 ||
      log_inputs > 15)
    return efail(LYA_EINVAL, "invalid emulator arguments");
  for (int i = 0; i < 4; ++i) {
    if (!(in_hi[i] > in_lo[i])) return efail(LYA_EINVAL, "input ranges must be increasing");
    if (((log_inputs >> i) & 1) && !(in_lo[i] > 0.0)) return efail(LYA_EINVAL, "log-scaled inputs need lo > 0");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  lya::EmuHeader h{};
  h.n_out = n_out;
  h.log_from = log_from;
  h.in_log = log_inputs;
  for (int i = 0; i < 4; ++i) {
    h.in_lo[i] = static_cast<float>(in_lo[i]);
    h.in_hi[i] = static_cast<float>(in_hi[i]);
    const bool lg = (log_inputs >> i) & 1;
    const double lo = lg ? log(in_lo[i]) : in_lo[i], hi = lg ? log(in_hi[i]) : in_hi[i];
    h.in_mul[i] = static_cast<float>(2.0 / (hi - lo));
    h.in_add[i] = static_cast<float>(-(hi + lo) / (hi - lo));
  }
  for (int o = 0; o < lya::kMaxOut; ++o) {
    h.out_mean[o] = 0.0f;
    h.out_std[o] = 1.0f;
    h.out_mask[o] = o < n_out ? 1.0f : 0.0f;
  }
  hipError_t e = hipMemcpyAsync(emu, &h, sizeof(h), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
  const size_t np = lya::n_params(n_out);
  float* p = lya::emu_params(emu);
  const size_t stride = lya::al(np * sizeof(float)) / sizeof(float);
  hipLaunchKernelGGL(lya::k_emu_init, dim3(256), dim3(256), 0, st, p, p + stride, p + 2 * stride, n_out, seed);
  e = hipGetLastError();
  if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
  return LYA_OK;
}

size_t lya_emulator_train_workspace_size(int32_t batch, int32_t n_out) {
  if (batch < 1 || n_out < 1 || n_out > lya::kMaxOut) return 0;
  return lya::carve_train(nullptr, batch, n_out).total;
}

int lya_emulator_set_scaling(void* emu, const float* y, int64_t n, void* stream) {
  if (!emu || !y || n < 1) return efail(LYA_EINVAL, "invalid scaling arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  lya::EmuHeader h;
  hipError_t e = hipMemcpyAsync(&h, emu, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
  hipLaunchKernelGGL(lya::k_emu_stats, dim3(h.n_out), dim3(256), 0, st, y, n, h.n_out, h.log_from,
                     static_cast<lya::EmuHeader*>(emu));
  e = hipGetLastError();
  return e == hipSuccess ? LYA_OK : efail(LYA_EHIP, hipGetErrorString(e));
}

int lya_emulator_loss_grad(const void* emu, const float* x0, const float* t, int32_t batch, int32_t use_bf16,
                           float* grad, float* loss, void* work, size_t work_bytes, void* stream) {
  if (!emu || !x0 || !t || batch < 1 || !grad) return efail(LYA_EINVAL, "invalid gradient arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  lya::EmuHeader h;
  hipError_t e = hipMemcpyAsync(&h, emu, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
  lya::TrainBufs tb = lya::carve_train(static_cast<char*>(work), batch, h.n_out);
  if (!work || work_bytes < tb.total) return efail(LYA_EWORKSPACE, "workspace too small for the emulator batch");
  const size_t np = lya::n_params(h.n_out);
  e = hipMemcpyAsync(tb.x0, x0, sizeof(float) * batch * lya::kIn, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(tb.tgt, t, sizeof(float) * batch * h.n_out, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = lya::emu_fwd_bwd(static_cast<const lya::EmuHeader*>(emu), lya::emu_params(emu), h.n_out, batch, use_bf16 != 0,
                         tb, st);
  if (e == hipSuccess) e = hipMemcpyAsync(grad, tb.grad, sizeof(float) * np, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, tb.loss, sizeof(float), hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? LYA_OK : efail(LYA_EHIP, hipGetErrorString(e));
}

int lya_emulator_train(void* emu, const float* x, const float* y, int64_t n, int32_t steps, int32_t batch,
                       double lr, int32_t use_bf16, float* loss_hist, void* work, size_t work_bytes, void* stream) {
  if (!emu || !x || !y || n < 1 || steps < 0 || batch < 1 || !(lr > 0.0))
    return efail(LYA_EINVAL, "invalid training arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  lya::EmuHeader h;
  hipError_t e = hipMemcpyAsync(&h, emu, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
  lya::TrainBufs tb = lya::carve_train(static_cast<char*>(work), batch, h.n_out);
  if (!work || work_bytes < tb.total) return efail(LYA_EWORKSPACE, "workspace too small for the emulator batch");
  const size_t np = lya::n_params(h.n_out);
  float* p = lya::emu_params(emu);
  const size_t stride = lya::al(np * sizeof(float)) / sizeof(float);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  int step = h.step;
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(lya::k_emu_gather, dim3(64), dim3(256), 0, st, x, y, n, static_cast<int64_t>(step), batch,
                       static_cast<const lya::EmuHeader*>(emu), tb.x0, tb.tgt);
    e = lya::emu_fwd_bwd(static_cast<const lya::EmuHeader*>(emu), p, h.n_out, batch, use_bf16 != 0, tb, st);
    if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
    ++step;
    const float bc1 = 1.0f - powf(b1, static_cast<float>(step));
    const float bc2 = 1.0f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(lya::k_adam, dim3(512), dim3(256), 0, st, p, p + stride, p + 2 * stride, tb.grad, np,
                       static_cast<float>(lr), b1, b2, eps, bc1, bc2);
    if (loss_hist) {
      e = hipMemcpyAsync(loss_hist + s, tb.loss, sizeof(float), hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return efail(LYA_EHIP, hipGetErrorString(e));
    }
  }
  e = hipMemcpyAsync(reinterpret_cast<char*>(emu) + offsetof(lya::EmuHeader, step), &step, sizeof(step),
                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? LYA_OK : efail(LYA_EHIP, hipGetErrorString(e));
}

int lya_emulator_predict(const void* emu, const float* x, int64_t n, float* y, void* stream) {
  if (!emu || !x || !y || n < 0) return efail(LYA_EINVAL, "invalid prediction arguments");
  if (n == 0) return LYA_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(lya::k_emu_predict, dim3(static_cast<unsigned>((n + 7) / 8)), dim3(256), 0, st,
                     static_cast<const lya::EmuHeader*>(emu), lya::emu_params(emu), x, n, y);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LYA_OK : efail(LYA_EHIP, hipGetErrorString(e));
}

}  // extern "C"
