// Device helpers shared by the lyamock HIP kernels (gfx950).
//
// Counter-based noise: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11):
//   round: (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,
//          c <- (hi1^c1^k0, lo1, hi0^c3^k1, lo0); key += (W0, W1); 10 rounds.
// Counter (idx lo, idx hi, stream, 0), key (seed lo, seed hi).  One call
// serves two consecutive linear indices: index L uses counter L>>1 and the
// word pair (2b, 2b+1), b = L & 1.  Uniform u = ((w>>9)+0.5)*2^-23 (exact in
// FP32), normals by Box-Muller (Box & Muller 1958).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lya {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply each (v_mad_u64_u32) instead of separate hi/lo products
    const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * c.z;
    c = make_uint4(static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0, static_cast<uint32_t>(p1),
                   static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1, static_cast<uint32_t>(p0));
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// Philox4x32-10 as above with each 3-input xor in one v_bitop3_b32 (truth
// table 0x96): the hot synthesis loop spends most of its integer work here.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint4 philox10_x3(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * c.z;
    c = make_uint4(xor3(static_cast<uint32_t>(p1 >> 32), c.y, k0), static_cast<uint32_t>(p1),
                   xor3(static_cast<uint32_t>(p0 >> 32), c.w, k1), static_cast<uint32_t>(p0));
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// ((w >> 9) + 1/2) 2^-23 exactly: one fma on the converted 23-bit integer
// (every intermediate is exact in FP32).
__device__ __forceinline__ float u01(uint32_t w) {
  return __builtin_fmaf(static_cast<float>(w >> 9), 1.1920928955078125e-07f, 5.9604644775390625e-08f);
}

// Box-Muller in FP32: (z1, z2) from the word pair (wa, wb), on the hardware
// transcendental units: v_log_f32 (log2), v_sqrt_f32, and v_sin_f32/v_cos_f32,
// which take their argument in revolutions, so sin(2 pi u) is one instruction.
// On gfx950 these agree with FP64 to ~1.2e-7 relative (log2) and ~1.3e-7
// absolute (sin, cos) over the uniforms used here.
__device__ __forceinline__ float2 box_muller(uint32_t wa, uint32_t wb) {
  constexpr float kMinus2Ln2 = -1.3862943611198906f;  // -2 ln 2
  const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u01(wa)));
  const float t = u01(wb);
  return make_float2(r * __builtin_amdgcn_cosf(t), r * __builtin_amdgcn_sinf(t));
}

// The Box-Muller pair scaled by sqrt(1/2) (the unit complex noise of a
// Hermitian pair), the scale folded into the radius: sqrt(-ln2 log2 u).
__device__ __forceinline__ float2 box_muller_half(uint32_t wa, uint32_t wb) {
  constexpr float kMinusLn2 = -0.6931471805599453f;
  const float r = __builtin_amdgcn_sqrtf(kMinusLn2 * __builtin_amdgcn_logf(u01(wa)));
  const float t = u01(wb);
  return make_float2(r * __builtin_amdgcn_cosf(t), r * __builtin_amdgcn_sinf(t));
}

// Normal pair for linear index lin of a stream.
__device__ __forceinline__ float2 normal_pair(uint64_t seed, uint32_t stream, uint64_t lin) {
  const uint64_t ctr = lin >> 1;
  const uint4 w = philox10(make_uint4(static_cast<uint32_t>(ctr), static_cast<uint32_t>(ctr >> 32), stream, 0u),
                           static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  return (lin & 1u) ? box_muller(w.z, w.w) : box_muller(w.x, w.y);
}

// ---- complex helpers (float2 = re, im) ----
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// explicit fused multiply-adds: every kernel that uses it then rounds the
// product the same way, whatever contraction the compiler would pick in context
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmul_i(float2 a) { return make_float2(-a.y, a.x); }  // i*a

// ---- inverse DFT butterflies (sign +), in place on v[0..R) ----
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = cmul_i(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kCos8 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kSin8 = 0.38268343236508977173f;  // sin(pi/8)

template <int R>
__device__ __forceinline__ void dft(float2* v);

template <>
__device__ __forceinline__ void dft<2>(float2* v) { dft2(v[0], v[1]); }

template <>
__device__ __forceinline__ void dft<4>(float2* v) { dft4(v[0], v[1], v[2], v[3]); }

// radix 8: two radix-4 on even/odd inputs, then twiddles exp(+2 pi i s/8)
template <>
__device__ __forceinline__ void dft<8>(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  o1 = make_float2(kSqrtHalf * (o1.x - o1.y), kSqrtHalf * (o1.x + o1.y));
  o2 = cmul_i(o2);
  o3 = make_float2(-kSqrtHalf * (o3.x + o3.y), kSqrtHalf * (o3.x - o3.y));
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// radix 16 as 4 x 4: X[k1 + 4 k2] = sum_n2 w16^(n2 k1) [dft4 over n1 of v[4 n1 + n2]](k1) w4^(n2 k2)
template <>
__device__ __forceinline__ void dft<16>(float2* v) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // after the first dft4, v[4*k1 + n2] holds Y[n2][k1]; apply w16^(n2*k1)
  // w16^1 = (c8, s8), w16^2 = (r, r), w16^3 = (s8, c8), w16^4 = i, w16^6 = (-r, r), w16^9 = (-c8, -s8)
  v[4 + 1] = cmul(v[4 + 1], make_float2(kCos8, kSin8));          // n2=1,k1=1: w^1
  v[8 + 1] = make_float2(kSqrtHalf * (v[9].x - v[9].y), kSqrtHalf * (v[9].x + v[9].y));  // n2=1,k1=2: w^2
  v[12 + 1] = cmul(v[13], make_float2(kSin8, kCos8));            // n2=1,k1=3: w^3
  v[4 + 2] = make_float2(kSqrtHalf * (v[6].x - v[6].y), kSqrtHalf * (v[6].x + v[6].y));  // n2=2,k1=1: w^2
  v[8 + 2] = cmul_i(v[10]);                                      // n2=2,k1=2: w^4
  v[12 + 2] = make_float2(-kSqrtHalf * (v[14].x + v[14].y), kSqrtHalf * (v[14].x - v[14].y));  // w^6
  v[4 + 3] = cmul(v[7], make_float2(kSin8, kCos8));              // n2=3,k1=1: w^3
  v[8 + 3] = make_float2(-kSqrtHalf * (v[11].x + v[11].y), kSqrtHalf * (v[11].x - v[11].y));  // w^6
  v[12 + 3] = cmul(v[15], make_float2(-kCos8, -kSin8));          // n2=3,k1=3: w^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1 + 0], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // now v[4*k1 + k2] holds X[k1 + 4 k2]; transpose to natural order
  float2 t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

// bf16 (round to nearest even) packing of two floats
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  uint32_t ua = __float_as_uint(a), ub = __float_as_uint(b);
  ua += 0x7FFFu + ((ua >> 16) & 1u);
  ub += 0x7FFFu + ((ub >> 16) & 1u);
  return (ua >> 16) | (ub & 0xFFFF0000u);
}
__device__ __forceinline__ float2 unpack_bf16x2(uint32_t w) {
  return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
}

}  // namespace lya
