// Box synthesis and inverse 3D FFT (gfx950).
//
// Computes the packed real-space field C_a + i C_b = IDFT3(X) with
//   X(k) = s(n^2) W(k) (m_a(k) + i m_b(k))      (eq:deltaL, eq:eta)
// where W is Hermitian-paired unit complex noise drawn from Philox in
// k-space (the footnote of section "Mock generation" allows drawing in
// k-space directly), s the amplitude table and m the component multiplier
// (1 for delta, f k_p k_q/k^2 for eta_pq).  For the pair (delta, eta_zz) the
// real part is delta and the imaginary part eta_par along z, both real fields
// because X_a and X_b are each Hermitian.
//
// Three passes over the [x][y][z] complex64 box (x planes padded, see
// plane_pitch), in place:
//   pass Z: synthesises the modes of T pencils along z straight into
//           registers (no spectrum is ever written to memory), FFT along z;
//   pass Y: tiles of N (y) x T (z contiguous) elements, FFT along y;
//   pass X: tiles of N (x) x T (z contiguous) elements, FFT along x.
// The X pass reads pencils whose elements lie in N planes 32 MB apart (at
// 2048^3), which costs address translation.  With a second box buffer the
// passes run in the two-buffer order instead:
//   pass Z writes the pencil of modes (kx, ky) at plane ky, row kx of buffer A;
//   pass YT transforms along the rows of A (over kx) and writes plane kx,
//           row ky of the field: a strided write, and writes do not wait;
//   pass Y  transforms the field in place along its rows (over ky).
// Both strided passes then read within one plane, the result is the same
// box with the two 1D transforms in the other order (equal up to rounding).
// Each tile is transformed by a Stockham autosort FFT with radix-4/8/16
// butterflies: stage 0 works on registers filled from global memory (or the
// synthesiser), middle stages exchange through LDS, the last stage writes
// global memory directly in natural order.  Tiles are mapped to blocks so that
// each XCD walks a contiguous range of tiles (neighbouring z chunks share
// cache lines).
#include <atomic>
#include <type_traits>

#include "lya_internal.h"

namespace lya {

enum { KIND_GENZ = 0, KIND_Y = 1, KIND_X = 2, KIND_YT = 3 };

constexpr int radix_of(int n, int s) {
  return n == 2048 ? (s < 2 ? 16 : 8)
       : n == 1024 ? (s < 2 ? 16 : 4)
       : n == 512  ? 8
       : n == 256  ? 16
       : n == 128  ? (s == 0 ? 16 : 8)
       : n == 64   ? 8
       : n == 32   ? (s == 0 ? 8 : 4)
       : 0;
}
constexpr int nstages_of(int n) {
  return (n == 2048 || n == 1024 || n == 512) ? 3 : 2;
}
constexpr int ns_before(int n, int s) { return s == 0 ? 1 : ns_before(n, s - 1) * radix_of(n, s - 1); }

__device__ __forceinline__ int xcd_tile(int b, int nb) {
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

// Tile order of the strided passes (block -> (outer, z0)):
//   0: each XCD walks consecutive tiles, z chunks fastest;
//   1: each XCD walks pairs of neighbouring z chunks (which share cache lines)
//      with the outer index changing between pairs, so the requests in flight
//      spread over more rows of the box;
//   2: plain order, z chunks fastest;
//   3: each XCD walks tiles with the outer index fastest.
template <int N, int T, int ORDER>
__device__ __forceinline__ void strided_tile(int b, int& outer, int& t0) {
  constexpr int nb = N * (N / T);
  if (ORDER == 2) {
    outer = b / (N / T);
    t0 = (b % (N / T)) * T;
    return;
  }
  const int u = xcd_tile(b, nb);
  if (ORDER == 0) {
    outer = u / (N / T);
    t0 = (u % (N / T)) * T;
  } else if (ORDER == 1) {
    const int rest = u >> 1;
    outer = rest % N;
    t0 = (2 * (rest / N) + (u & 1)) * T;
  } else {
    outer = u % N;
    t0 = (u / N) * T;
  }
}

__device__ __forceinline__ int sfreq(int i, int n) { return i < n / 2 ? i : i - n; }

__device__ __forceinline__ float comp_mult(int comp, int nx, int ny, int nz, int n2, int n, float f) {
  if (comp == 0) return 1.0f;
  if (comp < 0 || n2 == 0) return 0.0f;
  int a, b;
  switch (comp) {
    case 1: a = nx; b = nx; break;
    case 2: a = ny; b = ny; break;
    case 3: a = nz; b = nz; break;
    case 4: a = nx; b = ny; break;
    case 5: a = nx; b = nz; break;
    default: a = ny; b = nz; break;
  }
  if (comp >= 4 && (a == -(n / 2) || b == -(n / 2))) return 0.0f;
  // a*b and n2 are exact in FP32 (|n|^2 < 2^24); reciprocal good to 1 ulp
  return f * static_cast<float>(a * b) * __builtin_amdgcn_rcpf(static_cast<float>(n2));
}

// Complex multiplier (re, im) of a component: delta and eta_pq real (above);
// the velocity v_j = i f (aH)_0 k_j / k^2 delta_hat (eq:velocity, (aH)_0 =
// 100 km/s per Mpc/h) is i vscale n_j / |n|^2 with vscale = f 100 L / (2 pi).
// It is odd in k, so it vanishes on the Nyquist plane of j, where a mode is
// its own partner.
__device__ __forceinline__ float2 comp_mult2(int comp, int nx, int ny, int nz, int n2, int n, float f,
                                             float vscale) {
  if (comp < 7) return make_float2(comp_mult(comp, nx, ny, nz, n2, n, f), 0.0f);
  const int a = comp == 7 ? nx : (comp == 8 ? ny : nz);
  if (n2 == 0 || a == -(n / 2)) return make_float2(0.0f, 0.0f);
  return make_float2(0.0f, vscale * static_cast<float>(a) * __builtin_amdgcn_rcpf(static_cast<float>(n2)));
}

// Mode (ix, iy, iz) of the packed spectrum (a second amplitude table and the
// complex multipliers only in the generic synthesiser).
template <int N, bool GENERIC>
__device__ __forceinline__ float2 gen_mode(const GenParams& g, int ix, int iy, int iz) {
  const int nx = sfreq(ix, N), ny = sfreq(iy, N), nz = sfreq(iz, N);
  const int n2 = nx * nx + ny * ny + nz * nz;
  float s = g.table[n2];
  float sb = (GENERIC && g.table_b) ? g.table_b[n2] : s;
  if (g.only_n2 >= 0 && n2 != g.only_n2) s = sb = 0.0f;
  if (s == 0.0f && sb == 0.0f) return make_float2(0.0f, 0.0f);
  const uint64_t lin = (static_cast<uint64_t>(ix) * N + iy) * N + iz;
  const uint64_t plin = (static_cast<uint64_t>((N - ix) & (N - 1)) * N + ((N - iy) & (N - 1))) * N + ((N - iz) & (N - 1));
  const uint64_t own = lin < plin ? lin : plin;
  const float2 z = normal_pair(g.seed, 0u, own);
  float2 w;
  if (lin == plin) {
    w = make_float2(z.x, 0.0f);
  } else {
    w = make_float2(z.x * kSqrtHalf, (lin == own ? z.y : -z.y) * kSqrtHalf);
  }
  if (g.fixed_amp) {
    const float m = rsqrtf(w.x * w.x + w.y * w.y);
    w.x *= m;
    w.y *= m;
  }
  if (GENERIC) {
    // X = W (s c_a + i sb c_b)
    const float2 ca = comp_mult2(g.comp_a, nx, ny, nz, n2, N, g.f, g.vscale);
    const float2 cb = comp_mult2(g.comp_b, nx, ny, nz, n2, N, g.f, g.vscale);
    const float pr = s * ca.x - sb * cb.y, pi = s * ca.y + sb * cb.x;
    return make_float2(w.x * pr - w.y * pi, w.y * pr + w.x * pi);
  }
  const float ma = comp_mult(g.comp_a, nx, ny, nz, n2, N, g.f);
  const float mb = comp_mult(g.comp_b, nx, ny, nz, n2, N, g.f);
  return make_float2(s * (w.x * ma - w.y * mb), s * (w.y * ma + w.x * mb));
}

// SWZ (pass Z of the two-buffer order): pencil (kx, ky) goes to plane ky, row kx.
template <int N, int T, int E, int KIND, bool SWZ = false>
struct Pass {
  static constexpr int NT = N * T / E;
  static constexpr bool PF = KIND != KIND_GENZ;  // lanes walk the T contiguous pencils first
  static constexpr int NSTAGE = nstages_of(N);

  // Synthesising pass: a tile holds T pencils along z.  "Paired" tiles hold
  // H = T/2 pencils (ix, iy0..iy0+H-1) with 0 < ix < N/2, which own all their
  // modes, followed by their Hermitian partner pencils (N-ix, -iy mod N); the
  // remaining rows ix = 0 and ix = N/2 are cut into unpaired tiles of T pencils.
  static constexpr int H = T / 2;
  static constexpr size_t kPitch = plane_pitch(N);
  static constexpr int kPairedTiles = (N / 2 - 1) * (N / H);

  // global element index of element i of pencil p in tile (outer, t0); for the
  // synthesising pass outer is ix and t0 is iy0 (paired flags the tile kind)
  __device__ static __forceinline__ size_t gidx(int outer, int t0, int i, int p, bool paired = false) {
    if (KIND == KIND_GENZ) {
      const int px = paired && p >= H ? N - outer : outer;
      const int py = paired && p >= H ? (N - t0 - (p - H)) & (N - 1) : t0 + p;
      return SWZ ? static_cast<size_t>(py) * kPitch + static_cast<size_t>(px) * N + i
                 : static_cast<size_t>(px) * kPitch + static_cast<size_t>(py) * N + i;
    }
    if (KIND == KIND_Y || KIND == KIND_YT)
      return static_cast<size_t>(outer) * kPitch + static_cast<size_t>(i) * N + t0 + p;
    return static_cast<size_t>(i) * kPitch + static_cast<size_t>(outer) * N + t0 + p;
  }
  // where the last stage stores element i of pencil p: KIND_YT writes plane
  // i, row outer (of the other buffer); every other pass where it read
  __device__ static __forceinline__ size_t gidx_out(int outer, int t0, int i, int p, bool paired) {
    if (KIND == KIND_YT) return static_cast<size_t>(i) * kPitch + static_cast<size_t>(outer) * N + t0 + p;
    return gidx(outer, t0, i, p, paired);
  }
  // The same addresses split as base + offset, so that an access costs one
  // add: the y passes read (and KIND_Y writes) within plane outer, offset
  // i N + p in 32 bits from a block-uniform base; a synthesised pencil is
  // contiguous, offset i from its start; KIND_YT writes at i kPitch + p from
  // the block-uniform row (outer, t0).
  __device__ static __forceinline__ size_t base_in(int outer, int t0) {
    return static_cast<size_t>(outer) * kPitch + t0;
  }
  __device__ static __forceinline__ uint32_t off_in(int i, int p) {
    return static_cast<uint32_t>(i) * N + static_cast<uint32_t>(p);
  }
  // LDS layout with one padding slot per R0 elements along the FFT axis (R0 =
  // first radix): the first stage scatters its outputs with stride R0, which
  // without padding lands every lane group on the same banks.
  static constexpr int R0 = radix_of(N, 0);
  static constexpr int LDS_ELEMS = T * (N + N / R0);
  __device__ static __forceinline__ int lidx(int i, int p) {
    return PF ? (i + i / R0) * T + p : p * (N + N / R0) + i + i / R0;
  }

  template <int R>
  __device__ static __forceinline__ void coords(int w, int& p, int& j) {
    if (PF) {
      p = w % T;
      j = w / T;
    } else {
      j = w % (N / R);
      p = w / (N / R);
    }
  }

  template <int S>
  __device__ static __forceinline__ void butterflies(float2 (&v)[E], const float2* __restrict__ tw, int tid) {
    constexpr int R = radix_of(N, S), NS = ns_before(N, S), B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      int p, j;
      coords<R>(tid + b * NT, p, j);
      if (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], tw[r * k * (N / (NS * R))]);
      }
      dft<R>(&v[b * R]);
    }
  }

  // stage-0 registers of a strided tile straight from global memory
  // (EL..EH: the part of the thread's elements b R + r to load)
  template <int EL = 0, int EH = E>
  __device__ static __forceinline__ void load_global0(float2 (&v)[E], const float2* __restrict__ data, int outer,
                                                      int t0, int tid) {
    constexpr int R = radix_of(N, 0), B = E / R;
    if constexpr (KIND == KIND_Y || KIND == KIND_YT) {
      const float2* __restrict__ plane = data + base_in(outer, t0);
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (b * R + R <= EL || b * R >= EH) continue;
        int p, j;
        coords<R>(tid + b * NT, p, j);
        const uint32_t o = off_in(j, p);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (b * R + r >= EL && b * R + r < EH) v[b * R + r] = plane[o + static_cast<uint32_t>(r * (N / R) * N)];
      }
    } else {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (b * R + R <= EL || b * R >= EH) continue;
        int p, j;
        coords<R>(tid + b * NT, p, j);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (b * R + r >= EL && b * R + r < EH) v[b * R + r] = data[gidx(outer, t0, j + r * (N / R), p)];
      }
    }
  }

  // stages 0.. of the tile held in v, the results left in v for
  // store_global<NSTAGE - 1>; hook(k) runs before stage k's butterflies
  template <typename H>
  __device__ static __forceinline__ void transform(float2 (&v)[E], float2* lds, const float2* __restrict__ tw,
                                                   int tid, H hook) {
    hook(std::integral_constant<int, 0>());
    butterflies<0>(v, tw, tid);
    store_lds<0>(v, lds, tid);
    __syncthreads();
    load_lds<1>(v, lds, tid);
    hook(std::integral_constant<int, 1>());
    butterflies<1>(v, tw, tid);
    if constexpr (NSTAGE == 3) {
      __syncthreads();
      store_lds<1>(v, lds, tid);
      __syncthreads();
      load_lds<2>(v, lds, tid);
      hook(std::integral_constant<int, 2>());
      butterflies<2>(v, tw, tid);
    }
  }

  // stages 0.. of the tile held in v, ending with the natural-order global store
  __device__ static __forceinline__ void transform_store(float2 (&v)[E], float2* lds, float2* data,
                                                         uint32_t* out_bf16, const float2* __restrict__ tw,
                                                         bool zero_b, int outer, int t0, bool paired, int tid) {
    butterflies<0>(v, tw, tid);
    store_lds<0>(v, lds, tid);
    __syncthreads();
    load_lds<1>(v, lds, tid);
    butterflies<1>(v, tw, tid);
    if constexpr (NSTAGE == 2) {
      store_global<1>(v, data, out_bf16, zero_b, outer, t0, paired, tid);
    } else {
      __syncthreads();
      store_lds<1>(v, lds, tid);
      __syncthreads();
      load_lds<2>(v, lds, tid);
      butterflies<2>(v, tw, tid);
      store_global<2>(v, data, out_bf16, zero_b, outer, t0, paired, tid);
    }
  }

  template <int S>
  __device__ static __forceinline__ void load_lds(float2 (&v)[E], const float2* lds, int tid) {
    constexpr int R = radix_of(N, S), B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      int p, j;
      coords<R>(tid + b * NT, p, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = lds[lidx(j + r * (N / R), p)];
    }
  }

  // outputs of stage S go to element (j/NS)*NS*R + j%NS + r*NS
  template <int S>
  __device__ static __forceinline__ void store_lds(const float2 (&v)[E], float2* lds, int tid) {
    constexpr int R = radix_of(N, S), NS = ns_before(N, S), B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      int p, j;
      coords<R>(tid + b * NT, p, j);
      const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lidx(base + r * NS, p)] = v[b * R + r];
    }
  }

  // EL..EH: the part of the thread's elements (b R + r) to store
  template <int S, int EL = 0, int EH = E>
  __device__ static __forceinline__ void store_global(const float2 (&v)[E], float2* data, uint32_t* out_bf16,
                                                      bool zero_b, int outer, int t0, bool paired, int tid) {
    constexpr int R = radix_of(N, S), B = E / R;
    static_assert(ns_before(N, S) * R == N, "last stage");
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (b * R + R <= EL || b * R >= EH) continue;
      int p, j;
      coords<R>(tid + b * NT, p, j);
      // base + offset of element j + r N/R (see base_in)
      size_t base;
      if constexpr (KIND == KIND_Y) {
        base = base_in(outer, t0) + off_in(j, p);
      } else if constexpr (KIND == KIND_YT) {
        base = static_cast<size_t>(outer) * N + t0 + static_cast<size_t>(j) * kPitch + p;
      } else if constexpr (KIND == KIND_GENZ) {
        base = gidx(outer, t0, j, p, paired);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (b * R + r < EL || b * R + r >= EH) continue;
        size_t gi;
        if constexpr (KIND == KIND_Y) {
          gi = base + static_cast<uint32_t>(r * (N / R) * N);
        } else if constexpr (KIND == KIND_YT) {
          gi = base + static_cast<size_t>(r * (N / R)) * kPitch;
        } else if constexpr (KIND == KIND_GENZ) {
          gi = base + static_cast<uint32_t>(r * (N / R));
        } else {
          gi = gidx_out(outer, t0, j + r * (N / R), p, paired);
        }
        // a single requested component: the other half is exactly zero, not FFT rounding residue
        const float2 o = make_float2(v[b * R + r].x, zero_b ? 0.0f : v[b * R + r].y);
        if (out_bf16) {
          out_bf16[gi] = pack_bf16x2(o.x, o.y);
        } else if (KIND == KIND_GENZ) {
          // nontemporal: the synthesising pass writes lines it never read, and a
          // plain store first fetches each line into L2 (counter-measured)
          typedef float f2v __attribute__((ext_vector_type(2)));
          f2v w;
          w.x = o.x;
          w.y = o.y;
          __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(data + gi));
        } else {
          data[gi] = o;
        }
      }
    }
  }
};

// Paired synthesis: one Philox call per two consecutive owner modes (counter
// lin >> 1, words (x, y) for even iz and (z, w) for odd iz), one Box-Muller per
// owner mode, and each owner mode also fills its partner (N-ix, -iy, -iz) with
// the conjugate noise.  Result goes to LDS in pencil-major order.
// GM selects the synthesiser: GEN_GENERIC handles any component pair and the
// test hooks; GEN_DELTA_ETAZ ({delta, f mu_z^2 delta}) and GEN_DELTA ({delta, 0})
// are the branch-free forms used by lya_make_box.
enum { GEN_GENERIC = 0, GEN_DELTA_ETAZ = 1, GEN_DELTA = 2 };

template <int N, int T, int NT, int GM, typename LIDX>
__device__ __forceinline__ void gen_paired(const GenParams& g, int ix, int iy0, float2* lds, LIDX lidx, float* stab,
                                           float* stab_b) {
  constexpr int H = T / 2, NZ = N / 2 + 1;
  constexpr int NG = (H * NZ + NT - 1) / NT;  // amplitude gathers per thread
  constexpr int NP = H * (N / 2) / NT;        // Philox calls per thread
  static_assert(H * (N / 2) % NT == 0, "whole Philox calls per thread");
  const int nx = ix;  // 0 < ix < N/2
  // The amplitudes a pencil needs depend on |nz| only: gather them once into
  // LDS (the table is far larger than L2).  All of a thread's gathers are
  // issued first and stay in flight while it draws its Philox words; they are
  // written to LDS only after that.
  float ga[NG], gb[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int w = static_cast<int>(threadIdx.x) + i * NT;
    if (w < H * NZ) {
      const int po = w / NZ, az = w % NZ;
      const int ny = sfreq(iy0 + po, N);
      ga[i] = g.table[nx * nx + ny * ny + az * az];
      if (GM == GEN_GENERIC && g.table_b) gb[i] = g.table_b[nx * nx + ny * ny + az * az];
    }
  }
  uint4 wds[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int w = static_cast<int>(threadIdx.x) + p * NT;
    const int po = w / (N / 2), m = w % (N / 2);
    const uint64_t ctr = (static_cast<uint64_t>(ix) * N + iy0 + po) * (N / 2) + m;
    wds[p] = philox10_x3(make_uint4(static_cast<uint32_t>(ctr), static_cast<uint32_t>(ctr >> 32), 0u, 0u),
                         static_cast<uint32_t>(g.seed), static_cast<uint32_t>(g.seed >> 32));
  }
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int w = static_cast<int>(threadIdx.x) + i * NT;
    if (w < H * NZ) {
      stab[w] = ga[i];
      if (GM == GEN_GENERIC && g.table_b) stab_b[w] = gb[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int w = static_cast<int>(threadIdx.x) + p * NT;
    const int po = w / (N / 2), m = w % (N / 2);
    const int iy = iy0 + po;
    const int ny = sfreq(iy, N);
    const uint4 wd = wds[p];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int iz = 2 * m + e;
      const int nz = sfreq(iz, N);
      const int n2 = nx * nx + ny * ny + nz * nz;
      float s = stab[po * NZ + (nz < 0 ? -nz : nz)];
      float2 wv = e ? box_muller_half(wd.z, wd.w) : box_muller_half(wd.x, wd.y);
      float ma, mb;
      if (GM == GEN_GENERIC) {
        float sb = g.table_b ? stab_b[po * NZ + (nz < 0 ? -nz : nz)] : s;
        if (g.only_n2 >= 0 && n2 != g.only_n2) s = sb = 0.0f;
        if (g.fixed_amp) {
          const float r = rsqrtf(wv.x * wv.x + wv.y * wv.y);
          wv.x *= r;
          wv.y *= r;
        }
        // X = W P, X' = conj(W) P' with P = s c_a + i sb c_b at the mode and P'
        // the same at its partner (-nx, -ny, -nz): P' = P for the even
        // components, P' = -P for the velocities
        const int pny = sfreq((N - iy) & (N - 1), N), pnz = sfreq((N - iz) & (N - 1), N);
        const float2 ca = comp_mult2(g.comp_a, nx, ny, nz, n2, N, g.f, g.vscale);
        const float2 cb = comp_mult2(g.comp_b, nx, ny, nz, n2, N, g.f, g.vscale);
        const float2 da = comp_mult2(g.comp_a, -nx, pny, pnz, n2, N, g.f, g.vscale);
        const float2 db = comp_mult2(g.comp_b, -nx, pny, pnz, n2, N, g.f, g.vscale);
        const float pr = s * ca.x - sb * cb.y, pi = s * ca.y + sb * cb.x;
        const float qr = s * da.x - sb * db.y, qi = s * da.y + sb * db.x;
        lds[lidx(iz, po)] = make_float2(wv.x * pr - wv.y * pi, wv.y * pr + wv.x * pi);
        lds[lidx((N - iz) & (N - 1), H + po)] = make_float2(wv.x * qr + wv.y * qi, wv.x * qi - wv.y * qr);
        continue;
      } else {
        ma = s;  // n2 > 0 here (ix > 0)
        mb = GM == GEN_DELTA_ETAZ ? s * g.f * static_cast<float>(nz * nz) * __builtin_amdgcn_rcpf(static_cast<float>(n2))
                                  : 0.0f;
      }
      // X = W (ma + i mb), X' = conj(W) (ma + i mb)
      lds[lidx(iz, po)] = make_float2(wv.x * ma - wv.y * mb, wv.y * ma + wv.x * mb);
      lds[lidx((N - iz) & (N - 1), H + po)] = make_float2(wv.x * ma + wv.y * mb, wv.x * mb - wv.y * ma);
    }
  }
}

// SWZ: pass Z of the two-buffer order; LAST: the box's last pass (BF16 output,
// exact zeros for a single requested component).  KIND_YT stores to g.dst.
template <int N, int T, int E, int KIND, int ORDER = 1, int GM = GEN_GENERIC, bool SWZ = false,
          bool LAST = KIND == KIND_X>
__global__ void __launch_bounds__(N * T / E) k_fft_pass(float2* __restrict__ data, uint32_t* __restrict__ out_bf16,
                                                        const float2* __restrict__ tw, GenParams g) {
  using P = Pass<N, T, E, KIND, SWZ>;
  constexpr int NT = P::NT;
  __shared__ float2 lds[P::LDS_ELEMS];
  float2 v[E];
  const int tid = threadIdx.x;
  const int ntiles = N * (N / T);
  const int tile = xcd_tile(blockIdx.x, ntiles);  // synthesising pass
  int outer, t0;
  bool paired = false;
  if (KIND == KIND_GENZ) {
    if (P::H == 1 && tile < P::kPairedTiles && g.order) {
      // in bands of nx^2 + ny^2 (k_zo_band_write)
      paired = true;
      const uint32_t o = g.order[tile];
      outer = static_cast<int>(o >> 16);
      t0 = static_cast<int>(o & 0xffffu);
    } else if (tile < P::kPairedTiles) {
      paired = true;
      outer = 1 + tile / (N / P::H);
      // iy blocks in mirrored pairs: blocks j and N/H - j follow each other,
      // so the pencils (ix, iy) and (ix, -iy), which need the same amplitude
      // table entries (n^2 = nx^2 + ny^2 + nz^2), are made back to back on one
      // XCD and the second finds the entries in its L2
      constexpr int nb = N / P::H;
      const int r = tile % nb;
      t0 = (r == 0 ? 0 : r == 1 ? nb / 2 : (r & 1) ? nb - (r >> 1) : (r >> 1)) * P::H;
    } else {
      const int u = tile - P::kPairedTiles;
      outer = u < N / T ? 0 : N / 2;
      t0 = (u % (N / T)) * T;
    }
  } else {
    strided_tile<N, T, ORDER>(blockIdx.x, outer, t0);
  }

  // stage 0: registers from global memory or from the synthesiser
  if (KIND == KIND_GENZ && paired) {
    __shared__ float stab[KIND == KIND_GENZ ? (T / 2) * (N / 2 + 1) : 1];
    // second amplitude table: only the generic synthesiser serves two spectra
    __shared__ float stab_b[KIND == KIND_GENZ && GM == GEN_GENERIC ? (T / 2) * (N / 2 + 1) : 1];
    gen_paired<N, T, NT, GM>(g, outer, t0, lds, [](int i, int p) { return P::lidx(i, p); }, stab, stab_b);
    __syncthreads();
    P::template load_lds<0>(v, lds, tid);
    __syncthreads();
  } else if (KIND == KIND_GENZ) {
    constexpr int R = radix_of(N, 0), B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      int p, j;
      P::template coords<R>(tid + b * NT, p, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = gen_mode<N, GM == GEN_GENERIC>(g, outer, t0 + p, j + r * (N / R));
    }
  } else {
    P::load_global0(v, data, outer, t0, tid);
  }
  P::transform_store(v, lds, KIND == KIND_YT ? g.dst : data, LAST ? out_bf16 : nullptr, tw, LAST && g.comp_b < 0,
                     outer, t0, paired, tid);
}

// Persistent, software-pipelined strided pass: each block walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... (gridDim.x a multiple of 8, so a
// block stays on one XCD's range of tiles) and issues the global loads of its
// next tile before transforming the current one, so that their latency hides
// behind the FFT and the stores.  Two register copies of a tile: the waves
// are allowed the larger register budget of two waves per SIMD.  DEFER keeps
// a third copy, the transformed tile, and issues its stores in the next
// iteration after that iteration's loads: a store waits for its address
// translation, and loads issued behind it wait too, which for stores spread
// over N planes (the transposing pass) held the next tile's loads back
// (2048^3: 37.0-37.2 ms against 37.9-38.0 ms, bit-identical).  SPLIT issues
// the next tile's loads (and the deferred stores) in three parts, one before
// each FFT stage, instead of all at the start of the iteration: a wave that
// issues its 16 loads and 16 stores at once stalls on the full memory queue
// before it reaches the FFT, while in parts the memory traffic runs under the
// stages (the transposing pass at 2048^3: 31.6-31.8 ms, bit-identical; the
// same kernel without its FFT moves the box in 29.4 ms).
template <int N, int T, int E, int KIND, int ORDER, bool LAST = KIND == KIND_X, bool DEFER = false, bool SPLIT = false>
__global__ void __launch_bounds__(N * T / E) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_fft_pipe(float2* __restrict__ data, uint32_t* __restrict__ out_bf16, const float2* __restrict__ tw, GenParams g) {
  using P = Pass<N, T, E, KIND>;
  constexpr int ntiles = N * (N / T);
  __shared__ float2 lds[P::LDS_ELEMS];
  // twiddles in LDS: a global twiddle load issued after the next tile's loads
  // would wait for them (vector memory loads complete in order)
  __shared__ float2 stw[N];
  for (int i = threadIdx.x; i < N; i += P::NT) stw[i] = tw[i];
  __syncthreads();
  float2 v[E], nv[E];
  [[maybe_unused]] float2 ov[DEFER ? E : 1];
  [[maybe_unused]] int po = 0, pt = 0;
  [[maybe_unused]] bool have = false;
  int b = blockIdx.x;
  if (b >= ntiles) return;
  int outer, t0;
  strided_tile<N, T, ORDER>(b, outer, t0);
  P::load_global0(v, data, outer, t0, static_cast<int>(threadIdx.x));
  for (;;) {
    // a thread index the compiler cannot prove loop-invariant: hoisted out of
    // the loop, every LDS, twiddle and global address of the tile would stay
    // live in registers for the whole kernel (and spill)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int bn = b + static_cast<int>(gridDim.x);
    const bool more = bn < ntiles;
    int on = 0, tn = 0;
    if (more) strided_tile<N, T, ORDER>(bn, on, tn);
    float2* dst = KIND == KIND_YT ? g.dst : data;
    uint32_t* bf = LAST ? out_bf16 : nullptr;
    const bool zb = LAST && g.comp_b < 0;
    constexpr int NS = P::NSTAGE, LS = NS - 1;
    if constexpr (SPLIT) {
      // the next tile's loads, and the previous tile's deferred stores, in
      // parts before each stage of this tile's FFT
      P::transform(v, lds, stw, tid, [&](auto k) {
        constexpr int K = decltype(k)::value, EL = E * K / NS, EH = E * (K + 1) / NS;
        if (more) P::template load_global0<EL, EH>(nv, data, on, tn, tid);
        if constexpr (DEFER)
          if (have) P::template store_global<LS, EL, EH>(ov, dst, bf, zb, po, pt, false, tid);
      });
    } else {
      if (more) P::load_global0(nv, data, on, tn, tid);
      if constexpr (DEFER) {
        // the previous tile's stores, issued after the next tile's loads
        if (have) P::template store_global<LS>(ov, dst, bf, zb, po, pt, false, tid);
        P::transform(v, lds, stw, tid, [](auto) {});
      } else {
        P::transform_store(v, lds, dst, bf, stw, zb, outer, t0, false, tid);
      }
    }
    if constexpr (DEFER) {
#pragma unroll
      for (int e = 0; e < E; ++e) ov[e] = v[e];
      po = outer;
      pt = t0;
      have = true;
    } else if constexpr (SPLIT) {
      P::template store_global<LS>(v, dst, bf, zb, outer, t0, false, tid);
    }
    if (!more) break;
    __syncthreads();  // every thread has read this tile's LDS before the next one is written
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = nv[e];
    b = bn;
    outer = on;
    t0 = tn;
  }
  if constexpr (DEFER) {
    int tid = threadIdx.x;
    P::template store_global<P::NSTAGE - 1>(ov, KIND == KIND_YT ? g.dst : data, LAST ? out_bf16 : nullptr,
                                            LAST && g.comp_b < 0, po, pt, false, tid);
  }
}

// Tile shapes: (pencils per tile T, elements per thread E) for the
// synthesising pass and the strided passes.
template <int N>
struct Shape;
template <> struct Shape<32>   { static constexpr int TZ = 16, EZ = 8,  TS = 16, ES = 8; };
template <> struct Shape<64>   { static constexpr int TZ = 16, EZ = 8,  TS = 16, ES = 8; };
template <> struct Shape<128>  { static constexpr int TZ = 8,  EZ = 16, TS = 16, ES = 16; };
template <> struct Shape<256>  { static constexpr int TZ = 8,  EZ = 16, TS = 16, ES = 16; };
template <> struct Shape<512>  { static constexpr int TZ = 8,  EZ = 16, TS = 16, ES = 16; };
template <> struct Shape<1024> { static constexpr int TZ = 4,  EZ = 16, TS = 16, ES = 32; };
template <> struct Shape<2048> { static constexpr int TZ = 2,  EZ = 16, TS = 8,  ES = 32; };

// Variants of the strided passes (y and x), chosen per N by the autotuner:
//   0/1: tile of the table's T pencils, one tile per block, tile order 0/1;
//   2/3: half the pencils per tile (half the LDS: two blocks per CU), order 0/1;
//   4/5: half tiles in the persistent pipelined kernel, order 0/1;
//   6/7: full tiles with half the elements per thread (twice the waves), order 0/1;
//   8/9: as 6/7 in the persistent pipelined kernel;
//   10/11: full tiles, one per block, tile order 2 (plain) / 3 (outer index fastest);
//   12/13: full tiles in the persistent pipelined kernel, order 0/1;
//   14/15: as 8/9 with the next tile's loads issued in parts before the FFT
//          stages (SPLIT).
// Boxes below 1024 have variants 0 and 1 only.
namespace {
// [pass y/x][log2 N]; defaults: below 1024 one tile per block, y with tile
// order 0 and x with order 1; from 1024 up the pipelined kernel with full
// tiles of half the elements per thread, y order 0 (variant 8), x order 1
// with its loads split over the FFT stages (15: 36.6 ms against 42.0 ms for
// 9 at 2048^3, bit-identical; for y the split measured 31.4 against 31.1 ms)
std::atomic<int> g_variant[2][12] = {{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 8, 8}, {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 15, 15}};
int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n && l < 11) ++l;
  return l;
}
}  // namespace

int fft_variant(int n, int pass) { return g_variant[pass][ilog2(n)].load(std::memory_order_relaxed); }

int set_fft_variant(int n, int pass, int v) {
  if (v < 0 || v >= kFftVariants || pass < 0 || pass > 1) return -1;
  if (n < 1024 && v > 1) return -1;  // smaller boxes: one tile per block, order 0 or 1
  g_variant[pass][ilog2(n)].store(v, std::memory_order_relaxed);
  return 0;
}

template <int N, int T, int E, int KIND, int ORDER, bool PIPE, bool SPL = false>
hipError_t launch_strided_tile(float2* field, uint32_t* bf16, const float2* tw, const GenParams& g, hipStream_t st) {
  const char* name = KIND == KIND_Y ? "fft_y" : "fft_x";
  constexpr int ntiles = N * (N / T), nt = N * T / E;
  if constexpr (PIPE) {
    int blocks = (device_cus() + 7) / 8 * 8;
    if (blocks > ntiles) blocks = ntiles;
    LYA_TIMED(name, st,
              hipLaunchKernelGGL((k_fft_pipe<N, T, E, KIND, ORDER, KIND == KIND_X, false, SPL>), dim3(blocks), dim3(nt),
                                 0, st, field, bf16, tw, g));
  } else {
    LYA_TIMED(name, st,
              hipLaunchKernelGGL((k_fft_pass<N, T, E, KIND, ORDER>), dim3(ntiles), dim3(nt), 0, st, field, bf16, tw,
                                 g));
  }
  return hipGetLastError();
}

template <int N, int KIND>
hipError_t launch_strided(int variant, float2* field, uint32_t* bf16, const float2* tw, const GenParams& g,
                          hipStream_t st) {
  using S = Shape<N>;
  if constexpr (N >= 1024) {
    constexpr int TH = S::TS / 2, EH = S::ES / 2;
    switch (variant) {
      case 2: return launch_strided_tile<N, TH, EH, KIND, 0, false>(field, bf16, tw, g, st);
      case 3: return launch_strided_tile<N, TH, EH, KIND, 1, false>(field, bf16, tw, g, st);
      case 4: return launch_strided_tile<N, TH, EH, KIND, 0, true>(field, bf16, tw, g, st);
      case 5: return launch_strided_tile<N, TH, EH, KIND, 1, true>(field, bf16, tw, g, st);
      case 6: return launch_strided_tile<N, S::TS, EH, KIND, 0, false>(field, bf16, tw, g, st);
      case 7: return launch_strided_tile<N, S::TS, EH, KIND, 1, false>(field, bf16, tw, g, st);
      case 8: return launch_strided_tile<N, S::TS, EH, KIND, 0, true>(field, bf16, tw, g, st);
      case 9: return launch_strided_tile<N, S::TS, EH, KIND, 1, true>(field, bf16, tw, g, st);
      case 10: return launch_strided_tile<N, S::TS, S::ES, KIND, 2, false>(field, bf16, tw, g, st);
      case 11: return launch_strided_tile<N, S::TS, S::ES, KIND, 3, false>(field, bf16, tw, g, st);
      case 12: return launch_strided_tile<N, S::TS, S::ES, KIND, 0, true>(field, bf16, tw, g, st);
      case 13: return launch_strided_tile<N, S::TS, S::ES, KIND, 1, true>(field, bf16, tw, g, st);
      case 14: return launch_strided_tile<N, S::TS, EH, KIND, 0, true, true>(field, bf16, tw, g, st);
      case 15: return launch_strided_tile<N, S::TS, EH, KIND, 1, true, true>(field, bf16, tw, g, st);
      default: break;
    }
  }
  if (variant == 1) return launch_strided_tile<N, S::TS, S::ES, KIND, 1, false>(field, bf16, tw, g, st);
  return launch_strided_tile<N, S::TS, S::ES, KIND, 0, false>(field, bf16, tw, g, st);
}

// Tile order of the synthesising pass (boxes from kZOrderMinN up, where a
// paired tile is one pencil and its partner).  Pencil (nx, ny) reads the
// amplitude-table entries nx^2 + ny^2 + nz^2 for every nz: pencils with close
// key nx^2 + ny^2 read the same cache lines of the table (whose entries are
// spaced 2|nz| + 1 apart, one line each for most nz).  The paired tiles are
// visited band by band of kZoBand consecutive keys, so that the tiles in
// flight on one XCD span a few hundred keys and share their table lines in
// its L2.  Within a band the order is ix, then |ny|, then +ny before -ny (a
// pencil and its mirror, which read the same entries, back to back).  Built
// on every call without atomics, so the order is deterministic: the tiles of
// each band counted per band (closed form per ix), the band counts scanned,
// then each band's tiles written from the scan of its per-ix counts.
constexpr int kZoBand = 128;
constexpr int kZoNT = 256;

// floor(sqrt(x)) for 0 <= x < 2^24
__device__ __forceinline__ int zo_isqrt(int x) {
  int r = static_cast<int>(sqrtf(static_cast<float>(x)));
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return r;
}

// |ny| range [m0, m1] of the pencils (ix, ny) with key in [lo, lo + kZoBand)
__device__ __forceinline__ void zo_range(int ix, int lo, int n, int& m0, int& m1) {
  const int a = lo - ix * ix, b = a + kZoBand;
  m0 = a <= 0 ? 0 : zo_isqrt(a - 1) + 1;
  m1 = b <= 0 ? -1 : zo_isqrt(b - 1);
  if (m1 > n / 2) m1 = n / 2;
}

// tiles of (ix, +-m), m in [m0, m1]: +m exists up to n/2 - 1, -m from 1 to n/2
__device__ __forceinline__ int zo_count(int m0, int m1, int n) {
  if (m1 < m0) return 0;
  const int hp = m1 < n / 2 - 1 ? m1 : n / 2 - 1, lm = m0 > 1 ? m0 : 1;
  return (hp >= m0 ? hp - m0 + 1 : 0) + (m1 >= lm ? m1 - lm + 1 : 0);
}

template <int N>
__device__ __forceinline__ int zo_band_tiles(int band, int (&cnt)[(N / 2 + kZoNT - 1) / kZoNT]) {
  constexpr int PER = (N / 2 + kZoNT - 1) / kZoNT;
  int tot = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ix = 1 + static_cast<int>(threadIdx.x) * PER + k;
    int m0 = 0, m1 = -1;
    if (ix < N / 2) zo_range(ix, band * kZoBand, N, m0, m1);
    cnt[k] = zo_count(m0, m1, N);
    tot += cnt[k];
  }
  return tot;
}

// block-wide exclusive scan of one value per thread (kZoNT threads)
__device__ __forceinline__ int zo_exclusive(int v, int* s, int& total) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < kZoNT; d <<= 1) {
    const int a = static_cast<int>(threadIdx.x) >= d ? s[threadIdx.x - d] : 0;
    __syncthreads();
    s[threadIdx.x] += a;
    __syncthreads();
  }
  total = s[kZoNT - 1];
  return s[threadIdx.x] - v;
}

// tiles per band (a block per band)
template <int N>
__global__ void __launch_bounds__(kZoNT) k_zo_band_count(int* __restrict__ bcount) {
  __shared__ int s[kZoNT];
  int cnt[(N / 2 + kZoNT - 1) / kZoNT];
  int total;
  zo_exclusive(zo_band_tiles<N>(blockIdx.x, cnt), s, total);
  if (threadIdx.x == 0) bcount[blockIdx.x] = total;
}

// exclusive scan of the band counts in place (one block, each thread a run)
__global__ void __launch_bounds__(kZoNT) k_zo_band_scan(int* __restrict__ bcount, int nbands) {
  __shared__ int s[kZoNT];
  const int per = (nbands + kZoNT - 1) / kZoNT, c0 = static_cast<int>(threadIdx.x) * per;
  int tot = 0;
  for (int k = 0; k < per && c0 + k < nbands; ++k) tot += bcount[c0 + k];
  int total;
  int run = zo_exclusive(tot, s, total);
  for (int k = 0; k < per && c0 + k < nbands; ++k) {
    const int c = bcount[c0 + k];
    bcount[c0 + k] = run;
    run += c;
  }
}

// order[position] = (ix << 16) | iy for the tiles of each band (a block per band)
template <int N>
__global__ void __launch_bounds__(kZoNT) k_zo_band_write(const int* __restrict__ boff, uint32_t* __restrict__ order) {
  constexpr int PER = (N / 2 + kZoNT - 1) / kZoNT;
  __shared__ int s[kZoNT];
  int cnt[PER];
  int total;
  int pos = boff[blockIdx.x] + zo_exclusive(zo_band_tiles<N>(blockIdx.x, cnt), s, total);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (cnt[k] == 0) continue;
    const int ix = 1 + static_cast<int>(threadIdx.x) * PER + k;
    int m0, m1;
    zo_range(ix, blockIdx.x * kZoBand, N, m0, m1);
    for (int m = m0; m <= m1; ++m) {
      if (m <= N / 2 - 1) order[pos++] = (static_cast<uint32_t>(ix) << 16) | static_cast<uint32_t>(m);
      if (m >= 1) order[pos++] = (static_cast<uint32_t>(ix) << 16) | static_cast<uint32_t>(N - m);
    }
  }
}

struct ZOrderSizes {
  int ntiles, nbands;
  size_t words;  // order + band counts
};

template <int N>
constexpr ZOrderSizes zorder_sizes() {
  static_assert(Shape<N>::TZ == 2, "one pencil and its partner per paired tile");
  constexpr int ntiles = (N / 2 - 1) * N;
  constexpr int nkeys = (N / 2 - 1) * (N / 2 - 1) + (N / 2) * (N / 2) + 1;
  constexpr int nbands = (nkeys + kZoBand - 1) / kZoBand;
  return ZOrderSizes{ntiles, nbands, static_cast<size_t>(ntiles) + nbands};
}

template <int N>
hipError_t launch_zorder(uint32_t* work, hipStream_t st) {
  constexpr ZOrderSizes z = zorder_sizes<N>();
  uint32_t* order = work;
  int* bcount = reinterpret_cast<int*>(work + z.ntiles);
  LYA_TIMED("zorder", st, {
    hipLaunchKernelGGL(k_zo_band_count<N>, dim3(z.nbands), dim3(kZoNT), 0, st, bcount);
    hipLaunchKernelGGL(k_zo_band_scan, dim3(1), dim3(kZoNT), 0, st, bcount, z.nbands);
    hipLaunchKernelGGL(k_zo_band_write<N>, dim3(z.nbands), dim3(kZoNT), 0, st, bcount, order);
  });
  return hipGetLastError();
}

template <int N, bool SWZ>
hipError_t launch_zgen(const GenParams& g, int gm, const float2* tw, float2* out, hipStream_t st) {
  using S = Shape<N>;
  const int tz = N * (N / S::TZ);
  if (gm == GEN_DELTA_ETAZ) {
    LYA_TIMED("fft_z_gen", st,
              hipLaunchKernelGGL((k_fft_pass<N, S::TZ, S::EZ, KIND_GENZ, 0, GEN_DELTA_ETAZ, SWZ>), dim3(tz),
                                 dim3(N * S::TZ / S::EZ), 0, st, out, nullptr, tw, g));
  } else if (gm == GEN_DELTA) {
    LYA_TIMED("fft_z_gen", st,
              hipLaunchKernelGGL((k_fft_pass<N, S::TZ, S::EZ, KIND_GENZ, 0, GEN_DELTA, SWZ>), dim3(tz),
                                 dim3(N * S::TZ / S::EZ), 0, st, out, nullptr, tw, g));
  } else {
    LYA_TIMED("fft_z_gen", st,
              hipLaunchKernelGGL((k_fft_pass<N, S::TZ, S::EZ, KIND_GENZ, 0, GEN_GENERIC, SWZ>), dim3(tz),
                                 dim3(N * S::TZ / S::EZ), 0, st, out, nullptr, tw, g));
  }
  return hipGetLastError();
}

// The two strided passes of the two-buffer order: the transposing pass
// (second -> field, over kx) and the last pass (field in place, over ky);
// from 1024 up in the pipelined kernel with full tiles of half the elements
// per thread (the shape of strided variant 9) and tile order 1, the
// transposing pass with deferred stores and its loads and stores split over
// the FFT stages.  At 2048^3: 31.5 + 30.3 ms.  The last pass took 32.0 ms
// with the full element count per thread and 32.7 ms with its loads split,
// 33.4 ms in tile order 0 (it ran at 33.8 ms with half the elements and
// 32.0 ms with the full count while the transposing pass still issued its
// stores at once).  Below 1024 one tile per block.
template <int N>
hipError_t launch_two_buffer(GenParams g, const float2* tw, float2* second, float2* field, uint32_t* field_bf16,
                             hipStream_t st) {
  using S = Shape<N>;
  g.dst = field;
  if constexpr (N >= 1024) {
    constexpr int T = S::TS, E = S::ES / 2, ntiles = N * (N / T), nt = N * T / E;
    int blocks = (device_cus() + 7) / 8 * 8;
    if (blocks > ntiles) blocks = ntiles;
    LYA_TIMED("fft_x2", st,
              hipLaunchKernelGGL((k_fft_pipe<N, T, E, KIND_YT, 1, false, true, true>), dim3(blocks), dim3(nt), 0, st,
                                 second, nullptr, tw, g));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LYA_TIMED("fft_y2", st,
              hipLaunchKernelGGL((k_fft_pipe<N, T, E, KIND_Y, 1, true>), dim3(blocks), dim3(nt), 0, st, field,
                                 field_bf16, tw, g));
  } else {
    constexpr int T = S::TS, E = S::ES, ntiles = N * (N / T), nt = N * T / E;
    LYA_TIMED("fft_x2", st,
              hipLaunchKernelGGL((k_fft_pass<N, T, E, KIND_YT, 0>), dim3(ntiles), dim3(nt), 0, st, second, nullptr,
                                 tw, g));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LYA_TIMED("fft_y2", st,
              hipLaunchKernelGGL((k_fft_pass<N, T, E, KIND_Y, 0, GEN_GENERIC, false, true>), dim3(ntiles), dim3(nt),
                                 0, st, field, field_bf16, tw, g));
  }
  return hipGetLastError();
}

template <int N>
hipError_t run_box_fft(GenParams g, const float2* tw, float2* field, uint32_t* field_bf16, float2* second,
                       uint32_t* zorder, hipStream_t st) {
  const bool hooks = g.fixed_amp || g.only_n2 >= 0 || g.table_b;
  const int gm = (!hooks && g.comp_a == 0 && g.comp_b == 3)    ? GEN_DELTA_ETAZ
                 : (!hooks && g.comp_a == 0 && g.comp_b == -1) ? GEN_DELTA
                                                               : GEN_GENERIC;
  hipError_t e;
  g.order = nullptr;
  if constexpr (N >= kZOrderMinN) {
    if (zorder) {
      if ((e = launch_zorder<N>(zorder, st)) != hipSuccess) return e;
      g.order = zorder;
    }
  }
  if (second) {
    if ((e = launch_zgen<N, true>(g, gm, tw, second, st)) != hipSuccess) return e;
    return launch_two_buffer<N>(g, tw, second, field, field_bf16, st);
  }
  if ((e = launch_zgen<N, false>(g, gm, tw, field, st)) != hipSuccess) return e;
  if ((e = launch_strided<N, KIND_Y>(fft_variant(N, 0), field, nullptr, tw, g, st)) != hipSuccess) return e;
  return launch_strided<N, KIND_X>(fft_variant(N, 1), field, field_bf16, tw, g, st);
}

// One strided pass alone (autotuning): pass 0 = y, 1 = x, on the box in place.
hipError_t launch_fft_strided_pass(int n, int pass, int variant, const float2* tw, float2* field, hipStream_t st) {
  GenParams g{};
  g.comp_b = 3;
  switch (n) {
#define LYA_CASE(NN)                                                                                        \
  case NN:                                                                                                  \
    return pass == 0 ? launch_strided<NN, KIND_Y>(variant, field, nullptr, tw, g, st)                       \
                     : launch_strided<NN, KIND_X>(variant, field, nullptr, tw, g, st);
    LYA_CASE(32) LYA_CASE(64) LYA_CASE(128) LYA_CASE(256) LYA_CASE(512) LYA_CASE(1024) LYA_CASE(2048)
#undef LYA_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_box_fft(int n, const GenParams& g, const float2* tw, float2* field, uint32_t* field_bf16,
                          float2* second, uint32_t* zorder, hipStream_t st) {
  switch (n) {
    case 32: return run_box_fft<32>(g, tw, field, field_bf16, second, zorder, st);
    case 64: return run_box_fft<64>(g, tw, field, field_bf16, second, zorder, st);
    case 128: return run_box_fft<128>(g, tw, field, field_bf16, second, zorder, st);
    case 256: return run_box_fft<256>(g, tw, field, field_bf16, second, zorder, st);
    case 512: return run_box_fft<512>(g, tw, field, field_bf16, second, zorder, st);
    case 1024: return run_box_fft<1024>(g, tw, field, field_bf16, second, zorder, st);
    case 2048: return run_box_fft<2048>(g, tw, field, field_bf16, second, zorder, st);
    default: return hipErrorInvalidValue;
  }
}

size_t zorder_words(int n) { return n == 2048 ? zorder_sizes<2048>().words : 0; }

}  // namespace lya
