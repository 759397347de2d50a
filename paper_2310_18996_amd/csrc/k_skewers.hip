// Lines of sight, small-scale field and FGPA (gfx950).
//
// For every quasar line of sight (section "Gaussian fields along lines of
// sight" and eq:gfield, eq:FGPA):
//   * pixel j sits at the int64 fixed-point position origin + j*step (cell
//     units x 2^32); delta_L and eta_par come from periodic trilinear
//     interpolation of the packed {delta, eta} box;
//   * delta_S: Philox normals (stream 1, counter (q<<33)+m) on modes
//     m = 0..N_S/2 of a length N_S = next_pow2(n_q) line, scaled by
//     sqrt(P_s(k_m)/(N_S dpix)), P_s = amp exp(-(k/kcut)^2), then the real
//     inverse DFT, computed as one complex inverse FFT of length N_S/2 whose
//     output holds the even pixels in its real part and the odd pixels in
//     its imaginary part;
//   * wide-angle variant: eta_par = u_p u_q eta^pq at each corner voxel from
//     four packed boxes ({delta, eta_zz}, {eta_xx, eta_yy}, {eta_xy, eta_xz},
//     {eta_yz, 0}), u the skewer's direction, then interpolated like delta;
//   * Gaussian-kernel variant: the paper's average over the 7^3 voxels around
//     the pixel (standard deviation one voxel) in place of trilinear;
//   * g = delta_L + delta_S + c(z) eta_par, F = exp(-a(z) exp(b(z) g)), with
//     a, b, c quadratics in (1+z) and z the unperturbed redshift of
//     chi_j = chi0 - j*dchi (section "FGPA");
//   * per redshift bin, the sum of F and the pixel count, accumulated as
//     exact 64-bit integers of round(F 2^32), so the result does not depend on
//     the order in which work is scheduled.
// One persistent launch; each wavefront pulls chunks of skewers from an
// atomic queue and owns a skewer at a time (its small-scale FFT lives in the
// wave's slice of LDS, so no block-wide barrier is needed per skewer).
#include "lya_internal.h"
#include "lya_wavefft.h"

namespace lya {

constexpr int kSkWaves = 4;
constexpr int kSkNT = 64 * kSkWaves;

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

// Box element loads, the storage type fixed at compile time (a run-time test
// per corner splits the gathers into separate blocks that each wait for their
// load, instead of issuing all of a pixel's gathers together).
template <bool B16>
__device__ __forceinline__ float2 ld_field(const SkewerArgs& a, size_t i) {
  if constexpr (B16) return unpack_bf16x2(a.field_bf16[i]);
  else return a.field[i];
}

template <bool B16>
__device__ __forceinline__ float2 ld_wide(const SkewerArgs& a, int k, size_t i) {
  if constexpr (B16) return unpack_bf16x2(a.wide_bf16[k][i]);
  else return a.wide[k][i];
}

// Interpolation modes of the skewer kernel.
enum { kSkTri = 0, kSkWide = 1, kSkGauss = 2 };

// Gaussian-kernel average over the 7^3 voxels around the pixel's nearest grid
// point c (standard deviation one voxel, section "Gaussian fields along lines
// of sight"): the weights separate into 7 per axis, exp(-(o - t)^2/2) with
// t = u - c in [-1/2, 1/2), and the average divides by their product sum.
// Each z run of 7 voxels is contiguous in memory.
template <bool B16>
__device__ __forceinline__ void gauss7_at(const SkewerArgs& a, int64_t px, int64_t py, int64_t pz, int N, size_t NN,
                                          float& d, float& e) {
  float g[3][7], s[3];
  int c[3];
  const int64_t p3[3] = {px, py, pz};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const uint32_t fr = static_cast<uint32_t>(p3[ax]);
    const int up = static_cast<int>(fr >> 31);
    c[ax] = static_cast<int>(((p3[ax] >> 32) + up) & (N - 1));
    const float t = static_cast<float>(fr) * 2.3283064365386963e-10f - static_cast<float>(up);
    s[ax] = 0.0f;
#pragma unroll
    for (int o = 0; o < 7; ++o) {
      const float dd = static_cast<float>(o - 3) - t;
      g[ax][o] = __expf(-0.5f * dd * dd);
      s[ax] += g[ax][o];
    }
  }
  float ax_ = 0.0f, ay_ = 0.0f;
  for (int i = 0; i < 7; ++i) {
    const size_t rx = static_cast<size_t>((c[0] + i - 3) & (N - 1)) * NN;
    float bx = 0.0f, by = 0.0f;
#pragma unroll
    for (int jy = 0; jy < 7; ++jy) {
      const size_t row = rx + static_cast<size_t>((c[1] + jy - 3) & (N - 1)) * N;
      float rx_ = 0.0f, ry_ = 0.0f;
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const float2 f = ld_field<B16>(a, row + ((c[2] + k - 3) & (N - 1)));
        rx_ += g[2][k] * f.x;
        ry_ += g[2][k] * f.y;
      }
      bx += g[1][jy] * rx_;
      by += g[1][jy] * ry_;
    }
    ax_ += g[0][i] * bx;
    ay_ += g[0][i] * by;
  }
  const float inv = 1.0f / (s[0] * s[1] * s[2]);
  d = ax_ * inv;
  e = ay_ * inv;
}

// Staged form for 64 consecutive pixels of one skewer (one per lane, valid
// lanes only): their 7^3 neighbourhoods lie in a bounding box of cells that
// the wave loads into its LDS slice once (z runs contiguous), then each lane
// sums its 343 voxels from LDS.  Returns false (nothing done) when the box
// holds more than kGaussCap cells; the caller then gathers from global memory.
constexpr int kGaussCap = 1024;
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) v = min(v, __shfl_xor(v, w));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) v = max(v, __shfl_xor(v, w));
  return v;
}
template <bool B16>
__device__ __forceinline__ bool gauss7_staged(const SkewerArgs& a, int64_t px, int64_t py, int64_t pz, bool valid,
                                              int64_t base_x, int64_t base_y, int64_t base_z, int N, size_t NN,
                                              float2* lds, int lane, float& d, float& e) {
  const int64_t p3[3] = {px, py, pz};
  const int64_t b3[3] = {base_x, base_y, base_z};
  int c[3], lo[3], sz[3];
  float g[3][7], s[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const uint32_t fr = static_cast<uint32_t>(p3[ax]);
    const int up = static_cast<int>(fr >> 31);
    // nearest grid point relative to the chunk's base cell (small integers)
    c[ax] = static_cast<int>((p3[ax] >> 32) - b3[ax]) + up;
    const float t = static_cast<float>(fr) * 2.3283064365386963e-10f - static_cast<float>(up);
    s[ax] = 0.0f;
#pragma unroll
    for (int o = 0; o < 7; ++o) {
      const float dd = static_cast<float>(o - 3) - t;
      g[ax][o] = __expf(-0.5f * dd * dd);
      s[ax] += g[ax][o];
    }
    lo[ax] = wave_min(valid ? c[ax] : INT_MAX) - 3;
    sz[ax] = wave_max(valid ? c[ax] : INT_MIN) + 4 - lo[ax];
  }
  const int vol = sz[0] * sz[1] * sz[2];
  if (vol > kGaussCap || sz[0] > 64 || sz[1] > 64 || sz[2] > 64) return false;
  const int sxy = sz[1] * sz[2];
  for (int v = lane; v < vol; v += 64) {
    const int vx = v / sxy, r = v - vx * sxy, vy = r / sz[2], vz = r - vy * sz[2];
    const int gx = static_cast<int>((base_x + lo[0] + vx) & (N - 1));
    const int gy = static_cast<int>((base_y + lo[1] + vy) & (N - 1));
    const int gz = static_cast<int>((base_z + lo[2] + vz) & (N - 1));
    lds[v] = ld_field<B16>(a, gx * NN + static_cast<size_t>(gy) * N + gz);
  }
  wave_sync();
  float ax_ = 0.0f, ay_ = 0.0f;
  if (valid) {
    const int o0 = ((c[0] - 3 - lo[0]) * sz[1] + (c[1] - 3 - lo[1])) * sz[2] + (c[2] - 3 - lo[2]);
    for (int i = 0; i < 7; ++i) {
      float bx = 0.0f, by = 0.0f;
#pragma unroll
      for (int jy = 0; jy < 7; ++jy) {
        const float2* row = lds + o0 + i * sxy + jy * sz[2];
        float rx_ = 0.0f, ry_ = 0.0f;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          const float2 f = row[k];
          rx_ += g[2][k] * f.x;
          ry_ += g[2][k] * f.y;
        }
        bx += g[1][jy] * rx_;
        by += g[1][jy] * ry_;
      }
      ax_ += g[0][i] * bx;
      ay_ += g[0][i] * by;
    }
  }
  wave_sync();  // the slice is reloaded for the next 64 pixels
  const float inv = 1.0f / (s[0] * s[1] * s[2]);
  d = ax_ * inv;
  e = ay_ * inv;
  return true;
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

template <int U, int MODE, bool B16>
__global__ void __launch_bounds__(kSkNT) k_skewers(SkewerArgs a) {
  __shared__ float2 sbuf[kSkWaves][kHalfBuf];
  __shared__ float2 sgauss[MODE == kSkGauss ? kSkWaves : 1][MODE == kSkGauss ? kGaussCap : 1];
  __shared__ int sjb[kSkWaves][kMaxZBins + 1];
  __shared__ unsigned long long s_sum[kMaxZBins], s_cnt[kMaxZBins];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = tid; b < kMaxZBins; b += kSkNT) {
    s_sum[b] = 0ull;
    s_cnt[b] = 0ull;
  }
  __syncthreads();
  const int N = a.n;
  const size_t NN = plane_pitch(N);
  const bool gather = a.in_dens == nullptr;
  const bool want_bins = a.n_bins > 0 && a.do_flux;
  float2* buf = sbuf[wv];
  int* jb = sjb[wv];
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
      const double chi0 = a.chi0[q];
      int ns = 1;
      while (ns < np) ns <<= 1;
      const bool with_ds = (gather || a.ds_in_apply) && a.ps_amp > 0.0 && ns >= 2;
      // delta_S is drawn on lines of next_pow2(npix) <= 2048 pixels (the wave's
      // LDS line): a longer skewer is an input error, marked by NaN in every
      // output and left out of the bins
      if (with_ds && ns > 2 * kHalfMax) {
        const float qnan = __builtin_nanf("");
        for (int j = lane; j < np; j += 64) {
          if (a.dens) a.dens[off + j] = qnan;
          if (a.eta) a.eta[off + j] = qnan;
          if (a.flux) a.flux[off + j] = qnan;
        }
        continue;
      }
      // twiddles from global memory: a copy in LDS would cost this kernel its fourth block per CU
      if (with_ds) small_scale_wave(a, a.ps_amp, a.ps_kcut, a.id_base + q, ns, buf, a.tw2048, lane);
      // bin boundaries: jb[b] = first pixel with chi_j < edges[b] (chi_j decreases with j)
      if (want_bins) {
        bin_bounds(a.chi_edges, a.n_bins, chi0, a.dchi, np, jb, lane);
        wave_sync();
      }
      int64_t ox = 0, oy = 0, oz = 0, sx = 0, sy = 0, sz = 0;
      if (gather) {
        ox = a.origin_fx[3 * q];
        oy = a.origin_fx[3 * q + 1];
        oz = a.origin_fx[3 * q + 2];
        sx = a.step_fx[3 * q];
        sy = a.step_fx[3 * q + 1];
        sz = a.step_fx[3 * q + 2];
      }
      // wide-angle weights u_p u_q (off-diagonal ones doubled), u = step/|step|
      float wxx = 0.0f, wyy = 0.0f, wzz = 0.0f, wxy = 0.0f, wxz = 0.0f, wyz = 0.0f;
      if (MODE == kSkWide) {
        const double ux = static_cast<double>(sx), uy = static_cast<double>(sy), uz = static_cast<double>(sz);
        const double r2 = ux * ux + uy * uy + uz * uz;
        const double ir2 = r2 > 0.0 ? 1.0 / r2 : 0.0;
        wxx = static_cast<float>(ux * ux * ir2);
        wyy = static_cast<float>(uy * uy * ir2);
        wzz = static_cast<float>(uz * uz * ir2);
        wxy = static_cast<float>(2.0 * ux * uy * ir2);
        wxz = static_cast<float>(2.0 * ux * uz * ir2);
        wyz = static_cast<float>(2.0 * uy * uz * ir2);
      }
      // fixed-point positions of the lane's pixels j = lane + 64 u, advanced by
      // one addition per step of 64 U pixels (pixels past the end wrap like any
      // other and are dropped)
      int64_t pos[U][3];
      const int64_t adv[3] = {64 * U * sx, 64 * U * sy, 64 * U * sz};
      // position of the lane's pixels in the z(chi) table, in table steps
      // times 2^32 (chi_j / kZTabH = chi0 / kZTabH - j dchi / kZTabH, each term
      // rounded to 2^-32 steps: at most 2^-22 Mpc/h off at j = 2048)
      int64_t zpos[U];
      const int64_t zstep = llrint(a.dchi * (4294967296.0 / kZTabH));
      if (a.do_flux) {
        const int64_t z0 = llrint(chi0 * (4294967296.0 / kZTabH));
#pragma unroll
        for (int u = 0; u < U; ++u) zpos[u] = z0 - (lane + 64 * u) * zstep;
      }
      if (MODE != kSkGauss) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = lane + 64 * u;
          pos[u][0] = ox + j * sx;
          pos[u][1] = oy + j * sy;
          pos[u][2] = oz + j * sz;
        }
      }
      // pixel j is in bin b when jb[b+1] <= j < jb[b]; each lane walks j upward
      // and therefore the bins downward, accumulating one bin at a time.  U
      // pixels per lane per step: all their gathers are issued before any is used.
      int bin = a.n_bins - 1;
      int cur = -1;
      unsigned long long acc = 0ull, cnt = 0ull;
      // the Gaussian mode runs every lane through every 64-pixel chunk (its
      // wave reductions need all lanes); lanes past the end are not stored
      for (int it = (MODE == kSkGauss ? 0 : lane); it < np; it += 64 * U) {
        const int j0 = MODE == kSkGauss ? it + lane : it;
        float dd[U], ee[U];
        if (gather) {
          float dl[U], el[U];
          if constexpr (MODE == kSkGauss) {
            static_assert(U == 1, "one pixel per lane");
            const int j = j0;
            const bool valid = j < np;
            const int jj = valid ? j : j0 - lane;  // the chunk's first pixel (always valid)
            const int64_t px = ox + jj * sx, py = oy + jj * sy, pz = oz + jj * sz;
            // base cell: the chunk's first pixel, the same for every lane
            const int j1 = j0 - lane;
            const int64_t bx = (ox + j1 * sx) >> 32, by = (oy + j1 * sy) >> 32, bz = (oz + j1 * sz) >> 32;
            if (!gauss7_staged<B16>(a, px, py, pz, valid, bx, by, bz, N, NN, sgauss[wv], lane, dl[0], el[0]))
              gauss7_at<B16>(a, px, py, pz, N, NN, dl[0], el[0]);
          } else {
          float2 c[U][8];
          float t3[U][3];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t px = pos[u][0], py = pos[u][1], pz = pos[u][2];
            pos[u][0] = px + adv[0];
            pos[u][1] = py + adv[1];
            pos[u][2] = pz + adv[2];
            const uint32_t msk = static_cast<uint32_t>(N - 1);
            const uint32_t ix = static_cast<uint32_t>(px >> 32) & msk;
            const uint32_t iy = static_cast<uint32_t>(py >> 32) & msk;
            const uint32_t iz = static_cast<uint32_t>(pz >> 32) & msk;
            const uint32_t jx = (ix + 1) & msk, jy = (iy + 1) & msk, jz = (iz + 1) & msk;
            t3[u][0] = static_cast<float>(static_cast<uint32_t>(px)) * 2.3283064365386963e-10f;
            t3[u][1] = static_cast<float>(static_cast<uint32_t>(py)) * 2.3283064365386963e-10f;
            t3[u][2] = static_cast<float>(static_cast<uint32_t>(pz)) * 2.3283064365386963e-10f;
            if (MODE == kSkWide) {
              // plane offsets in 64 bits, offsets within a plane (< n^2) in 32
              const size_t x0 = static_cast<size_t>(ix) * NN, x1 = static_cast<size_t>(jx) * NN;
              const uint32_t y0 = iy * static_cast<uint32_t>(N), y1 = jy * static_cast<uint32_t>(N);
              const size_t ci[8] = {x0 + (y0 + iz), x0 + (y0 + jz), x0 + (y1 + iz), x0 + (y1 + jz),
                                    x1 + (y0 + iz), x1 + (y0 + jz), x1 + (y1 + iz), x1 + (y1 + jz)};
              // all 32 gathers first, then eta_par = u_p u_q eta^pq per corner
              float2 w0[8], w1[8], w2[8], w3[8];
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                w0[k] = ld_field<B16>(a, ci[k]);
                w1[k] = ld_wide<B16>(a, 0, ci[k]);
                w2[k] = ld_wide<B16>(a, 1, ci[k]);
                w3[k] = ld_wide<B16>(a, 2, ci[k]);
              }
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const float e = wzz * w0[k].y + wxx * w1[k].x + wyy * w1[k].y + wxy * w2[k].x + wxz * w2[k].y +
                                wyz * w3[k].x;
                c[u][k] = make_float2(w0[k].x, e);
              }
            } else {
              // byte addresses: each x plane's start as one 32 x 32 -> 64-bit
              // multiply-add on the box pointer, the corner's offset within the
              // plane (below 2^25 bytes) added to it
              constexpr uint32_t ES = B16 ? 4u : 8u;
              const char* fb = B16 ? reinterpret_cast<const char*>(a.field_bf16) : reinterpret_cast<const char*>(a.field);
              const uint32_t pb = static_cast<uint32_t>(NN) * ES;  // plane pitch in bytes (< 2^32)
              const char* p0 = fb + static_cast<uint64_t>(ix) * pb;
              const char* p1 = fb + static_cast<uint64_t>(jx) * pb;
              const uint32_t y0 = iy * (static_cast<uint32_t>(N) * ES), y1 = jy * (static_cast<uint32_t>(N) * ES);
              const uint32_t z0 = iz * ES, z1 = jz * ES;
              const uint32_t o[4] = {y0 + z0, y0 + z1, y1 + z0, y1 + z1};
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const char* pk = (k < 4 ? p0 : p1) + o[k & 3];
                if constexpr (B16)
                  c[u][k] = unpack_bf16x2(*reinterpret_cast<const uint32_t*>(pk));
                else
                  c[u][k] = *reinterpret_cast<const float2*>(pk);
              }
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const float tx = t3[u][0], ty = t3[u][1], tz = t3[u][2];
            dl[u] = trilerp(tx, ty, tz, c[u][0].x, c[u][1].x, c[u][2].x, c[u][3].x, c[u][4].x, c[u][5].x,
                            c[u][6].x, c[u][7].x);
            el[u] = trilerp(tx, ty, tz, c[u][0].y, c[u][1].y, c[u][2].y, c[u][3].y, c[u][4].y, c[u][5].y,
                            c[u][6].y, c[u][7].y);
          }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int j = j0 + 64 * u;
            float d = dl[u];
            const float e = el[u];
            if (j < np) {
              if (with_ds) {
                const float2 z2 = buf[pidx(j >> 1)];
                d += (j & 1) ? z2.y : z2.x;
              }
              if (a.dens) a.dens[off + j] = d;
              if (a.eta) a.eta[off + j] = e;
            }
            dd[u] = d;
            ee[u] = e;
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int j = j0 + 64 * u;
            dd[u] = j < np ? a.in_dens[off + j] : 0.0f;
            ee[u] = j < np ? a.in_eta[off + j] : 0.0f;
            if (with_ds && j < np) {
              const float2 z2 = buf[pidx(j >> 1)];
              dd[u] += (j & 1) ? z2.y : z2.x;
            }
          }
        }
        if (a.do_flux) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int j = j0 + 64 * u;
            if (j >= np) break;
            const float d = dd[u], e = ee[u];
            const int64_t zp = zpos[u];
            const int64_t ip = zp >> 32;
            int iu;
            float t;
            if (ip >= 0 && ip <= kZTabN - 2) {
              iu = static_cast<int>(ip);
              t = static_cast<float>(static_cast<uint32_t>(zp)) * 2.3283064365386963e-10f;
            } else {  // beyond the table: the end interval continued linearly
              iu = ip < 0 ? 0 : kZTabN - 2;
              t = static_cast<float>(static_cast<double>(zp - (static_cast<int64_t>(iu) << 32)) *
                                     2.3283064365386963e-10);
            }
            const float zt0 = a.ztab[iu], zt1 = a.ztab[iu + 1];
            const float x = (zt0 + t * (zt1 - zt0)) + (1.0f - kFgpaX0);   // (1+z) - x0
            const float ca = a.cf[0][0] + x * (a.cf[0][1] + x * a.cf[0][2]);
            const float cb = a.cf[1][0] + x * (a.cf[1][1] + x * a.cf[1][2]);
            const float cc = a.cf[2][0] + x * (a.cf[2][1] + x * a.cf[2][2]);
            const float F = __expf(-ca * __expf(cb * (d + cc * e)));
            if (a.flux) a.flux[off + j] = F;
            if (want_bins) {
              while (bin >= 0 && j >= jb[bin]) --bin;  // pixel j lies below bin's upper edge
              const int key = (bin >= 0 && j >= jb[bin + 1]) ? bin : -1;
              if (key != cur) {
                if (cnt) {
                  atomicAdd(&s_sum[cur], acc);
                  atomicAdd(&s_cnt[cur], cnt);
                }
                acc = 0ull;
                cnt = 0ull;
                cur = key;
              }
              if (key >= 0) {
                acc += __float2ull_rn(F * 4294967296.0f);
                cnt += 1ull;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) zpos[u] -= 64 * U * zstep;
        }
      }
      if (cnt) {
        atomicAdd(&s_sum[cur], acc);
        atomicAdd(&s_cnt[cur], cnt);
      }
      wave_sync();  // the wave's LDS slice is reused by its next skewer
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

int device_cus() {
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

template <bool B16>
void launch_skewer_kernel(const SkewerArgs& a, int u, dim3 grid, hipStream_t st) {
  if (a.is_gauss) {
    // 343 gathers per pixel: one pixel per lane at a time
    LYA_TIMED("skewers_gauss", st, hipLaunchKernelGGL((k_skewers<1, kSkGauss, B16>), grid, dim3(kSkNT), 0, st, a));
  } else if (a.is_wide) {
    // four boxes per pixel: at most two pixels per lane in flight
    if (u == 1)
      LYA_TIMED("skewers_wide", st, hipLaunchKernelGGL((k_skewers<1, kSkWide, B16>), grid, dim3(kSkNT), 0, st, a));
    else
      LYA_TIMED("skewers_wide", st, hipLaunchKernelGGL((k_skewers<2, kSkWide, B16>), grid, dim3(kSkNT), 0, st, a));
  } else if (u == 1) {
    LYA_TIMED(a.in_dens ? "apply_fgpa" : "skewers", st,
              hipLaunchKernelGGL((k_skewers<1, kSkTri, B16>), grid, dim3(kSkNT), 0, st, a));
  } else if (u == 2) {
    LYA_TIMED(a.in_dens ? "apply_fgpa" : "skewers", st,
              hipLaunchKernelGGL((k_skewers<2, kSkTri, B16>), grid, dim3(kSkNT), 0, st, a));
  } else {
    LYA_TIMED(a.in_dens ? "apply_fgpa" : "skewers", st,
              hipLaunchKernelGGL((k_skewers<4, kSkTri, B16>), grid, dim3(kSkNT), 0, st, a));
  }
}

hipError_t launch_skewers(const SkewerArgs& a, hipStream_t st) {
  LYA_TIMED("skewer_reset", st,
            hipLaunchKernelGGL(k_skewer_reset, dim3(1), dim3(256), 0, st, a.queue, a.bin_sum, a.bin_cnt));
  const int64_t nchunks = (a.n_sk + a.chunk - 1) / a.chunk;
  int64_t blocks = static_cast<int64_t>(device_cus()) * (a.blocks_per_cu > 0 ? a.blocks_per_cu : 4);
  if (blocks * kSkWaves > nchunks) blocks = (nchunks + kSkWaves - 1) / kSkWaves;
  if (blocks < 1) blocks = 1;
  const int u = a.unroll == 1 || a.unroll == 4 ? a.unroll : 2;
  const dim3 grid(static_cast<unsigned>(blocks));
  if (a.field_bf16)
    launch_skewer_kernel<true>(a, u, grid, st);
  else
    launch_skewer_kernel<false>(a, u, grid, st);
  if (a.n_bins > 0 && a.do_flux)
    LYA_TIMED("skewer_finalize", st,
              hipLaunchKernelGGL(k_skewer_finalize, dim3(1), dim3(256), 0, st, a.n_bins, a.bin_sum, a.bin_cnt,
                                 a.out_fsum, a.out_count));
  return hipGetLastError();
}

}  // namespace lya
