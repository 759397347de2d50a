/* Exact FP64 evaluation of whole z-lines of a large periodic Gaussian box.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle): used for sampled parity of
 * boxes too large for a full FP64 inverse FFT on the host.
 *
 * Follows eq:deltaL and eq:eta with the same mode bookkeeping as
 * oracle/field.py (written independently here in plain C):
 *   W(k) from Philox4x32-10 (Salmon et al. SC'11), key = seed, counter =
 *   (lin>>1 lo, lin>>1 hi, stream 0, 0), words (2b, 2b+1) with b = lin & 1,
 *   uniforms ((w>>9)+0.5) 2^-23, Box-Muller in FP64; the owner of a Hermitian
 *   pair is the lower linear index; self-conjugate modes take W = z1.
 *   X(k) = s(n^2) W(k) * (mult_a + i mult_b) with mult from the component
 *   pair (delta, or f k_p k_q / k^2).
 * For each requested column (mx, my) the plain definition
 *   C(mx,my,mz) = sum_{ix,iy,iz} X exp(+2 pi i (ix mx + iy my + iz mz)/N)
 * is evaluated as A[iz] = sum_{ix,iy} X exp(2 pi i (ix mx + iy my)/N)
 * followed by a direct (O(N^2)) sum over iz.  No FFT, no blocking beyond
 * splitting the ix loop over threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint64_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = m0 * (uint64_t)c[0];
    uint64_t p1 = m1 * (uint64_t)c[2];
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

static void normals(uint64_t seed, uint32_t stream, uint64_t lin, double* z1, double* z2) {
  uint64_t ctr = lin >> 1;
  uint32_t c[4] = {(uint32_t)ctr, (uint32_t)(ctr >> 32), stream, 0u};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  int b = (int)(lin & 1u);
  double u1 = ((double)(c[2 * b] >> 9) + 0.5) * ldexp(1.0, -23);
  double u2 = ((double)(c[2 * b + 1] >> 9) + 0.5) * ldexp(1.0, -23);
  double r = sqrt(-2.0 * log(u1));
  *z1 = r * cos(2.0 * M_PI * u2);
  *z2 = r * sin(2.0 * M_PI * u2);
}

static long sgn_freq(long i, long n) { return i < n / 2 ? i : i - n; }

/* comp: 0 delta, 1 xx, 2 yy, 3 zz, 4 xy, 5 xz, 6 yz */
static double multiplier(int comp, long nx, long ny, long nz, long n, double f) {
  if (comp == 0) return 1.0;
  long v[3] = {nx, ny, nz};
  static const int P[7] = {0, 0, 1, 2, 0, 0, 1};
  static const int Q[7] = {0, 0, 1, 2, 1, 2, 2};
  long n2 = nx * nx + ny * ny + nz * nz;
  if (n2 == 0) return 0.0;
  int p = P[comp], q = Q[comp];
  if (p != q && (v[p] == -(n / 2) || v[q] == -(n / 2))) return 0.0;
  return f * (double)(v[p] * v[q]) / (double)n2;
}

/* Returns 0 on success.  out_re/out_im: [nlines][n]; line l at column
 * (mx[l], my[l]); out_re holds component a, out_im component b. */
int oracle_field_lines(int n, uint64_t seed, double f, int comp_a, int comp_b,
                       int fixed_amp, long only_n2, const double* table,
                       int nlines, const int* mx, const int* my,
                       double* out_re, double* out_im, int nthreads) {
  long N = n;
  double* acc = (double*)calloc((size_t)nthreads * nlines * N * 2, sizeof(double));
  if (!acc) return -1;
  double* ctab = (double*)malloc(sizeof(double) * N);
  double* stab = (double*)malloc(sizeof(double) * N);
  for (long r = 0; r < N; ++r) {
    ctab[r] = cos(2.0 * M_PI * (double)r / (double)N);
    stab[r] = sin(2.0 * M_PI * (double)r / (double)N);
  }
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
  for (long ix = 0; ix < N; ++ix) {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    double* a = acc + (size_t)t * nlines * N * 2;
    long nx = sgn_freq(ix, N);
    for (long iy = 0; iy < N; ++iy) {
      long ny = sgn_freq(iy, N);
      for (long iz = 0; iz < N; ++iz) {
        long nz = sgn_freq(iz, N);
        long n2 = nx * nx + ny * ny + nz * nz;
        if (only_n2 >= 0 && n2 != only_n2) continue;
        double s = table[n2];
        if (s == 0.0) continue;
        uint64_t lin = ((uint64_t)ix * N + iy) * N + iz;
        uint64_t plin = ((uint64_t)((N - ix) % N) * N + (N - iy) % N) * N + (N - iz) % N;
        uint64_t own = lin < plin ? lin : plin;
        double z1, z2;
        normals(seed, 0u, own, &z1, &z2);
        double wr, wi;
        if (lin == plin) { wr = z1; wi = 0.0; }
        else {
          wr = z1 / sqrt(2.0);
          wi = (lin == own ? z2 : -z2) / sqrt(2.0);
        }
        if (fixed_amp) {
          double m = sqrt(wr * wr + wi * wi);
          wr /= m; wi /= m;
        }
        double ma = multiplier(comp_a, nx, ny, nz, N, f);
        double mb = comp_b < 0 ? 0.0 : multiplier(comp_b, nx, ny, nz, N, f);
        /* X = s W (ma + i mb) */
        double xr = s * (wr * ma - wi * mb);
        double xi = s * (wi * ma + wr * mb);
        for (int l = 0; l < nlines; ++l) {
          long r = (ix * mx[l] + iy * my[l]) % N;
          double pr = ctab[r], pi = stab[r];
          a[((size_t)l * N + iz) * 2 + 0] += xr * pr - xi * pi;
          a[((size_t)l * N + iz) * 2 + 1] += xr * pi + xi * pr;
        }
      }
    }
  }
  for (int l = 0; l < nlines; ++l) {
    for (long mz = 0; mz < N; ++mz) {
      double sr = 0.0, si = 0.0;
      for (int t = 0; t < nthreads; ++t) {
        const double* a = acc + ((size_t)t * nlines + l) * N * 2;
        for (long iz = 0; iz < N; ++iz) {
          long r = (iz * mz) % N;
          double ar = a[iz * 2], ai = a[iz * 2 + 1];
          sr += ar * ctab[r] - ai * stab[r];
          si += ar * stab[r] + ai * ctab[r];
        }
      }
      out_re[(size_t)l * N + mz] = sr;
      out_im[(size_t)l * N + mz] = si;
    }
  }
  free(acc); free(ctab); free(stab);
  return 0;
}
