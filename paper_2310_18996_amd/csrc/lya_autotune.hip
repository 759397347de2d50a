// Launch-shape autotuning and HIP-graph capture of the hot path.
//
// The tuning table holds, per box size, the variant of each strided FFT pass
// (tile of 8 or 4 pencils, tile order, one tile per block or the persistent
// pipelined kernel) and the skewer kernel's work-chunk size and blocks per
// CU.  The autotuners time every candidate with HIP events on the caller's
// stream and keep the fastest; later calls for that box size use it.
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/lyamock.h"
#include "lya_internal.h"

namespace lya {

namespace {
std::mutex g_mu;
int g_chunk[12] = {4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4};
int g_bpc[12] = {4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4};
int g_unroll[12] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
int lg(int n) {
  int l = 0;
  while ((1 << l) < n && l < 11) ++l;
  return l;
}
}  // namespace

int sk_chunk(int n) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_chunk[lg(n)];
}
int sk_blocks_per_cu(int n) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_bpc[lg(n)];
}
int sk_unroll(int n) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_unroll[lg(n)];
}
void set_sk_shape(int n, int chunk, int bpc, int unroll) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_chunk[lg(n)] = chunk;
  g_bpc[lg(n)] = bpc;
  g_unroll[lg(n)] = unroll;
}

}  // namespace lya

namespace {

thread_local char g_aerr[256] = "";
int afail(int code, const char* msg) {
  snprintf(g_aerr, sizeof(g_aerr), "%s", msg);
  return code;
}
int ahip(hipError_t e, const char* where) {
  snprintf(g_aerr, sizeof(g_aerr), "%s: %s", where, hipGetErrorString(e));
  return LYA_EHIP;
}
bool box_ok(const lya_box* b) {
  return b && b->n >= 32 && b->n <= 2048 && (b->n & (b->n - 1)) == 0 && b->storage == LYA_F32;
}

constexpr int kChunks[] = {1, 2, 4, 8, 16, 32, 64};
constexpr int kBpc[] = {1, 2, 3, 4};
constexpr int kUnroll[] = {1, 2, 4};
constexpr int kNChunks = sizeof(kChunks) / sizeof(kChunks[0]);
constexpr int kNBpc = sizeof(kBpc) / sizeof(kBpc[0]);
constexpr int kNUnroll = sizeof(kUnroll) / sizeof(kUnroll[0]);

// mean milliseconds of `reps` runs of fn() on st, after one untimed run
template <typename F>
hipError_t time_ms(F&& fn, int reps, hipStream_t st, double* ms) {
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  float t = 0.0f;
  e = fn();
  if (e == hipSuccess) e = hipEventRecord(a, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = static_cast<double>(t) / reps;
  return e;
}

struct GraphHolder {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

}  // namespace

extern "C" {

const char* lya_autotune_last_error(void) { return g_aerr; }

int lya_get_tuning(int32_t n, lya_tuning* t) {
  if (!t || n < 32 || n > 2048 || (n & (n - 1))) return afail(LYA_EINVAL, "invalid box size or NULL output");
  t->fft_y = lya::fft_variant(n, 0);
  t->fft_x = lya::fft_variant(n, 1);
  t->sk_chunk = lya::sk_chunk(n);
  t->sk_blocks_per_cu = lya::sk_blocks_per_cu(n);
  t->sk_unroll = lya::sk_unroll(n);
  return LYA_OK;
}

int lya_set_tuning(int32_t n, const lya_tuning* t) {
  if (!t || n < 32 || n > 2048 || (n & (n - 1))) return afail(LYA_EINVAL, "invalid box size or NULL tuning");
  if (t->sk_chunk < 1 || t->sk_chunk > 1024 || t->sk_blocks_per_cu < 1 || t->sk_blocks_per_cu > 4 ||
      (t->sk_unroll != 1 && t->sk_unroll != 2 && t->sk_unroll != 4))
    return afail(LYA_EINVAL, "skewer chunk must be in [1, 1024], blocks per CU in [1, 4], unroll 1, 2 or 4");
  const int oy = lya::fft_variant(n, 0), ox = lya::fft_variant(n, 1);
  if (lya::set_fft_variant(n, 0, t->fft_y) || lya::set_fft_variant(n, 1, t->fft_x)) {
    lya::set_fft_variant(n, 0, oy);
    lya::set_fft_variant(n, 1, ox);
    return afail(LYA_EINVAL, "FFT variant out of range (boxes below 1024 have only the default variants 0 and 1)");
  }
  lya::set_sk_shape(n, t->sk_chunk, t->sk_blocks_per_cu, t->sk_unroll);
  return LYA_OK;
}

int lya_autotune_fft(const lya_box* box, void* field, void* work, size_t work_bytes, int32_t reps, double* ms,
                     lya_tuning* out, void* stream) {
  if (!box_ok(box)) return afail(LYA_EINVAL, "box must be FP32 with n a power of two in [32, 2048]");
  if (!field || !work || reps < 1) return afail(LYA_EINVAL, "field, work or reps invalid");
  const size_t need = ((sizeof(float2) * box->n) + 255) & ~static_cast<size_t>(255);
  if (work_bytes < need) return afail(LYA_EWORKSPACE, "workspace too small for the twiddles");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float2* tw = static_cast<float2*>(work);
  hipError_t e = lya::launch_twiddles(tw, box->n, st);
  if (e != hipSuccess) return ahip(e, "twiddles");
  const int n = box->n;
  const int nv = n >= 1024 ? lya::kFftVariants : 2;
  int best[2] = {lya::fft_variant(n, 0), lya::fft_variant(n, 1)};
  for (int pass = 0; pass < 2; ++pass) {
    double t_all[lya::kFftVariants];
    for (int v = 0; v < lya::kFftVariants; ++v) {
      double t = -1.0;
      if (v < nv) {
        e = time_ms([&] { return lya::launch_fft_strided_pass(n, pass, v, tw, static_cast<float2*>(field), st); },
                    reps, st, &t);
        if (e != hipSuccess) return ahip(e, "timing an FFT variant");
      }
      t_all[v] = t;
      if (ms) ms[pass * lya::kFftVariants + v] = t;
    }
    // the current variant stays unless another is at least 2% faster (timing
    // noise alone should not flip the choice from run to run)
    const int cur = best[pass];
    double bt = t_all[cur] * 0.98;
    for (int v = 0; v < nv; ++v) {
      if (t_all[v] < bt) {
        bt = t_all[v];
        best[pass] = v;
      }
    }
  }
  lya::set_fft_variant(n, 0, best[0]);
  lya::set_fft_variant(n, 1, best[1]);
  if (out) return lya_get_tuning(n, out);
  return LYA_OK;
}

int lya_autotune_skewers(const lya_box* box, const void* field, const lya_skewers* sk, const lya_ps1d* ps,
                         uint64_t seed, const lya_cosmo* cosmo, const lya_fgpa* fgpa, float* dens, float* eta,
                         float* flux, const lya_zbins* zb, void* work, size_t work_bytes, int32_t reps, double* ms,
                         lya_tuning* out, void* stream) {
  if (!box_ok(box)) return afail(LYA_EINVAL, "box must be FP32 with n a power of two in [32, 2048]");
  if (reps < 1) return afail(LYA_EINVAL, "reps must be >= 1");
  const int n = box->n;
  const int c0 = lya::sk_chunk(n), b0 = lya::sk_blocks_per_cu(n), u0 = lya::sk_unroll(n);
  double bt = 1e300;
  int bc = c0, bb = b0, bu = u0;
  for (int i = 0; i < kNChunks; ++i) {
    for (int j = 0; j < kNBpc; ++j) {
      for (int k = 0; k < kNUnroll; ++k) {
        lya::set_sk_shape(n, kChunks[i], kBpc[j], kUnroll[k]);
        int rc = LYA_OK;
        double t = 0.0;
        hipError_t e = time_ms(
            [&] {
              rc = lya_draw_skewers(box, field, sk, ps, seed, cosmo, fgpa, dens, eta, flux, zb, work, work_bytes,
                                    stream);
              return rc == LYA_OK ? hipSuccess : hipErrorUnknown;
            },
            reps, static_cast<hipStream_t>(stream), &t);
        if (rc != LYA_OK) {
          lya::set_sk_shape(n, c0, b0, u0);
          snprintf(g_aerr, sizeof(g_aerr), "lya_draw_skewers: %s", lya_last_error());
          return rc;
        }
        if (e != hipSuccess) {
          lya::set_sk_shape(n, c0, b0, u0);
          return ahip(e, "timing a skewer launch shape");
        }
        if (ms) ms[(i * kNBpc + j) * kNUnroll + k] = t;
        if (t < bt) {
          bt = t;
          bc = kChunks[i];
          bb = kBpc[j];
          bu = kUnroll[k];
        }
      }
    }
  }
  lya::set_sk_shape(n, bc, bb, bu);
  if (out) return lya_get_tuning(n, out);
  return LYA_OK;
}

int lya_graph_begin(void* stream) {
  hipError_t e = hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal);
  return e == hipSuccess ? LYA_OK : ahip(e, "begin capture");
}

int lya_graph_end(void* stream, lya_graph* out) {
  if (!out) return afail(LYA_EINVAL, "output is NULL");
  *out = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &g);
  if (e != hipSuccess) return ahip(e, "end capture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return ahip(e, "instantiate");
  }
  GraphHolder* h = new GraphHolder{g, x};
  *out = reinterpret_cast<lya_graph>(h);
  return LYA_OK;
}

int lya_graph_launch(lya_graph g, void* stream) {
  if (!g) return afail(LYA_EINVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(reinterpret_cast<GraphHolder*>(g)->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LYA_OK : ahip(e, "graph launch");
}

int lya_graph_destroy(lya_graph g) {
  if (!g) return LYA_OK;
  GraphHolder* h = reinterpret_cast<GraphHolder*>(g);
  hipError_t e1 = hipGraphExecDestroy(h->exec);
  hipError_t e2 = hipGraphDestroy(h->graph);
  delete h;
  if (e1 != hipSuccess) return ahip(e1, "graph exec destroy");
  if (e2 != hipSuccess) return ahip(e2, "graph destroy");
  return LYA_OK;
}

}  // extern "C"
