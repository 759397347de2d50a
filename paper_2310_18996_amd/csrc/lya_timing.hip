// Optional per-kernel timing: when enabled, every kernel the library launches
// is bracketed by two HIP events recorded on its own stream.  Reading the
// records waits for the last event and sums elapsed time per kernel name.
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lyamock.h"
#include "lya_internal.h"

namespace lya {
namespace {

struct Rec {
  const char* name;
  hipEvent_t a, b;
};

struct Agg {
  std::string name;
  double ms = 0.0;
  int64_t n = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Agg> g_agg;
thread_local hipEvent_t t_open = nullptr;
thread_local const char* t_name = nullptr;

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

void timer_begin(const char* name, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipEvent_t e = take();
  if (!e) return;
  if (hipEventRecord(e, st) != hipSuccess) {
    g_pool.push_back(e);
    return;
  }
  t_open = e;
  t_name = name;
}

void timer_end(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || !t_open) return;
  hipEvent_t e = take();
  if (e && hipEventRecord(e, st) == hipSuccess) {
    g_recs.push_back(Rec{t_name, t_open, e});
  } else {
    g_pool.push_back(t_open);
    if (e) g_pool.push_back(e);
  }
  t_open = nullptr;
}

}  // namespace lya

extern "C" {

int lya_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(lya::g_mu);
  for (auto& r : lya::g_recs) {
    lya::g_pool.push_back(r.a);
    lya::g_pool.push_back(r.b);
  }
  lya::g_recs.clear();
  lya::g_agg.clear();
  lya::g_on = on != 0;
  return LYA_OK;
}

int lya_timing_collect(void) {
  std::lock_guard<std::mutex> lk(lya::g_mu);
  lya::g_agg.clear();
  if (!lya::g_recs.empty() && hipEventSynchronize(lya::g_recs.back().b) != hipSuccess) return LYA_EHIP;
  for (auto& r : lya::g_recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return LYA_EHIP;
    bool found = false;
    for (auto& g : lya::g_agg) {
      if (g.name == r.name) {
        g.ms += ms;
        g.n += 1;
        found = true;
        break;
      }
    }
    if (!found) lya::g_agg.push_back(lya::Agg{r.name, static_cast<double>(ms), 1});
  }
  return static_cast<int>(lya::g_agg.size());
}

int lya_timing_get(int i, char* name, int name_len, double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(lya::g_mu);
  if (i < 0 || i >= static_cast<int>(lya::g_agg.size()) || !name || name_len < 1) return LYA_EINVAL;
  snprintf(name, name_len, "%s", lya::g_agg[i].name.c_str());
  if (total_ms) *total_ms = lya::g_agg[i].ms;
  if (launches) *launches = lya::g_agg[i].n;
  return LYA_OK;
}

}  // extern "C"
