// profile.cpp -- optional HIP-event timing of each entry point's dominant kernel.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"

namespace {

struct Slot {
  hipEvent_t a = nullptr, b = nullptr;
  int which = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Slot> g_pool;
size_t g_used = 0;
constexpr size_t kMaxSlots = 4096;

}  // namespace

namespace lam {

// Returns the slot to record around the kernel, or nullptr when timing is off
// or the pool is exhausted.
void *profile_begin(int which, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_on || g_used >= g_pool.size()) return nullptr;
  Slot *sl = &g_pool[g_used++];
  sl->which = which;
  if (hipEventRecord(sl->a, s) != hipSuccess) return nullptr;
  return sl;
}

void profile_end(void *slot, void *stream) {
  if (!slot) return;
  (void)hipEventRecord(static_cast<Slot *>(slot)->b, static_cast<hipStream_t>(stream));
}

}  // namespace lam

extern "C" LAM_API lam_status lam_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> g(g_mu);
  if (on && g_pool.empty()) {
    g_pool.resize(kMaxSlots);
    for (auto &sl : g_pool) {
      if (hipEventCreate(&sl.a) != hipSuccess || hipEventCreate(&sl.b) != hipSuccess) return LAM_EHIP;
    }
  }
  g_on = on != 0;
  g_used = 0;
  return LAM_OK;
}

extern "C" LAM_API lam_status lam_profile_read(double ms[LAM_PROFILE_SLOTS], int64_t launches[LAM_PROFILE_SLOTS]) {
  if (!ms || !launches) return LAM_EINVAL;
  std::lock_guard<std::mutex> g(g_mu);
  for (int i = 0; i < LAM_PROFILE_SLOTS; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (size_t i = 0; i < g_used; ++i) {
    Slot &sl = g_pool[i];
    if (hipEventSynchronize(sl.b) != hipSuccess) return LAM_EHIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, sl.a, sl.b) != hipSuccess) return LAM_EHIP;
    ms[sl.which] += t;
    launches[sl.which] += 1;
  }
  g_used = 0;
  return LAM_OK;
}
