#include "profile.h"

#include <vector>

#include "dmc_internal.h"

namespace dmc {
namespace prof {
namespace {

int g_selected = -1;
bool g_paused = false;  // no events while a stream is being captured into a graph
std::vector<hipEvent_t> g_pool;  // begin/end pairs, reused between sessions
size_t g_used = 0;

hipEvent_t next_event() {
  if (g_used == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_used++];
}

}  // namespace

void begin(hipStream_t s, int kernel) {
  if (kernel != g_selected || g_paused) return;
  hipEvent_t e = next_event();
  if (e) (void)hipEventRecord(e, s);
}

void end(hipStream_t s, int kernel) { begin(s, kernel); }

void pause(bool on) { g_paused = on; }

}  // namespace prof
}  // namespace dmc

extern "C" {

dmc_status dmc_profile_start(int32_t kernel) {
  if (kernel < 0 || kernel >= DMC_KERNEL_COUNT) return DMC_ERR_INVALID_ARG;
  dmc::prof::g_selected = kernel;
  dmc::prof::g_used = 0;
  return DMC_OK;
}

dmc_status dmc_profile_stop(int32_t* launches, double* ms_total) {
  using namespace dmc::prof;
  g_selected = -1;
  double total = 0.0;
  int32_t count = 0;
  for (size_t i = 0; i + 1 < g_used; i += 2) {
    if (hipEventSynchronize(g_pool[i + 1]) != hipSuccess) return DMC_ERR_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_pool[i], g_pool[i + 1]) != hipSuccess) return DMC_ERR_DEVICE;
    total += ms;
    ++count;
  }
  g_used = 0;
  if (launches) *launches = count;
  if (ms_total) *ms_total = total;
  return DMC_OK;
}

}  // extern "C"
