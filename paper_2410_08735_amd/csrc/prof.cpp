// HIP-event profiler for the library's hot kernels (off by default).
#include <mutex>

#include "rte_internal.h"

namespace rte {

namespace {
struct Slot {
  std::vector<hipEvent_t> a, b;
  std::vector<double> units;
  size_t used = 0;
};
bool g_on = false;
Slot g_slot[PROF_SLOTS];
std::mutex g_mu;
}  // namespace

bool prof_enabled() { return g_on; }

void prof_begin(int slot, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  Slot& S = g_slot[slot];
  if (S.used == S.a.size()) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return;
    S.a.push_back(e0);
    S.b.push_back(e1);
    S.units.push_back(0.0);
  }
  (void)hipEventRecord(S.a[S.used], s);
}

void prof_end(int slot, hipStream_t s, double units) {
  std::lock_guard<std::mutex> lk(g_mu);
  Slot& S = g_slot[slot];
  if (S.used >= S.a.size()) return;
  (void)hipEventRecord(S.b[S.used], s);
  S.units[S.used] = units;
  S.used++;
}

int prof_last(int slot) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_slot[slot].used - 1;
}

void prof_set_units(int slot, int idx, double units) {
  std::lock_guard<std::mutex> lk(g_mu);
  Slot& S = g_slot[slot];
  if (idx >= 0 && (size_t)idx < S.used) S.units[idx] = units;
}

// Empty kernel whose only purpose is to appear in kernel traces.
__global__ void k_region_marker(int) {}

}  // namespace rte

extern "C" int rte_prof_mark(int id, void* stream) {
  hipLaunchKernelGGL(rte::k_region_marker, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), id);
  return hipGetLastError() == hipSuccess ? RTE_OK : RTE_EHIP;
}

extern "C" int rte_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(rte::g_mu);
  rte::g_on = on != 0;
  for (auto& S : rte::g_slot) S.used = 0;
  return RTE_OK;
}

extern "C" int rte_prof_read(int slot, int64_t* launches, double* total_ms, double* total_units) {
  if (slot < 0 || slot >= rte::PROF_SLOTS || !launches || !total_ms || !total_units) return RTE_EINVAL;
  std::lock_guard<std::mutex> lk(rte::g_mu);
  auto& S = rte::g_slot[slot];
  double ms = 0.0, u = 0.0;
  int64_t n = 0;
  for (size_t i = 0; i < S.used; ++i) {
    if (hipEventSynchronize(S.b[i]) != hipSuccess) return RTE_EHIP;
    if (S.units[i] < 0.0) continue;  // withdrawn (a launch that found no work)
    float t = 0.f;
    if (hipEventElapsedTime(&t, S.a[i], S.b[i]) != hipSuccess) return RTE_EHIP;
    ms += t;
    u += S.units[i];
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  *total_units = u;
  return RTE_OK;
}
