// prof.cpp — opt-in per-kernel timing (see prof.h and mbx_profile_* in mbx.h).
#include "prof.h"

#include <mutex>
#include <vector>

#include "../../include/mbx.h"

namespace mbx {
namespace {

struct Rec {
  hipEvent_t a, b;
  double bytes;
  int launches;
};

std::mutex g_mu;
int g_kernel = PK_NONE;
std::vector<Rec> g_recs;      // recorded pairs not yet read
std::vector<hipEvent_t> g_pool;
hipEvent_t g_open = nullptr;

hipEvent_t take_event() {
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

bool prof_on(int k) { return k != PK_NONE && g_kernel == k; }
bool prof_active() { return g_kernel != PK_NONE; }

void prof_begin(int k, hipStream_t s) {
  if (!prof_on(k)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_open = take_event();
  if (g_open) (void)hipEventRecord(g_open, s);
}

void prof_end_n(int k, hipStream_t s, double bytes, int launches) {
  if (!prof_on(k)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_open) return;
  hipEvent_t e = take_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_recs.push_back(Rec{g_open, e, bytes, launches});
  g_open = nullptr;
}

void prof_end(int k, hipStream_t s, double bytes) { prof_end_n(k, s, bytes, 1); }

}  // namespace mbx

extern "C" {

int mbx_profile(int kernel) {
  std::lock_guard<std::mutex> lk(mbx::g_mu);
  if (kernel < mbx::PK_NONE || kernel > mbx::PK_GRAM) return MBX_EINVAL;
  mbx::g_kernel = kernel;
  for (auto& r : mbx::g_recs) {
    mbx::g_pool.push_back(r.a);
    mbx::g_pool.push_back(r.b);
  }
  mbx::g_recs.clear();
  return MBX_OK;
}

int mbx_profile_read(int64_t* launches, double* total_ms, double* total_bytes) {
  std::lock_guard<std::mutex> lk(mbx::g_mu);
  double ms = 0.0, by = 0.0;
  int64_t n = 0;
  for (auto& r : mbx::g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return MBX_EHIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return MBX_EHIP;
    ms += t;
    by += r.bytes;
    n += r.launches;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (total_bytes) *total_bytes = by;
  return MBX_OK;
}

}  // extern "C"
