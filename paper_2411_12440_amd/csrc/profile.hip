// Kernel timing with HIP events (ls_profile_enable / ls_profile_read).
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace lsplat {

namespace {

struct Rec {
  const char* name;
  hipEvent_t a, b;
};

struct Profiler {
  bool enabled = false;
  std::vector<hipEvent_t> pool;       // free events
  std::vector<Rec> pending;           // recorded, not yet read
  std::map<std::string, std::pair<int64_t, double>> totals;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

Profiler& prof() {
  static Profiler p;
  return p;
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), s_(s), slot_(-1) {
  Profiler& p = prof();
  if (!p.enabled || !name) return;   // a null name: untimed (creates no events)
  hipEvent_t a = p.get(), b = p.get();
  if (!a || !b) return;
  if (hipEventRecord(a, s) != hipSuccess) return;
  p.pending.push_back(Rec{name, a, b});
  slot_ = (int)p.pending.size() - 1;
}

ProfScope::~ProfScope() {
  if (slot_ < 0) return;
  Profiler& p = prof();
  if (slot_ < (int)p.pending.size()) (void)hipEventRecord(p.pending[slot_].b, s_);
}

}  // namespace lsplat

using namespace lsplat;

extern "C" {

ls_status ls_profile_enable(int enable) {
  prof().enabled = enable != 0;
  return LS_OK;
}

ls_status ls_profile_read(ls_kernel_time* out, int capacity, int* count, int reset) {
  Profiler& p = prof();
  for (Rec& r : p.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& t = p.totals[r.name];
      t.first += 1;
      t.second += ms;
    }
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.pending.clear();
  std::vector<std::pair<std::string, std::pair<int64_t, double>>> v(p.totals.begin(), p.totals.end());
  std::sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.second.second > y.second.second; });
  if (count) *count = (int)v.size();
  for (int i = 0; out && i < capacity && i < (int)v.size(); ++i) {
    memset(out[i].name, 0, sizeof(out[i].name));
    strncpy(out[i].name, v[i].first.c_str(), sizeof(out[i].name) - 1);
    out[i].launches = v[i].second.first;
    out[i].total_ms = v[i].second.second;
  }
  if (reset) p.totals.clear();
  return LS_OK;
}

}  // extern "C"
