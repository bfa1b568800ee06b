// Launch profiler (see prof.hpp) and its C entry points.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "prof.hpp"

namespace ie {

namespace {
struct Rec {
  std::string key;
  double bytes;
  long group = -1;
  hipEvent_t a = nullptr, b = nullptr;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
long g_next_group = 0;
thread_local long t_group = -1;
std::map<long, double> g_scale;
std::vector<size_t> g_open;  // indices of records whose end event is pending (nested scopes)

hipEvent_t get_event() {
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

bool prof_enabled() { return g_on; }

long prof_new_group() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_next_group++;
}
void prof_set_group(long g) { t_group = g; }
void prof_scale_group(long g, double scale) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_on && g >= 0) g_scale[g] = scale;
}

void prof_record(hipStream_t s, bool start, const std::string* key, double bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipEvent_t e = get_event();
  if (e == nullptr) return;
  if (start) {
    Rec r;
    r.key = *key;
    r.bytes = bytes;
    r.group = t_group;
    r.a = e;
    g_open.push_back(g_recs.size());
    g_recs.push_back(r);
  } else {
    if (g_open.empty()) {
      g_pool.push_back(e);
      return;
    }
    g_recs[g_open.back()].b = e;
    g_open.pop_back();
  }
  (void)hipEventRecord(e, s);
}

}  // namespace ie

using namespace ie;

extern "C" {

int ie_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_scale.clear();
  g_open.clear();
  g_on = true;
  return IE_OK;
}

int ie_profile_end(ie_kernel_stat* out, int32_t cap, int32_t* count) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = false;
  if (hipDeviceSynchronize() != hipSuccess) return fail(IE_EDEVICE, "hipDeviceSynchronize failed");
  struct Agg {
    int n = 0;
    double tot = 0, mn = 1e300, mx = 0, bytes = 0;
  };
  std::map<std::string, Agg> agg;
  for (auto& r : g_recs) {
    if (!r.a || !r.b) continue;
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    Agg& g = agg[r.key];
    g.n += 1;
    g.tot += ms;
    g.mn = std::min(g.mn, double(ms));
    g.mx = std::max(g.mx, double(ms));
    double sc = 1.0;
    if (r.group >= 0) {
      auto it = g_scale.find(r.group);
      if (it != g_scale.end()) sc = it->second;
    }
    g.bytes += r.bytes * sc;
  }
  for (auto& r : g_recs) {
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_scale.clear();
  std::vector<std::pair<std::string, Agg>> v(agg.begin(), agg.end());
  std::sort(v.begin(), v.end(), [](auto& x, auto& y) { return x.second.tot > y.second.tot; });
  int n = 0;
  for (auto& kv : v) {
    if (out != nullptr && n < cap) {
      ie_kernel_stat& k = out[n];
      std::memset(&k, 0, sizeof(k));
      std::strncpy(k.name, kv.first.c_str(), sizeof(k.name) - 1);
      k.launches = kv.second.n;
      k.total_ms = kv.second.tot;
      k.min_ms = kv.second.mn;
      k.max_ms = kv.second.mx;
      k.bytes_per_launch = kv.second.n ? kv.second.bytes / kv.second.n : 0;
    }
    ++n;
  }
  if (count) *count = n;
  return IE_OK;
}

}  // extern "C"
