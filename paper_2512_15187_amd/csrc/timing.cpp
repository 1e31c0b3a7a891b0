// Per-kernel timing with HIP events recorded around each library launch on
// the stream the kernel is launched on.  Off by default; when on, every launch
// (or every k-th launch of each kernel, pid_timing_sample) records one event
// pair, and pid_timing_get() resolves the pending pairs (waiting for them) and
// reports the accumulated time per kernel name.
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/pid.h"
#include "pid_timing.h"

namespace {

struct Pending {
  const char* name;
  hipEvent_t a, b;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<double, int64_t>> g_tot;
std::set<std::string> g_sel;   // kernels to time; empty = all
std::map<std::string, int64_t> g_seen;   // launches of each timed kernel since enabling
int64_t g_every = 1;                     // bracket launch 0, k, 2k, ... of each kernel
constexpr size_t kPoolEvents = 512;   // pre-created when timing is switched on

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

void resolve_locked() {
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& t = g_tot[p.name];
      t.first += ms;
      t.second += 1;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}

}  // namespace

namespace pidk {

KernelTimer::KernelTimer(const char* name, hipStream_t st, bool by_launch)
    : name_(name), st_(st), by_launch_(by_launch) {
  if (!g_on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_sel.empty() && g_sel.find(name) == g_sel.end()) return;
  if (g_every > 1 && g_seen[name]++ % g_every != 0) return;
  a_ = take_event();
  b_ = take_event();
  if (!a_ || !b_) {
    if (a_) g_pool.push_back(a_);
    if (b_) g_pool.push_back(b_);
    a_ = b_ = nullptr;
    return;
  }
  if (!by_launch_) hipEventRecord(a_, st_);
}

KernelTimer::~KernelTimer() {
  if (!a_ || !b_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!by_launch_) hipEventRecord(b_, st_);
  g_pending.push_back({name_, a_, b_});
}

}  // namespace pidk

extern "C" {

pid_status pid_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  g_tot.clear();
  g_seen.clear();
  // events are created here, not in the launches being timed
  while (on && g_pool.size() < kPoolEvents) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    g_pool.push_back(e);
  }
  g_on.store(on != 0);
  return PID_OK;
}

pid_status pid_timing_select(const char* names) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_sel.clear();
  if (!names) return PID_OK;
  std::string cur;
  for (const char* c = names;; ++c) {
    if (*c == ',' || *c == '\0') {
      if (!cur.empty()) g_sel.insert(cur);
      cur.clear();
      if (*c == '\0') break;
    } else if (*c != ' ') {
      cur.push_back(*c);
    }
  }
  return PID_OK;
}

pid_status pid_timing_sample(int every) {
  if (every < 1 || every > (1 << 20)) return PID_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  g_every = every;
  g_seen.clear();
  return PID_OK;
}

pid_status pid_timing_get(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return PID_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  auto it = g_tot.find(kernel);
  *total_ms = it == g_tot.end() ? 0.0 : it->second.first;
  *launches = it == g_tot.end() ? 0 : it->second.second;
  return PID_OK;
}

}  // extern "C"
