// Host-only test of the serving admission policy (sched.h) with a simulated
// executor: requests of random size and duration arrive over simulated time,
// the policy admits them, and "kernels" finish after their duration.  Checks
// the arena (in bounds, disjoint, merged back), the slot and footprint limits,
// waiting for memory, the starvation rule and cancellation.  Built with g++
// under AddressSanitizer and UndefinedBehaviorSanitizer by the test suite.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2512_15187_amd/csrc/sched.h"

using pidsched::Admission;
using pidsched::Arena;
using pidsched::Pending;
using pidsched::Policy;

static int g_fail = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                          \
    }                                                                    \
  } while (0)

static void arena_basics() {
  Arena a(4096);
  size_t o1 = 0, o2 = 0, o3 = 0, o4 = 0;
  CHECK(a.alloc(1000, &o1) && o1 == 0);          // rounds to 1024
  CHECK(a.alloc(1, &o2) && o2 == 1024);          // rounds to 256
  CHECK(a.alloc(2048, &o3) && o3 == 1280);
  CHECK(!a.alloc(1024, &o4));                    // 768 bytes left
  CHECK(a.free_bytes() == 768);
  a.release(o2, 1);
  CHECK(a.free_blocks() == 2);
  CHECK(!a.alloc(1024, &o4));                    // 256 + 768, not contiguous
  a.release(o1, 1000);                           // merges with the freed 256
  CHECK(a.free_blocks() == 2 && a.largest_free() == 1280);
  CHECK(a.alloc(1280, &o4) && o4 == 0);
  a.release(o4, 1280);
  a.release(o3, 2048);                           // everything merges back
  CHECK(a.free_blocks() == 1 && a.free_bytes() == 4096);
  size_t z = 0;
  CHECK(a.alloc(0, &z));                         // an empty request still takes one unit
  a.release(z, 0);
  CHECK(a.free_bytes() == 4096);
}

// A request that fits the arena alone but not next to the running one waits
// for memory although a slot is free, and starts when the memory is released.
static void waits_for_memory() {
  Policy p(100 * 1024, 4, 0.05);
  p.enqueue({1, 60 * 1024, 60 * 1024, 0.0});
  p.enqueue({2, 60 * 1024, 60 * 1024, 0.001});
  auto a = p.admit(0.002);
  CHECK(a.size() == 1 && a[0].ticket == 1);
  CHECK(p.busy_slots() == 1 && p.queued() == 1);
  CHECK(p.admit(0.003).empty());                 // slot free, memory not
  p.complete(a[0].slot);
  auto b = p.admit(0.004);
  CHECK(b.size() == 1 && b[0].ticket == 2 && b[0].ws_off == 0);
}

// Later requests pass a head that does not fit until the head has waited
// longer than the starvation limit; then nothing passes it.
static void bypass_until_starving() {
  Policy p(100 * 1024, 4, 0.05);
  p.enqueue({1, 70 * 1024, 0, 0.0});
  auto a = p.admit(0.0);
  CHECK(a.size() == 1);
  p.enqueue({2, 50 * 1024, 0, 0.010});           // head: does not fit beside 1
  p.enqueue({3, 10 * 1024, 0, 0.011});           // small: passes 2
  auto b = p.admit(0.012);
  CHECK(b.size() == 1 && b[0].ticket == 3);
  p.enqueue({4, 10 * 1024, 0, 0.070});
  auto c = p.admit(0.071);                       // head 2 waited 61 ms: 4 must wait
  CHECK(c.empty());
  p.complete(b[0].slot);
  CHECK(p.admit(0.072).empty());                 // 2 still does not fit (70 + 50 > 100)
  p.complete(a[0].slot);
  auto d = p.admit(0.073);                       // now 2 first, then 4
  CHECK(d.size() == 2 && d[0].ticket == 2 && d[1].ticket == 4);
}

static void slots_budget_cancel() {
  Policy p(1 << 20, 2, 0.05);
  p.set_budget(3000);
  CHECK(p.too_large(2 << 20, 0));
  CHECK(p.too_large(10, 3001));
  CHECK(!p.too_large(10, 3000));
  for (uint64_t t = 1; t <= 4; ++t) p.enqueue({t, 256, 1000, 0.0});
  auto a = p.admit(0.0);
  CHECK(a.size() == 2 && p.footprint_in_use() == 2000);   // two slots
  p.set_budget(2500);
  p.complete(a[0].slot);
  auto b = p.admit(0.001);
  CHECK(b.size() == 1 && p.footprint_in_use() == 2000);   // slot free, budget allows one more
  auto c = p.admit(0.002);
  CHECK(c.empty());                                        // 2000 + 1000 > 2500
  auto t = p.cancel_queued();
  CHECK(t.size() == 1 && t[0] == 4 && p.queued() == 0);
}

// Random arrivals, sizes and durations against a simulated executor.
static void simulated_executor(uint32_t seed) {
  std::mt19937_64 rng(seed);
  const size_t arena = 1 << 24;
  const int slots = 1 + (int)(rng() % 6);
  const double starve = 0.05;
  Policy p(arena, slots, starve);
  const size_t budget = (rng() % 2) ? (size_t)(arena * 1.5) : 0;
  p.set_budget(budget);
  struct Req { double arrive, dur; size_t ws, fp; double t_admit = -1, t_done = -1; int slot = -1; size_t off = 0; };
  std::vector<Req> reqs;
  double t = 0;
  for (int k = 0; k < 3000; ++k) {
    t += std::exponential_distribution<double>(400.0)(rng);
    Req r;
    r.arrive = t;
    r.dur = std::uniform_real_distribution<double>(0.0002, 0.02)(rng);
    r.ws = (size_t)(std::pow(2.0, std::uniform_real_distribution<double>(8, 23.5)(rng)));
    r.fp = r.ws + (size_t)(rng() % (1 << 22));
    if (p.too_large(r.ws, r.fp)) continue;
    reqs.push_back(r);
  }
  // event loop: arrivals, completions, admissions
  std::map<uint64_t, size_t> idx;
  size_t next = 0;
  double now = 0;
  std::multimap<double, int> finishing;   // time -> slot
  std::vector<uint64_t> on_slot(slots, 0);
  std::set<std::pair<size_t, size_t>> live;   // (offset, rounded bytes)
  while (next < reqs.size() || !finishing.empty() || p.queued()) {
    double t_arr = next < reqs.size() ? reqs[next].arrive : 1e300;
    double t_fin = finishing.empty() ? 1e300 : finishing.begin()->first;
    // also wake up when the head would start starving
    now = std::min(t_arr, t_fin);
    if (now >= 1e299) now += 0.001;   // only queued work: advance the clock
    if (t_fin <= t_arr && !finishing.empty()) {
      const int s = finishing.begin()->second;
      finishing.erase(finishing.begin());
      Req& r = reqs[idx[on_slot[s]]];
      r.t_done = now;
      live.erase({r.off, Arena::round(r.ws) ? Arena::round(r.ws) : 256});
      p.complete(s);
      on_slot[s] = 0;
    } else if (next < reqs.size()) {
      idx[next + 1] = next;
      p.enqueue({next + 1, reqs[next].ws, reqs[next].fp, reqs[next].arrive});
      ++next;
    }
    for (const Admission& a : p.admit(now)) {
      Req& r = reqs[idx[a.ticket]];
      CHECK(r.t_admit < 0);
      r.t_admit = now;
      r.slot = a.slot;
      r.off = a.ws_off;
      const size_t rb = Arena::round(r.ws) ? Arena::round(r.ws) : 256;
      CHECK(a.ws_off + rb <= arena);
      for (const auto& l : live) CHECK(a.ws_off + rb <= l.first || l.first + l.second <= a.ws_off);
      live.insert({a.ws_off, rb});
      CHECK(on_slot[a.slot] == 0);
      on_slot[a.slot] = a.ticket;
      finishing.emplace(now + r.dur, a.slot);
    }
    CHECK(p.busy_slots() <= slots);
    CHECK(!budget || p.footprint_in_use() <= budget);
  }
  CHECK(p.arena().free_bytes() == arena && p.arena().free_blocks() == 1);
  CHECK(p.footprint_in_use() == 0 && p.busy_slots() == 0);
  for (const Req& r : reqs) CHECK(r.t_admit >= r.arrive && r.t_done >= r.t_admit);
  // starvation rule: no request that arrived after a starving head started
  // before it
  for (size_t i = 0; i < reqs.size(); ++i)
    for (size_t j = i + 1; j < reqs.size() && j < i + 64; ++j)
      if (reqs[j].t_admit < reqs[i].t_admit && reqs[j].t_admit > reqs[i].arrive + starve + 1e-12) {
        // j started before i although i had been waiting longer than the
        // limit; allowed only if i was not the head (an earlier request still
        // queued at that time)
        bool earlier_queued = false;
        for (size_t k = 0; k < i; ++k)
          if (reqs[k].t_admit > reqs[j].t_admit - 1e-15 && reqs[k].arrive <= reqs[j].t_admit) earlier_queued = true;
        CHECK(earlier_queued);
      }
}

int main() {
  arena_basics();
  waits_for_memory();
  bypass_until_starving();
  slots_budget_cancel();
  for (uint32_t s = 1; s <= 12; ++s) simulated_executor(s);
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("sched policy: all checks passed\n");
  return 0;
}
