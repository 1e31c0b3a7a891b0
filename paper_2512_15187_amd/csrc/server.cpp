// Serving loop: continuous batching of PID requests of uneven ensemble and
// grid size on one GPU.
//
// A scheduler thread owns `max_slots` HIP streams (default priority) and a
// caller-provided device arena.  Requests wait in an admission queue until
//   (a) their workspace fits in the arena (first-fit over a free list), and
//   (b) an execution slot is free;
// they are then launched on the slot's stream, so requests admitted while
// others run overlap on the device.  Completion is detected with one HIP
// event per slot; the slot and the arena block are released at once and the
// queue is scanned again.  Admission scans the queue in arrival order and
// lets later requests pass a head request that does not fit, until the head
// has waited `kStarveMs`; from then on nothing is admitted ahead of it.
//
// A request runs exactly the kernels and launch geometry of the stand-alone
// calls, which depend on its own shape only, so its results are bitwise the
// same alone or in any mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/pid.h"

namespace pidapi {
pid_status workspace_size(const pid_ensemble*, const pid_iso*, int, int, size_t*);
pid_status run(int, const pid_ensemble*, const pid_iso*, int, const pid_out*, void*, size_t, void*);
pid_status set_error(pid_status, const char*);
}  // namespace pidapi

namespace {

constexpr double kStarveMs = 50.0;
using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t ticket = 0;
  pid_request req{};
  size_t ws_bytes = 0;
  size_t ws_off = 0;
  int slot = -1;
  bool done = false;
  pid_status result = PID_OK;
  double t_submit = 0, t_start = 0, t_done = 0;
};

// First-fit allocator over [0, size) with 256-byte granularity.
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes;
        size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace

struct pid_server {
  int device = 0;
  char* arena_base = nullptr;
  size_t arena_bytes = 0;
  Arena arena{0};
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<std::shared_ptr<Job>> running;   // per slot
  std::deque<std::shared_ptr<Job>> queue;
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  Clock::time_point t0 = Clock::now();
  std::thread thread;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  void finish(int slot, pid_status st) {
    auto j = running[slot];
    j->result = st;
    j->t_done = now();
    j->done = true;
    arena.release(j->ws_off, j->ws_bytes);
    running[slot].reset();
  }

  void loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // completions
      bool any_running = false;
      for (size_t s = 0; s < running.size(); ++s) {
        if (!running[s]) continue;
        hipError_t q = hipEventQuery(events[s]);
        if (q == hipSuccess) {
          finish((int)s, PID_OK);
        } else if (q != hipErrorNotReady) {
          pidapi::set_error(PID_ERR_DEVICE, hipGetErrorString(q));
          finish((int)s, PID_ERR_DEVICE);
        } else {
          any_running = true;
        }
      }
      cv_done.notify_all();
      if (stop) {
        for (auto& j : queue) {
          j->result = PID_ERR_CANCELLED;
          j->done = true;
        }
        queue.clear();
        cv_done.notify_all();
        if (!any_running) break;
      }
      // admission in arrival order, with bypass until the head starves
      const double tnow = now();
      bool head_starving = !queue.empty() && (tnow - queue.front()->t_submit) * 1e3 > kStarveMs;
      for (auto it = queue.begin(); it != queue.end();) {
        int slot = -1;
        for (size_t s = 0; s < running.size(); ++s)
          if (!running[s]) { slot = (int)s; break; }
        if (slot < 0) break;
        auto j = *it;
        size_t off = 0;
        if (!arena.alloc(j->ws_bytes, &off)) {
          if (it == queue.begin() && head_starving) break;
          ++it;
          continue;
        }
        j->ws_off = off;
        j->slot = slot;
        j->t_start = now();
        // inputs still being produced on the caller's stream
        if (j->req.ready) hipStreamWaitEvent(streams[slot], reinterpret_cast<hipEvent_t>(j->req.ready), 0);
        pid_status st = pidapi::run(j->req.variant, &j->req.ens, &j->req.iso, j->req.gemm, &j->req.out,
                                    arena_base + off, j->ws_bytes, streams[slot]);
        running[slot] = j;
        if (st != PID_OK) {
          finish(slot, st);
        } else if (hipEventRecord(events[slot], streams[slot]) != hipSuccess) {
          hipStreamSynchronize(streams[slot]);
          finish(slot, PID_ERR_DEVICE);
        }
        it = queue.erase(it);
        any_running = true;
      }
      if (stop && !any_running && queue.empty()) break;
      if (any_running) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        cv_sched.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
    cv_done.notify_all();
  }
};

extern "C" {

pid_status pid_server_create(int device, void* arena, size_t arena_bytes, int max_slots,
                             pid_server** server) {
  if (!server) return pidapi::set_error(PID_ERR_INVALID_ARG, "server is NULL");
  if (!arena || arena_bytes < 4096) return pidapi::set_error(PID_ERR_INVALID_ARG, "arena missing or too small");
  if (max_slots < 1 || max_slots > 64) return pidapi::set_error(PID_ERR_INVALID_ARG, "max_slots must be 1..64");
  if (hipSetDevice(device) != hipSuccess) return pidapi::set_error(PID_ERR_DEVICE, "hipSetDevice failed");
  auto* s = new pid_server();
  s->device = device;
  s->arena_base = static_cast<char*>(arena);
  s->arena_bytes = arena_bytes;
  s->arena = Arena(arena_bytes);
  s->streams.resize(max_slots);
  s->events.resize(max_slots);
  s->running.resize(max_slots);
  for (int i = 0; i < max_slots; ++i) {
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) != hipSuccess) {
      delete s;
      return pidapi::set_error(PID_ERR_DEVICE, "stream/event creation failed");
    }
  }
  s->thread = std::thread([s] { s->loop(); });
  *server = s;
  return PID_OK;
}

pid_status pid_submit(pid_server* s, const pid_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL argument");
  if (req->variant != 0 && req->variant != 1) return pidapi::set_error(PID_ERR_INVALID_ARG, "variant must be 0 or 1");
  size_t need = 0;
  pid_status st = pidapi::workspace_size(&req->ens, &req->iso, req->variant, req->gemm, &need);
  if (st != PID_OK) return st;
  if (need > s->arena_bytes) return pidapi::set_error(PID_ERR_OVER_BUDGET, "request workspace exceeds the arena");
  auto j = std::make_shared<Job>();
  j->req = *req;
  j->ws_bytes = need;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return pidapi::set_error(PID_ERR_CANCELLED, "server is stopping");
  j->ticket = s->next_ticket++;
  j->t_submit = s->now();
  s->jobs[j->ticket] = j;
  s->queue.push_back(j);
  *ticket = j->ticket;
  s->cv_sched.notify_one();
  return PID_OK;
}

pid_status pid_poll(pid_server* s, uint64_t ticket, int* done, pid_status* result) {
  if (!s || !done) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return pidapi::set_error(PID_ERR_INVALID_ARG, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  if (result) *result = it->second->done ? it->second->result : PID_OK;
  return PID_OK;
}

pid_status pid_wait(pid_server* s, uint64_t ticket, pid_status* result) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return pidapi::set_error(PID_ERR_INVALID_ARG, "unknown ticket");
  auto j = it->second;
  s->cv_done.wait(lk, [&] { return j->done; });
  if (result) *result = j->result;
  return PID_OK;
}

pid_status pid_request_times(pid_server* s, uint64_t ticket, double* t_submit, double* t_start,
                             double* t_done) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return pidapi::set_error(PID_ERR_INVALID_ARG, "unknown ticket");
  if (t_submit) *t_submit = it->second->t_submit;
  if (t_start) *t_start = it->second->t_start;
  if (t_done) *t_done = it->second->t_done;
  return PID_OK;
}

pid_status pid_server_destroy(pid_server* s) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  if (s->thread.joinable()) s->thread.join();
  for (size_t i = 0; i < s->streams.size(); ++i) {
    if (s->streams[i]) { hipStreamSynchronize(s->streams[i]); hipStreamDestroy(s->streams[i]); }
    if (s->events[i]) hipEventDestroy(s->events[i]);
  }
  delete s;
  return PID_OK;
}

}  // extern "C"
