// Serving loop: continuous batching of PID requests of uneven ensemble and
// grid size on one GPU.
//
// A scheduler thread owns `max_slots` HIP streams (default priority) and a
// caller-provided device arena.  The admission policy (sched.h) decides under
// the server's lock which queued requests start, on which slot and where in
// the arena; the scheduler then releases the lock and launches them on their
// slot streams, so that requests admitted while others run overlap on the
// device and no client waits on a launch.  Each request is bracketed by a
// pair of timing events on its slot stream: the end event signals completion
// (polled every 20 us), and both give the request's start and end on the
// device, relative to a reference event recorded when the server was created.
// On completion the slot, the arena block and the footprint are released and
// the queue is scanned again.
//
// A request runs exactly the kernels and launch geometry of the stand-alone
// calls, which depend on its own shape only, so its results are bitwise the
// same alone or in any mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pid.h"
#include "sched.h"

namespace pidapi {
pid_status workspace_size(const pid_ensemble*, const pid_iso*, int, int, size_t*);
pid_status run(int, const pid_ensemble*, const pid_iso*, int, const pid_out*, void*, size_t, void*);
pid_status set_error(pid_status, const char*);
}  // namespace pidapi

namespace {

constexpr double kStarveS = 0.050;   // a passed-over head request blocks the queue after 50 ms
using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t ticket = 0;
  pid_request req{};
  size_t ws_bytes = 0;
  size_t footprint = 0;
  size_t ws_off = 0;
  int slot = -1;
  bool done = false;
  pid_status result = PID_OK;
  std::string err;            // error text of a failed request
  double t_submit = 0, t_start = 0, t_done = 0;
  double dev_start_ms = -1, dev_end_ms = -1;
};

int dtype_bytes(int dtype) {
  switch (dtype) {
    case PID_F64: return 8;
    case PID_F32: return 4;
    case PID_F16: case PID_BF16: return 2;
    default: return 1;
  }
}

// Device bytes a request touches besides its workspace: the stored ensemble
// (its rows up to the last valid point), the weights and every output asked for.
size_t request_bytes(const pid_request& r) {
  const pid_ensemble& e = r.ens;
  size_t b = e.dtype == PID_B1 ? (size_t)((e.n - 1) * e.ld + e.m + 7) / 8
                               : (size_t)((e.n - 1) * e.ld + e.m) * (size_t)dtype_bytes(e.dtype);
  if (e.weights) b += (size_t)e.m * 4;
  const size_t n = (size_t)e.n;
  if (r.out.inclusion && r.variant == 0) b += n * n * 8;
  for (const void* p : {(const void*)r.out.mass, (const void*)r.out.in_in, (const void*)r.out.in_out,
                        (const void*)r.out.depth})
    if (p) b += n * 8;
  if (r.out.rank) b += n * 4;
  if (r.out.order) b += n * 4;
  return b;
}

}  // namespace

struct pid_server {
  int device = 0;
  char* arena_base = nullptr;
  size_t arena_bytes = 0;
  pidsched::Policy policy{0, 0, kStarveS};
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> ev_start, ev_end;   // per slot, timing enabled
  hipEvent_t ev_ref = nullptr;                // device time origin
  std::vector<std::shared_ptr<Job>> running;  // per slot
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  Clock::time_point t0 = Clock::now();
  std::thread thread;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // (lock held)
  void finish(int slot, pid_status st, const std::string& err) {
    auto j = running[(size_t)slot];
    j->result = st;
    j->err = err;
    j->t_done = now();
    j->done = true;
    policy.complete(slot);
    running[(size_t)slot].reset();
  }

  // Launch one admitted request on its slot stream (lock not held).  On a
  // failure the slot stream is drained before the caller frees the
  // workspace, since some kernels of the request may already be queued.
  pid_status launch(const Job& j, int slot, std::string* err) {
    hipStream_t s = streams[(size_t)slot];
    if (j.req.ready) {
      hipError_t e = hipStreamWaitEvent(s, reinterpret_cast<hipEvent_t>(j.req.ready), 0);
      if (e != hipSuccess) {
        *err = std::string("hipStreamWaitEvent: ") + hipGetErrorString(e);
        return PID_ERR_DEVICE;
      }
    }
    hipError_t e = hipEventRecord(ev_start[(size_t)slot], s);
    if (e != hipSuccess) {
      *err = std::string("hipEventRecord: ") + hipGetErrorString(e);
      hipStreamSynchronize(s);
      return PID_ERR_DEVICE;
    }
    pid_status st = pidapi::run(j.req.variant, &j.req.ens, &j.req.iso, j.req.gemm, &j.req.out,
                                arena_base + j.ws_off, j.ws_bytes, s);
    if (st != PID_OK) {
      *err = pid_last_error();   // this thread's text of the failed call
      hipStreamSynchronize(s);
      return st;
    }
    e = hipEventRecord(ev_end[(size_t)slot], s);
    if (e != hipSuccess) {
      *err = std::string("hipEventRecord: ") + hipGetErrorString(e);
      hipStreamSynchronize(s);
      return PID_ERR_DEVICE;
    }
    return PID_OK;
  }

  void loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // completions
      bool any_running = false;
      for (size_t s = 0; s < running.size(); ++s) {
        if (!running[s]) continue;
        hipError_t q = hipEventQuery(ev_end[s]);
        if (q == hipSuccess) {
          float a = 0.f, b = 0.f;
          if (hipEventElapsedTime(&a, ev_ref, ev_start[s]) == hipSuccess &&
              hipEventElapsedTime(&b, ev_ref, ev_end[s]) == hipSuccess) {
            running[s]->dev_start_ms = a;
            running[s]->dev_end_ms = b;
          }
          finish((int)s, PID_OK, "");
        } else if (q != hipErrorNotReady) {
          hipStreamSynchronize(streams[s]);
          finish((int)s, PID_ERR_DEVICE, std::string("request failed on the device: ") + hipGetErrorString(q));
        } else {
          any_running = true;
        }
      }
      if (stop) {
        for (uint64_t t : policy.cancel_queued()) {
          auto it = jobs.find(t);
          if (it == jobs.end()) continue;
          it->second->result = PID_ERR_CANCELLED;
          it->second->err = "the server stopped before the request started";
          it->second->done = true;
        }
      }
      cv_done.notify_all();
      if (stop && !any_running) break;
      // admissions: decided under the lock, launched outside it
      std::vector<pidsched::Admission> adm = stop ? std::vector<pidsched::Admission>{} : policy.admit(now());
      std::vector<std::shared_ptr<Job>> started;
      for (const auto& a : adm) {
        auto j = jobs[a.ticket];
        j->slot = a.slot;
        j->ws_off = a.ws_off;
        j->t_start = now();
        running[(size_t)a.slot] = j;
        started.push_back(j);
      }
      if (!started.empty()) {
        std::vector<std::pair<pid_status, std::string>> res(started.size());
        lk.unlock();
        for (size_t k = 0; k < started.size(); ++k)
          res[k].first = launch(*started[k], started[k]->slot, &res[k].second);
        lk.lock();
        for (size_t k = 0; k < started.size(); ++k) {
          if (res[k].first != PID_OK) finish(started[k]->slot, res[k].first, res[k].second);
          else any_running = true;
        }
        cv_done.notify_all();
      }
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

namespace {

pid_status find_job(pid_server* s, uint64_t ticket, std::shared_ptr<Job>* j) {
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return pidapi::set_error(PID_ERR_INVALID_ARG, "unknown ticket");
  *j = it->second;
  return PID_OK;
}

// The calling thread's last error becomes the request's error text.
void report(const Job& j) {
  if (j.done && j.result != PID_OK) pidapi::set_error(j.result, j.err.c_str());
}

}  // namespace

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
  s->policy = pidsched::Policy(arena_bytes, max_slots, kStarveS);
  s->streams.assign((size_t)max_slots, nullptr);
  s->ev_start.assign((size_t)max_slots, nullptr);
  s->ev_end.assign((size_t)max_slots, nullptr);
  s->running.resize((size_t)max_slots);
  auto cleanup = [s] {
    for (size_t i = 0; i < s->streams.size(); ++i) {
      if (s->streams[i]) hipStreamDestroy(s->streams[i]);
      if (s->ev_start[i]) hipEventDestroy(s->ev_start[i]);
      if (s->ev_end[i]) hipEventDestroy(s->ev_end[i]);
    }
    if (s->ev_ref) hipEventDestroy(s->ev_ref);
    delete s;
  };
  for (int i = 0; i < max_slots; ++i) {
    if (hipStreamCreateWithFlags(&s->streams[(size_t)i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev_start[(size_t)i]) != hipSuccess || hipEventCreate(&s->ev_end[(size_t)i]) != hipSuccess) {
      cleanup();
      return pidapi::set_error(PID_ERR_DEVICE, "stream/event creation failed");
    }
  }
  if (hipEventCreate(&s->ev_ref) != hipSuccess || hipEventRecord(s->ev_ref, s->streams[0]) != hipSuccess ||
      hipEventSynchronize(s->ev_ref) != hipSuccess) {
    cleanup();
    return pidapi::set_error(PID_ERR_DEVICE, "reference event failed");
  }
  s->t0 = Clock::now();
  s->thread = std::thread([s] { s->loop(); });
  *server = s;
  return PID_OK;
}

pid_status pid_server_set_budget(pid_server* s, size_t footprint_bytes) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->policy.set_budget(footprint_bytes);
  s->cv_sched.notify_one();
  return PID_OK;
}

pid_status pid_server_clock(pid_server* s, double* now_s) {
  if (!s || !now_s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL argument");
  *now_s = s->now();
  return PID_OK;
}

pid_status pid_submit(pid_server* s, const pid_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL argument");
  const double t = s->now();   // the request's submission, before any wait for the lock
  if (req->variant != 0 && req->variant != 1 && req->variant != 3)
    return pidapi::set_error(PID_ERR_INVALID_ARG, "variant must be 0 (all-pairs), 1 (PID-mean) or 3 (all-pairs depths)");
  size_t need = 0;
  pid_status st = pidapi::workspace_size(&req->ens, &req->iso, req->variant, req->gemm, &need);
  if (st != PID_OK) return st;
  auto j = std::make_shared<Job>();
  j->req = *req;
  j->ws_bytes = need;
  j->footprint = need + request_bytes(*req);
  j->t_submit = t;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return pidapi::set_error(PID_ERR_CANCELLED, "server is stopping");
  if (s->policy.too_large(j->ws_bytes, j->footprint))
    return pidapi::set_error(PID_ERR_OVER_BUDGET, "request exceeds the arena or the footprint budget");
  j->ticket = s->next_ticket++;
  s->jobs[j->ticket] = j;
  s->policy.enqueue({j->ticket, j->ws_bytes, j->footprint, j->t_submit});
  *ticket = j->ticket;
  s->cv_sched.notify_one();
  return PID_OK;
}

pid_status pid_poll(pid_server* s, uint64_t ticket, int* done, pid_status* result) {
  if (!s || !done) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::shared_ptr<Job> j;
  if (pid_status st = find_job(s, ticket, &j)) return st;
  *done = j->done ? 1 : 0;
  if (result) *result = j->done ? j->result : PID_OK;
  report(*j);
  return PID_OK;
}

pid_status pid_wait(pid_server* s, uint64_t ticket, pid_status* result) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  std::shared_ptr<Job> j;
  if (pid_status st = find_job(s, ticket, &j)) return st;
  s->cv_done.wait(lk, [&] { return j->done; });
  if (result) *result = j->result;
  report(*j);
  return PID_OK;
}

pid_status pid_request_times(pid_server* s, uint64_t ticket, double* t_submit, double* t_start,
                             double* t_done) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  std::shared_ptr<Job> j;
  if (pid_status st = find_job(s, ticket, &j)) return st;
  if (t_submit) *t_submit = j->t_submit;
  if (t_start) *t_start = j->t_start;
  if (t_done) *t_done = j->t_done;
  return PID_OK;
}

pid_status pid_request_device_times(pid_server* s, uint64_t ticket, double* start_ms, double* end_ms) {
  if (!s || !start_ms || !end_ms) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::shared_ptr<Job> j;
  if (pid_status st = find_job(s, ticket, &j)) return st;
  if (!j->done || j->result != PID_OK || j->dev_start_ms < 0)
    return pidapi::set_error(PID_ERR_INVALID_ARG, "the request has not completed successfully");
  *start_ms = j->dev_start_ms;
  *end_ms = j->dev_end_ms;
  return PID_OK;
}

pid_status pid_release(pid_server* s, uint64_t ticket) {
  if (!s) return pidapi::set_error(PID_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return pidapi::set_error(PID_ERR_INVALID_ARG, "unknown ticket");
  if (!it->second->done) return pidapi::set_error(PID_ERR_INVALID_ARG, "the request has not finished");
  s->jobs.erase(it);
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
    if (s->ev_start[i]) hipEventDestroy(s->ev_start[i]);
    if (s->ev_end[i]) hipEventDestroy(s->ev_end[i]);
  }
  if (s->ev_ref) hipEventDestroy(s->ev_ref);
  delete s;
  return PID_OK;
}

}  // extern "C"
