// Admission policy of the serving loop (continuous batching): which queued
// request starts next, on which execution slot and at which offset of the
// device arena.  Plain C++ with no device calls, so that the policy can be
// driven by the server (under its lock, with HIP streams executing the
// admitted requests) and by host-only tests with a simulated executor.
//
//   * Arena: first-fit over [0, size) with 256-byte granularity; a freed
//     block merges with its free neighbours.
//   * A request is admitted when an execution slot is free, its workspace
//     fits in the arena, and its footprint (masks, weights, outputs and
//     workspace) keeps the admitted total within the footprint budget
//     (0 = no budget).
//   * Requests are considered in arrival order.  One that does not fit yet
//     is passed over, so that smaller requests behind it can start, until
//     the head of the queue has waited longer than the starvation limit;
//     from then on nothing is admitted ahead of the head.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace pidsched {

class Arena {
 public:
  explicit Arena(size_t size = 0) : size_(size) {
    if (size) free_[0] = size;
  }
  static size_t round(size_t bytes) { return (bytes + 255) & ~size_t(255); }
  size_t size() const { return size_; }

  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    if (bytes == 0) bytes = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }

  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    if (bytes == 0) bytes = 256;
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

  size_t free_bytes() const {
    size_t t = 0;
    for (const auto& kv : free_) t += kv.second;
    return t;
  }
  size_t largest_free() const {
    size_t t = 0;
    for (const auto& kv : free_) t = kv.second > t ? kv.second : t;
    return t;
  }
  size_t free_blocks() const { return free_.size(); }

 private:
  size_t size_;
  std::map<size_t, size_t> free_;   // offset -> bytes, disjoint and not adjacent
};

struct Pending {
  uint64_t ticket = 0;
  size_t ws_bytes = 0;     // workspace carved from the arena
  size_t footprint = 0;    // bytes counted against the footprint budget
  double t_submit = 0.0;   // seconds on the caller's clock
};

struct Admission {
  uint64_t ticket;
  int slot;
  size_t ws_off;
};

class Policy {
 public:
  Policy(size_t arena_bytes, int slots, double starve_s)
      : arena_(arena_bytes), starve_s_(starve_s), slot_(slots) {}

  void set_budget(size_t footprint_bytes) { budget_ = footprint_bytes; }
  size_t budget() const { return budget_; }
  size_t arena_bytes() const { return arena_.size(); }

  // A request that could never be admitted, even alone.
  bool too_large(size_t ws_bytes, size_t footprint) const {
    return Arena::round(ws_bytes) > arena_.size() || (budget_ && footprint > budget_);
  }

  void enqueue(const Pending& p) { queue_.push_back(p); }

  // Admissions possible at time `now`, in the order they are made.
  std::vector<Admission> admit(double now) {
    std::vector<Admission> out;
    const bool head_starving = !queue_.empty() && (now - queue_.front().t_submit) > starve_s_;
    for (auto it = queue_.begin(); it != queue_.end();) {
      int slot = -1;
      for (size_t s = 0; s < slot_.size(); ++s)
        if (!slot_[s].busy) { slot = (int)s; break; }
      if (slot < 0) break;
      size_t off = 0;
      const bool fits_budget = !budget_ || in_use_ + it->footprint <= budget_;
      if (!fits_budget || !arena_.alloc(it->ws_bytes, &off)) {
        if (it == queue_.begin() && head_starving) break;
        ++it;
        continue;
      }
      Slot& sl = slot_[slot];
      sl.busy = true;
      sl.ticket = it->ticket;
      sl.ws_off = off;
      sl.ws_bytes = it->ws_bytes;
      sl.footprint = it->footprint;
      in_use_ += it->footprint;
      out.push_back({it->ticket, slot, off});
      it = queue_.erase(it);
    }
    return out;
  }

  // The request on `slot` has finished (or failed): its slot, workspace and
  // footprint are free again.  The caller must have made sure that nothing
  // on the device still uses the workspace.
  void complete(int slot) {
    Slot& sl = slot_[(size_t)slot];
    if (!sl.busy) return;
    arena_.release(sl.ws_off, sl.ws_bytes);
    in_use_ -= sl.footprint;
    sl = Slot{};
  }

  // Drop every queued request (server stopping); returns their tickets.
  std::vector<uint64_t> cancel_queued() {
    std::vector<uint64_t> t;
    for (const auto& p : queue_) t.push_back(p.ticket);
    queue_.clear();
    return t;
  }

  size_t queued() const { return queue_.size(); }
  int busy_slots() const {
    int b = 0;
    for (const auto& s : slot_) b += s.busy ? 1 : 0;
    return b;
  }
  bool slot_busy(int s) const { return slot_[(size_t)s].busy; }
  uint64_t slot_ticket(int s) const { return slot_[(size_t)s].ticket; }
  size_t footprint_in_use() const { return in_use_; }
  const Arena& arena() const { return arena_; }

 private:
  struct Slot {
    bool busy = false;
    uint64_t ticket = 0;
    size_t ws_off = 0, ws_bytes = 0, footprint = 0;
  };
  Arena arena_;
  double starve_s_;
  size_t budget_ = 0;
  size_t in_use_ = 0;
  std::vector<Slot> slot_;
  std::deque<Pending> queue_;
};

}  // namespace pidsched
