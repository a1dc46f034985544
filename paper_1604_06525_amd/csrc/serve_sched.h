// The batching server's scheduling, without the device: arena ranges, the
// request life cycle and the start policy.  opt_server.hip drives it with real
// launches; a CPU test drives it with a fake executor.
//
// Life cycle of a slot:
//   EMPTY --submit--> NEW --start (admission order, fill budget)--> RUN
//   RUN --its last outer iteration (or an LM stop, seen in a completed step)
//       is enqueued with its final cost--> DRAIN
//   NEW/RUN --cancel--> DRAIN (or EMPTY at once when no enqueued step uses it)
//   DRAIN --the last step that used it has completed--> EMPTY (range freed)
// A step enqueues one outer iteration for every runnable slot (RUN, not
// cancelled, iterations left, no LM stop) and the final cost of every RUN slot
// whose iterations are then all enqueued or whose LM solve has stopped.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <vector>

namespace optmi {
namespace sched {

// Arena byte ranges, first fit with coalescing.
class RangeAlloc {
 public:
  void reset(size_t off, size_t bytes) {
    free_.clear();
    if (bytes) free_[off] = bytes;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
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
    for (auto& kv : free_) t += kv.second;
    return t;
  }
  // the free ranges, in address order (for checks)
  const std::map<size_t, size_t>& ranges() const { return free_; }

 private:
  std::map<size_t, size_t> free_;
};

enum class SlotState { EMPTY, NEW, RUN, DRAIN };

// What scheduling reads and writes of a request.
struct SlotCore {
  SlotState state = SlotState::EMPTY;
  int64_t ticket = -1;
  size_t ws_off = 0, ws_bytes = 0;
  int outer = 0;          // outer iterations asked for
  bool lm = false;        // Levenberg-Marquardt (its stop is read back per step)
  int it = 0;             // outer iterations enqueued
  bool lm_done = false;   // LM radius fell below its minimum (seen in a completed step)
  bool cancelled = false;
  bool graph_pending = false;  // incidence lists not built yet: may not start
  double fill = 1.0;      // estimated share of the GPU one of its launches occupies
  int64_t last_step = -1; // last step that enqueued work for it
};

inline bool runnable(const SlotCore& s) {
  return s.state == SlotState::RUN && !s.cancelled && s.it < s.outer && !s.lm_done;
}

// Start NEW requests in admission (ticket) order while the running set's fill
// stays within the budget; at least one request runs.  A request whose graph
// lists are pending is passed over without holding up those behind it.
// Returns the slots started.
template <class S>
std::vector<int> start_requests(std::vector<S>& slots, double budget) {
  double running = 0.0;
  for (const S& s : slots)
    if (runnable(s)) running += s.fill;
  std::vector<int> order;
  for (int i = 0; i < (int)slots.size(); ++i)
    if (slots[(size_t)i].state == SlotState::NEW) order.push_back(i);
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return slots[(size_t)a].ticket < slots[(size_t)b].ticket; });
  std::vector<int> fresh;
  for (int i : order) {
    S& s = slots[(size_t)i];
    if (s.graph_pending) continue;
    if (running > 0.0 && running + s.fill > budget) break;
    s.state = SlotState::RUN;
    running += s.fill;
    fresh.push_back(i);
  }
  return fresh;
}

// The work of one step: run (one outer iteration), lm (their LM scalars read
// back), fin (final cost; the slot retires with this step).
struct StepPlan {
  std::vector<int> run, lm, fin;
  bool empty() const { return run.empty() && fin.empty(); }
};

template <class S>
StepPlan plan_step(const std::vector<S>& slots) {
  StepPlan p;
  for (int i = 0; i < (int)slots.size(); ++i) {
    const S& s = slots[(size_t)i];
    if (!runnable(s)) continue;
    p.run.push_back(i);
    if (s.lm) p.lm.push_back(i);
  }
  for (int i = 0; i < (int)slots.size(); ++i) {
    const S& s = slots[(size_t)i];
    if (s.state != SlotState::RUN || s.cancelled) continue;
    const int after = s.it + (runnable(s) ? 1 : 0);
    if (after >= s.outer || s.lm_done) p.fin.push_back(i);
  }
  return p;
}

// After the step's work is enqueued as step `idx`.
template <class S>
void commit_step(std::vector<S>& slots, const std::vector<int>& fresh, const StepPlan& p, int64_t idx) {
  for (int i : p.run) slots[(size_t)i].it += 1;
  for (int i : fresh) slots[(size_t)i].last_step = idx;
  for (int i : p.run) slots[(size_t)i].last_step = idx;
  for (int i : p.fin) {
    S& s = slots[(size_t)i];
    s.last_step = idx;
    s.state = SlotState::DRAIN;
  }
}

// When step n_done - 1 has completed: the LM stops it read back (stopped(i)
// for each slot of gathered), then every DRAIN slot that no pending step uses is
// released (release(slot index)).
template <class S, class Stopped, class Release>
void complete_step(std::vector<S>& slots, const std::vector<int>& gathered, int64_t n_done, Stopped stopped,
                   Release release) {
  for (int i : gathered) {
    S& s = slots[(size_t)i];
    if (s.state == SlotState::RUN && stopped(i)) s.lm_done = true;
  }
  for (int i = 0; i < (int)slots.size(); ++i)
    if (slots[(size_t)i].state == SlotState::DRAIN && slots[(size_t)i].last_step < n_done) release(i);
}

// Cancel the live request with this ticket: released at once (release(slot))
// if no step in flight uses it, else DRAIN.  False if there is none.
template <class S, class Release>
bool cancel(std::vector<S>& slots, int64_t ticket, int64_t n_done, Release release) {
  for (int i = 0; i < (int)slots.size(); ++i) {
    S& s = slots[(size_t)i];
    if (s.state == SlotState::EMPTY || s.ticket != ticket || s.cancelled) continue;
    s.cancelled = true;
    if (s.last_step < n_done) {
      release(i);
    } else {
      s.state = SlotState::DRAIN;
    }
    return true;
  }
  return false;
}

}  // namespace sched
}  // namespace optmi
