// CPU harness for the batching server's scheduling (serve_sched.h), driven by a
// fake executor instead of the device: requests are submitted, cancelled and
// stepped at random; steps "complete" in order after a random number of calls,
// up to three in flight as in the server; LM requests stop at random.  After
// every operation it checks the invariants the server relies on:
//  * arena: live ranges and free ranges tile the arena exactly (no overlap, no
//    leak), and free ranges are coalesced;
//  * start policy: requests start in ticket order (a graph request whose lists
//    are pending is skipped, never started); the running fill stays within the
//    budget unless a single request runs;
//  * life cycle: a request gets at most its outer iterations, each in a
//    distinct step; a slot is released only after the last step that used it
//    has completed; every request that is not cancelled retires exactly once,
//    with all its iterations or after an LM stop; after the stream ends every
//    slot is empty and the whole arena is free.
// Also checks RangeAlloc against a byte map.  Prints "ok" or the first failure.
//   usage: serve_sched_harness <seed> <operations>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "serve_sched.h"

using namespace optmi::sched;

#define CHECK(c, ...)                                 \
  do {                                                \
    if (!(c)) {                                       \
      std::printf("FAIL line %d: ", __LINE__);        \
      std::printf(__VA_ARGS__);                       \
      std::printf("\n");                              \
      std::exit(1);                                   \
    }                                                 \
  } while (0)

struct FSlot : SlotCore {
  int pending_steps = 0;  // steps until its graph lists are built
};

struct Step {
  int64_t idx;
  std::vector<int> gathered, retiring;
  int delay;  // calls until it completes
};

static void check_ranges(const RangeAlloc& ra, size_t arena, const std::vector<FSlot>& slots) {
  std::map<size_t, size_t> all = ra.ranges();
  for (auto it = all.begin(); it != all.end(); ++it) {
    auto nx = std::next(it);
    if (nx != all.end()) CHECK(it->first + it->second < nx->first, "free ranges not coalesced at %zu", it->first);
  }
  for (const FSlot& s : slots)
    if (s.state != SlotState::EMPTY) all.emplace(s.ws_off, s.ws_bytes);
  size_t pos = 0;
  for (auto& kv : all) {
    CHECK(kv.first == pos, "gap or overlap at %zu (range starts %zu)", pos, kv.first);
    pos += kv.second;
  }
  CHECK(pos == arena, "ranges cover %zu of %zu bytes", pos, arena);
}

static void range_alloc_model(std::mt19937_64& rng) {
  const size_t N = 4096;
  RangeAlloc ra;
  ra.reset(0, N);
  std::vector<int> owner(N, -1);
  std::map<int, std::pair<size_t, size_t>> live;
  int next = 0;
  for (int op = 0; op < 4000; ++op) {
    if (live.empty() || rng() % 3) {
      const size_t b = 1 + rng() % 300;
      size_t off = 0;
      const bool ok = ra.alloc(b, &off);
      // first fit: the lowest offset with b free bytes
      size_t want = N + 1;
      for (size_t s = 0, run = 0; s < N; ++s) {
        run = owner[s] < 0 ? run + 1 : 0;
        if (run == b) {
          want = s + 1 - b;
          break;
        }
      }
      CHECK(ok == (want <= N), "alloc(%zu) ok=%d, model %zu", b, (int)ok, want);
      if (!ok) continue;
      CHECK(off == want, "alloc(%zu) at %zu, first fit is %zu", b, off, want);
      for (size_t s = off; s < off + b; ++s) owner[s] = next;
      live[next++] = {off, b};
    } else {
      auto it = live.begin();
      std::advance(it, rng() % live.size());
      ra.release(it->second.first, it->second.second);
      for (size_t s = it->second.first; s < it->second.first + it->second.second; ++s) owner[s] = -1;
      live.erase(it);
    }
    size_t fr = 0;
    for (int o : owner) fr += o < 0;
    CHECK(fr == ra.free_bytes(), "free bytes %zu, model %zu", ra.free_bytes(), fr);
  }
}

int main(int argc, char** argv) {
  const uint64_t seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
  const int ops = argc > 2 ? std::atoi(argv[2]) : 20000;
  std::mt19937_64 rng(seed);
  range_alloc_model(rng);

  const int max_slots = 3 + (int)(rng() % 14);
  const size_t arena = 1 << 16;
  const double budget = 0.5 + (double)(rng() % 40) / 10.0;
  const int kDepth = 3;
  std::vector<FSlot> slots((size_t)max_slots);
  RangeAlloc ra;
  ra.reset(0, arena);
  std::deque<Step> inflight;
  int64_t n_steps = 0, n_done = 0, next_ticket = 1;
  std::map<int64_t, int> retired;       // ticket -> times retired
  std::set<int64_t> cancelled_t, submitted;
  std::map<int64_t, std::set<int64_t>> steps_of;  // ticket -> steps that ran an iteration of it
  std::map<int64_t, int> outer_of;
  std::map<int64_t, bool> stopped_of;   // LM stop decided by the fake device

  auto release = [&](int i) {
    FSlot& s = slots[(size_t)i];
    CHECK(s.last_step < n_done, "slot %d released while step %lld may still use it (done %lld)", i,
          (long long)s.last_step, (long long)n_done);
    ra.release(s.ws_off, s.ws_bytes);
    s = FSlot();
  };
  auto complete_one = [&]() {
    Step st = inflight.front();
    inflight.pop_front();
    CHECK(st.idx == n_done, "steps complete in order");
    for (int i : st.retiring) {
      const FSlot& s = slots[(size_t)i];
      if (s.cancelled) continue;
      retired[s.ticket]++;
      CHECK((int)steps_of[s.ticket].size() == s.outer || s.lm_done,
            "ticket %lld retired after %zu of %d iterations without an LM stop", (long long)s.ticket,
            steps_of[s.ticket].size(), s.outer);
    }
    n_done++;
    complete_step(slots, st.gathered, n_done, [&](int i) { return stopped_of[slots[(size_t)i].ticket]; }, release);
  };
  auto harvest = [&](bool block) {
    bool first = true;
    while (!inflight.empty()) {
      if (block && first) inflight.front().delay = 0;
      first = false;
      if (inflight.front().delay > 0) {
        inflight.front().delay--;
        break;
      }
      complete_one();
    }
  };
  auto step = [&]() {
    harvest(false);
    if (n_steps - n_done >= kDepth) harvest(true);
    for (FSlot& s : slots)
      if (s.state == SlotState::NEW && s.graph_pending && --s.pending_steps <= 0) s.graph_pending = false;
    // the start policy
    std::vector<FSlot> before = slots;
    const std::vector<int> fresh = start_requests(slots, budget);
    std::set<int> fs(fresh.begin(), fresh.end());
    int64_t max_started = -1;
    for (int i : fresh) {
      CHECK(before[(size_t)i].state == SlotState::NEW && !before[(size_t)i].graph_pending, "bad start");
      max_started = std::max(max_started, slots[(size_t)i].ticket);
    }
    for (int i = 0; i < max_slots; ++i)
      if (slots[(size_t)i].state == SlotState::NEW && !slots[(size_t)i].graph_pending)
        CHECK(slots[(size_t)i].ticket > max_started, "ticket %lld passed over by %lld",
              (long long)slots[(size_t)i].ticket, (long long)max_started);
    double running = 0.0;
    int nrun = 0;
    for (const FSlot& s : slots)
      if (runnable(s)) running += s.fill, nrun++;
    if (!fresh.empty()) CHECK(nrun == 1 || running <= budget + 1e-12, "fill %g over budget %g", running, budget);
    const StepPlan plan = plan_step(slots);
    if (fresh.empty() && plan.empty()) {
      if (!inflight.empty()) harvest(true);
      return;
    }
    for (int i : plan.run) {
      const FSlot& s = slots[(size_t)i];
      CHECK(s.it < s.outer && !s.cancelled && !s.lm_done, "runs a finished request");
      CHECK(steps_of[s.ticket].insert(n_steps).second, "two iterations in one step");
    }
    Step st;
    st.idx = n_steps;
    st.gathered = plan.lm;
    st.retiring = plan.fin;
    st.delay = (int)(rng() % 4);
    // the fake device: an LM request may stop in this step
    for (int i : plan.lm)
      if (rng() % 5 == 0) stopped_of[slots[(size_t)i].ticket] = true;
    commit_step(slots, fresh, plan, n_steps++);
    inflight.push_back(st);
  };
  auto submit = [&]() {
    int slot = -1;
    for (int k = 0; k < max_slots; ++k)
      if (slots[(size_t)k].state == SlotState::EMPTY) {
        slot = k;
        break;
      }
    if (slot < 0) return;
    const size_t need = 256 * (1 + rng() % 24);
    size_t off = 0;
    if (!ra.alloc(need, &off)) return;
    FSlot s;
    s.state = SlotState::NEW;
    s.ticket = next_ticket++;
    s.ws_off = off;
    s.ws_bytes = need;
    s.outer = (int)(rng() % 6);
    s.lm = rng() % 2;
    s.fill = 0.05 + (double)(rng() % 30) / 10.0;
    s.graph_pending = rng() % 4 == 0;
    s.pending_steps = 1 + (int)(rng() % 3);
    slots[(size_t)slot] = s;
    submitted.insert(s.ticket);
    outer_of[s.ticket] = s.outer;
  };
  auto cancel_one = [&]() {
    std::vector<int64_t> live;
    for (const FSlot& s : slots)
      if (s.state != SlotState::EMPTY && !s.cancelled) live.push_back(s.ticket);
    if (live.empty()) return;
    const int64_t t = live[rng() % live.size()];
    CHECK(cancel(slots, t, n_done, release), "cancel of a live ticket failed");
    cancelled_t.insert(t);
    CHECK(!cancel(slots, t, n_done, release), "second cancel of a ticket succeeded");
  };

  for (int op = 0; op < ops; ++op) {
    const unsigned r = rng() % 100;
    if (r < 45) {
      submit();
    } else if (r < 50) {
      cancel_one();
    } else {
      step();
    }
    check_ranges(ra, arena, slots);
  }
  // the stream ends: step until everything has retired
  for (int guard = 0; guard < 100000; ++guard) {
    bool busy = !inflight.empty();
    for (const FSlot& s : slots) busy = busy || s.state != SlotState::EMPTY;
    if (!busy) break;
    step();
    check_ranges(ra, arena, slots);
  }
  for (const FSlot& s : slots) CHECK(s.state == SlotState::EMPTY, "slot left in state %d", (int)s.state);
  CHECK(ra.free_bytes() == arena, "arena not all free at the end");
  for (int64_t t : submitted) {
    const int n = retired.count(t) ? retired[t] : 0;
    if (cancelled_t.count(t)) {
      CHECK(n <= 1, "cancelled ticket %lld retired %d times", (long long)t, n);
    } else {
      CHECK(n == 1, "ticket %lld retired %d times", (long long)t, n);
      CHECK((int)steps_of[t].size() == outer_of[t] || stopped_of[t], "ticket %lld ran %zu of %d iterations",
            (long long)t, steps_of[t].size(), outer_of[t]);
    }
  }
  std::printf("ok seed %llu: %zu requests, %zu cancelled, %lld steps, budget %.1f, %d slots\n",
              (unsigned long long)seed, submitted.size(), cancelled_t.size(), (long long)n_steps, budget, max_slots);
  return 0;
}
