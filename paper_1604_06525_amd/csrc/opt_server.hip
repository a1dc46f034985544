// Serving many solves at once (continuous batching).
//
// The paper notes that a GPU solver is inefficient on problems with few
// unknowns (Sec. 8, on the small examples): one problem of a few thousand sites
// fills a small fraction of the chip, and every kernel launch costs about as
// much as the work it carries.  The server runs many requests together: each
// step advances every running request by one outer iteration, and every stage of
// that iteration is one launch per energy kind covering all requests of that
// kind (k_batch), each over the block range it would have alone.
//
// Scheduling.  Requests are admitted (workspace carved from the arena) when a
// slot and a range are free, and started in admission order while the running
// set's estimated GPU fill (the wavefront slots of each request's widest launch
// over the device's) stays within a budget.  The requests of one energy kind
// share each launch; the kinds run on streams of their own, so they overlap.  Steps are pipelined: a step is enqueued without
// waiting for the GPU (up to kDepth in flight); its scalars and results come back
// through pinned memory behind an event, and the host harvests completed steps
// whenever it calls in.
//
// Each request's arithmetic, partial sums and reduction order are those of the
// single-problem solve, so a request gives the same bits whether it runs alone
// or in any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "opt.h"
#include "host.h"
#include "serve_sched.h"

using namespace optmi;
using namespace optmi::host;
using optmi::sched::SlotState;

namespace {

constexpr int kStageKinds = 12;  // table kinds that one step can write
constexpr int kMaxKinds = 56;    // energy form (7) x precision x method x PCG form
constexpr int kDepth = 3;        // steps in flight
constexpr int kLanes = kMaxLanes - 1;  // streams the energy-kind groups of a step run on
// Default fill budget: the running set may hold about four GPUs' worth of
// launches.  A launch of a mid-sized problem fills the wavefront slots but is
// short, so its time is mostly latency that co-running launches hide
// (saturation throughput of the serving mix measured 157 / 251 / 216 solves/s
// at budgets 1 / 4 / unlimited).
constexpr double kDefaultFillBudget = 4.0;

// A request: its scheduling state (serve_sched.h: the life cycle NEW, RUN, DRAIN and
// the start policy) and what its launches need.
struct Slot : sched::SlotCore {
  std::unique_ptr<opt_problem> p;
  void* x = nullptr;
  opt_solve_params sp{};
  bool fused = false;     // PCG form used
  // A graph request's edge list is copied to pinned memory behind the work on
  // the server's stream; its incidence lists are built on the host by the first
  // step after that copy has completed (graph_pending until then), and the
  // request starts from then on.
  hipEvent_t ev_edges = nullptr;
  int* edges_pin = nullptr;  // 2E ints; freed once the lists are built
  int* inc_pin = nullptr;    // incidence_words ints; their upload reads them, so kept until release
};

// Free a slot's graph staging (waiting for the edge copy if it may still run).
void free_graph_staging(Slot& s) {
  if (s.ev_edges) {
    (void)hipEventSynchronize(s.ev_edges);
    (void)hipEventDestroy(s.ev_edges);
    s.ev_edges = nullptr;
  }
  if (s.edges_pin) (void)hipHostFree(s.edges_pin);
  if (s.inc_pin) (void)hipHostFree(s.inc_pin);
  s.edges_pin = s.inc_pin = nullptr;
}

// Pinned per-slot landing area for a finished request.
struct ResultArea {
  DevScalars scal;
  double trace[kTraceCap];
};

struct TuneEntry {
  int32_t energy, precision;
  int64_t min_sites, max_sites;
  opt_tuning t;
};

struct Result {
  opt_solve_report rep{};
  std::vector<double> trace;
  bool nonfinite = false;
  int code = OPT_OK;  // a request dropped before it ran (its edge list was invalid)
  std::string msg;
};

struct StepRec {
  hipEvent_t ev = nullptr;
  std::vector<int> gathered;  // LM slots whose scalars this step reads back
  std::vector<int> retiring;  // slots whose final cost this step computes
};

// Every table kind holds, over all energy kinds, one argument row and two start
// entries per problem, one block-to-problem entry per block (at most kMaxBlocks
// per problem, plus up to kXcdCount - 1 idle blocks before it), and per kind
// three alignment gaps.
size_t table_area_bytes(int max_slots) {
  const size_t per_stage =
      (size_t)max_slots * (kMaxArgBytes + 2 * sizeof(int) + sizeof(int) * (kMaxBlocks + kXcdCount)) +
      (size_t)kMaxKinds * 3 * kAlign;
  return align_up((size_t)kStageKinds * per_stage);
}

size_t gather_bytes(int max_slots) { return align_up((size_t)max_slots * sizeof(DevScalars)); }

}  // namespace

struct opt_server {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int max_slots = 0;
  hipStream_t stream = nullptr;
  double fill_budget = kDefaultFillBudget;
  Batcher B;
  char* staging[kDepth] = {};           // pinned argument tables, one per step in flight
  DevScalars* dev_gather = nullptr;     // device, one row per slot
  DevScalars* host_gather[kDepth] = {}; // pinned, one per step in flight
  ResultArea* res = nullptr;            // pinned, one per slot
  StepRec steps[kDepth];
  // Each group of requests that share launches (one energy kind) runs on a lane
  // stream of its own, so that the groups of a step overlap on the device.  A
  // step forks the lanes from the server's stream after its table copy and joins
  // them back before its read-backs.
  hipStream_t lanes[kLanes] = {};
  hipEvent_t ev_fork[kDepth] = {};
  hipEvent_t ev_join[kDepth][kLanes] = {};
  int64_t n_steps = 0, n_done = 0;      // steps enqueued, steps completed and harvested
  sched::RangeAlloc ranges;
  std::vector<Slot> slots;
  std::map<int64_t, Result> results;
  std::vector<TuneEntry> tuning;  // later entries take precedence
  int64_t next_ticket = 1;

  ~opt_server() {
    if (n_steps > n_done) (void)hipStreamSynchronize(stream);
    for (Slot& s : slots) free_graph_staging(s);
    for (int k = 0; k < kDepth; ++k) {
      if (staging[k]) (void)hipHostFree(staging[k]);
      if (host_gather[k]) (void)hipHostFree(host_gather[k]);
      if (steps[k].ev) (void)hipEventDestroy(steps[k].ev);
      if (ev_fork[k]) (void)hipEventDestroy(ev_fork[k]);
      for (hipEvent_t e : ev_join[k])
        if (e) (void)hipEventDestroy(e);
    }
    for (hipStream_t l : lanes)
      if (l) (void)hipStreamDestroy(l);
    if (res) (void)hipHostFree(res);
  }
};

namespace {

// Requests that can share one launch: same energy, domain (ARAP warping has a
// grid and a graph form), precision, method (the damped and undamped fused
// kernels differ) and PCG form; bit 0 is the form.
int key_of(const Slot& s) {
  const int dom = s.p->desc.domain == OPT_GRAPH ? 1 : 0;
  return (((s.p->desc.energy * 2 + dom) * 2 + s.p->desc.precision) * 2 + (s.sp.method == OPT_LM ? 1 : 0)) * 2 +
         (s.fused ? 1 : 0);
}

SlotRef ref_of(Slot& s) {
  SlotRef r;
  r.p = s.p.get();
  r.x = s.x;
  const int lm = s.sp.method == OPT_LM;
  r.pa = PrecondArgs{0.0, s.sp.lm_diag_min, s.sp.lm_diag_max, s.sp.use_precond, lm != 0};
  r.lm = lm;
  r.L = s.sp.pcg_iters;
  return r;
}

// Record `stage` for the slots listed, one batched launch per energy kind.
int record_stage(opt_server* sv, Stage st, const std::vector<int>& ids) {
  std::map<int, std::vector<SlotRef>> groups;
  for (int i : ids) groups[key_of(sv->slots[(size_t)i])].push_back(ref_of(sv->slots[(size_t)i]));
  for (auto& kv : groups) {
    std::vector<SlotRef>& g = kv.second;
    const bool fused = (kv.first & 1) != 0;
    TRY(g[0].p->impl->batch(st, g.data(), (int)g.size(), fused, sv->B));
  }
  return OPT_OK;
}

template <class A, class F>
int record_scalar(opt_server* sv, const std::vector<int>& ids, F make, const char* name) {
  if (ids.empty()) return OPT_OK;
  std::vector<A> rows;
  std::vector<int> grids(ids.size(), 1);
  for (int i : ids) rows.push_back(make(sv->slots[(size_t)i], i));
  return batch_record(sv->B, rows.data(), grids.data(), (int)rows.size(), 0, 1, name);
}

void release_slot(opt_server* sv, Slot& s) {
  free_graph_staging(s);
  sv->ranges.release(s.ws_off, s.ws_bytes);
  s = Slot();
}

// Graph requests whose edge list has arrived: build their incidence lists and
// enqueue the upload (before this step's launches).  A request whose edges are
// invalid is dropped and reported by poll.
int finish_graph_admissions(opt_server* sv) {
  for (size_t i = 0; i < sv->slots.size(); ++i) {
    Slot& s = sv->slots[i];
    if (s.state != SlotState::NEW || !s.graph_pending) continue;
    const hipError_t q = hipEventQuery(s.ev_edges);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(OPT_EHIP, "hipEventQuery failed: %s", hipGetErrorString(q));
    bool gfused = false;
    const int rc = build_incidence_host(s.p->sh, s.edges_pin, s.inc_pin, &gfused);
    if (rc != OPT_OK) {
      Result r;
      r.code = rc;
      r.msg = last_error();
      sv->results[s.ticket] = std::move(r);
      release_slot(sv, s);
      continue;
    }
    TRY(upload_incidence(s.p.get(), s.inc_pin));
    // the form is known now: the fused one if the lists fit their caps
    s.p->gfused = gfused;
    s.fused = s.sp.pcg_variant == OPT_PCG_FUSED && s.p->impl->has_fused() && !s.p->impl->fused_is_big();
    s.fill = s.p->impl->gpu_fill(s.fused, s.sp.method == OPT_LM);
    (void)hipEventDestroy(s.ev_edges);
    s.ev_edges = nullptr;
    (void)hipHostFree(s.edges_pin);
    s.edges_pin = nullptr;
    s.graph_pending = false;
  }
  return OPT_OK;
}

// The report of a finished request, as opt_solve fills it.
void finish_result(opt_server* sv, int i) {
  Slot& s = sv->slots[(size_t)i];
  const ResultArea& ra = sv->res[i];
  const DevScalars& hs = ra.scal;
  const int K = s.sp.outer_iters, lm = s.sp.method == OPT_LM;
  const int done = lm ? hs.outer_done : K;
  Result r;
  r.trace.assign(ra.trace, ra.trace + K + 1);
  for (int j = done; j <= K; ++j) r.trace[(size_t)j] = hs.E_final;
  r.rep.cost_initial = K > 0 ? r.trace[0] : hs.E_final;
  r.rep.cost_final = hs.E_final;
  r.rep.outer_done = done;
  r.rep.steps_accepted = lm ? hs.n_accepted : K;
  r.rep.cost_trace = nullptr;
  r.nonfinite = hs.nonfinite != 0;
  sv->results[s.ticket] = std::move(r);
}

// Process completed steps in order.  block: wait for the oldest one in flight.
int harvest(opt_server* sv, bool block) {
  bool first = true;
  while (sv->n_done < sv->n_steps) {
    const int ring = (int)(sv->n_done % kDepth);
    StepRec& r = sv->steps[ring];
    if (block && first) {
      HIP_TRY(hipEventSynchronize(r.ev));
    } else {
      const hipError_t q = hipEventQuery(r.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return fail(OPT_EHIP, "hipEventQuery failed: %s", hipGetErrorString(q));
    }
    first = false;
    for (int i : r.retiring)
      if (!sv->slots[(size_t)i].cancelled) finish_result(sv, i);
    sv->n_done++;
    const DevScalars* g = sv->host_gather[ring];
    sched::complete_step(sv->slots, r.gathered, sv->n_done, [g](int i) { return g[i].done != 0; },
                         [sv](int i) { release_slot(sv, sv->slots[(size_t)i]); });
  }
  return OPT_OK;
}

}  // namespace

extern "C" {

int opt_server_reserved_bytes(int32_t max_slots, size_t* bytes) {
  if (!bytes) return fail(OPT_EINVAL, "bytes is NULL");
  if (max_slots < 1 || max_slots > 4096) return fail(OPT_EINVAL, "max_slots %d outside [1, 4096]", max_slots);
  *bytes = table_area_bytes(max_slots) + gather_bytes(max_slots);
  return OPT_OK;
}

int opt_server_create(void* arena, size_t arena_bytes, int32_t max_slots, void* hip_stream,
                      opt_server** out) {
  if (!out) return fail(OPT_EINVAL, "out is NULL");
  *out = nullptr;
  size_t reserved = 0;
  TRY(opt_server_reserved_bytes(max_slots, &reserved));
  if (!arena) return fail(OPT_EINVAL, "arena is NULL");
  if (((uintptr_t)arena) % kAlign) return fail(OPT_EINVAL, "arena must be %zu-byte aligned", kAlign);
  if (arena_bytes < reserved)
    return fail(OPT_ENOMEM, "arena of %zu bytes is smaller than the %zu the server keeps", arena_bytes,
                reserved);
  std::unique_ptr<opt_server> sv(new (std::nothrow) opt_server());
  if (!sv) return fail(OPT_ENOMEM, "host allocation failed");
  sv->arena = (char*)arena;
  sv->arena_bytes = arena_bytes;
  sv->max_slots = max_slots;
  sv->stream = (hipStream_t)hip_stream;
  sv->slots.resize((size_t)max_slots);
  const size_t tb = table_area_bytes(max_slots), gb = gather_bytes(max_slots);
  for (int k = 0; k < kDepth; ++k) {
    HIP_TRY(hipHostMalloc((void**)&sv->staging[k], tb, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&sv->host_gather[k], gb, hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&sv->steps[k].ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&sv->ev_fork[k], hipEventDisableTiming));
    for (int l = 0; l < kLanes; ++l) HIP_TRY(hipEventCreateWithFlags(&sv->ev_join[k][l], hipEventDisableTiming));
  }
  for (int l = 0; l < kLanes; ++l) HIP_TRY(hipStreamCreateWithFlags(&sv->lanes[l], hipStreamNonBlocking));
  HIP_TRY(hipHostMalloc((void**)&sv->res, sizeof(ResultArea) * (size_t)max_slots, hipHostMallocDefault));
  sv->B.dev = sv->arena;
  sv->B.cap = tb;
  sv->B.stream = sv->stream;
  sv->dev_gather = (DevScalars*)(sv->arena + tb);
  sv->ranges.reset(tb + gb, (arena_bytes - tb - gb) / kAlign * kAlign);
  *out = sv.release();
  return OPT_OK;
}

int opt_server_destroy(opt_server* sv) {
  delete sv;
  return OPT_OK;
}

int opt_server_set_fill_budget(opt_server* sv, double budget) {
  if (!sv) return fail(OPT_EINVAL, "server is NULL");
  if (!(budget >= 0.0)) return fail(OPT_EINVAL, "fill budget %g must be >= 0", budget);
  sv->fill_budget = budget;
  return OPT_OK;
}

int opt_server_submit(opt_server* sv, const opt_problem_desc* desc, void* unknowns,
                      const opt_solve_params* sp, int64_t* ticket) {
  if (!sv || !unknowns || !ticket) return fail(OPT_EINVAL, "server, unknowns or ticket is NULL");
  *ticket = -1;
  Shape sh;
  TRY(check_desc(desc, &sh));
  TRY(check_params(sp));
  TRY(check_method(desc, sp));
  TRY(harvest(sv, false));
  const size_t need = align_up(make_layout(sh).total);
  size_t slot = (size_t)sv->max_slots;
  for (size_t k = 0; k < sv->slots.size(); ++k)
    if (sv->slots[k].state == SlotState::EMPTY) {
      slot = k;
      break;
    }
  if (slot == (size_t)sv->max_slots) return fail(OPT_EAGAIN, "all %d slots are busy", sv->max_slots);
  size_t off = 0;
  if (!sv->ranges.alloc(need, &off))
    return fail(OPT_EAGAIN, "no free arena range of %zu bytes (%zu free in total)", need,
                sv->ranges.free_bytes());
  std::unique_ptr<opt_problem> p(new (std::nothrow) opt_problem());
  if (!p) {
    sv->ranges.release(off, need);
    return fail(OPT_ENOMEM, "host allocation failed");
  }
  const int rc = problem_init(p.get(), desc, sh, sv->arena + off, sv->stream, /*defer_graph=*/true);
  if (rc != OPT_OK) {
    sv->ranges.release(off, need);
    return rc;
  }
  int* edges_pin = nullptr;
  int* inc_pin = nullptr;
  hipEvent_t ev_edges = nullptr;
  if (sh.graph) {
    // the edge list comes back behind the work already on the server's stream,
    // without waiting for it
    const size_t ne = std::max<size_t>(1, 2 * (size_t)sh.n_edges);
    hipError_t e = hipHostMalloc((void**)&edges_pin, sizeof(int) * ne, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&inc_pin, sizeof(int) * incidence_words(sh), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_edges, hipEventDisableTiming);
    if (e == hipSuccess && sh.n_edges > 0)
      e = hipMemcpyAsync(edges_pin, desc->edges, sizeof(int) * 2 * (size_t)sh.n_edges, hipMemcpyDeviceToHost,
                         sv->stream);
    if (e == hipSuccess) e = hipEventRecord(ev_edges, sv->stream);
    if (e != hipSuccess) {
      if (ev_edges) (void)hipEventSynchronize(ev_edges), (void)hipEventDestroy(ev_edges);
      (void)hipStreamSynchronize(sv->stream);
      if (edges_pin) (void)hipHostFree(edges_pin);
      if (inc_pin) (void)hipHostFree(inc_pin);
      sv->ranges.release(off, need);
      return fail(OPT_EHIP, "staging the edge list failed: %s", hipGetErrorString(e));
    }
  }
  // (launch shapes are those of the 2D grid kernels: a graph request of the same
  // energy, the Laplacian's, takes none)
  for (auto it = sv->tuning.rbegin(); it != sv->tuning.rend() && desc->domain == OPT_GRID2D; ++it)
    if (it->energy == desc->energy && it->precision == desc->precision && sh.n >= it->min_sites &&
        sh.n <= it->max_sites) {
      p->tune = it->t;
      break;
    }
  Slot& s = sv->slots[slot];
  s = Slot();
  s.state = SlotState::NEW;
  s.ticket = sv->next_ticket++;
  s.ws_off = off;
  s.ws_bytes = need;
  s.x = unknowns;
  s.sp = *sp;
  s.outer = sp->outer_iters;
  s.lm = sp->method == OPT_LM;
  s.fused = sp->pcg_variant == OPT_PCG_FUSED && p->impl->has_fused() && !p->impl->fused_is_big();
  s.fill = p->impl->gpu_fill(s.fused, sp->method == OPT_LM);
  s.p = std::move(p);
  s.graph_pending = sh.graph;
  s.ev_edges = ev_edges;
  s.edges_pin = edges_pin;
  s.inc_pin = inc_pin;
  *ticket = s.ticket;
  return OPT_OK;
}

int opt_server_step(opt_server* sv) {
  if (!sv) return fail(OPT_EINVAL, "server is NULL");
  TRY(harvest(sv, false));
  if (sv->n_steps - sv->n_done >= kDepth) TRY(harvest(sv, true));
  TRY(finish_graph_admissions(sv));
  // start admitted requests (serve_sched.h: admission order, fill budget), then plan
  // the step: one outer iteration for every runnable request, the final cost
  // for those whose iterations are then all enqueued (or whose LM solve stopped)
  const std::vector<int> fresh = sched::start_requests(sv->slots, sv->fill_budget);
  const sched::StepPlan plan = sched::plan_step(sv->slots);
  const std::vector<int>&run = plan.run, &lm_run = plan.lm, &fin = plan.fin;
  if (fresh.empty() && plan.empty()) {
    // nothing to enqueue: wait for the oldest step in flight, if any, or for a
    // pending edge list
    if (sv->n_steps > sv->n_done) {
      TRY(harvest(sv, true));
    } else {
      for (Slot& s : sv->slots)
        if (s.state == SlotState::NEW && s.graph_pending) {
          HIP_TRY(hipEventSynchronize(s.ev_edges));
          break;
        }
    }
    return OPT_OK;
  }

  const int ring = (int)(sv->n_steps % kDepth);
  sv->B.reset();
  sv->B.host = sv->staging[ring];
  // lane 0: the server's stream, before the fork (setup of the requests that start)
  sv->B.lane = 0;
  sv->B.stream = sv->stream;
  TRY(record_scalar<SetupArgs>(sv, fresh, [](Slot& s, int) {
    return setup_args(s.p->S(), 0.0, s.sp.lm_radius0, s.sp.method == OPT_LM ? 1 : 0, s.sp.lm_radius_min);
  }, "setup[batch]"));
  // one outer iteration (Sec. 4) for every running request, and the final cost
  // of those that finish: each group of requests sharing launches on a lane
  struct Group {
    std::vector<int> run, lm, fin;
  };
  std::map<int, Group> groups;
  for (int i : run) groups[key_of(sv->slots[(size_t)i])].run.push_back(i);
  for (int i : lm_run) groups[key_of(sv->slots[(size_t)i])].lm.push_back(i);
  for (int i : fin) groups[key_of(sv->slots[(size_t)i])].fin.push_back(i);
  DevScalars* dg = sv->dev_gather;
  int gi = 0;
  for (auto& kv : groups) {
    const Group& g = kv.second;
    const int lane = gi++ % kLanes;
    sv->B.lane = 1 + lane;
    sv->B.stream = sv->lanes[lane];
    TRY(record_stage(sv, Stage::LIN, g.run));
    TRY(record_stage(sv, Stage::INIT, g.run));
    TRY(record_stage(sv, Stage::PCG, g.run));
    TRY(record_stage(sv, Stage::MODEL, g.lm));
    TRY(record_stage(sv, Stage::TRIAL_COST, g.lm));
    TRY(record_scalar<DecideArgs>(sv, g.lm, [](Slot& s, int) {
      return decide_args(s.p->S(), s.p->part(P_M), s.p->part(P_COST), s.p->nblk, s.sp);
    }, "decide[batch]"));
    TRY(record_stage(sv, Stage::STEP, g.run));
    TRY(record_stage(sv, Stage::COST, g.fin));
    TRY(record_scalar<FinishArgs>(sv, g.fin, [](Slot& s, int) {
      return finish_args(s.p->S(), s.p->part(P_COST), s.p->nblk);
    }, "finish[batch]"));
    TRY(record_scalar<GatherArgs>(sv, g.lm, [dg](Slot& s, int i) {
      return GatherArgs{s.p->S(), dg + i};
    }, "gather[batch]"));
  }
  // enqueue: tables, setup, fork, the lanes' launches round robin, join,
  // read-backs, event; no wait
  if (sv->B.used) HIP_TRY(hipMemcpyAsync(sv->B.dev, sv->B.host, sv->B.used, hipMemcpyHostToDevice, sv->stream));
  for (auto& f : sv->B.q[0]) TRY(f());
  const int n_lanes = std::min(kLanes, gi);
  if (n_lanes > 0) {
    HIP_TRY(hipEventRecord(sv->ev_fork[ring], sv->stream));
    for (int l = 0; l < n_lanes; ++l) HIP_TRY(hipStreamWaitEvent(sv->lanes[l], sv->ev_fork[ring], 0));
    size_t next[kMaxLanes] = {};
    for (bool more = true; more;) {
      more = false;
      for (int l = 1; l <= n_lanes; ++l) {
        std::vector<std::function<int()>>& q = sv->B.q[l];
        if (next[l] < q.size()) {
          TRY(q[next[l]++]());
          more = more || next[l] < q.size();
        }
      }
    }
    for (int l = 0; l < n_lanes; ++l) {
      HIP_TRY(hipEventRecord(sv->ev_join[ring][l], sv->lanes[l]));
      HIP_TRY(hipStreamWaitEvent(sv->stream, sv->ev_join[ring][l], 0));
    }
  }
  if (!lm_run.empty())
    HIP_TRY(hipMemcpyAsync(sv->host_gather[ring], sv->dev_gather, sizeof(DevScalars) * (size_t)sv->max_slots,
                           hipMemcpyDeviceToHost, sv->stream));
  for (int i : fin) {
    Slot& s = sv->slots[(size_t)i];
    HIP_TRY(hipMemcpyAsync(&sv->res[i].scal, s.p->S(), sizeof(DevScalars), hipMemcpyDeviceToHost, sv->stream));
    if (s.sp.outer_iters > 0)
      HIP_TRY(hipMemcpyAsync(sv->res[i].trace, s.p->trace(), sizeof(double) * (size_t)s.sp.outer_iters,
                             hipMemcpyDeviceToHost, sv->stream));
  }
  StepRec& rec = sv->steps[ring];
  rec.gathered = lm_run;
  rec.retiring = fin;
  HIP_TRY(hipEventRecord(rec.ev, sv->stream));
  sched::commit_step(sv->slots, fresh, plan, sv->n_steps++);
  return OPT_OK;
}

int opt_server_poll(opt_server* sv, int64_t ticket, int32_t* done, opt_solve_report* report) {
  if (!sv || !done) return fail(OPT_EINVAL, "server or done is NULL");
  *done = 0;
  TRY(harvest(sv, false));
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) {
    for (const Slot& s : sv->slots)
      if (s.state != SlotState::EMPTY && s.ticket == ticket && !s.cancelled) return OPT_OK;
    return fail(OPT_EINVAL, "ticket %lld is not known (or was already collected)", (long long)ticket);
  }
  *done = 1;
  const Result& r = it->second;
  if (r.code != OPT_OK) {
    const int code = r.code;
    const std::string msg = r.msg;
    sv->results.erase(it);
    return fail(code, "request dropped: %s", msg.c_str());
  }
  const bool nonfinite = r.nonfinite;
  if (report) {
    double* dst = report->cost_trace;
    *report = r.rep;
    report->cost_trace = dst;
    if (dst) memcpy(dst, r.trace.data(), sizeof(double) * r.trace.size());
  }
  sv->results.erase(it);
  if (nonfinite) return fail(OPT_ENUMERIC, "a cost was NaN or infinite");
  return OPT_OK;
}

int opt_server_cancel(opt_server* sv, int64_t ticket) {
  if (!sv) return fail(OPT_EINVAL, "server is NULL");
  if (sv->results.erase(ticket)) return OPT_OK;
  // work already enqueued for it must complete before its range is reused
  if (sched::cancel(sv->slots, ticket, sv->n_done, [sv](int i) { release_slot(sv, sv->slots[(size_t)i]); }))
    return OPT_OK;
  return fail(OPT_EINVAL, "ticket %lld is not known", (long long)ticket);
}

int opt_server_wait(opt_server* sv) {
  if (!sv) return fail(OPT_EINVAL, "server is NULL");
  while (sv->n_done < sv->n_steps) TRY(harvest(sv, true));
  return OPT_OK;
}

int opt_server_add_tuning(opt_server* sv, int32_t energy, int32_t precision, int64_t min_sites,
                          int64_t max_sites, const opt_tuning* t) {
  if (!sv || !t) return fail(OPT_EINVAL, "server or tuning is NULL");
  TRY(check_tuning(t));
  if (min_sites > max_sites) return fail(OPT_EINVAL, "empty site range");
  sv->tuning.push_back(TuneEntry{energy, precision, min_sites, max_sites, *t});
  return OPT_OK;
}

int opt_server_info(opt_server* sv, int32_t* active, size_t* arena_free) {
  if (!sv) return fail(OPT_EINVAL, "server is NULL");
  TRY(harvest(sv, false));
  int n = 0;
  for (const Slot& s : sv->slots) n += s.state != SlotState::EMPTY && !s.cancelled;
  if (active) *active = n;
  if (arena_free) *arena_free = sv->ranges.free_bytes();
  return OPT_OK;
}

}  // extern "C"
