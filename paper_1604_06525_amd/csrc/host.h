// Host-side internals shared by the single-problem API (opt_capi.hip) and the
// batching server (opt_server.hip): error reporting, the workspace layout, the
// problem handle and the per-energy launch interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstring>
#include <functional>
#include <memory>
#include <vector>

#include "opt.h"
#include "common.h"
#include "kernels.h"

namespace optmi {
namespace host {

// Record a formatted message as the calling thread's last error; returns code.
int fail(int code, const char* fmt, ...);
const char* last_error();

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::optmi::host::fail(OPT_EHIP, "%s failed: %s (%s:%d)", #call,                \
                                 hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

#define HIP_LAUNCHED(name)                                                                \
  do {                                                                                    \
    hipError_t e_ = hipGetLastError();                                                    \
    if (e_ != hipSuccess)                                                                 \
      return ::optmi::host::fail(OPT_EHIP, "launch of %s failed: %s", name,               \
                                 hipGetErrorString(e_));                                  \
  } while (0)

#define TRY(x)                     \
  do {                             \
    int rc_ = (x);                 \
    if (rc_ != OPT_OK) return rc_; \
  } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kMaxArgBytes = 1024;  // bound on any argument row of a batched launch
constexpr int kTraceCap = 4097;  // outer iterations + 1 that a report can hold
constexpr int kMaxOuter = kTraceCap - 1;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Shape {
  int C = 0;           // unknown channels
  int state_planes = 0;
  int n = 0;           // sites
  size_t tsize = 0;    // bytes of the bulk type
  int n_edges = 0;     // graph: listed undirected edges
  int stage_w = 0;     // graph: values per vertex pcg_a stages (0: not staged)
  bool graph = false;
  bool gfz = false;    // graph: the fused PCG form's per-chunk lists are built
  // materialised Jacobian (OPT_PCG_MATERIALIZED): rows per site, entries per
  // row, entries per J^T column
  bool mat = false;
  int mat_rows = 0, mat_slots = 0, mat_tslots = 0;
};

// Byte offsets of every region of a problem's workspace.
struct Layout {
  size_t r0, r1, p0, p1, q, diag, minv, damp, delta, state, flags, csr, halo, gfz, jval, jcol, jt, jy, parts,
      scal, trace, rows, total;
};

// Argument rows a single problem launches with, one device slot of kMaxArgBytes
// each in its workspace (the batching server keeps its own tables).
enum RowKind {
  ROW_SETUP, ROW_LIN, ROW_INIT, ROW_PCGA, ROW_APPLY, ROW_PCGB, ROW_FUSED, ROW_STEP, ROW_COST,
  ROW_TRIAL, ROW_MODEL, ROW_DECIDE, ROW_FINISH, ROW_PLANES, ROW_EVALJ, ROW_MATP, ROW_MATA, ROW_MATB, ROW_PCGA_LIT,
  kNumRows
};

// Partial-sum buffers of kMaxBlocks doubles each; the fused form uses two pairs.
enum { P_LIN = 0, P_RZ0 = 1, P_RZ1 = 2, P_PQ = 3, P_COST = 4, P_M = 5, P_F0 = 6, P_F1 = 8 };
constexpr int kNumPartBufs = 10;

Layout make_layout(const Shape& sh);
int check_desc(const opt_problem_desc* d, Shape* sh);
int check_params(const opt_solve_params* sp);
int check_method(const opt_problem_desc* d, const opt_solve_params* sp);
int check_tuning(const opt_tuning* t);

struct PrecondArgs {
  double lam, dmin, dmax;
  int use;
  bool damped;  // LM: write and apply the damping vector
};

// ---------------------------------------------------------------- batching
// Argument tables of batched launches are written into pinned host staging
// memory while a step is planned, copied to device memory in one transfer, and
// then the recorded launches are enqueued.  Launches are recorded into lanes:
// each lane's launches go to one stream, in recording order; the server
// enqueues the lanes round robin, one launch of each in turn, so that lanes on
// different streams start together.
constexpr int kMaxLanes = 4;

struct Batcher {
  char* host = nullptr;   // pinned staging
  char* dev = nullptr;    // device table area of the same size
  size_t cap = 0, used = 0;
  hipStream_t stream = nullptr;  // stream of the lane being recorded
  int lane = 0;                  // lane being recorded
  std::vector<std::function<int()>> q[kMaxLanes];

  void reset() {
    used = 0;
    lane = 0;
    for (auto& l : q) l.clear();
  }
  void push(std::function<int()> f) { q[lane].push_back(std::move(f)); }
  // Reserve `bytes` (256-aligned); returns the offset or -1 if full.
  long long reserve(size_t bytes) {
    const size_t off = align_up(used);
    if (off + bytes > cap) return -1;
    used = off + bytes;
    return (long long)off;
  }
};

// One problem's part in a batched launch.
struct SlotRef {
  opt_problem* p;
  void* x;
  PrecondArgs pa;
  int lm;
  int L;          // PCG iterations
};

enum class Stage { LIN, INIT, PCG, MODEL, TRIAL_COST, STEP, COST };

// Strip partition of a grid for the fused kernel (opt_capi.hip: strip_geom).
struct StripGeom {
  int n_sx, n_sy, sw, rq, rr, grid;
};

// Launch sequence for one energy and bulk type.
class Impl {
 public:
  virtual ~Impl() = default;
  virtual int linearize(const void* x, int lm_gate) = 0;
  // u_form: the fused form follows (write u_0 = M^-1 b where b would go)
  virtual int init(const void* x, double* trace, PrecondArgs pa, int lm_gate, int u_form) = 0;
  virtual int pcg_a(int k, int L, PrecondArgs pa, int lm_gate) = 0;
  virtual int pcg_b(int k, int L, PrecondArgs pa, int lm_gate) = 0;
  // pcg_a with the stored per-site state recomputed inside the product
  // (OPT_PCG_RECOMPUTE; shape from shading only)
  virtual bool has_recompute() const { return false; }
  virtual int pcg_a_recompute(int k, int L, PrecondArgs pa, int lm_gate) = 0;
  virtual int fused(int iter, int L, PrecondArgs pa, int lm_gate) = 0;
  virtual bool has_fused() const = 0;
  // materialised form (OPT_PCG_MATERIALIZED): evaluate J at the linearisation
  // point, then per iteration y = J p and q = J^T y (+ damping), then pcg_b
  virtual bool has_mat() const { return false; }
  virtual int eval_j() = 0;
  virtual int mat_a(int k, int L, PrecondArgs pa, int lm_gate) = 0;
  virtual int mat_b(int k, int L, PrecondArgs pa, int lm_gate) = 0;
  // the fused form runs the instantiation for vectors past 256 MB (solo only:
  // the server runs such problems in the split form)
  virtual bool fused_is_big() const { return false; }
  virtual int apply_jtj(const void* p, void* q, PrecondArgs pa) = 0;
  virtual int apply_step(void* x, int lm_gate) = 0;
  virtual int cost(const void* x, const void* delta, int lm_gate) = 0;
  virtual int model(const void* x) = 0;
  // Copy an internal vector (interleaved) out to channel planes.
  virtual int to_planes(const void* src, void* dst) = 0;
  // Fused-kernel strip partition in force (grid energies).
  virtual StripGeom strip_geometry(bool damped) const = 0;
  // Estimated share of the GPU one PCG launch of this problem occupies (its
  // wavefronts over those the device holds at the kernel's occupancy), <= 1.
  virtual double gpu_fill(bool fused, bool damped) const = 0;
  // Record one batched launch of `stage` over n problems of this energy and
  // type (the PCG stage records all of its launches); `fused` picks the form.
  virtual int batch(Stage stage, const SlotRef* slots, int n, bool fused, Batcher& B) = 0;
};

}  // namespace host
}  // namespace optmi

struct opt_problem {
  opt_problem_desc desc;
  optmi::host::Shape sh;
  optmi::host::Layout L;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int nblk = 1;
  int n_simd = 1024;  // SIMDs of the device (fused kernel launch shape)
  const void* last_x = nullptr;
  bool gfused = false;  // graph: the fused PCG form's lists are built and fit
  // last bytes stored in each device argument row (a row is stored again only
  // when it changes)
  std::vector<std::vector<unsigned char>> row_cache =
      std::vector<std::vector<unsigned char>>(optmi::host::kNumRows);
  opt_tuning tune{};
  std::unique_ptr<optmi::host::Impl> impl;
  // PCG-phase timing (opt_profile_enable)
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;   // created on demand, reused
  size_t ev_used = 0;                // events recorded since the last read
  int64_t prof_iters = 0;
  // Graph replay of repeated solves (opt_problem_set_graph_replay): the launch
  // sequence of a solve is determined by the unknowns pointer, the parameters and
  // the tuning; when a solve repeats the previous one's, that sequence is
  // recorded once as a HIP graph (on a private stream) and replayed.
  struct SolveKey {
    const void* x = nullptr;
    opt_solve_params sp{};
    opt_tuning tune{};
    bool valid = false;
  };
  bool graphs = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  SolveKey gkey, last_eager;
  // argument rows as the graph leaves them (restored into row_cache after a replay)
  std::vector<std::vector<unsigned char>> rows_after_graph;

  void drop_graph() {
    if (gexec) {
      (void)hipStreamSynchronize(stream);
      (void)hipGraphExecDestroy(gexec);
    }
    gexec = nullptr;
    gkey.valid = false;
  }

  ~opt_problem() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }

  void* at(size_t off) const { return ws + off; }
  double* part(int k) const { return (double*)(ws + L.parts) + (size_t)k * optmi::kMaxBlocks; }
  optmi::DevScalars* S() const { return (optmi::DevScalars*)(ws + L.scal); }
  double* trace() const { return (double*)(ws + L.trace); }
};

namespace optmi {
namespace host {

// Build the handle's state inside `workspace` (validated descriptor); for a
// graph this sorts the edges into the incidence list and synchronises, unless
// defer_graph (the caller then builds and uploads it: build_incidence_host,
// upload_incidence).
int problem_init(opt_problem* p, const opt_problem_desc* desc, const Shape& sh, void* workspace,
                 hipStream_t stream, bool defer_graph = false);

// Graph incidence and staging lists as one host array (see opt_capi.hip);
// *gfused tells whether the fused PCG form's lists fit their caps.
size_t incidence_words(const Shape& sh);
int build_incidence_host(const Shape& sh, const int* edges, int* out, bool* gfused);
int upload_incidence(opt_problem* p, const int* words);

// opt_solve on a created problem (parameters validated here).
int solve(opt_problem* p, void* x, const opt_solve_params* sp, opt_solve_report* rep);

// An argument struct with every byte zero (padding included) before its fields
// are set, so equal arguments compare equal byte for byte.
template <class A>
A blank() {
  A a;
  std::memset(static_cast<void*>(&a), 0, sizeof(A));
  return a;
}

// Argument rows of the one-block scalar stages.
inline SetupArgs setup_args(DevScalars* S, double lambda, double radius0, int lm, double radius_min) {
  SetupArgs a = blank<SetupArgs>();
  a.S = S;
  a.lambda = lambda;
  a.radius0 = radius0;
  a.lm = lm;
  a.radius_min = radius_min;
  return a;
}
inline FinishArgs finish_args(DevScalars* S, const double* part, int nb) {
  FinishArgs a = blank<FinishArgs>();
  a.S = S;
  a.part = part;
  a.nb = nb;
  return a;
}
inline DecideArgs decide_args(DevScalars* S, const double* m_part, const double* c_part, int nb,
                              const opt_solve_params& sp) {
  DecideArgs a = blank<DecideArgs>();
  a.S = S;
  a.m_part = m_part;
  a.c_part = c_part;
  a.nb = nb;
  a.lc.radius_min = sp.lm_radius_min;
  a.lc.radius_max = sp.lm_radius_max;
  a.lc.min_rel_decrease = sp.lm_min_rel_decrease;
  return a;
}

// Launch one stage of a single problem: store its argument row in the problem's
// workspace (only if it changed since the last store) and run the stage kernel
// over `grid` blocks, in the problem's stream.
template <class A>
int launch_row(opt_problem* p, int kind, const A& a, int grid, int iter, const char* name) {
  static_assert(sizeof(A) <= kMaxArgBytes, "argument row larger than its slot");
  A* dev = (A*)(p->ws + p->L.rows + (size_t)kind * kMaxArgBytes);
  std::vector<unsigned char>& c = p->row_cache[(size_t)kind];
  if (c.size() != sizeof(A) || std::memcmp(c.data(), &a, sizeof(A)) != 0) {
    k_put<A><<<1, 64, 0, p->stream>>>(dev, a);
    HIP_LAUNCHED(name);
    c.assign((const unsigned char*)&a, (const unsigned char*)&a + sizeof(A));
  }
  k_batch<A><<<grid, kBlock, 0, p->stream>>>(dev, nullptr, nullptr, 1, iter);
  HIP_LAUNCHED(name);
  return OPT_OK;
}

// A batched argument table in the staging area: one row per problem and the
// first block of each problem's range.
// Each problem's blocks start at a multiple of kXcdCount (the hardware deals
// blocks to the XCDs round-robin), so they fall on the XCDs as when alone.
constexpr int kXcdCount = 8;

template <class A>
struct BatchTable {
  const A* rows = nullptr;      // device, one per problem
  const int* start = nullptr;   // device, 2n entries: first block and grid of each problem
  const int* slot_of = nullptr; // device, problem of each block (-1: idle)
  int n = 0, total = 0;         // problems, blocks
};

template <class A>
int batch_table(Batcher& B, const A* rows, const int* grids, int n, BatchTable<A>* t) {
  static_assert(sizeof(A) <= kMaxArgBytes, "argument row larger than the table area allows");
  long long total = 0;
  for (int k = 0; k < n; ++k) {
    if (grids[k] < 1 || grids[k] > kMaxBlocks) return fail(OPT_EINVAL, "grid of %d blocks", grids[k]);
    total = (total + kXcdCount - 1) / kXcdCount * kXcdCount + grids[k];
  }
  const size_t tbytes = sizeof(A) * (size_t)n, sbytes = sizeof(int) * 2 * (size_t)n;
  const long long ot = B.reserve(tbytes), os = B.reserve(sbytes), om = B.reserve(sizeof(int) * total);
  if (ot < 0 || os < 0 || om < 0) return fail(OPT_ENOMEM, "server table area is full");
  A* ht = (A*)(B.host + ot);
  int* hs = (int*)(B.host + os);
  int* hm = (int*)(B.host + om);
  int b = 0;
  for (int k = 0; k < n; ++k) {
    const int b0 = (b + kXcdCount - 1) / kXcdCount * kXcdCount;
    for (; b < b0; ++b) hm[b] = -1;
    ht[k] = rows[k];
    hs[2 * k] = b0;
    hs[2 * k + 1] = grids[k];
    for (int q = 0; q < grids[k]; ++q) hm[b0 + q] = k;
    b = b0 + grids[k];
  }
  t->rows = (const A*)(B.dev + ot);
  t->start = (const int*)(B.dev + os);
  t->slot_of = (const int*)(B.dev + om);
  t->n = n;
  t->total = b;
  return OPT_OK;
}

template <class A>
int batch_launch(const BatchTable<A>& t, int iter, hipStream_t st, const char* name) {
  k_batch<A><<<t.total, kBlock, 0, st>>>(t.rows, t.start, t.slot_of, t.n, iter);
  HIP_LAUNCHED(name);
  return OPT_OK;
}

// Record a batched launch of `A` rows (one per problem) with the given block
// counts, for iterations [iter_lo, iter_hi) (one recorded launch each).
template <class A>
int batch_record(Batcher& B, const A* rows, const int* grids, int n, int iter_lo, int iter_hi,
                 const char* name) {
  if (n <= 0 || iter_lo >= iter_hi) return OPT_OK;
  BatchTable<A> t;
  TRY(batch_table(B, rows, grids, n, &t));
  hipStream_t st = B.stream;
  for (int it = iter_lo; it < iter_hi; ++it) B.push([=]() -> int { return batch_launch(t, it, st, name); });
  return OPT_OK;
}

}  // namespace host
}  // namespace optmi
