// Host side of the C ABI declared in include/opt.h: descriptor validation,
// workspace layout, and the order in which the kernels of a solve are enqueued
// (Sec. 4: per outer iteration linearise, PCG-init, L PCG iterations, update;
// LM adds the model decrease, the trial cost and the step decision).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "opt.h"
#include "host.h"
#include "energies.h"
#include "fused_sfs.h"
#include "fused_graph.h"
#include "graph_lists.h"

namespace optmi {
namespace host {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

// Ints of the fused graph form's lists: a row per chunk.
size_t gfz_words(const Shape& sh) { return lists::gfz_words(sh.n); }

Layout make_layout(const Shape& sh) {
  Layout L{};
  size_t off = 0;
  const size_t vec = align_up((size_t)sh.C * sh.n * sh.tsize);
  for (size_t* v : {&L.r0, &L.r1, &L.p0, &L.p1, &L.q, &L.diag, &L.minv, &L.damp, &L.delta}) {
    *v = off;
    off += vec;
  }
  L.state = off; off += align_up((size_t)sh.state_planes * sh.n * sh.tsize);
  L.flags = off; off += align_up((size_t)sh.n);
  L.csr = off;  // graph: row offsets [n+1], then neighbour ids [2E]
  if (sh.graph) off += align_up(sizeof(int) * ((size_t)sh.n + 1 + 2 * (size_t)sh.n_edges));
  L.halo = off;  // graph: chunk-local neighbour slots [2E], halo counts [chunks], halo ids [chunks][cap]
  if (sh.graph)
    off += align_up(sizeof(int) * (2 * (size_t)sh.n_edges + (size_t)(sh.n + kBlock - 1) / kBlock *
                                                                  (1 + (size_t)halo_cap(sh.tsize, sh.stage_w))));
  L.gfz = off;  // graph, fused form: per-chunk lists [chunks][kGfRow]
  if (sh.gfz) off += align_up(sizeof(int) * gfz_words(sh));
  // materialised Jacobian: entries (values, columns), J^T lists, y = J p
  const size_t jrows = sh.mat ? (size_t)sh.n * sh.mat_rows : 0;
  L.jval = off; off += align_up(jrows * sh.mat_slots * sh.tsize);
  L.jcol = off; off += align_up(jrows * sh.mat_slots * sizeof(int));
  L.jt = off; off += align_up((size_t)(sh.mat ? sh.n : 0) * sh.C * sh.mat_tslots * sizeof(int));
  L.jy = off; off += align_up(jrows * sh.tsize);
  L.parts = off; off += align_up(kNumPartBufs * (size_t)kMaxBlocks * sizeof(double));
  L.scal = off; off += align_up(sizeof(DevScalars));
  L.trace = off; off += align_up((size_t)kTraceCap * sizeof(double));
  L.rows = off; off += align_up((size_t)kNumRows * kMaxArgBytes);
  L.total = off;
  return L;
}

namespace {

int energy_channels(int e) {
  switch (e) {
    case OPT_E_LAPLACIAN: return LaplacianGrid<float>::C;
    case OPT_E_ARAP_WARP: return ArapWarp<float>::C;
    case OPT_E_POISSON: return Poisson<float>::C;
    case OPT_E_FLOW: return OpticalFlow<float>::C;
    case OPT_E_SFS: return ShapeFromShading<float>::C;
    case OPT_E_ARAP_MESH: return ArapMesh<float>::C;
    case OPT_E_ARAP_VOLUME: return ArapVolume<float>::C;
    case OPT_E_LP_SMOOTH: return LpSmoothGrid<float>::C;
    case OPT_E_INTRINSIC: return IntrinsicImage<float>::C;
    default: return 0;
  }
}

int energy_state_planes(int e) {
  switch (e) {
    case OPT_E_LAPLACIAN: return 0;
    case OPT_E_ARAP_WARP: return ArapWarp<float>::kOwnState;
    case OPT_E_POISSON: return Poisson<float>::kOwnState;
    case OPT_E_FLOW: return OpticalFlow<float>::kOwnState;
    case OPT_E_SFS: return ShapeFromShading<float>::kOwnState;
    case OPT_E_ARAP_MESH: return ArapMesh<float>::kOwnState;
    case OPT_E_ARAP_VOLUME: return ArapVolume<float>::kOwnState;
    case OPT_E_LP_SMOOTH: return LpSmoothGrid<float>::kOwnState;
    case OPT_E_INTRINSIC: return IntrinsicImage<float>::kOwnState;
    default: return 0;
  }
}

// Values per vertex pcg_a stages for a graph energy: p and the energy's own
// (0: the energy is not staged).
template <class E>
constexpr int stage_width_of() {
  if constexpr (optmi::StagedOf<E>::value) return E::C + E::kStageVals;
  return 0;
}

int stage_width(int e) {
  switch (e) {
    case OPT_E_ARAP_WARP: return stage_width_of<ArapWarpGraph<float>>();
    case OPT_E_ARAP_MESH: return stage_width_of<ArapMesh<float>>();
    default: return 0;
  }
}

// Materialised-Jacobian dimensions of an energy on a domain (rows per site,
// entries per row, entries per J^T column); false if it has none.
bool mat_dims(int e, int domain, int* rows, int* slots, int* tslots) {
  if (e == OPT_E_ARAP_WARP && domain == OPT_GRID2D) {
    *rows = ArapWarp<float>::kJRows;
    *slots = ArapWarp<float>::kJSlots;
    *tslots = ArapWarp<float>::kJTSlots;
    return true;
  }
  if (e == OPT_E_SFS && domain == OPT_GRID2D) {
    *rows = ShapeFromShading<float>::kJRows;
    *slots = ShapeFromShading<float>::kJSlots;
    *tslots = ShapeFromShading<float>::kJTSlots;
    return true;
  }
  return false;
}

int n_params_needed(int e) {
  switch (e) {
    case OPT_E_LAPLACIAN: return 2;
    case OPT_E_ARAP_WARP: return 2;
    case OPT_E_POISSON: return 0;
    case OPT_E_FLOW: return 2;
    case OPT_E_SFS: return 16;
    case OPT_E_ARAP_MESH: return 2;
    case OPT_E_ARAP_VOLUME: return 2;
    case OPT_E_LP_SMOOTH: return 4;
    case OPT_E_INTRINSIC: return 5;
    default: return 0;
  }
}

int n_arrays_needed(int e) {
  switch (e) {
    case OPT_E_LAPLACIAN: return 1;
    case OPT_E_ARAP_WARP: return 3;
    case OPT_E_POISSON: return 2;
    case OPT_E_FLOW: return 4;
    case OPT_E_SFS: return 4;
    case OPT_E_ARAP_MESH: return 2;
    case OPT_E_ARAP_VOLUME: return 2;
    case OPT_E_LP_SMOOTH: return 1;
    case OPT_E_INTRINSIC: return 1;
    default: return 0;
  }
}

}  // namespace

int check_desc(const opt_problem_desc* d, Shape* sh) {
  if (!d) return fail(OPT_EINVAL, "descriptor is NULL");
  if (d->precision != OPT_FP64 && d->precision != OPT_MIXED)
    return fail(OPT_EINVAL, "precision %d is not OPT_FP64 or OPT_MIXED", d->precision);
  const int C = energy_channels(d->energy);
  if (C == 0) return fail(OPT_EUNSUPPORTED, "energy %d is not built", d->energy);
  const bool volume_energy = d->energy == OPT_E_ARAP_VOLUME;
  const bool grid_energy = d->energy != OPT_E_ARAP_MESH && !volume_energy;
  // ARAP warping and the Laplacian run on either 2D domain (the graph form
  // takes an edge list)
  const bool both = d->energy == OPT_E_ARAP_WARP || d->energy == OPT_E_LAPLACIAN;
  if (volume_energy != (d->domain == OPT_GRID3D))
    return fail(OPT_EUNSUPPORTED, "energy %d and domain %d do not go together (OPT_E_ARAP_VOLUME is the "
                "OPT_GRID3D energy)", d->energy, d->domain);
  if (d->domain == OPT_GRID3D) {
    if (d->width < 1 || d->height < 1 || d->depth < 1)
      return fail(OPT_EINVAL, "grid size %d x %d x %d must be positive", d->width, d->height, d->depth);
    if ((long long)d->width * d->height * d->depth > (1LL << 28))
      return fail(OPT_EINVAL, "grid of %lld sites is too large", (long long)d->width * d->height * d->depth);
    sh->n = d->width * d->height * d->depth;
  } else if (d->domain == OPT_GRID2D) {
    if (!grid_energy) return fail(OPT_EUNSUPPORTED, "energy %d needs the graph domain", d->energy);
    if (d->width < 1 || d->height < 1)
      return fail(OPT_EINVAL, "grid size %d x %d must be positive", d->width, d->height);
    // (every fused kernel's strips of one grid row fit in the partial-sum buffers)
    if (d->width > kSfsCols * kWaves * kMaxBlocks)
      return fail(OPT_EINVAL, "grid width %d exceeds %d", d->width, kSfsCols * kWaves * kMaxBlocks);
    if ((long long)d->width * d->height > (1LL << 30))
      return fail(OPT_EINVAL, "grid of %lld sites is too large", (long long)d->width * d->height);
    sh->n = d->width * d->height;
  } else if (d->domain == OPT_GRAPH) {
    if (grid_energy && !both) return fail(OPT_EUNSUPPORTED, "energy %d needs the grid domain", d->energy);
    if (d->n_vertices < 1 || d->n_edges < 0)
      return fail(OPT_EINVAL, "graph of %d vertices and %d edges", d->n_vertices, d->n_edges);
    if (d->n_edges > (1 << 29)) return fail(OPT_EINVAL, "%d edges is too many", d->n_edges);
    if (d->n_edges > 0 && !d->edges) return fail(OPT_EINVAL, "edges is NULL");
    sh->n = d->n_vertices;
    sh->n_edges = d->n_edges;
    sh->graph = true;
    sh->stage_w = stage_width(d->energy);
    sh->gfz = d->energy == OPT_E_ARAP_MESH || d->energy == OPT_E_LAPLACIAN;
  } else {
    return fail(OPT_EINVAL, "domain %d is not OPT_GRID2D or OPT_GRAPH", d->domain);
  }
  if (d->n_params < n_params_needed(d->energy) || d->n_params > 16)
    return fail(OPT_EINVAL, "energy %d needs %d params, got %d", d->energy,
                n_params_needed(d->energy), d->n_params);
  for (int k = 0; k < n_arrays_needed(d->energy); ++k)
    if (!d->arrays[k]) return fail(OPT_EINVAL, "arrays[%d] is NULL", k);
  if (d->energy == OPT_E_LP_SMOOTH || d->energy == OPT_E_INTRINSIC) {
    const int at = d->energy == OPT_E_LP_SMOOTH ? 2 : 3;  // p, then eps
    const double p = d->params[at], eps = d->params[at + 1];
    if (!(p > 0.0 && p <= 2.0)) return fail(OPT_EINVAL, "p = %g is outside (0, 2]", p);
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(OPT_EINVAL, "eps = %g must be positive", eps);
  }
  // the graph Laplacian smooths a float3 per vertex (the grid one a scalar)
  sh->C = d->energy == OPT_E_LAPLACIAN && d->domain == OPT_GRAPH ? LaplacianGraph<float>::C : C;
  sh->state_planes = energy_state_planes(d->energy);
  sh->tsize = d->precision == OPT_FP64 ? sizeof(double) : sizeof(float);
  if (d->materialize != 0 && d->materialize != 1)
    return fail(OPT_EINVAL, "materialize %d is not 0 or 1", d->materialize);
  if (d->materialize) {
    if (!mat_dims(d->energy, d->domain, &sh->mat_rows, &sh->mat_slots, &sh->mat_tslots))
      return fail(OPT_EUNSUPPORTED, "energy %d on domain %d has no materialised Jacobian", d->energy, d->domain);
    // every entry index fits an int32
    if ((long long)sh->n * sh->mat_rows * sh->mat_slots >= (1LL << 31))
      return fail(OPT_EINVAL, "materialised Jacobian of %lld entries is too large",
                  (long long)sh->n * sh->mat_rows * sh->mat_slots);
    sh->mat = true;
  }
  return OPT_OK;
}

namespace {

// Partition of a W x H grid into strips for the fused kernel: n_sx strips
// across of sw produced columns each (sw <= 60, as even as possible), n_sy
// strips down of rq or rq + 1 rows.
//   t.strip_rows > 0: strips of that many rows;
//   otherwise about w strips per SIMD with the rows split evenly, w =
//   t.waves_per_simd or, by default, min(kAutoWavesPerSimd, the kernel's
//   occupancy in waves per SIMD); never under 4 rows.
// Balance matters: a launch is set by its slowest SIMD, so every SIMD should
// get the same number of equal strips (measured best: two where two fit, which
// lets each SIMD overlap one strip's memory waits with the other's arithmetic).
constexpr int kAutoWavesPerSimd = 2;

StripGeom strip_geom(int W, int H, const opt_tuning& t, int n_simd, int occupancy, int cols) {
  StripGeom g;
  g.n_sx = (W + cols - 1) / cols;
  g.sw = (W + g.n_sx - 1) / g.n_sx;
  const int max_sy = std::max(1, H / 4);
  int n_sy;
  if (t.strip_rows > 0) {
    n_sy = (H + t.strip_rows - 1) / t.strip_rows;
  } else {
    const int w = t.waves_per_simd > 0 ? t.waves_per_simd
                                       : std::max(1, std::min(kAutoWavesPerSimd, occupancy));
    n_sy = std::min(max_sy, std::max(1, w * n_simd / g.n_sx));
  }
  n_sy = std::max(1, std::min(n_sy, kWaves * kMaxBlocks / g.n_sx));
  g.n_sy = n_sy;
  g.rq = H / n_sy;
  g.rr = H % n_sy;
  g.grid = (g.n_sx * g.n_sy + kWaves - 1) / kWaves;
  return g;
}

template <class E>
class ImplT final : public Impl {
 public:
  using T = typename E::Real;
  // fused PCG kernels: the generic one (grid operators of radius 1) and the
  // residual-streaming one for shape from shading (radius 2)
  static constexpr bool kSfs = std::is_same_v<E, ShapeFromShading<T>>;
  static constexpr bool kFusedOk = !E::kGraph && (E::kRadius == 1 || kSfs);
  // graph energies with the fused graph kernel's hooks
  static constexpr bool kGFused = E::kGraph && GraphFusedOf<E>::value;
  static constexpr int kCols = kSfs ? kSfsCols : kStripCols;
  ImplT(opt_problem* p, const E& e) : p_(p), e_(e) {}

  Precond<T> pc(PrecondArgs a) const {
    Precond<T> c = blank<Precond<T>>();
    c.lam = (T)a.lam;
    c.dmin = (T)a.dmin;
    c.use = a.use;
    c.dmax = (T)a.dmax;
    return c;
  }
  T* vec(size_t off) const { return (T*)p_->at(off); }
  T* pbuf(int k) const { return vec((k & 1) ? p_->L.p1 : p_->L.p0); }
  T* rbuf(int k) const { return vec((k & 1) ? p_->L.r1 : p_->L.r0); }
  T* damp(PrecondArgs pa) const { return pa.damped ? vec(p_->L.damp) : nullptr; }
  int nblk() const { return p_->nblk; }

  // ------------------------------------------------ argument builders
  LinArgs<E> lin_args(const void* x, int lm) const {
    LinArgs<E> a = blank<LinArgs<E>>();
    a.e = e_;
    a.x = (const T*)x;
    a.part = p_->part(P_LIN);
    a.S = p_->S();
    a.lm_gate = lm;
    return a;
  }
  InitArgs<E> init_args(const void* x, double* trace, PrecondArgs pa, int lm, int u_form) const {
    InitArgs<E> a = blank<InitArgs<E>>();
    a.e = e_;
    a.x = (const T*)x;
    a.o = InitOut<T>{rbuf(0), vec(p_->L.diag), vec(p_->L.minv), damp(pa), vec(p_->L.delta)};
    a.lin_part = p_->part(P_LIN);
    a.n_lin = p_->nblk;
    a.rz_part = p_->part(P_RZ0);
    a.S = p_->S();
    a.trace = trace;
    a.pc = pc(pa);
    a.lm_gate = lm;
    a.u_form = u_form;
    return a;
  }
  SplitBufs<T> split_bufs(PrecondArgs pa) const {
    SplitBufs<T> b = blank<SplitBufs<T>>();
    b.r = rbuf(0);
    b.minv = vec(p_->L.minv);
    b.damp = damp(pa);
    b.p[0] = pbuf(0);
    b.p[1] = pbuf(1);
    b.q = vec(p_->L.q);
    b.rz_part[0] = p_->part(P_RZ0);
    b.rz_part[1] = p_->part(P_RZ1);
    b.pq_part = p_->part(P_PQ);
    return b;
  }
  template <int MODE>
  SplitAArgs<E, MODE> split_a_args(const SplitBufs<T>& b, int L, int lm) const {
    SplitAArgs<E, MODE> a = blank<SplitAArgs<E, MODE>>();
    a.e = e_;
    a.b = b;
    a.n_part = p_->nblk;
    a.S = p_->S();
    a.lm_gate = lm;
    a.L = L;
    return a;
  }
  SplitAArgs<E, 0> pcga_args(int L, PrecondArgs pa, int lm) const {
    return split_a_args<0>(split_bufs(pa), L, lm);
  }
  SplitBArgs<T, E::C> pcgb_args(int L, int lm) const {
    SplitBArgs<T, E::C> a = blank<SplitBArgs<T, E::C>>();
    a.n = e_.n;
    a.delta = vec(p_->L.delta);
    a.r = rbuf(0);
    a.p[0] = pbuf(0);
    a.p[1] = pbuf(1);
    a.q = vec(p_->L.q);
    a.minv = vec(p_->L.minv);
    a.pq_part = p_->part(P_PQ);
    a.rz_part[0] = p_->part(P_RZ0);
    a.rz_part[1] = p_->part(P_RZ1);
    a.n_part = p_->nblk;
    a.S = p_->S();
    a.lm_gate = lm;
    a.L = L;
    return a;
  }
  // Waves per SIMD the fused kernel can hold (blocks per CU of four waves).
  template <bool DAMP>
  static int fused_occupancy() {
    static const int occ = [] {
      int blocks = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<FusedArgs<E, DAMP>>, kBlock, 0) !=
          hipSuccess)
        return 1;
      return std::max(1, blocks * kWaves / 4);
    }();
    return occ;
  }
  StripGeom geom(bool damped) const {
    if constexpr (E::kGraph) {
      (void)damped;
      return StripGeom{};
    } else if constexpr (!kFusedOk) {
      (void)damped;
      return strip_geom(e_.W, e_.H, p_->tune, p_->n_simd, 1, kStripCols);
    } else {
      return strip_geom(e_.W, e_.H, p_->tune, p_->n_simd,
                        damped ? fused_occupancy<true>() : fused_occupancy<false>(), kCols);
    }
  }

  template <bool DAMP, bool BIG = false>
  FusedArgs<E, DAMP, BIG> fused_args(int L, PrecondArgs pa, int lm, int* grid) const {
    const StripGeom g = geom(DAMP);
    FusedArgs<E, DAMP, BIG> a = blank<FusedArgs<E, DAMP, BIG>>();
    a.e = e_;
    a.b.u[0] = rbuf(0);
    a.b.u[1] = rbuf(1);
    a.b.p[0] = pbuf(0);
    a.b.p[1] = pbuf(1);
    a.b.x = vec(p_->L.delta);
    a.b.part[0] = p_->part(P_F0);
    a.b.part[1] = p_->part(P_F1);
    a.b.diag = vec(p_->L.diag);
    a.pc = pc(pa);
    a.n_part = g.grid;
    a.S = p_->S();
    a.lm_gate = lm;
    a.n_sx = g.n_sx;
    a.n_sy = g.n_sy;
    a.sw = g.sw;
    a.rq = g.rq;
    a.rr = g.rr;
    a.L = L;
    *grid = g.grid;
    return a;
  }
  // Blocks per CU the fused graph kernel holds (its LDS decides).
  template <bool DAMP>
  static int gfused_blocks_per_cu() {
    static const int occ = [] {
      int blocks = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<GraphFusedArgs<E, DAMP>>, kBlock, 0) !=
          hipSuccess)
        return 1;
      return std::max(1, blocks);
    }();
    return occ;
  }
  // One block per chunk, at most as many as are resident at once (each then
  // walks its chunks with a fixed stride) and at most kMaxBlocks.
  int gfused_grid(bool damped) const {
    const int nch = (e_.n + kBlock - 1) / kBlock;
    const int per_cu = damped ? gfused_blocks_per_cu<true>() : gfused_blocks_per_cu<false>();
    return std::max(1, std::min({nch, kMaxBlocks, per_cu * std::max(1, p_->n_simd / 4)}));
  }
  template <bool DAMP>
  GraphFusedArgs<E, DAMP> gfused_args(int L, PrecondArgs pa, int lm, int* grid) const {
    GraphFusedArgs<E, DAMP> a = blank<GraphFusedArgs<E, DAMP>>();
    a.e = e_;
    a.b.u[0] = rbuf(0);
    a.b.u[1] = rbuf(1);
    a.b.p[0] = pbuf(0);
    a.b.p[1] = pbuf(1);
    a.b.x = vec(p_->L.delta);
    a.b.part[0] = p_->part(P_F0);
    a.b.part[1] = p_->part(P_F1);
    a.b.diag = vec(p_->L.diag);
    a.gl.rows = (const int*)p_->at(p_->L.gfz);
    a.pc = pc(pa);
    a.S = p_->S();
    a.lm_gate = lm;
    a.L = L;
    *grid = gfused_grid(DAMP);
    a.n_part = *grid;
    return a;
  }
  StepArgs<E> step_args(void* x, int lm) const {
    StepArgs<E> a = blank<StepArgs<E>>();
    a.e = e_;
    a.x = (T*)x;
    a.delta = vec(p_->L.delta);
    a.S = p_->S();
    a.lm_gate = lm;
    return a;
  }
  CostArgs<E> cost_args(const void* x, const void* delta, int lm) const {
    CostArgs<E> a = blank<CostArgs<E>>();
    a.e = e_;
    a.x = (const T*)x;
    a.delta = (const T*)delta;
    a.part = p_->part(P_COST);
    a.S = p_->S();
    a.lm_gate = lm;
    return a;
  }
  ModelArgs<E> model_args(const void* x) const {
    ModelArgs<E> a = blank<ModelArgs<E>>();
    a.e = e_;
    a.x = (const T*)x;
    a.delta = vec(p_->L.delta);
    a.part = p_->part(P_M);
    a.S = p_->S();
    return a;
  }

  // ------------------------------------------------ single-problem launches
  template <class A>
  int go(int kind, const A& a, int grid, int iter, const char* name) {
    return launch_row(p_, kind, a, grid, iter, name);
  }

  int linearize(const void* x, int lm) override {
    xlin_ = (const T*)x;
    return go(ROW_LIN, lin_args(x, lm), nblk(), 0, "linearize");
  }
  int init(const void* x, double* trace, PrecondArgs pa, int lm, int u_form) override {
    return go(ROW_INIT, init_args(x, trace, pa, lm, u_form), nblk(), 0, "init");
  }
  int pcg_a(int k, int L, PrecondArgs pa, int lm) override {
    return go(ROW_PCGA, pcga_args(L, pa, lm), nblk(), k, "pcg_a");
  }
  int pcg_b(int k, int L, PrecondArgs, int lm) override {
    return go(ROW_PCGB, pcgb_args(L, lm), nblk(), k, "pcg_b");
  }
  bool has_recompute() const override { return kSfs; }
  int pcg_a_recompute(int k, int L, PrecondArgs pa, int lm) override {
    if constexpr (!kSfs) {
      return fail(OPT_EUNSUPPORTED, "OPT_PCG_RECOMPUTE is built for shape from shading only");
    } else {
      if (!xlin_) return fail(OPT_EINVAL, "OPT_PCG_RECOMPUTE needs a linearisation point");
      SplitAArgs<ShapeFromShadingLit<T>, 0> a = blank<SplitAArgs<ShapeFromShadingLit<T>, 0>>();
      static_cast<ShapeFromShading<T>&>(a.e) = e_;
      a.e.xlin = xlin_;
      const SplitAArgs<E, 0> b = pcga_args(L, pa, lm);
      a.b = b.b;
      a.n_part = b.n_part;
      a.S = b.S;
      a.lm_gate = b.lm_gate;
      a.L = b.L;
      return go(ROW_PCGA_LIT, a, nblk(), k, "pcg_a_recompute");
    }
  }
  // ------------------------------------------------ materialised form
  bool has_mat() const override { return MatOf<E>::value; }
  MatBufs<T> mat_bufs() const {
    MatBufs<T> m = blank<MatBufs<T>>();
    m.val = vec(p_->L.jval);
    m.col = (const int*)p_->at(p_->L.jcol);
    m.jt = (const int*)p_->at(p_->L.jt);
    m.y = vec(p_->L.jy);
    m.rows = (long long)e_.n * p_->sh.mat_rows;
    return m;
  }
  int eval_j() override {
    if constexpr (!MatOf<E>::value) {
      return fail(OPT_EUNSUPPORTED, "no materialised Jacobian for this energy");
    } else {
      EvalJArgs<E> a = blank<EvalJArgs<E>>();
      a.e = e_;
      a.val = vec(p_->L.jval);
      a.col = (int*)p_->at(p_->L.jcol);
      a.jt = (int*)p_->at(p_->L.jt);
      return go(ROW_EVALJ, a, nblk(), 0, "eval_j");
    }
  }
  // p_k, then y = J p_k (one thread per row, over as many blocks as rows fill)
  int mat_a(int k, int L, PrecondArgs, int lm) override {
    if constexpr (!MatOf<E>::value) {
      return fail(OPT_EUNSUPPORTED, "no materialised Jacobian for this energy");
    } else {
      MatPArgs<T, E::C> ap = blank<MatPArgs<T, E::C>>();
      ap.n = e_.n;
      ap.r = rbuf(0);
      ap.minv = vec(p_->L.minv);
      ap.p[0] = pbuf(0);
      ap.p[1] = pbuf(1);
      ap.rz_part[0] = p_->part(P_RZ0);
      ap.rz_part[1] = p_->part(P_RZ1);
      ap.n_part = p_->nblk;
      ap.S = p_->S();
      ap.lm_gate = lm;
      ap.L = L;
      TRY(go(ROW_MATP, ap, nblk(), k, "mat_p"));
      MatAArgs<E> a = blank<MatAArgs<E>>();
      a.m = mat_bufs();
      a.p = pbuf(k);
      a.S = p_->S();
      a.lm_gate = lm;
      a.L = L;
      const long long blocks = (a.m.rows + kBlock - 1) / kBlock;
      return go(ROW_MATA, a, (int)std::min<long long>(blocks, 65535), k, "mat_a");
    }
  }
  int mat_b(int k, int L, PrecondArgs pa, int lm) override {
    if constexpr (!MatOf<E>::value) {
      return fail(OPT_EUNSUPPORTED, "no materialised Jacobian for this energy");
    } else {
      MatBArgs<E> a = blank<MatBArgs<E>>();
      a.m = mat_bufs();
      a.n = e_.n;
      a.p = pbuf(k);
      a.damp = damp(pa);
      a.q = vec(p_->L.q);
      a.pq_part = p_->part(P_PQ);
      a.S = p_->S();
      a.lm_gate = lm;
      a.L = L;
      return go(ROW_MATB, a, nblk(), k, "mat_b");
    }
  }
  // The fused kernels address memory through raw buffers whose in-range byte
  // offsets stay under 2^28.  Whole vectors (and the state) of at most 256 MB:
  // the regular instantiation.  Past that the radius-1 kernel's BIG
  // instantiation bases its buffers at each strip's first row, so only the
  // rows one strip touches (its own plus two halo rows each side) must span
  // less; the shape-from-shading kernel has no such form.
  bool whole_fits() const {
    const size_t rec = std::max<size_t>((size_t)E::C, (size_t)std::max(E::kStatePlanes, 1)) * sizeof(T);
    return rec * e_.n <= (size_t(1) << 28);
  }
  bool span_fits() const {
    const size_t rec = std::max<size_t>((size_t)E::C, (size_t)std::max(E::kStatePlanes, 1)) * sizeof(T);
    for (bool damped : {false, true}) {
      const StripGeom g = geom(damped);
      const size_t rows = (size_t)g.rq + (g.rr > 0 ? 1 : 0) + 4;
      if (rows * (size_t)e_.W * rec >= (size_t(1) << 28)) return false;
    }
    return true;
  }
  bool has_fused() const override {
    if constexpr (kGFused) {
      return p_->gfused;
    } else if constexpr (!kFusedOk) {
      return false;
    } else if constexpr (kSfs) {
      return whole_fits();
    } else {
      return whole_fits() || span_fits();
    }
  }
  bool fused_is_big() const override {
    if constexpr (!kFusedOk || kSfs) {
      return false;
    } else {
      return has_fused() && (!whole_fits() || (p_->tune.large_grid_form && span_fits()));
    }
  }
  // iter = -1 is the priming launch (it writes only partials).
  int fused(int iter, int L, PrecondArgs pa, int lm) override {
    if constexpr (kGFused) {
      if (!p_->gfused) return fail(OPT_EUNSUPPORTED, "the graph's lists do not fit the fused form");
      int grid = 0;
      if (pa.damped) return go(ROW_FUSED, gfused_args<true>(L, pa, lm, &grid), grid, iter, "fused");
      return go(ROW_FUSED, gfused_args<false>(L, pa, lm, &grid), grid, iter, "fused");
    } else if constexpr (!kFusedOk) {
      return fail(OPT_EUNSUPPORTED, "no fused PCG kernel for this energy");
    } else {
      int grid = 0;
      if constexpr (!kSfs) {
        if (fused_is_big()) {
          if (pa.damped) return go(ROW_FUSED, fused_args<true, true>(L, pa, lm, &grid), grid, iter, "fused");
          return go(ROW_FUSED, fused_args<false, true>(L, pa, lm, &grid), grid, iter, "fused");
        }
      }
      if (pa.damped) return go(ROW_FUSED, fused_args<true>(L, pa, lm, &grid), grid, iter, "fused");
      return go(ROW_FUSED, fused_args<false>(L, pa, lm, &grid), grid, iter, "fused");
    }
  }
  int apply_jtj(const void* pin, void* qout, PrecondArgs pa) override {
    SplitBufs<T> b = blank<SplitBufs<T>>();
    b.damp = damp(pa);
    b.p[0] = (T*)pin;
    b.q = (T*)qout;
    SplitAArgs<E, 1> a = split_a_args<1>(b, 1, 0);
    a.n_part = 0;
    return go(ROW_APPLY, a, nblk(), 0, "apply");
  }
  int apply_step(void* x, int lm) override { return go(ROW_STEP, step_args(x, lm), nblk(), 0, "step"); }
  int cost(const void* x, const void* delta, int lm) override {
    return go(delta ? ROW_TRIAL : ROW_COST, cost_args(x, delta, lm), nblk(), 0, "cost");
  }
  int model(const void* x) override { return go(ROW_MODEL, model_args(x), nblk(), 0, "model"); }
  StripGeom strip_geometry(bool damped) const override { return geom(damped); }
  double gpu_fill(bool use_fused, bool damped) const override {
    double waves = (double)nblk() * kWaves;
    int occ = 2;
    if constexpr (kGFused) {
      if (use_fused && has_fused()) {
        waves = (double)gfused_grid(damped) * kWaves;
        occ = std::max(1, (damped ? gfused_blocks_per_cu<true>() : gfused_blocks_per_cu<false>()) * kWaves / 4);
      }
    }
    if constexpr (kFusedOk) {
      if (use_fused && has_fused()) {
        const StripGeom g = geom(damped);
        waves = (double)g.n_sx * g.n_sy;
        occ = damped ? fused_occupancy<true>() : fused_occupancy<false>();
      }
    }
    return std::min(1.0, waves / ((double)occ * p_->n_simd));
  }
  int to_planes(const void* src, void* dst) override {
    PlanesArgs<T, E::C> a = blank<PlanesArgs<T, E::C>>();
    a.src = (const T*)src;
    a.dst = (T*)dst;
    a.n = e_.n;
    return go(ROW_PLANES, a, nblk(), 0, "to_planes");
  }

  // ------------------------------------------------ batched launches
  // Every problem keeps the grid it has alone, so its per-block partials and
  // results are the same bits in a batch as in a single-problem solve.
  template <class A, class F>
  static int rec(Batcher& B, const SlotRef* s, int n, F make, int lo, int hi, const char* name) {
    std::vector<A> rows((size_t)n);
    std::vector<int> grids((size_t)n);
    for (int k = 0; k < n; ++k) {
      const ImplT* im = static_cast<const ImplT*>(s[k].p->impl.get());
      rows[(size_t)k] = make(*im, s[k], &grids[(size_t)k]);
    }
    return batch_record(B, rows.data(), grids.data(), n, lo, hi, name);
  }

  int batch(Stage st, const SlotRef* s, int n, bool use_fused, Batcher& B) override {
    if (n <= 0) return OPT_OK;
    int Lmax = 0;
    for (int k = 0; k < n; ++k) Lmax = std::max(Lmax, s[k].L);
    switch (st) {
      case Stage::LIN:
        return rec<LinArgs<E>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
          *g = m.nblk();
          return m.lin_args(r.x, r.lm);
        }, 0, 1, "linearize[batch]");
      case Stage::INIT:
        return rec<InitArgs<E>>(B, s, n, [use_fused](const ImplT& m, const SlotRef& r, int* g) {
          *g = m.nblk();
          return m.init_args(r.x, r.p->trace(), r.pa, r.lm, use_fused ? 1 : 0);
        }, 0, 1, "init[batch]");
      case Stage::PCG:
        if (use_fused) {
          if constexpr (kGFused) {
            if (s[0].pa.damped)
              return rec<GraphFusedArgs<E, true>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
                return m.template gfused_args<true>(r.L, r.pa, r.lm, g);
              }, -1, Lmax, "fused[batch]");
            return rec<GraphFusedArgs<E, false>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
              return m.template gfused_args<false>(r.L, r.pa, r.lm, g);
            }, -1, Lmax, "fused[batch]");
          } else if constexpr (!kFusedOk) {
            return fail(OPT_EUNSUPPORTED, "no fused PCG kernel for this energy");
          } else {
            // one group holds problems of one method (the server keys groups by
            // it), so the damping form is the same for all
            if (s[0].pa.damped)
              return rec<FusedArgs<E, true>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
                return m.template fused_args<true>(r.L, r.pa, r.lm, g);
              }, -1, Lmax, "fused[batch]");
            return rec<FusedArgs<E, false>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
              return m.template fused_args<false>(r.L, r.pa, r.lm, g);
            }, -1, Lmax, "fused[batch]");
          }
        } else {
          // the two kernels of each iteration alternate, so record them in turn
          std::vector<SplitAArgs<E, 0>> ra((size_t)n);
          std::vector<SplitBArgs<T, E::C>> rb((size_t)n);
          std::vector<int> grids((size_t)n);
          for (int k = 0; k < n; ++k) {
            const ImplT* im = static_cast<const ImplT*>(s[k].p->impl.get());
            ra[(size_t)k] = im->pcga_args(s[k].L, s[k].pa, s[k].lm);
            rb[(size_t)k] = im->pcgb_args(s[k].L, s[k].lm);
            grids[(size_t)k] = im->nblk();
          }
          BatchTable<SplitAArgs<E, 0>> ta;
          BatchTable<SplitBArgs<T, E::C>> tb;
          TRY(batch_table(B, ra.data(), grids.data(), n, &ta));
          TRY(batch_table(B, rb.data(), grids.data(), n, &tb));
          hipStream_t stream = B.stream;
          for (int it = 0; it < Lmax; ++it)
            B.push([=]() -> int {
              TRY(batch_launch(ta, it, stream, "pcg_a[batch]"));
              return batch_launch(tb, it, stream, "pcg_b[batch]");
            });
          return OPT_OK;
        }
      case Stage::MODEL:
        return rec<ModelArgs<E>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
          *g = m.nblk();
          return m.model_args(r.x);
        }, 0, 1, "model[batch]");
      case Stage::TRIAL_COST:
        return rec<CostArgs<E>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
          *g = m.nblk();
          return m.cost_args(r.x, r.p->at(r.p->L.delta), 1);
        }, 0, 1, "trial_cost[batch]");
      case Stage::STEP:
        return rec<StepArgs<E>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
          *g = m.nblk();
          return m.step_args(r.x, r.lm);
        }, 0, 1, "step[batch]");
      case Stage::COST:
        return rec<CostArgs<E>>(B, s, n, [](const ImplT& m, const SlotRef& r, int* g) {
          *g = m.nblk();
          return m.cost_args(r.x, nullptr, 0);
        }, 0, 1, "cost[batch]");
    }
    return fail(OPT_EINVAL, "unknown stage");
  }

 private:
  opt_problem* p_;
  E e_;
  const T* xlin_ = nullptr;  // the last linearisation point (OPT_PCG_RECOMPUTE reads it)
};

// The staging lists build_incidence writes after the incidence list.
Halo halo_of(const opt_problem* p) {
  Halo h;
  h.nbl = (const int*)p->at(p->L.halo);
  h.hcnt = h.nbl + 2 * (size_t)p->sh.n_edges;
  h.hid = h.hcnt + (p->sh.n + kBlock - 1) / kBlock;
  return h;
}

template <typename T>
std::unique_ptr<Impl> make_impl_t(opt_problem* p) {
  const opt_problem_desc& d = p->desc;
  switch (d.energy) {
    case OPT_E_ARAP_WARP: {
      if (d.domain == OPT_GRAPH) {
        ArapWarpGraph<T> e;
        e.n = p->sh.n;
        e.rp = (const int*)p->at(p->L.csr);
        e.nb = e.rp + (p->sh.n + 1);
        e.U = (const T*)d.arrays[0];
        e.Ct = (const T*)d.arrays[1];
        e.mask = (const uint8_t*)d.arrays[2];
        e.st = (T*)p->at(p->L.state);
        e.flags = (uint8_t*)p->at(p->L.flags);
        e.halo = halo_of(p);
        e.wf = (T)d.params[0];
        e.wr = (T)d.params[1];
        e.wf_d = d.params[0];
        e.wr_d = d.params[1];
        return std::unique_ptr<Impl>(new ImplT<ArapWarpGraph<T>>(p, e));
      }
      ArapWarp<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.U = (const T*)d.arrays[0];
      e.Ct = (const T*)d.arrays[1];
      e.mask = (const uint8_t*)d.arrays[2];
      e.st = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf = (T)d.params[0];
      e.wr = (T)d.params[1];
      e.wf_d = d.params[0];
      e.wr_d = d.params[1];
      return std::unique_ptr<Impl>(new ImplT<ArapWarp<T>>(p, e));
    }
    case OPT_E_POISSON: {
      Poisson<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.Tg = (const T*)d.arrays[0];
      e.mask = (const uint8_t*)d.arrays[1];
      e.flags = (uint8_t*)p->at(p->L.flags);
      return std::unique_ptr<Impl>(new ImplT<Poisson<T>>(p, e));
    }
    case OPT_E_FLOW: {
      OpticalFlow<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.I = (const T*)d.arrays[0];
      e.Ih = (const T*)d.arrays[1];
      e.Idx = (const T*)d.arrays[2];
      e.Idy = (const T*)d.arrays[3];
      e.jf = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf = (T)d.params[0];
      e.wr = (T)d.params[1];
      e.wf_d = d.params[0];
      e.wr_d = d.params[1];
      return std::unique_ptr<Impl>(new ImplT<OpticalFlow<T>>(p, e));
    }
    case OPT_E_SFS: {
      ShapeFromShading<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.D = (const T*)d.arrays[0];
      e.Im = (const T*)d.arrays[1];
      e.eR = (const uint8_t*)d.arrays[2];
      e.eC = (const uint8_t*)d.arrays[3];
      e.st = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.sw_p = std::sqrt(d.params[0]);
      e.sw_s = std::sqrt(d.params[1]);
      e.sw_g = std::sqrt(d.params[2]);
      e.fx = d.params[3];
      e.fy = d.params[4];
      e.ux = d.params[5];
      e.uy = d.params[6];
      for (int k = 0; k < 9; ++k) e.L[k] = d.params[7 + k];
      e.sw_pT = (T)e.sw_p;
      e.sw_sT = (T)e.sw_s;
      e.sw_gT = (T)e.sw_g;
      return std::unique_ptr<Impl>(new ImplT<ShapeFromShading<T>>(p, e));
    }
    case OPT_E_LAPLACIAN: {
      if (d.domain == OPT_GRAPH) {
        LaplacianGraph<T> e;
        e.n = p->sh.n;
        e.rp = (const int*)p->at(p->L.csr);
        e.nb = e.rp + (p->sh.n + 1);
        e.A = (const T*)d.arrays[0];
        e.flags = (uint8_t*)p->at(p->L.flags);
        e.wf2 = (T)(d.params[0] * d.params[0]);
        e.wr2 = (T)(d.params[1] * d.params[1]);
        e.wf_d = d.params[0];
        e.wr_d = d.params[1];
        return std::unique_ptr<Impl>(new ImplT<LaplacianGraph<T>>(p, e));
      }
      LaplacianGrid<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.A = (const T*)d.arrays[0];
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf2 = (T)(d.params[0] * d.params[0]);
      e.wr2 = (T)(d.params[1] * d.params[1]);
      e.wf_d = d.params[0];
      e.wr_d = d.params[1];
      return std::unique_ptr<Impl>(new ImplT<LaplacianGrid<T>>(p, e));
    }
    case OPT_E_LP_SMOOTH: {
      LpSmoothGrid<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.A = (const T*)d.arrays[0];
      e.st = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf2 = (T)(d.params[0] * d.params[0]);
      e.wr2 = (T)(d.params[1] * d.params[1]);
      e.wf_d = d.params[0];
      e.wr_d = d.params[1];
      e.p_d = d.params[2];
      e.eps2_d = d.params[3] * d.params[3];
      return std::unique_ptr<Impl>(new ImplT<LpSmoothGrid<T>>(p, e));
    }
    case OPT_E_INTRINSIC: {
      IntrinsicImage<T> e;
      e.W = d.width;
      e.H = d.height;
      e.n = p->sh.n;
      e.I = (const T*)d.arrays[0];
      e.st = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf2 = (T)(d.params[0] * d.params[0]);
      e.wa2 = (T)(d.params[1] * d.params[1]);
      e.ws2 = (T)(d.params[2] * d.params[2]);
      e.wf_d = d.params[0];
      e.wa_d = d.params[1];
      e.ws_d = d.params[2];
      e.p_d = d.params[3];
      e.eps2_d = d.params[4] * d.params[4];
      return std::unique_ptr<Impl>(new ImplT<IntrinsicImage<T>>(p, e));
    }
    case OPT_E_ARAP_VOLUME: {
      ArapVolume<T> e;
      e.n = p->sh.n;
      e.W = d.width;
      e.H = d.height;
      e.D = d.depth;
      e.U = (const T*)d.arrays[0];
      e.Ct = (const T*)d.arrays[1];
      e.trig = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf = (T)d.params[0];
      e.wr = (T)d.params[1];
      e.wf_d = d.params[0];
      e.wr_d = d.params[1];
      return std::unique_ptr<Impl>(new ImplT<ArapVolume<T>>(p, e));
    }
    case OPT_E_ARAP_MESH: {
      ArapMesh<T> e;
      e.n = p->sh.n;
      e.rp = (const int*)p->at(p->L.csr);
      e.nb = e.rp + (p->sh.n + 1);
      e.halo = halo_of(p);
      e.U = (const T*)d.arrays[0];
      e.Ct = (const T*)d.arrays[1];
      e.trig = (T*)p->at(p->L.state);
      e.flags = (uint8_t*)p->at(p->L.flags);
      e.wf = (T)d.params[0];
      e.wr = (T)d.params[1];
      e.wf_d = d.params[0];
      e.wr_d = d.params[1];
      return std::unique_ptr<Impl>(new ImplT<ArapMesh<T>>(p, e));
    }
    default:
      return nullptr;
  }
}

std::unique_ptr<Impl> make_impl(opt_problem* p) {
  if (p->desc.precision == OPT_FP64) return make_impl_t<double>(p);
  return make_impl_t<float>(p);
}

}  // namespace

// Graph domain: the per-vertex incidence list (CSR) and the staging lists, as
// one host array (graph_lists.h has the layout and the builders).
lists::GraphShape graph_shape(const Shape& sh) {
  return lists::GraphShape{sh.n, sh.n_edges, halo_cap(sh.tsize, sh.stage_w), sh.gfz};
}

size_t incidence_words(const Shape& sh) { return lists::words(graph_shape(sh)); }

int build_incidence_host(const Shape& sh, const int* edges, int* out, bool* gfused) {
  const long long bad = lists::build(graph_shape(sh), edges, out, gfused);
  if (bad >= 0)
    return fail(OPT_EINVAL, "edge %lld = (%d, %d) names a vertex outside [0, %d)", bad, edges[2 * bad],
                edges[2 * bad + 1], sh.n);
  return OPT_OK;
}

// Enqueue the copies of the incidence arrays into the workspace on the
// problem's stream (`words` must stay valid until they have run).
int upload_incidence(opt_problem* p, const int* words) {
  const size_t V = (size_t)p->sh.n, E = (size_t)p->sh.n_edges;
  const size_t csr = V + 1 + 2 * E, total = incidence_words(p->sh);
  const size_t gfz = p->sh.gfz ? gfz_words(p->sh) : 0, halo = total - csr - gfz;
  HIP_TRY(hipMemcpyAsync(p->at(p->L.csr), words, sizeof(int) * csr, hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->at(p->L.halo), words + csr, sizeof(int) * halo, hipMemcpyHostToDevice, p->stream));
  if (gfz)
    HIP_TRY(hipMemcpyAsync(p->at(p->L.gfz), words + csr + halo, sizeof(int) * gfz, hipMemcpyHostToDevice,
                           p->stream));
  return OPT_OK;
}

// Copy the edge list to the host (on the problem's stream, behind the work
// already there), build the lists and upload them; synchronises the stream.
int build_incidence(opt_problem* p) {
  const int E = p->sh.n_edges;
  std::vector<int> edges((size_t)2 * E), words(incidence_words(p->sh));
  if (E > 0) {
    HIP_TRY(hipMemcpyAsync(edges.data(), p->desc.edges, sizeof(int) * 2 * (size_t)E, hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  bool gfused = false;
  TRY(build_incidence_host(p->sh, edges.data(), words.data(), &gfused));
  TRY(upload_incidence(p, words.data()));
  p->gfused = gfused;
  HIP_TRY(hipStreamSynchronize(p->stream));
  return OPT_OK;
}

int problem_init(opt_problem* p, const opt_problem_desc* desc, const Shape& sh, void* workspace,
                 hipStream_t stream, bool defer_graph) {
  p->desc = *desc;
  p->sh = sh;
  p->L = make_layout(sh);
  p->stream = stream;
  p->ws = (char*)workspace;
  p->nblk = (int)std::min<long long>(kMaxBlocks, (sh.n + kBlock - 1) / kBlock);
  if (p->nblk < 1) p->nblk = 1;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  p->n_simd = std::max(1, cus) * 4;  // four SIMDs per compute unit
  p->impl = make_impl(p);
  if (!p->impl) return fail(OPT_EUNSUPPORTED, "energy %d is not built", desc->energy);
  if (sh.graph && !defer_graph) TRY(build_incidence(p));
  TRY(launch_row(p, ROW_SETUP, setup_args(p->S(), 0.0, 1.0, 0, 0.0), 1, 0, "setup"));
  return OPT_OK;
}

int check_tuning(const opt_tuning* t) {
  if (t->strip_rows < 0 || t->strip_rows > (1 << 20))
    return fail(OPT_EINVAL, "strip_rows %d outside [0, 2^20]", t->strip_rows);
  if (t->waves_per_simd < 0 || t->waves_per_simd > 64)
    return fail(OPT_EINVAL, "waves_per_simd %d outside [0, 64]", t->waves_per_simd);
  if (t->large_grid_form != 0 && t->large_grid_form != 1)
    return fail(OPT_EINVAL, "large_grid_form %d is not 0 or 1", t->large_grid_form);
  return OPT_OK;
}

// A method the energy offers: the IRLS energy takes Gauss-Newton steps only.
int check_method(const opt_problem_desc* d, const opt_solve_params* sp) {
  if ((d->energy == OPT_E_LP_SMOOTH || d->energy == OPT_E_INTRINSIC) && sp->method == OPT_LM)
    return fail(OPT_EUNSUPPORTED, "energy %d is solved by IRLS, which takes Gauss-Newton steps", d->energy);
  return OPT_OK;
}

int check_params(const opt_solve_params* sp) {
  if (!sp) return fail(OPT_EINVAL, "solve params are NULL");
  if (sp->method != OPT_GN && sp->method != OPT_LM)
    return fail(OPT_EINVAL, "method %d is not OPT_GN or OPT_LM", sp->method);
  if (sp->outer_iters < 0 || sp->outer_iters > kMaxOuter)
    return fail(OPT_EINVAL, "outer_iters %d outside [0, %d]", sp->outer_iters, kMaxOuter);
  if (sp->pcg_iters < 0 || sp->pcg_iters > 1000000)
    return fail(OPT_EINVAL, "pcg_iters %d outside [0, 1000000]", sp->pcg_iters);
  if (sp->method == OPT_LM) {
    if (!(sp->lm_radius0 > 0) || !(sp->lm_radius_max > 0) || !(sp->lm_radius_min >= 0))
      return fail(OPT_EINVAL, "LM radii must be positive");
  }
  if (sp->pcg_variant < OPT_PCG_FUSED || sp->pcg_variant > OPT_PCG_RECOMPUTE)
    return fail(OPT_EINVAL, "pcg_variant %d is not an opt_pcg_variant", sp->pcg_variant);
  if (!(sp->lm_diag_min >= 0) || !(sp->lm_diag_max >= sp->lm_diag_min))
    return fail(OPT_EINVAL, "LM diagonal clamp [%g, %g] is invalid", sp->lm_diag_min,
                sp->lm_diag_max);
  return OPT_OK;
}

namespace {

int sync_scalars(opt_problem* p, DevScalars* hs) {
  HIP_TRY(hipMemcpyAsync(hs, p->S(), sizeof(DevScalars), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return OPT_OK;
}

// Record the next profiling event on the problem's stream.
int record_event(opt_problem* p) {
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    p->ev_pool.push_back(e);
  }
  HIP_TRY(hipEventRecord(p->ev_pool[p->ev_used], p->stream));
  p->ev_used++;
  return OPT_OK;
}

// The L iterations of the inner solve after init, in the chosen form.  Energies
// whose operator reaches further than one site (shape from shading) always use
// the split form.
// Whether the inner solve runs in the fused form (which starts from u_0 = M^-1 b).
int uses_fused(opt_problem* p, int variant) {
  return variant == OPT_PCG_FUSED && p->impl->has_fused() ? 1 : 0;
}

int run_pcg(opt_problem* p, PrecondArgs pa, int lm, int L, int variant) {
  if (variant == OPT_PCG_RECOMPUTE) {
    if (!p->impl->has_recompute())
      return fail(OPT_EUNSUPPORTED, "OPT_PCG_RECOMPUTE is built for shape from shading only");
    for (int k = 0; k < L; ++k) {
      TRY(p->impl->pcg_a_recompute(k, L, pa, lm));
      TRY(p->impl->pcg_b(k, L, pa, lm));
    }
    return OPT_OK;
  }
  if (variant == OPT_PCG_MATERIALIZED) {
    if (!p->sh.mat) return fail(OPT_EINVAL, "OPT_PCG_MATERIALIZED needs a problem created with materialize = 1");
    TRY(p->impl->eval_j());
    for (int k = 0; k < L; ++k) {
      TRY(p->impl->mat_a(k, L, pa, lm));
      TRY(p->impl->mat_b(k, L, pa, lm));
      TRY(p->impl->pcg_b(k, L, pa, lm));
    }
    return OPT_OK;
  }
  if (uses_fused(p, variant)) {
    if (L > 0) TRY(p->impl->fused(-1, L, pa, lm));
    for (int i = 0; i < L; ++i) TRY(p->impl->fused(i, L, pa, lm));
  } else {
    for (int k = 0; k < L; ++k) {
      TRY(p->impl->pcg_a(k, L, pa, lm));
      TRY(p->impl->pcg_b(k, L, pa, lm));
    }
  }
  return OPT_OK;
}


// Enqueue the whole solve of Sec. 4 on a created problem: setup, K outer
// iterations (linearise, init, L PCG iterations, LM decision, update), final
// cost.  Every decision inside is taken on the device.
int enqueue_solve(opt_problem* p, void* x, const opt_solve_params* sp) {
  const int K = sp->outer_iters, Lp = sp->pcg_iters;
  const int lm = sp->method == OPT_LM;
  double* trace = p->trace();
  TRY(launch_row(p, ROW_SETUP, setup_args(p->S(), 0.0, sp->lm_radius0, lm, sp->lm_radius_min), 1, 0, "setup"));
  PrecondArgs pa{0.0, sp->lm_diag_min, sp->lm_diag_max, sp->use_precond, lm != 0};
  for (int k = 0; k < K; ++k) {
    TRY(p->impl->linearize(x, lm));
    TRY(p->impl->init(x, trace, pa, lm, uses_fused(p, sp->pcg_variant)));
    if (p->profile) TRY(record_event(p));
    TRY(run_pcg(p, pa, lm, Lp, sp->pcg_variant));
    if (p->profile) {
      TRY(record_event(p));
      p->prof_iters += Lp;
    }
    if (lm) {
      TRY(p->impl->model(x));
      TRY(p->impl->cost(x, p->at(p->L.delta), 1));
      TRY(launch_row(p, ROW_DECIDE, decide_args(p->S(), p->part(P_M), p->part(P_COST), p->nblk, *sp), 1, 0,
                      "decide"));
    }
    TRY(p->impl->apply_step(x, lm));
  }
  TRY(p->impl->cost(x, nullptr, 0));
  TRY(launch_row(p, ROW_FINISH, finish_args(p->S(), p->part(P_COST), p->nblk), 1, 0, "finish"));
  return OPT_OK;
}

bool same_params(const opt_solve_params& a, const opt_solve_params& b) {
  return a.method == b.method && a.outer_iters == b.outer_iters && a.pcg_iters == b.pcg_iters &&
         a.use_precond == b.use_precond && a.lm_radius0 == b.lm_radius0 && a.lm_radius_min == b.lm_radius_min &&
         a.lm_radius_max == b.lm_radius_max && a.lm_diag_min == b.lm_diag_min && a.lm_diag_max == b.lm_diag_max &&
         a.lm_min_rel_decrease == b.lm_min_rel_decrease && a.pcg_variant == b.pcg_variant;
}

bool same_key(const opt_problem::SolveKey& a, const opt_problem::SolveKey& b) {
  return a.valid && b.valid && a.x == b.x && same_params(a.sp, b.sp) && a.tune.strip_rows == b.tune.strip_rows &&
         a.tune.waves_per_simd == b.tune.waves_per_simd && a.tune.large_grid_form == b.tune.large_grid_form;
}

// Record the solve's launch sequence as a graph on the problem's private
// stream, instantiate it and launch it on the problem's stream.  Every argument
// row is stored inside the graph (the row cache is emptied first), so a replay
// does not depend on what other calls left in the rows.
int capture_solve(opt_problem* p, void* x, const opt_solve_params* sp, const opt_problem::SolveKey& key) {
  p->drop_graph();
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  // launch-shape queries (occupancy) are answered before recording starts
  (void)p->impl->gpu_fill(true, false);
  (void)p->impl->gpu_fill(true, true);
  for (auto& c : p->row_cache) c.clear();
  hipStream_t user = p->stream;
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  p->stream = p->cap_stream;
  const int rc = enqueue_solve(p, x, sp);
  p->stream = user;
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(p->cap_stream, &g);
  hipGraphExec_t ex = nullptr;
  hipError_t ei = hipSuccess;
  if (rc == OPT_OK && ec == hipSuccess) ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (rc != OPT_OK || ec != hipSuccess || ei != hipSuccess) {
    // nothing recorded was executed: no row is known to be stored
    for (auto& c : p->row_cache) c.clear();
    if (rc != OPT_OK) return rc;
    return fail(OPT_EHIP, "recording the solve as a graph failed: %s",
                hipGetErrorString(ec != hipSuccess ? ec : ei));
  }
  p->gexec = ex;
  p->gkey = key;
  p->rows_after_graph = p->row_cache;
  HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
  return OPT_OK;
}

// The whole solve (opt_solve): enqueue it (or replay its graph) and, if a
// report is asked for, read the scalars and the cost trace back.
int solve_problem(opt_problem* p, void* x, const opt_solve_params* sp, opt_solve_report* rep) {
  TRY(check_params(sp));
  TRY(check_method(&p->desc, sp));
  const int K = sp->outer_iters;
  const int lm = sp->method == OPT_LM;
  opt_problem::SolveKey key;
  key.x = x;
  key.sp = *sp;
  key.tune = p->tune;
  key.valid = true;
  const bool graphs = p->graphs && !p->profile;
  if (graphs && p->gexec && same_key(p->gkey, key)) {
    HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
    p->row_cache = p->rows_after_graph;
  } else if (graphs && same_key(p->last_eager, key)) {
    TRY(capture_solve(p, x, sp, key));
  } else {
    TRY(enqueue_solve(p, x, sp));
    p->last_eager = key;
  }
  p->last_x = nullptr;
  if (!rep) return OPT_OK;
  // the scalars and the cost trace come back in one synchronisation of the
  // problem's stream
  DevScalars hs;
  std::vector<double> tr((size_t)K + 1, 0.0);
  HIP_TRY(hipMemcpyAsync(&hs, p->S(), sizeof(DevScalars), hipMemcpyDeviceToHost, p->stream));
  if (K > 0)
    HIP_TRY(hipMemcpyAsync(tr.data(), p->trace(), sizeof(double) * (size_t)K, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  const int done = lm ? hs.outer_done : K;
  for (int k = done; k <= K; ++k) tr[(size_t)k] = hs.E_final;
  rep->cost_initial = K > 0 ? tr[0] : hs.E_final;
  rep->cost_final = hs.E_final;
  rep->outer_done = done;
  rep->steps_accepted = lm ? hs.n_accepted : K;
  if (rep->cost_trace) memcpy(rep->cost_trace, tr.data(), sizeof(double) * ((size_t)K + 1));
  if (hs.nonfinite) return fail(OPT_ENUMERIC, "a cost was NaN or infinite");
  return OPT_OK;
}

// ---------------------------------------------------------------- static scratch
// The workspace of opt_solve_scratch: one file-scope device array, which every
// GPU the library runs on holds (its own copy) until the process ends.  Host
// code never uses the array's name as an address: the device address of each
// GPU's copy is looked up once per device and kept.
constexpr size_t kScratchBytes = OPT_SCRATCH_BYTES;
static_assert(kScratchBytes % kAlign == 0, "scratch is a whole number of aligned blocks");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // by device ordinal; nullptr until looked up

int scratch_of_current_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[(size_t)dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr) % kAlign) return fail(OPT_EHIP, "static scratch has no usable address");
    g_scratch_ptr[(size_t)dev] = ptr;
  }
  *out = g_scratch_ptr[(size_t)dev];
  return OPT_OK;
}
}  // namespace

int solve(opt_problem* p, void* x, const opt_solve_params* sp, opt_solve_report* rep) {
  return solve_problem(p, x, sp, rep);
}

}  // namespace host
}  // namespace optmi

using namespace optmi;
using namespace optmi::host;

extern "C" {

const char* opt_last_error(void) { return last_error(); }

int opt_energy_channels(int32_t energy) { return energy_channels(energy); }

void opt_default_params(opt_solve_params* p) {
  if (!p) return;
  p->method = OPT_GN;
  p->outer_iters = 10;
  p->pcg_iters = 50;
  p->use_precond = 1;
  p->lm_radius0 = 1e4;
  p->lm_radius_min = 1e-32;
  p->lm_radius_max = 1e16;
  p->lm_diag_min = 1e-6;
  p->lm_diag_max = 1e32;
  p->lm_min_rel_decrease = 1e-3;
  p->pcg_variant = OPT_PCG_FUSED;
}

int opt_workspace_size(const opt_problem_desc* desc, size_t* bytes) {
  if (!bytes) return fail(OPT_EINVAL, "bytes is NULL");
  Shape sh;
  TRY(check_desc(desc, &sh));
  *bytes = make_layout(sh).total;
  return OPT_OK;
}

int opt_problem_create(const opt_problem_desc* desc, void* workspace, size_t workspace_bytes,
                       void* hip_stream, opt_problem** out) {
  if (!out) return fail(OPT_EINVAL, "out is NULL");
  *out = nullptr;
  Shape sh;
  TRY(check_desc(desc, &sh));
  const Layout L = make_layout(sh);
  if (!workspace) return fail(OPT_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace) % kAlign)
    return fail(OPT_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < L.total)
    return fail(OPT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes,
                L.total);
  std::unique_ptr<opt_problem> p(new (std::nothrow) opt_problem());
  if (!p) return fail(OPT_ENOMEM, "host allocation failed");
  TRY(problem_init(p.get(), desc, sh, workspace, (hipStream_t)hip_stream));
  *out = p.release();
  return OPT_OK;
}

int opt_problem_destroy(opt_problem* prob) {
  delete prob;
  return OPT_OK;
}

int opt_linearize(opt_problem* p, const void* x, double* cost) {
  if (!p || !x) return fail(OPT_EINVAL, "problem or unknowns is NULL");
  TRY(p->impl->linearize(x, 0));
  p->last_x = x;
  if (cost) {
    TRY(launch_row(p, ROW_FINISH, finish_args(p->S(), p->part(P_LIN), p->nblk), 1, 0, "finish"));
    DevScalars hs;
    TRY(sync_scalars(p, &hs));
    *cost = hs.E_final;
    if (!std::isfinite(hs.E_final)) return fail(OPT_ENUMERIC, "cost is not finite");
  }
  return OPT_OK;
}

int opt_eval_jtf(opt_problem* p, void* b_out, void* diag_out) {
  if (!p) return fail(OPT_EINVAL, "problem is NULL");
  if (!p->last_x) return fail(OPT_EINVAL, "opt_linearize has not been called");
  PrecondArgs pa{0.0, 0.0, 0.0, 1, false};
  TRY(p->impl->init(p->last_x, nullptr, pa, 0, 0));
  if (b_out) TRY(p->impl->to_planes(p->at(p->L.r0), b_out));
  if (diag_out) TRY(p->impl->to_planes(p->at(p->L.diag), diag_out));
  return OPT_OK;
}

int opt_apply_jtj(opt_problem* p, const void* pin, void* qout, double lambda,
                  const opt_solve_params* sp) {
  if (!p || !pin || !qout) return fail(OPT_EINVAL, "problem, p or q is NULL");
  if (!p->last_x) return fail(OPT_EINVAL, "opt_linearize has not been called");
  if (pin == qout) return fail(OPT_EINVAL, "p and q must not overlap");
  PrecondArgs pa{0.0, 0.0, 0.0, 1, false};
  if (lambda != 0.0) {
    if (!sp) return fail(OPT_EINVAL, "params are needed when lambda != 0");
    pa = PrecondArgs{lambda, sp->lm_diag_min, sp->lm_diag_max, 1, true};
    TRY(p->impl->init(p->last_x, nullptr, pa, 0, 0));
  }
  return p->impl->apply_jtj(pin, qout, pa);
}

int opt_pcg(opt_problem* p, const opt_solve_params* sp, double lambda, void* delta_out) {
  if (!p) return fail(OPT_EINVAL, "problem is NULL");
  TRY(check_params(sp));
  if (!p->last_x) return fail(OPT_EINVAL, "opt_linearize has not been called");
  PrecondArgs pa{lambda, sp->lm_diag_min, sp->lm_diag_max, sp->use_precond, lambda != 0.0};
  TRY(launch_row(p, ROW_SETUP, setup_args(p->S(), lambda, 1.0, 0, 0.0), 1, 0, "setup"));
  TRY(p->impl->init(p->last_x, nullptr, pa, 0, uses_fused(p, sp->pcg_variant)));
  TRY(run_pcg(p, pa, 0, sp->pcg_iters, sp->pcg_variant));
  if (delta_out) TRY(p->impl->to_planes(p->at(p->L.delta), delta_out));
  return OPT_OK;
}

int opt_problem_set_tuning(opt_problem* p, const opt_tuning* t) {
  if (!p || !t) return fail(OPT_EINVAL, "problem or tuning is NULL");
  TRY(check_tuning(t));
  p->tune = *t;
  return OPT_OK;
}

int opt_problem_set_graph_replay(opt_problem* p, int enable) {
  if (!p) return fail(OPT_EINVAL, "problem is NULL");
  p->graphs = enable != 0;
  if (!p->graphs) p->drop_graph();
  p->last_eager.valid = false;
  return OPT_OK;
}

int opt_problem_pcg_form(opt_problem* p, int variant, int* form) {
  if (!p || !form) return fail(OPT_EINVAL, "problem or form is NULL");
  if (variant < OPT_PCG_FUSED || variant > OPT_PCG_RECOMPUTE)
    return fail(OPT_EINVAL, "pcg_variant %d is not an opt_pcg_variant", variant);
  if (variant == OPT_PCG_RECOMPUTE && !p->impl->has_recompute())
    return fail(OPT_EUNSUPPORTED, "OPT_PCG_RECOMPUTE is built for shape from shading only");
  *form = variant == OPT_PCG_MATERIALIZED || variant == OPT_PCG_RECOMPUTE
              ? variant
              : (uses_fused(p, variant) ? OPT_PCG_FUSED : OPT_PCG_SPLIT);
  return OPT_OK;
}

int opt_problem_get_tuning(opt_problem* p, opt_tuning* t) {
  if (!p || !t) return fail(OPT_EINVAL, "problem or tuning is NULL");
  *t = p->tune;
  if (!p->sh.graph) {
    const StripGeom g = p->impl->strip_geometry(false);
    t->strip_rows = g.rq + (g.rr > 0 ? 1 : 0);
    t->waves_per_simd = (g.n_sx * g.n_sy + p->n_simd - 1) / p->n_simd;
  }
  return OPT_OK;
}

int opt_profile_enable(opt_problem* p, int enable) {
  if (!p) return fail(OPT_EINVAL, "problem is NULL");
  p->profile = enable != 0;
  return OPT_OK;
}

int opt_profile_read(opt_problem* p, double* pcg_ms, int64_t* pcg_iters) {
  if (!p || !pcg_ms || !pcg_iters) return fail(OPT_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(p->stream));
  double total = 0.0;
  for (size_t k = 0; k + 1 < p->ev_used; k += 2) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev_pool[k], p->ev_pool[k + 1]));
    total += ms;
  }
  *pcg_ms = total;
  *pcg_iters = p->prof_iters;
  p->ev_used = 0;
  p->prof_iters = 0;
  return OPT_OK;
}

int opt_cost(opt_problem* p, const void* x, double* cost) {
  if (!p || !x || !cost) return fail(OPT_EINVAL, "problem, unknowns or cost is NULL");
  TRY(p->impl->cost(x, nullptr, 0));
  TRY(launch_row(p, ROW_FINISH, finish_args(p->S(), p->part(P_COST), p->nblk), 1, 0, "finish"));
  DevScalars hs;
  TRY(sync_scalars(p, &hs));
  *cost = hs.E_final;
  if (!std::isfinite(hs.E_final)) return fail(OPT_ENUMERIC, "cost is not finite");
  return OPT_OK;
}

int opt_solve(opt_problem* p, void* x, const opt_solve_params* sp, opt_solve_report* rep) {
  if (!p || !x) return fail(OPT_EINVAL, "problem or unknowns is NULL");
  return solve_problem(p, x, sp, rep);
}

int opt_solve_scratch(const opt_problem_desc* desc, void* unknowns, const opt_solve_params* params,
                      opt_solve_report* report, void* hip_stream) {
  if (!unknowns) return fail(OPT_EINVAL, "unknowns is NULL");
  Shape sh;
  TRY(check_desc(desc, &sh));
  TRY(check_params(params));
  TRY(check_method(desc, params));
  const Layout L = make_layout(sh);
  if (L.total > kScratchBytes)
    return fail(OPT_ENOMEM, "the problem needs %zu bytes of workspace; the static scratch holds %zu",
                L.total, kScratchBytes);
  void* ws = nullptr;
  TRY(scratch_of_current_device(&ws));
  opt_problem p;
  TRY(problem_init(&p, desc, sh, ws, (hipStream_t)hip_stream));
  return solve_problem(&p, unknowns, params, report);
}

}  // extern "C"
