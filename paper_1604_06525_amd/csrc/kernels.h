// Kernels of one solve, generic over the energy.
//
// Each stage is an argument struct plus a device function run(args, grid, iter).
// k_batch launches one problem, or many problems of one kind at once, each over
// its own contiguous range of blocks, and gives every block the grid it would
// have had alone, so results do not depend on the batch.
//
// Kernel boundaries are the only grid-wide synchronisation.  A scalar that
// needs a sum over the whole problem is produced as per-block FP64 partials by
// one kernel and summed, in a fixed order, by every block of the next kernel, so
// no fence or atomic is needed and every run gives the same bits.
//
// Two forms of the preconditioned CG inner solve (Sec. 4.1) are built.
//
// Split (two kernels per iteration, the textbook recurrence):
//   pcg_a(k):  beta = rz_k / rz_{k-1} (k > 0);  p_k = z_k + beta p_{k-1}, z = M^-1 r,
//              evaluated for each site and the neighbours its product reads;
//              q = A p_k;  write p_k, q;  partials of p_k . q.
//   pcg_b(k):  alpha = rz_k / (p.q);  d += alpha p;  r -= alpha q;  partials of r.z.
//
// Fused (one kernel per iteration): the single-reduction recurrence of
// Chronopoulos and Gear, which gives the same iterates in exact arithmetic.  With
// u = M^-1 r, gamma = r.u and delta = u.(A u) summed by the previous kernel:
//   beta_i = gamma_i/gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i/alpha_{i-1})
//   p_i = u_i + beta_i p_{i-1};  s_i = A p_i;  d += alpha_i p_i;
//   u_{i+1} = u_i - alpha_i M^-1 s_i  (= M^-1 r_{i+1});
//   partials of gamma_{i+1} = r_{i+1}.u_{i+1} = sum M u_{i+1}^2 and of
//   delta_{i+1} = |J u_{i+1}|^2 + u_{i+1}.(lambda D) u_{i+1}.
// The kernel carries u instead of r, and M (the Jacobi diagonal, damped for LM)
// is recomputed per site from the state and flags it reads anyway, so neither r
// nor M^-1 is read.  s_i = A p_i is formed exactly (not by its own recurrence).
// Init writes u_0 = M^-1 b; a first "priming" launch (iter = -1, alpha = beta =
// 0, no stores) produces gamma_0 and delta_0.
//
// If the curvature p.Ap is not positive the solve stops (DevScalars::stopped):
// every later iteration kernel returns at once and d keeps its value.
#pragma once
#include <type_traits>
#include <utility>

#include "common.h"

namespace optmi {

// Element i (0 or 1) of a pair held in kernel arguments.  A select rather than
// an index: a runtime index into an argument struct copied to a local would put
// the whole struct in scratch memory.
template <typename P>
__device__ __forceinline__ P pick(P const (&pair)[2], int i) {
  return i ? pair[1] : pair[0];
}

// The unit of work of a block, XCD-aware: blocks go to the 8 XCDs round-robin
// (block b to XCD b % 8), and each XCD takes one contiguous run of units, so
// neighbouring sites (grid rows, Morton-ordered graph vertices) share its L2.
// XCD x holds q + (x < r) of the nb blocks (q = nb / 8, r = nb % 8); the map is
// a bijection of [0, nb).  (In a batch the hardware placement differs; only
// speed depends on it.)
__device__ __forceinline__ int unit_of_block(VG g) {
  const int q = g.nb >> 3, r = g.nb & 7, x = g.bid & 7;
  return x * q + min(x, r) + (g.bid >> 3);
}

// Grid-stride loop over sites with a fixed per-thread order (the grid size
// depends only on n), so the partial sums are reproducible; block b takes the
// chunks unit_of_block(b), + nb, ...
#define OPT_SITE_LOOP(s, n, g) \
  for (int s = unit_of_block(g) * kBlock + threadIdx.x; s < (n); s += (g).nb * kBlock)

// Views over global memory centred at site s = (vi_, vj_) of a W x H grid; every
// read off the grid returns 0 (flags 0: not on the grid).
#define OPT_GRID_VIEWS(e, s)                                                          \
  const int vi_ = (s) % (e).W, vj_ = (s) / (e).W;                                     \
  auto inb_ = [&](int di, int dj) {                                                   \
    const int ii = vi_ + di, jj = vj_ + dj;                                           \
    return ii >= 0 && ii < (e).W && jj >= 0 && jj < (e).H;                            \
  };                                                                                  \
  auto Fg = [&](int di, int dj) -> uint32_t {                                         \
    return inb_(di, dj) ? (uint32_t)(e).flags[(s) + dj * (e).W + di] : 0u;            \
  };                                                                                  \
  auto Sg = [&](int k, int di, int dj) -> typename E::Real {                          \
    return inb_(di, dj) ? (e).state_at(k, (s) + dj * (e).W + di) : typename E::Real(0);  \
  };

// b = -J^T F and diag(J^T J) at an active site s at the linearisation point x.
template <class E>
__device__ __forceinline__ void site_jtf_diag(const E& e, const typename E::Real* __restrict__ x,
                                              int s, typename E::Real* b, typename E::Real* d) {
  using T = typename E::Real;
  const int n = e.n;
  if constexpr (E::kGraph) {
    auto X = [&](int c, int v) -> T { return x[(size_t)c * n + v]; };
    e.jtf_diag_site(X, s, b, d);
  } else {
    OPT_GRID_VIEWS(e, s)
    auto Xg = [&](int c, int di, int dj) -> T {
      return inb_(di, dj) ? x[(size_t)c * n + s + dj * e.W + di] : T(0);
    };
    e.jtf_diag(Xg, Sg, Fg, s, vi_, vj_, b, d);
  }
}

// g = J^T J P at an active site s; P(c, site) reads the direction.
template <class E, class PA>
__device__ __forceinline__ void site_apply(const E& e, int s, PA P, typename E::Real* g) {
  using T = typename E::Real;
  if constexpr (E::kGraph) {
    e.apply_site(P, s, g);
  } else {
    OPT_GRID_VIEWS(e, s)
    auto Pv = [&](int c, int di, int dj) -> T {
      return inb_(di, dj) ? P(c, s + dj * e.W + di) : T(0);
    };
    e.apply(Pv, Sg, Fg, vi_, vj_, g);
  }
}

// ---------------------------------------------------------------- linearize
template <class E>
struct LinArgs {
  E e;
  const typename E::Real* x;
  double* part;
  const DevScalars* S;
  int lm_gate;
};

template <class E>
__device__ __forceinline__ void run(const LinArgs<E>& a, VG g, int) {
  if (a.lm_gate && (a.S->done || !a.S->need_lin)) return;
  double acc = 0.0;
  const int n = a.e.n;
  auto X = [&](int ch, int s) -> double { return (double)a.x[(size_t)ch * n + s]; };
  OPT_SITE_LOOP(s, n, g) {
    a.e.linearize(a.x, s);
    acc += a.e.cost(X, s);
  }
  block_store(acc, a.part, g);
}

// ---------------------------------------------------------------- init
// r = b = -J^T F, diag = diag(J^T J), M^-1 and (LM) the damping lambda*D, d = 0,
// and partials of r.z for the split form; also finishes the cost of the
// linearisation (trace entry) and resets the PCG state.
template <typename T>
struct InitOut {
  T* r;
  T* diag;
  T* minv;
  T* damp;   // nullptr unless LM
  T* delta;
};

template <class E>
struct InitArgs {
  E e;
  const typename E::Real* x;
  InitOut<typename E::Real> o;
  const double* lin_part;
  int n_lin;
  double* rz_part;
  DevScalars* S;
  double* trace;  // cost trace (entry S->trace_k), or nullptr
  Precond<typename E::Real> pc;
  int lm_gate;
  int u_form;  // fused form: write u_0 = M^-1 b (not b) to o.r
};

template <class E>
__device__ __forceinline__ void run(const InitArgs<E>& a, VG g, int) {
  using T = typename E::Real;
  constexpr int C = E::C;
  DevScalars* S = a.S;
  if (a.lm_gate && S->done) return;
  // LM re-solves at the same x after a rejected step: the cost is then kept.
  const bool fresh = !a.lm_gate || S->need_lin;
  double E0 = 0.0;
  if (fresh) E0 = reduce_partials(a.lin_part, a.n_lin);
  if (is_block_leader(g)) {
    if (fresh) {
      S->E0 = E0;
      if (!finite_d(E0)) S->nonfinite = 1;
    } else {
      E0 = S->E0;
    }
    if (a.trace) {
      a.trace[S->trace_k] = E0;
      S->trace_k += 1;
    }
    S->stopped = 0;
  }
  Precond<T> pc = a.pc;
  if (a.lm_gate) pc.lam = (T)S->lambda;
  const int n = a.e.n;
  double rz = 0.0;
  OPT_SITE_LOOP(s, n, g) {
    T b[C], d[C];
    if (a.e.flags[s] & E::ACTIVE) {
      site_jtf_diag(a.e, a.x, s, b, d);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) { b[c] = T(0); d[c] = T(0); }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t k = vix<C>(c, s);
      const T m = pc.minv(d[c]);
      a.o.r[k] = a.u_form ? m * b[c] : b[c];
      a.o.diag[k] = d[c];
      a.o.minv[k] = m;
      if (a.o.damp) a.o.damp[k] = pc.lam != T(0) ? pc.damp(d[c]) : T(0);
      a.o.delta[k] = T(0);
      rz += (double)b[c] * (double)(m * b[c]);
    }
  }
  block_store(rz, a.rz_part, g);
}

// ---------------------------------------------------------------- split: pcg_a
// Iteration k of the split form (MODE 0), or the plain product
// q = (J^T J + damp) p_in (MODE 1, with p_in in p[0] and q in the caller's
// channel-plane layout; the damping vector stays in the internal layout).
template <typename T>
struct SplitBufs {
  const T* r;
  const T* minv;
  const T* damp;   // nullptr: no damping
  T* p[2];         // iteration k writes p[k & 1] and reads p_{k-1} from p[(k + 1) & 1]
  T* q;
  double* rz_part[2];  // r.z partials of iteration k are read from rz_part[k & 1]
  double* pq_part;
};

// Graph energies whose pcg_a stages a chunk of vertices in LDS (E::kStaged).
template <class E, class = void>
struct StagedOf : std::false_type {};
template <class E>
struct StagedOf<E, std::void_t<decltype(E::kStaged)>> : std::bool_constant<E::kStaged> {};

template <class E, int MODE>
struct SplitAArgs {
  E e;
  SplitBufs<typename E::Real> b;
  int n_part;
  DevScalars* S;
  int lm_gate;
  int L;  // iterations of this problem; later ones return at once
};

template <class E, int MODE>
__device__ __forceinline__ void run(const SplitAArgs<E, MODE>& a, VG g, int k) {
  using T = typename E::Real;
  constexpr int C = E::C;
  const int n = a.e.n;
  const SplitBufs<T>& b = a.b;
  DevScalars* S = a.S;
  T beta = T(0);
  if (MODE == 0) {
    if (k >= a.L || S->stopped || (a.lm_gate && S->done)) return;
    const double rz = reduce_partials(pick(b.rz_part, k & 1), a.n_part);
    if (k > 0) beta = (T)(rz / S->rz[(k - 1) & 1]);
    if (is_block_leader(g)) S->rz[k & 1] = rz;
  }
  const T* pold = MODE == 1 ? b.p[0] : pick(b.p, (k + 1) & 1);
  T* pnew = pick(b.p, k & 1);
  auto Pg = [&](int c, int site) -> T {
    if (MODE == 1) return pold[(size_t)c * n + site];
    const size_t o = vix<C>(c, site);
    const T z = b.minv[o] * b.r[o];
    return k == 0 ? z : fma(beta, pold[o], z);
  };
  double pq = 0.0;
  // p, q and the partial of p.q at site s, given its p (pv) and (J^T J p)_s
  auto finish = [&](int s, bool act, const T* pv_in, const T* gv) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = vix<C>(c, s);
      T pv = T(0), qv = T(0);
      if (act) {
        pv = pv_in[c];
        qv = gv[c];
        if (b.damp) qv += b.damp[o] * pv;
      }
      if (MODE == 0) pnew[o] = pv;
      b.q[MODE == 1 ? (size_t)c * n + s : o] = qv;
      pq += (double)pv * (double)qv;
    }
  };
  if constexpr (StagedOf<E>::value) {
    // The block's chunk of vertices is staged in LDS first (their p and the
    // values the energy reads of a neighbour), after it the chunk's halo: the
    // outside neighbours listed for it when the problem was created (about 13%
    // of the edges of a Morton-ordered icosphere at 256 vertices per chunk
    // leave it), and the chunk's neighbour slots.  Every neighbour is then read
    // from LDS, except those of a chunk whose halo overflowed the cap (read
    // from global memory).
    constexpr int NS = E::kStageVals, H = halo_cap(sizeof(T), C + NS), NBC = nbl_cap(sizeof(T));
    __shared__ T sp[kBlock + H][C];
    __shared__ T sst[kBlock + H][NS];
    __shared__ int snb[NBC];
    const Halo& hl = a.e.halo;
    for (int chunk = unit_of_block(g); chunk * kBlock < n; chunk += g.nb) {
      const int v0 = chunk * kBlock, t = threadIdx.x, v = v0 + t;
      const bool in = v < n;
      // Every index the chunk needs is requested before any load that depends
      // on one: the halo count and the halo row (a fixed-stride row, read
      // whole), the chunk's and the vertex's incidence ranges, the flags.
      const int nh = hl.hcnt[chunk];
      const int* hrow = hl.hid + (size_t)chunk * H;
      const int kb = a.e.rp[v0], ke = a.e.rp[min(v0 + kBlock, n)];
      const int k0 = in ? a.e.rp[v] : 0, k1 = in ? a.e.rp[v + 1] : 0;
      const uint32_t fl = in ? (uint32_t)a.e.flags[v] : 0u;
      T pv[C];
#pragma unroll
      for (int c = 0; c < C; ++c) pv[c] = in ? Pg(c, v) : T(0);
      if (in) {
#pragma unroll
        for (int c = 0; c < C; ++c) sp[t][c] = pv[c];
        const Vals<T, NS> sv = a.e.stage_vals(v);
#pragma unroll
        for (int k2 = 0; k2 < NS; ++k2) sst[t][k2] = sv.v[k2];
      }
      for (int j = t; j < H; j += kBlock) {
        const int u = hrow[j];
        if (j < nh) {
#pragma unroll
          for (int c = 0; c < C; ++c) sp[kBlock + j][c] = Pg(c, u);
          const Vals<T, NS> sv = a.e.stage_vals(u);
#pragma unroll
          for (int k2 = 0; k2 < NS; ++k2) sst[kBlock + j][k2] = sv.v[k2];
        }
      }
      const int nk = min(ke - kb, NBC);
      for (int j = t; j < nk; j += kBlock) snb[j] = hl.nbl[kb + j];
      __syncthreads();
      // slot s >= 0: LDS; s < 0: vertex -s - 1 in global memory
      auto Pl = [&](int c, int s) -> T { return s >= 0 ? sp[s][c] : Pg(c, -s - 1); };
      auto Sl = [&](int s) {
        if (s < 0) return a.e.stage_vals(-s - 1);
        Vals<T, NS> r;
#pragma unroll
        for (int k2 = 0; k2 < NS; ++k2) r.v[k2] = sst[s][k2];
        return r;
      };
      auto NBl = [&](int k) { return k - kb < nk ? snb[k - kb] : hl.nbl[k]; };
      const bool act = in && (fl & E::ACTIVE);
      T gv[C];
      if (act) a.e.apply_staged(Pl, Sl, NBl, t, k0, k1, fl, gv);
      if (in) finish(v, act, pv, gv);
      __syncthreads();  // the next chunk reuses the stage
    }
  } else {
    OPT_SITE_LOOP(s, n, g) {
      T gv[C], pv[C];
      const bool act = a.e.flags[s] & E::ACTIVE;
      if (act) {
        site_apply(a.e, s, Pg, gv);
#pragma unroll
        for (int c = 0; c < C; ++c) pv[c] = Pg(c, s);
      }
      finish(s, act, pv, gv);
    }
  }
  if (MODE == 0) block_store(pq, b.pq_part, g);
}

// ---------------------------------------------------------------- split: pcg_b
template <typename T, int C>
struct SplitBArgs {
  int n;
  T* delta;
  T* r;
  T* p[2];
  const T* q;
  const T* minv;
  const double* pq_part;
  double* rz_part[2];  // iteration k writes rz_part[(k + 1) & 1]
  int n_part;
  DevScalars* S;
  int lm_gate;
  int L;
};

template <typename T, int C>
__device__ __forceinline__ void run(const SplitBArgs<T, C>& a, VG g, int k) {
  DevScalars* S = a.S;
  if (k >= a.L || S->stopped || (a.lm_gate && S->done)) return;
  const double pq = reduce_partials(a.pq_part, a.n_part);
  if (!(pq > 0.0)) {
    if (is_block_leader(g)) S->stopped = 1;
    return;
  }
  const T alpha = (T)(S->rz[k & 1] / pq);
  const T* p = pick(a.p, k & 1);
  double rz = 0.0;
  OPT_SITE_LOOP(s, a.n, g) {
    // all loads of the site before its stores (the arrays may alias as far as
    // the compiler knows, so interleaving would serialise them)
    T pv[C], dv[C], qv[C], rv[C], mv[C];
    const size_t o0 = vix<C>(0, s);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      pv[c] = p[o0 + c];
      dv[c] = a.delta[o0 + c];
      qv[c] = a.q[o0 + c];
      rv[c] = a.r[o0 + c];
      mv[c] = a.minv[o0 + c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      dv[c] = fma(alpha, pv[c], dv[c]);
      rv[c] = fma(-alpha, qv[c], rv[c]);
      rz += (double)rv[c] * (double)(mv[c] * rv[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      a.delta[o0 + c] = dv[c];
      a.r[o0 + c] = rv[c];
    }
  }
  block_store(rz, pick(a.rz_part, (k + 1) & 1), g);
}

// ---------------------------------------------------------------- materialised PCG
// The alternative to the matrix-free products that Sec. 7 compares them with:
// J is evaluated once per linearisation into device memory (evalJ; a fixed
// number of entries per residual row, the energy's eval_j) and every PCG
// iteration multiplies by it twice, y = J p then q = J^T y.  J^T is not stored:
// each unknown's list of the J entries in its column (built once from the
// structure by evalJ) gathers them.  The recurrence is the split form's: per
// iteration p = z + beta p (MatP), y = J p (MatA), q = J^T y (MatB, with the
// partials of p.q), then pcg_b unchanged.

// Energies that can materialise their Jacobian (E::kJRows).
template <class E, class = void>
struct MatOf : std::false_type {};
template <class E>
struct MatOf<E, std::void_t<decltype(E::kJRows)>> : std::true_type {};

template <class E>
struct EvalJArgs {
  E e;
  typename E::Real* val;  // [n][kJRows][kJSlots]
  int* col;
  int* jt;                // [n][C][kJTSlots]
};

template <class E>
__device__ __forceinline__ void run(const EvalJArgs<E>& a, VG g, int) {
  constexpr int RS = E::kJRows * E::kJSlots, CT = E::C * E::kJTSlots;
  OPT_SITE_LOOP(s, a.e.n, g) {
    a.e.eval_j(s, a.val + (size_t)s * RS, a.col + (size_t)s * RS);
    a.e.eval_jt(s, a.jt + (size_t)s * CT);
  }
}

template <typename T>
struct MatBufs {
  const T* val;    // J entries, rows x slots
  const int* col;  // their internal vector index (-1: none)
  const int* jt;   // per unknown, tslots indices into val (-1: none), row order
  T* y;            // J p, one per row
  long long rows;
};

// p_k = z + beta p_{k-1} with z = M^-1 r (beta from the r.z partials of the
// previous pcg_b, or of init); stored for the two products and pcg_b.
template <typename T, int C>
struct MatPArgs {
  int n;
  const T* r;
  const T* minv;
  T* p[2];
  const double* rz_part[2];
  int n_part;
  DevScalars* S;
  int lm_gate;
  int L;
};

template <typename T, int C>
__device__ __forceinline__ void run(const MatPArgs<T, C>& a, VG g, int k) {
  DevScalars* S = a.S;
  if (k >= a.L || S->stopped || (a.lm_gate && S->done)) return;
  const double rz = reduce_partials(pick(a.rz_part, k & 1), a.n_part);
  const T beta = k > 0 ? (T)(rz / S->rz[(k - 1) & 1]) : T(0);
  if (is_block_leader(g)) S->rz[k & 1] = rz;
  const T* pold = pick(a.p, (k + 1) & 1);
  T* pnew = pick(a.p, k & 1);
  OPT_SITE_LOOP(s, a.n, g) {
    T rv[C], mv[C], po[C];
    const size_t o = vix<C>(0, s);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      rv[c] = a.r[o + c];
      mv[c] = a.minv[o + c];
      po[c] = k > 0 ? pold[o + c] : T(0);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) pnew[o + c] = fma(beta, po[c], mv[c] * rv[c]);
  }
}

// y = J p, one thread per residual row.
template <class E>
struct MatAArgs {
  MatBufs<typename E::Real> m;
  const typename E::Real* p;
  const DevScalars* S;
  int lm_gate;
  int L;
};

template <class E>
__device__ __forceinline__ void run(const MatAArgs<E>& a, VG g, int k) {
  using T = typename E::Real;
  constexpr int NS = E::kJSlots;
  const DevScalars* S = a.S;
  if (k >= a.L || S->stopped || (a.lm_gate && S->done)) return;
  const MatBufs<T>& m = a.m;
  for (long long r = (long long)unit_of_block(g) * kBlock + threadIdx.x; r < m.rows;
       r += (long long)g.nb * kBlock) {
    int cl[NS];
    T vl[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      cl[t] = m.col[r * NS + t];
      vl[t] = m.val[r * NS + t];
    }
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < NS; ++t)
      if (cl[t] >= 0) acc = fma(vl[t], a.p[cl[t]], acc);
    m.y[r] = acc;
  }
}

// q = J^T y (+ damping p), partials of p . q.
template <class E>
struct MatBArgs {
  MatBufs<typename E::Real> m;
  int n;
  const typename E::Real* p;
  const typename E::Real* damp;
  typename E::Real* q;
  double* pq_part;
  DevScalars* S;
  int lm_gate;
  int L;
};

template <class E>
__device__ __forceinline__ void run(const MatBArgs<E>& a, VG g, int k) {
  using T = typename E::Real;
  constexpr int C = E::C, NS = E::kJSlots, NT = E::kJTSlots;
  DevScalars* S = a.S;
  if (k >= a.L || S->stopped || (a.lm_gate && S->done)) return;
  const MatBufs<T>& m = a.m;
  double pq = 0.0;
  OPT_SITE_LOOP(s, a.n, g) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t u = vix<C>(c, s);
      int e[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) e[t] = m.jt[u * NT + t];
      T acc = T(0);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if (e[t] >= 0) acc = fma(m.val[e[t]], m.y[e[t] / NS], acc);
      const T pv = a.p[u];
      if (a.damp) acc = fma(a.damp[u], pv, acc);
      a.q[u] = acc;
      pq += (double)pv * (double)acc;
    }
  }
  block_store(pq, a.pq_part, g);
}

// ---------------------------------------------------------------- fused iteration
// Value that lane l-1 (from_left) or l+1 (from_right) of the wave holds; 0 past
// the ends of the wave.  DPP wave shifts, so no LDS traffic.
__device__ __forceinline__ uint32_t dpp_from_left(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, true);  // wave_shr:1
}
__device__ __forceinline__ uint32_t dpp_from_right(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, true);  // wave_shl:1
}
__device__ __forceinline__ float from_left(float v) {
  return __uint_as_float(dpp_from_left(__float_as_uint(v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __uint_as_float(dpp_from_right(__float_as_uint(v)));
}
__device__ __forceinline__ double from_left(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = dpp_from_left((uint32_t)u), hi = dpp_from_left((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(lo | (hi << 32)));
}
__device__ __forceinline__ double from_right(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = dpp_from_right((uint32_t)u), hi = dpp_from_right((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(lo | (hi << 32)));
}
__device__ __forceinline__ uint32_t from_left(uint32_t v) { return dpp_from_left(v); }
__device__ __forceinline__ uint32_t from_right(uint32_t v) { return dpp_from_right(v); }

// The value lane i (uniform, below 64) holds, in every lane.
__device__ __forceinline__ float lane_value(float v, int i) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), i));
}
__device__ __forceinline__ double lane_value(double v, int i) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), i);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One wave per strip of 64 columns: 60 produced, 2 halo columns on each side.
constexpr int kStripCols = 60;

// Edge geometry an energy may keep from apply (on a row) for jsq (on the same
// row one step later): E::JCache with apply_c and jsq_c, else nothing.
template <class E, class = void>
struct JCacheOf {
  struct type {};
  static constexpr bool kOn = false;
};
template <class E>
struct JCacheOf<E, std::void_t<typename E::JCache>> {
  using type = typename E::JCache;
  static constexpr bool kOn = true;
};

// An energy may form J^T J p row by row in the streaming kernel, passing each
// residual of an edge between rows to the next step (E::Carry, edge_next and
// apply_stream); else the fused kernel uses apply.
template <class E, class = void>
struct StreamApplyOf {
  struct Carry {};
  static constexpr bool kOn = false;
};
template <class E>
struct StreamApplyOf<E, std::void_t<typename E::Carry>> {
  using Carry = typename E::Carry;
  static constexpr bool kOn = true;
};

// One grid row as one lane sees it (its column), for the streaming kernel.
template <class E, bool DAMP>
struct StreamRow {
  using T = typename E::Real;
  static constexpr int C = E::C, NS = E::kStatePlanes > 0 ? E::kStatePlanes : 1;
  T u[C];    // u_i, later u_{i+1}
  T p[C];    // p_{i-1}, later p_i
  T x[C];    // d (loaded one step before it is updated)
  T po[C];   // p_{i-1}, kept for the deferred update of d
  T st[NS];
  uint32_t f;
  T aw;  // 1 where the site is active, else 0 (set with p)
  typename JCacheOf<E>::type jc;  // set by apply on this row, read by its jsq
};

// Stencil views centred on row R (rows U before and D after it in the walk); V
// selects the vector.  Horizontal neighbours come from the adjacent lanes
// (DPP), vertical ones from the row ring.  Views: P (vector), S (state), F
// (flags), A (active weight).  With flip (a walk up the grid) a view at dj < 0
// reads D and one at dj > 0 reads U, so the body sees the grid's orientation.
// Lane exchanges whose values the body does not read are dropped by the
// compiler.
template <class E, bool DAMP, class VSel, class Body>
__device__ __forceinline__ auto with_views(const StreamRow<E, DAMP>& U, const StreamRow<E, DAMP>& R,
                                           const StreamRow<E, DAMP>& D, VSel V, Body body, bool flip = false) {
  using T = typename E::Real;
  constexpr int C = E::C, NS = StreamRow<E, DAMP>::NS;
  T vl[C], vr[C], sl[NS], sr[NS];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    vl[c] = from_left(V(R, c));
    vr[c] = from_right(V(R, c));
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    sl[q] = from_left(R.st[q]);
    sr[q] = from_right(R.st[q]);
  }
  const uint32_t fl = from_left(R.f), fr = from_right(R.f);
  const T al = from_left(R.aw), ar = from_right(R.aw);
  // dj is a constant at every call, so a view off the row is one select of
  // the two rows' values on the uniform flag.  Both values are read first: a
  // choice between two places in the row ring, read once, would send the ring
  // to scratch memory.
  auto pick_ud = [](bool down, auto u, auto d) { return down ? d : u; };
  auto Pv = [&](int c, int di, int dj) -> T {
    return dj != 0 ? pick_ud((dj > 0) != flip, V(U, c), V(D, c)) : di < 0 ? vl[c] : di > 0 ? vr[c] : V(R, c);
  };
  auto Sv = [&](int q, int di, int dj) -> T {
    return dj != 0 ? pick_ud((dj > 0) != flip, U.st[q], D.st[q]) : di < 0 ? sl[q] : di > 0 ? sr[q] : R.st[q];
  };
  auto Fv = [&](int di, int dj) -> uint32_t {
    return dj != 0 ? pick_ud((dj > 0) != flip, U.f, D.f) : di < 0 ? fl : di > 0 ? fr : R.f;
  };
  auto Av = [&](int di, int dj) -> T {
    return dj != 0 ? pick_ud((dj > 0) != flip, U.aw, D.aw) : di < 0 ? al : di > 0 ? ar : R.aw;
  };
  return body(Pv, Sv, Fv, Av);
}


template <typename T>
struct FusedBufs {
  T* u[2];         // iteration i reads u_i from u[i & 1], writes u_{i+1} to u[(i + 1) & 1]
  T* p[2];         // iteration i writes p_i to p[i & 1], reads p_{i-1} from p[(i + 1) & 1]
  T* x;            // the PCG solution d, updated in place
  double* part[2]; // [gamma | delta] partials, kMaxBlocks apart; iteration i writes
                   // part[i & 1] (the priming launch writes part[1]) and reads the other
  const T* diag;   // diag(J^T J) from init (read by energies that do not recompute it)
};

// BIG: the instantiation for grids whose internal vectors pass 256 MB; its
// raw buffers are based at each strip's first row (see run).
template <class E, bool DAMP, bool BIG = false>
struct FusedArgs {
  E e;
  FusedBufs<typename E::Real> b;
  Precond<typename E::Real> pc;  // lam taken from the device scalars when lm_gate
  int n_part;  // blocks of this problem
  DevScalars* S;
  int lm_gate;
  int n_sx, n_sy;  // strips across, strips down
  int sw;          // produced columns per strip (<= kStripCols)
  int rq, rr;      // rows per strip: rq, one more for the first rr strips down
  int L;
};

// f(integral_constant<int, I>) for each I of the sequence, in order.
// Cache policy of the fused kernel's vector stores.  FP32 rows: device scope
// (the stores write through to the level every XCD sees, so little is left to
// write back when the kernel ends; measured 1-9% faster than the default, the
// non-temporal hint 10% slower).  FP64 rows: the default (device scope made
// those launches 40-70% slower).
template <typename T>
constexpr int kFusedStoreAux = sizeof(T) == 4 ? 16 : 0;

template <int... I, class F>
__device__ __forceinline__ void unroll_seq(std::integer_sequence<int, I...>, F f) {
  (f(std::integral_constant<int, I>{}), ...);
}

// Rows of loads in flight ahead of the row being started (FP64 rows are twice
// as large, so fewer fit in registers).
template <typename T>
constexpr int kPrefetchOf = sizeof(T) > 4 ? 2 : 4;

// How an energy's strip walk is laid out (chosen per energy from measurement:
// both choices cost registers, and with them waves per SIMD).
//  * kPrefetchD: d of a produced row is loaded with the row's other data, so
//    the update of d waits on no load issued later (else it is loaded one step
//    before it is updated, and the wait for it also drains the rows in flight).
//  * kPeel: the steps before the pipeline is full run apart from the loop (see
//    walk_steps).
// An energy sets them with `static constexpr int kFusedWalk` (bit 0: kPrefetchD,
// bit 1: kPeel), and the rows prefetched ahead (kPrefetchOf by default) with
// `static constexpr int kFusedPrefetch`.
template <class E, class = void>
struct FusedWalkOf {
  static constexpr bool kPrefetchD = false, kPeel = false;
};
template <class E>
struct FusedWalkOf<E, std::void_t<decltype(E::kFusedWalk)>> {
  static constexpr bool kPrefetchD = (E::kFusedWalk & 1) != 0, kPeel = (E::kFusedWalk & 2) != 0;
};
template <class E, class = void>
struct FusedPrefetchOf {
  static constexpr int value = kPrefetchOf<typename E::Real>;
};
template <class E>
struct FusedPrefetchOf<E, std::void_t<decltype(E::kFusedPrefetch)>> {
  static constexpr int value = E::kFusedPrefetch;
};
// The record an energy stores per site may hold fewer values than the state
// planes its products read (`static constexpr int kStateRec`): the walk loads
// it into the last kStateRec places of a row's state and the energy's
// expand_state fills the rest once the row's loads have landed.
template <class E, class = void>
struct StateRecOf {
  static constexpr int value = E::kStatePlanes;
  static constexpr bool kExpand = false;
};
template <class E>
struct StateRecOf<E, std::void_t<decltype(E::kStateRec)>> {
  static constexpr int value = E::kStateRec;
  static constexpr bool kExpand = E::kStateRec != E::kStatePlanes;
};

// The K steps of a strip walk; step(PH, k, steady) gets the ring slot k % N as
// a constant.  Plain form: groups of N steps, each step tested against K.
// Peeled form: steps 0 .. P-1 one at a time (their tests for a pipeline not yet
// full fold away), then groups of N steps with no test at all, then the rest.
// In the plain form a loop iteration has branches whose paths carry different
// numbers of loads in flight; the wait after such a merge drains every load,
// prefetched rows included.  steady is true from step P on in the peeled form
// and always false in the plain one.
template <int N, int P, bool PEEL, class Step>
__device__ __forceinline__ void walk_steps(int K, Step step) {
  static_assert(P < N, "the start-up steps fit one turn of the ring");
  if constexpr (PEEL) {
    unroll_seq(std::make_integer_sequence<int, P>{}, [&](auto J) {
      constexpr int j = decltype(J)::value;
      if (j < K) step(std::integral_constant<int, j % N>{}, j, std::false_type{});
    });
    int k = P;
    for (; k + N <= K; k += N) {
      unroll_seq(std::make_integer_sequence<int, N>{}, [&](auto J) {
        constexpr int j = decltype(J)::value;
        step(std::integral_constant<int, (P + j) % N>{}, k + j, std::true_type{});
      });
    }
    unroll_seq(std::make_integer_sequence<int, N - 1>{}, [&](auto J) {
      constexpr int j = decltype(J)::value;
      if (k + j < K) step(std::integral_constant<int, (P + j) % N>{}, k + j, std::true_type{});
    });
  } else {
    for (int k = 0; k < K; k += N) {
      unroll_seq(std::make_integer_sequence<int, N>{}, [&](auto J) {
        constexpr int j = decltype(J)::value;
        if (k + j < K) step(std::integral_constant<int, j>{}, k + j, std::false_type{});
      });
    }
  }
}

template <class E, bool DAMP, bool BIG>
__device__ __forceinline__ void run(const FusedArgs<E, DAMP, BIG>& a, VG g, int iter) {
  using T = typename E::Real;
  using Row = StreamRow<E, DAMP>;
  constexpr int C = E::C, NS = E::kStatePlanes;
  constexpr int kPrefetch = FusedPrefetchOf<E>::value;
  static_assert(kPrefetch >= 1, "at least the next row is in flight");
  constexpr int N = kPrefetch + 4;  // ring slots: four rows in use, the rest in flight
  const E& e = a.e;
  DevScalars* S = a.S;
  if (iter >= a.L) return;
  const bool read_pold = iter > 0, write_out = iter >= 0;
  // d = sum_i alpha_i p_i is updated every second iteration: an odd iteration
  // adds alpha_{i-1} p_{i-1} (the p it reads) and then alpha_i p_i, rounding as
  // two successive updates would; an even one leaves d alone unless it is the
  // last.  That halves the traffic of d.
  const bool xupd = write_out && ((iter & 1) || iter == a.L - 1);
  const bool xtwo = xupd && (iter & 1);
  const int W = e.W, H = e.H, n = e.n, n_sy = a.n_sy, sw = a.sw;
  const int lane = threadIdx.x & 63;
  // the wave's strip and every row quantity below are wave-uniform (scalar)
  const int strip = unit_of_block(g) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool has_strip = strip < a.n_sx * n_sy;
  // Strips are numbered along grid rows, so horizontally adjacent strips run
  // side by side (and mostly on one XCD).  Vertically adjacent strips walk in
  // opposite directions, so both reach the halo rows they share at about the
  // same time and the second read is served by the L2.  A site's operator sees
  // its rows in grid orientation either way (the streaming energy's, symmetric
  // in the two, in walk order).
  const int sy = strip / a.n_sx, sx = strip % a.n_sx;
  const int col = sx * sw - 2 + lane;
  const int y0 = sy * a.rq + min(sy, a.rr), y1 = min(y0 + a.rq + (sy < a.rr ? 1 : 0), H);
  const int dir = (sy & 1) ? -1 : 1;
  const int ybeg = dir > 0 ? y0 - 2 : y1 + 1;  // row of step 0
  const int ylo = max(y0 - 2, 0), yhi = min(y1 + 1, H - 1);
  const bool colin = has_strip && col >= 0 && col < W;
  const bool out_lane = colin && lane >= 2 && lane < 2 + sw;
  const int K = (y1 - y0) + 4;  // rows y0-2 .. y1+1
  // One raw buffer per vector and for the per-site state and flags.  A site's
  // channels are adjacent, so each row of a vector is one wide load per lane.
  // A lane or row off the strip uses an out-of-range offset: its loads return
  // 0, its stores are dropped.  The BIG instantiation bases every buffer at
  // the first row the strip touches (yb) and covers only its rows ylo..yhi, so
  // that offsets stay small however large the grid is (the other keeps whole
  // vectors: fewer live registers, which the FP32 warp kernel needs).
  using SR = StateRecOf<E>;
  constexpr int NR = SR::value;  // values stored per site
  constexpr unsigned VB = C * sizeof(T), SB = (NR > 0 ? NR : 1) * sizeof(T);
  const int yb = BIG ? ylo : 0;
  const size_t span = BIG ? (has_strip ? (size_t)(yhi - ylo + 1) * W : 0) : (size_t)n;  // sites
  const size_t rb = BIG && has_strip ? (size_t)yb * W : 0;                               // first site
  const size_t vbytes = span * VB;
  const Buf<T> Buin = Buf<T>::make(pick(a.b.u, iter < 0 ? 0 : (iter & 1)) + rb * C, vbytes);
  const Buf<T> Bpin = Buf<T>::make(pick(a.b.p, (iter + 1) & 1) + rb * C, read_pold ? vbytes : 0);
  const Buf<T> Bx = Buf<T>::make(a.b.x + rb * C, xupd ? vbytes : 0);
  const Buf<T> Buout = Buf<T>::make(pick(a.b.u, (iter + 1) & 1) + rb * C, write_out ? vbytes : 0);
  const Buf<T> Bpout = Buf<T>::make(pick(a.b.p, iter & 1) + rb * C, write_out ? vbytes : 0);
  const Buf<T> Bst = Buf<T>::make(e.state_base() + (NR > 0 ? rb * NR : 0), NR > 0 ? span * SB : 0);
  const Buf<uint8_t> Bf = Buf<uint8_t>::make(e.flags + rb, span);
  // Byte offsets are a per-lane column part plus a scalar row part (rows
  // counted from yb).  Either part may be kBufOutOfRange; the sum then stays at
  // or above 2^28 (no part in range reaches 2^28: the host launches a form
  // only where that holds), so the access is out of range as required.
  const unsigned lane_v = colin ? (unsigned)col * VB : kBufOutOfRange;
  const unsigned lane_s = colin ? (unsigned)col * SB : kBufOutOfRange;
  const unsigned lane_f = colin ? (unsigned)col : kBufOutOfRange;
  const unsigned lane_o = out_lane ? (unsigned)col * VB : kBufOutOfRange;
  // The row of step k lives in ring slot k % N; its loads are issued
  // kPrefetch steps before it is started.
  using FW = FusedWalkOf<E>;
  Row ring[N];
  auto issue = [&](Row& R, int y) {
    const bool in = y >= ylo && y <= yhi;
    const unsigned rs = (unsigned)((y - yb) * W);
    if constexpr (NR > 0) {
      buf_loadv<NR>(Bst, lane_s + (in ? rs * SB : kBufOutOfRange), 0, R.st + (NS - NR));
    } else {
      R.st[0] = T(0);
    }
    R.f = Bf.load(lane_f + (in ? rs : kBufOutOfRange), 0);
    const unsigned o = lane_v + (in ? rs * VB : kBufOutOfRange);
    buf_loadv<C>(Buin, o, 0, R.u);
    buf_loadv<C>(Bpin, o, 0, R.p);
    if constexpr (FW::kPrefetchD) {
      // d of a produced row, when this launch updates it
      const bool prod = y >= y0 && y < y1;
      buf_loadv<C>(Bx, lane_o + ((prod && xupd) ? rs * VB : kBufOutOfRange), 0, R.x);
    }
  };
  // The first rows do not depend on alpha and beta: fetch them while the
  // previous launch's partial sums are reduced.
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) issue(ring[k], ybeg + dir * k);

  // The scalars that earlier launches left, read together up front.
  // S->stopped holds 1 + the iteration at which the PCG stopped; the blocks of
  // that launch all take the stop path (a sibling may already have set it, so
  // a block only returns here for a stop of an earlier launch).
  const int stopped_at = S->stopped;
  const int lm_done = a.lm_gate ? S->done : 0;
  const double gam_old = iter > 0 ? S->gam[(iter - 1) & 1] : 1.0;
  const double alpha_old = iter > 0 ? S->alpha[(iter - 1) & 1] : 1.0;
  const double lam_now = a.lm_gate ? S->lambda : 0.0;
  if ((stopped_at != 0 && stopped_at != iter + 1) || lm_done) return;
  const double* part_in = pick(a.b.part, (iter + 1) & 1);
  double* part_out = pick(a.b.part, iter & 1);
  double alpha = 0.0, beta = 0.0;
  const double alpha_prev = (iter & 1) ? alpha_old : 0.0;
  if (iter >= 0) {
    double gam, del;
    reduce_partials2(part_in, part_in + kMaxBlocks, a.n_part, &gam, &del);
    double den = del;
    if (iter > 0) {
      beta = gam / gam_old;
      den = del - beta * gam / alpha_old;
    }
    if (!(den > 0.0)) {
      if (is_block_leader(g)) S->stopped = iter + 1;
      if ((iter & 1) && out_lane) {
        // the update alpha_{i-1} p_{i-1} deferred from the previous iteration
        const T ap = (T)alpha_prev;
        for (int y = y0; y < y1; ++y) {
          const unsigned s = (unsigned)((y - yb) * W + col);
          if (!(Bf.load(s, 0) & E::ACTIVE)) continue;
          T pv[C], xv[C];
          buf_loadv<C>(Bpin, s * VB, 0, pv);
          buf_loadv<C>(Bx, s * VB, 0, xv);
#pragma unroll
          for (int c = 0; c < C; ++c) xv[c] = fma(ap, pv[c], xv[c]);
          buf_storev<C>(Bx, s * VB, 0, xv);
        }
      }
      return;
    }
    alpha = gam / den;
    if (is_block_leader(g)) {
      S->gam[iter & 1] = gam;
      S->alpha[iter & 1] = alpha;
    }
  }
  const T aT = (T)alpha, bT = (T)beta, apT = (T)alpha_prev;
  Precond<T> pc = a.pc;
  if (a.lm_gate) pc.lam = (T)lam_now;
  double g_acc = 0.0, d_acc = 0.0;

  if (has_strip) {
    auto selp = [](const Row& R, int c) { return R.p[c]; };
    auto selu = [](const Row& R, int c) { return R.u[c]; };

    using SA = StreamApplyOf<E>;
    typename SA::Carry cprev{};  // residuals of the edge (y - 2 dir, y - dir)
    auto shift = [](T v, int di) { return di > 0 ? from_right(v) : from_left(v); };
    auto step = [&](auto PH, int k, auto steady) {
      constexpr int ph = decltype(PH)::value;
      constexpr bool st = decltype(steady)::value;
      Row& R0 = ring[ph];                // row y = ybeg + dir k
      Row& R1 = ring[(ph + N - 1) % N];  // y - dir
      Row& R2 = ring[(ph + N - 2) % N];  // y - 2 dir
      Row& R3 = ring[(ph + N - 3) % N];  // y - 3 dir
      const int y = ybeg + dir * k;
      issue(ring[(ph + kPrefetch) % N], y + dir * kPrefetch);
      if constexpr (SR::kExpand) E::expand_state(R0.st);
      // p_i = u_i + beta p_{i-1} on row y
#pragma unroll
      for (int c = 0; c < C; ++c) {
        // at iteration 0 (and in the priming launch) beta is 0 and p_{i-1}
        // reads as 0, so this is p_0 = u_0 exactly
        R0.po[c] = R0.p[c];
        R0.p[c] = fma(bT, R0.p[c], R0.u[c]);
      }
      R0.aw = (R0.f & E::ACTIVE) ? T(1) : T(0);
      typename SA::Carry cnext{};  // residuals of the edge (y - dir, y)
      if constexpr (SA::kOn) {
        if (st || k >= 1) cnext = e.edge_next(R1, R0);
      }
      if (st || k >= 2) {
        // on row y - dir: s = A p (with the LM damping), the diagonal M from the
        // state, u_{i+1} = u_i - alpha M^-1 s and the partial of gamma = sum M u^2;
        // d of that row is fetched now (unless it came with the row), to be
        // updated in the next step
        const int y1r = y - dir;
        T gv[C], dg[C];
        if constexpr (SA::kOn) {
          with_views(R2, R1, R0, selp, [&](auto Pv, auto Sv, auto Fv, auto Av) {
            e.apply_stream(Pv, Sv, Fv, Av, shift, cprev, cnext, gv, R1.jc);
            e.diag_stream(Sv, Fv, Av, dg);
            return 0;
          });
        } else {
          // the views in grid orientation (row above, row below), whichever way
          // the strip walks: an energy may keep a value per edge at one of its
          // ends (a weight of the edge below a site)
          with_views(R2, R1, R0, selp, [&](auto Pv, auto Sv, auto Fv, auto) {
            if constexpr (JCacheOf<E>::kOn) {
              e.apply_c(Pv, Sv, Fv, col, y1r, gv, R1.jc);
            } else {
              e.apply(Pv, Sv, Fv, col, y1r, gv);
            }
            e.diag(Sv, Fv, dg);
            return 0;
          }, dir < 0);
        }
        const bool act = R1.f & E::ACTIVE;
        const bool prod = y1r >= y0 && y1r < y1;  // uniform
        if constexpr (!FW::kPrefetchD) {
          const unsigned ox = act ? lane_o + ((prod && xupd) ? (unsigned)((y1r - yb) * W) * VB : kBufOutOfRange)
                                  : kBufOutOfRange;
          buf_loadv<C>(Bx, ox, 0, R1.x);
        }
        T gs = 0, dd = 0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          T sv = gv[c];
          T dmp = T(0);
          if constexpr (DAMP) {
            dmp = pc.lam != T(0) ? pc.damp(dg[c]) : T(0);
            sv = fma(dmp, R1.p[c], sv);
          }
          // M and M^-1 as Precond gives them (without damping, lam is 0)
          // (branch-free: the reciprocal is taken even where it is not used)
          const T m = DAMP ? pc.den(dg[c]) : (pc.use ? dg[c] : T(1));
          const T rm = recip(m);
          const T mi = pc.use ? (m > T(0) ? rm : T(0)) : T(1);
          R1.u[c] = act ? fma(-aT, mi * sv, R1.u[c]) : T(0);
          gs = fma(m * R1.u[c], R1.u[c], gs);
          if constexpr (DAMP) dd = fma(dmp * R1.u[c], R1.u[c], dd);
        }
        g_acc += (double)((out_lane && prod) ? gs : T(0));
        // the damping part of delta, u.(lambda D) u, is pointwise: taken here
        if constexpr (DAMP) d_acc += (double)((out_lane && prod && (R1.f & E::INGRID)) ? dd : T(0));
      }
      if constexpr (SA::kOn) cprev = cnext;
      if (st || k >= 4) {
        // row y - 2 dir is final: partial of delta = |J u|^2 (+ u.(lambda D) u),
        // and the stores of d, u, p
        const int yo = y - 2 * dir;
        // grid orientation as for the product (the streaming energy's rows are
        // symmetric and stay in walk order)
        const T jq = with_views(R3, R2, R1, selu, [&](auto Pv, auto Sv, auto Fv, auto Av) {
          if constexpr (JCacheOf<E>::kOn) {
            return e.jsq_c(Pv, Fv, Av, R2.jc);
          } else {
            return e.jsq(Pv, Sv, Fv, col, yo);
          }
        }, !SA::kOn && dir < 0);
        const bool act = R2.f & E::ACTIVE;
        d_acc += (double)((out_lane && (R2.f & E::INGRID)) ? jq : T(0));
        const unsigned o = lane_o + (unsigned)((yo - yb) * W) * VB;
        const unsigned ox = (act && xupd) ? o : kBufOutOfRange;
        T pv[C], xv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          pv[c] = act ? R2.p[c] : T(0);
          const T xo = xtwo ? fma(apT, R2.po[c], R2.x[c]) : R2.x[c];
          xv[c] = fma(aT, pv[c], xo);
        }
        buf_storev<C, kFusedStoreAux<T>>(Bx, ox, 0, xv);
        buf_storev<C, kFusedStoreAux<T>>(Buout, o, 0, R2.u);
        buf_storev<C, kFusedStoreAux<T>>(Bpout, o, 0, pv);
      }
    };
    walk_steps<N, 4, FW::kPeel>(K, step);
  }
  double gs, ds;
  block_sum2(g_acc, d_acc, &gs, &ds);
  if (threadIdx.x == 0) {
    part_out[g.bid] = gs;
    part_out[kMaxBlocks + g.bid] = ds;
  }
}

// ---------------------------------------------------------------- updates
// GN: x += d on active sites.  LM: the same, only if the step was accepted.
template <class E>
struct StepArgs {
  E e;
  typename E::Real* x;
  const typename E::Real* delta;
  const DevScalars* S;
  int lm_gate;
};

template <class E>
__device__ __forceinline__ void run(const StepArgs<E>& a, VG g, int) {
  constexpr int C = E::C;
  if (a.lm_gate && !a.S->accepted) return;
  const int n = a.e.n;
  OPT_SITE_LOOP(s, n, g) {
    if (!(a.e.flags[s] & E::ACTIVE)) continue;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      a.x[o] = a.x[o] + a.delta[vix<C>(c, s)];
    }
  }
}

// ---------------------------------------------------------------- cost
// FP64 cost partials at x (delta == nullptr) or at the trial point x + delta,
// rounded to the bulk type exactly as the step update would store it.
template <class E>
struct CostArgs {
  E e;
  const typename E::Real* x;
  const typename E::Real* delta;
  double* part;
  const DevScalars* S;
  int lm_gate;
};

template <class E>
__device__ __forceinline__ void run(const CostArgs<E>& a, VG g, int) {
  using T = typename E::Real;
  if (a.lm_gate && a.S->done) return;
  const int n = a.e.n;
  auto X = [&](int c, int s) -> double {
    const size_t o = (size_t)c * n + s;
    if (a.delta == nullptr) return (double)a.x[o];
    return (double)(T)(a.x[o] + a.delta[vix<E::C>(c, s)]);
  };
  double acc = 0.0;
  OPT_SITE_LOOP(s, n, g) acc += a.e.cost(X, s);
  block_store(acc, a.part, g);
}

// LM model partials: sum_r (J d)_r (2 F_r + (J d)_r) at x.
template <class E>
struct ModelArgs {
  E e;
  const typename E::Real* x;
  const typename E::Real* delta;
  double* part;
  const DevScalars* S;
};

template <class E>
__device__ __forceinline__ void run(const ModelArgs<E>& a, VG g, int) {
  if (a.S->done) return;
  const int n = a.e.n;
  auto X = [&](int c, int s) -> double { return (double)a.x[(size_t)c * n + s]; };
  auto D = [&](int c, int s) -> double { return (double)a.delta[vix<E::C>(c, s)]; };
  double acc = 0.0;
  OPT_SITE_LOOP(s, n, g) acc += a.e.model(X, D, s);
  block_store(acc, a.part, g);
}

// ---------------------------------------------------------------- scalar kernels (one block)
struct LMConsts {
  double radius_min, radius_max, min_rel_decrease;
};

// Sets up the scalars of a solve.
struct SetupArgs {
  DevScalars* S;
  double lambda, radius0;
  int lm;
  double radius_min;  // LM: a solve whose initial radius is below this does nothing
};

__device__ __forceinline__ void run(const SetupArgs& a, VG, int) {
  if (threadIdx.x == 0) {
    DevScalars* S = a.S;
    S->rz[0] = S->rz[1] = 0.0;
    S->gam[0] = S->gam[1] = 0.0;
    S->alpha[0] = S->alpha[1] = 0.0;
    S->E0 = S->E1 = S->m = 0.0;
    S->radius = a.radius0;
    S->nu = 2.0;
    S->lambda = a.lm ? 1.0 / a.radius0 : a.lambda;
    S->E_final = 0.0;
    S->stopped = 0;
    S->accepted = 0;
    S->need_lin = 1;
    S->done = a.lm && a.radius0 < a.radius_min ? 1 : 0;
    S->n_accepted = 0;
    S->outer_done = 0;
    S->nonfinite = 0;
    S->trace_k = 0;
  }
}

// LM step decision (gain ratio, Nielsen radius update).
struct DecideArgs {
  DevScalars* S;
  const double* m_part;
  const double* c_part;
  int nb;
  LMConsts lc;
};

__device__ __forceinline__ void run(const DecideArgs& a, VG, int) {
  DevScalars* S = a.S;
  if (S->done) {
    // the solve has ended: the update of this outer iteration must not repeat
    // the last accepted step
    if (threadIdx.x == 0) S->accepted = 0;
    return;
  }
  // the partials hold sum (J d)(2F + J d); the model decrease is its negation
  const double m = -reduce_partials(a.m_part, a.nb);
  const double E1 = reduce_partials(a.c_part, a.nb);
  if (threadIdx.x == 0) {
    S->m = m;
    S->E1 = E1;
    if (!finite_d(E1)) S->nonfinite = 1;
    const double rho = m != 0.0 ? (S->E0 - E1) / m : -INFINITY;
    if (m > 0.0 && rho > a.lc.min_rel_decrease) {
      const double t = 2.0 * rho - 1.0;
      const double f = fmax(1.0 / 3.0, 1.0 - t * t * t);
      S->radius = fmin(S->radius / f, a.lc.radius_max);
      S->nu = 2.0;
      S->accepted = 1;
      S->need_lin = 1;
      S->E0 = E1;
      S->n_accepted += 1;
    } else {
      S->radius = S->radius / S->nu;
      S->nu = 2.0 * S->nu;
      S->accepted = 0;
      S->need_lin = 0;
    }
    S->outer_done += 1;
    if (S->radius < a.lc.radius_min) S->done = 1;
    S->lambda = 1.0 / S->radius;
  }
}

// Finish a cost reduction into E_final.
struct FinishArgs {
  DevScalars* S;
  const double* part;
  int nb;
};

__device__ __forceinline__ void run(const FinishArgs& a, VG, int) {
  const double E = reduce_partials(a.part, a.nb);
  if (threadIdx.x == 0) {
    a.S->E_final = E;
    if (!finite_d(E)) a.S->nonfinite = 1;
  }
}

// An internal vector (sites x C, interleaved) copied out to the caller's layout
// of C planes of n values.
template <typename T, int C>
struct PlanesArgs {
  const T* src;
  T* dst;
  int n;
};

template <typename T, int C>
__device__ __forceinline__ void run(const PlanesArgs<T, C>& a, VG g, int) {
  OPT_SITE_LOOP(s, a.n, g) {
#pragma unroll
    for (int c = 0; c < C; ++c) a.dst[(size_t)c * a.n + s] = a.src[vix<C>(c, s)];
  }
}

// Copy a problem's scalars into a gathering area (one read-back for many problems).
struct GatherArgs {
  const DevScalars* src;
  DevScalars* dst;
};

__device__ __forceinline__ void run(const GatherArgs& a, VG, int) {
  if (threadIdx.x == 0) *a.dst = *a.src;
}

// ---------------------------------------------------------------- launchers
// Every stage runs through this one kernel per argument type, alone (n == 1:
// the problem's own argument row, the hardware grid) or batched: problem j owns
// blocks [start[2j], start[2j] + start[2j+1]), slot_of[b] names the problem of
// block b (-1: an idle block), and its arguments are table[j].  Each batched
// range starts at a multiple of 8, so a problem's block i runs on XCD i mod 8 as
// it would alone.  One kernel binary for both means a problem computes the same
// bits alone and in any batch.
// The BIG FP32 fused iteration is held to the registers of two waves per SIMD
// (its per-strip buffer bases cost two spills instead of a third register bank).
template <class A>
struct MinWavesOf {
  static constexpr int value = 1;
};
template <class E, bool DAMP>
struct MinWavesOf<FusedArgs<E, DAMP, true>> {
  static constexpr int value = sizeof(typename E::Real) == 4 ? 2 : 1;
};

template <class A>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MinWavesOf<A>::value)))
k_batch(const A* __restrict__ table,
                                                  const int* __restrict__ start,
                                                  const int* __restrict__ slot_of, int n, int iter) {
  const int b = blockIdx.x;
  int j = 0;
  VG g{b, (int)gridDim.x};
  if (n != 1) {
    j = slot_of[b];
    if (j < 0) return;
    g = VG{b - start[2 * j], start[2 * j + 1]};
  }
  // read in place: the row's fields are loaded where used (uniform addresses,
  // scalar loads); a local copy of the whole row would be kept in scratch memory
  const A& a = table[j];
  run(a, g, iter);
}

// Store one argument row in device memory, in stream order.
template <class A>
__global__ void k_put(A* __restrict__ dst, A a) {
  if (threadIdx.x == 0) *dst = a;
}

}  // namespace optmi
