// Kernels of one solve on a 2D grid, generic over the energy.
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
// u = M^-1 r, w = A u, gamma = r.u and delta = w.u summed by the previous kernel:
//   beta_i = gamma_i/gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i/alpha_{i-1})
//   p_i = u_i + beta_i p_{i-1};  s_i = A p_i;  d += alpha_i p_i;  r_{i+1} = r_i - alpha_i s_i
//   partials of gamma_{i+1} = r_{i+1}.u_{i+1} and delta_{i+1} = (A u_{i+1}).u_{i+1}.
// A block stages r_i, p_{i-1}, M^-1 and the energy's state for its tile plus a
// halo of twice the operator radius in LDS, computes p_i on all of it, s_i and
// r_{i+1} on the tile plus one operator radius, and A u_{i+1} on the tile, so
// only r, p and d cross HBM once per iteration.  s_i = A p_i is formed exactly
// (not by its own recurrence).  A first "priming" launch with alpha = beta = 0
// produces gamma_0 and delta_0.
//
// If the curvature p.Ap is not positive the solve stops (DevScalars::stopped):
// every later iteration kernel returns at once and d keeps its value.
#pragma once
#include <type_traits>

#include "common.h"

namespace optmi {

// Grid-stride loop over sites with a fixed per-thread order (the grid size
// depends only on n), so the partial sums are reproducible.
#define OPT_SITE_LOOP(s, n) \
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < (n); s += gridDim.x * kBlock)

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
    return inb_(di, dj) ? (e).state_plane(k)[(s) + dj * (e).W + di] : typename E::Real(0); \
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
__global__ void __launch_bounds__(kBlock)
k_linearize(E e, const typename E::Real* __restrict__ x, double* __restrict__ part,
            const DevScalars* __restrict__ S, int lm_gate) {
  if (lm_gate && (S->done || !S->need_lin)) return;
  double acc = 0.0;
  const int n = e.n;
  auto X = [&](int ch, int s) -> double { return (double)x[(size_t)ch * n + s]; };
  OPT_SITE_LOOP(s, n) {
    e.linearize(x, s);
    acc += e.cost(X, s);
  }
  block_store(acc, part);
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
__global__ void __launch_bounds__(kBlock)
k_init(E e, const typename E::Real* __restrict__ x, InitOut<typename E::Real> o,
       const double* __restrict__ lin_part, int n_lin, double* __restrict__ rz_part,
       DevScalars* S, double* __restrict__ trace, int trace_idx, Precond<typename E::Real> pc,
       int lm_gate) {
  using T = typename E::Real;
  constexpr int C = E::C;
  if (lm_gate && S->done) return;
  // LM re-solves at the same x after a rejected step: the cost is then kept.
  const bool fresh = !lm_gate || S->need_lin;
  double E0 = 0.0;
  if (fresh) E0 = reduce_partials(lin_part, n_lin);
  if (is_block_leader()) {
    if (fresh) {
      S->E0 = E0;
      if (!finite_d(E0)) S->nonfinite = 1;
    } else {
      E0 = S->E0;
    }
    if (trace) trace[trace_idx] = E0;
    S->stopped = 0;
  }
  if (lm_gate) pc.lam = (T)S->lambda;
  const int n = e.n;
  double rz = 0.0;
  OPT_SITE_LOOP(s, n) {
    T b[C], d[C];
    if (e.flags[s] & E::ACTIVE) {
      site_jtf_diag(e, x, s, b, d);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) { b[c] = T(0); d[c] = T(0); }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t k = (size_t)c * n + s;
      const T m = pc.minv(d[c]);
      o.r[k] = b[c];
      o.diag[k] = d[c];
      o.minv[k] = m;
      if (o.damp) o.damp[k] = pc.lam != T(0) ? pc.damp(d[c]) : T(0);
      o.delta[k] = T(0);
      rz += (double)b[c] * (double)(m * b[c]);
    }
  }
  block_store(rz, rz_part);
}

// ---------------------------------------------------------------- split: pcg_a
// MODE 0: PCG iteration (p from r, the previous p and beta).
// MODE 1: plain product q = (J^T J + damp) p_in (p_in passed as `pold`).
template <typename T>
struct SplitBufs {
  const T* r;
  const T* minv;
  const T* damp;  // nullptr: no damping
  const T* pold;
  T* pnew;
  T* q;
};

template <class E, int MODE>
__global__ void __launch_bounds__(kBlock)
k_pcg_a(E e, int k, SplitBufs<typename E::Real> b, const double* __restrict__ rz_part, int n_rz,
        double* __restrict__ pq_part, DevScalars* S, int lm_gate) {
  using T = typename E::Real;
  constexpr int C = E::C;
  const int n = e.n;
  T beta = T(0);
  if (MODE == 0) {
    if (S->stopped || (lm_gate && S->done)) return;
    const double rz = reduce_partials(rz_part, n_rz);
    if (k > 0) beta = (T)(rz / S->rz[(k - 1) & 1]);
    if (is_block_leader()) S->rz[k & 1] = rz;
  }
  double pq = 0.0;
  auto Pg = [&](int c, int site) -> T {
    const size_t o = (size_t)c * n + site;
    if (MODE == 1) return b.pold[o];
    const T z = b.minv[o] * b.r[o];
    return k == 0 ? z : fma(beta, b.pold[o], z);
  };
  OPT_SITE_LOOP(s, n) {
    T g[C];
    const bool act = e.flags[s] & E::ACTIVE;
    if (act) site_apply(e, s, Pg, g);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      T pv = T(0), qv = T(0);
      if (act) {
        pv = Pg(c, s);
        qv = g[c];
        if (b.damp) qv += b.damp[o] * pv;
      }
      if (MODE == 0) b.pnew[o] = pv;
      b.q[o] = qv;
      pq += (double)pv * (double)qv;
    }
  }
  if (MODE == 0) block_store(pq, pq_part);
}

// ---------------------------------------------------------------- split: pcg_b
template <typename T, int C>
__global__ void __launch_bounds__(kBlock)
k_pcg_b(int n, int k, T* __restrict__ delta, T* __restrict__ r, const T* __restrict__ p,
        const T* __restrict__ q, const T* __restrict__ minv, const double* __restrict__ pq_part,
        int n_pq, double* __restrict__ rz_part, DevScalars* S, int lm_gate) {
  if (S->stopped || (lm_gate && S->done)) return;
  const double pq = reduce_partials(pq_part, n_pq);
  if (!(pq > 0.0)) {
    if (is_block_leader()) S->stopped = 1;
    return;
  }
  const T alpha = (T)(S->rz[k & 1] / pq);
  double rz = 0.0;
  OPT_SITE_LOOP(s, n) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      delta[o] = fma(alpha, p[o], delta[o]);
      const T rv = fma(-alpha, q[o], r[o]);
      r[o] = rv;
      rz += (double)rv * (double)(minv[o] * rv);
    }
  }
  block_store(rz, rz_part);
}

// ---------------------------------------------------------------- fused iteration
template <typename T>
struct FusedBufs {
  const T* r_in;
  T* r_out;
  const T* p_in;
  T* p_out;
  T* x;            // the PCG solution d, updated in place
  const T* minv;
  const T* damp;   // nullptr: no damping
  const double* part_in;   // [gamma partials | delta partials], kMaxBlocks apart
  double* part_out;
  int n_part_in;
};

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

// Geometry of the fused kernel on a grid: one wave per strip of 64 columns
// (60 produced, 2 halo columns on each side) and kStripRows-or-fewer rows.
constexpr int kStripCols = 60;

// One grid row as one lane sees it (its column), for the streaming kernel.
template <class E>
struct StreamRow {
  using T = typename E::Real;
  static constexpr int C = E::C, NS = E::kStatePlanes > 0 ? E::kStatePlanes : 1;
  T r[C];    // r_i, later r_{i+1}
  T m[C];    // M^-1, later u_{i+1} = M^-1 r_{i+1}
  T p[C];    // p_i
  T x[C];    // d (only on produced rows)
  T dmp[C];  // LM damping (only when damped)
  T st[NS];
  uint32_t f;
};

// Apply the energy's operator at the centre row R with rows U (above) and D
// (below); V selects the vector (p or u).  Horizontal neighbours come from the
// adjacent lanes.
template <class E, class VSel>
__device__ __forceinline__ void stream_apply(const E& e, const StreamRow<E>& U,
                                             const StreamRow<E>& R, const StreamRow<E>& D,
                                             VSel V, int col, int row, typename E::Real* g) {
  using T = typename E::Real;
  constexpr int C = E::C, NS = StreamRow<E>::NS;
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
  auto Pv = [&](int c, int di, int dj) -> T {
    return dj < 0 ? V(U, c) : dj > 0 ? V(D, c) : di < 0 ? vl[c] : di > 0 ? vr[c] : V(R, c);
  };
  auto Sv = [&](int q, int di, int dj) -> T {
    return dj < 0 ? U.st[q] : dj > 0 ? D.st[q] : di < 0 ? sl[q] : di > 0 ? sr[q] : R.st[q];
  };
  auto Fv = [&](int di, int dj) -> uint32_t {
    return dj < 0 ? U.f : dj > 0 ? D.f : di < 0 ? fl : di > 0 ? fr : R.f;
  };
  e.apply(Pv, Sv, Fv, col, row, g);
}

// The k-th unit of work of this block, XCD-aware: blocks go to the 8 XCDs
// round-robin, and each XCD takes one contiguous run of units so neighbouring
// strips share its L2.
__device__ __forceinline__ int unit_of_block(int n_units) {
  const int G = gridDim.x;
  if (G % 8 != 0) return blockIdx.x;
  const int per = G / 8;
  return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <class E>
__global__ void __launch_bounds__(kBlock)
k_fused(E e, FusedBufs<typename E::Real> b, DevScalars* S, int iter, int lm_gate, int n_sx,
        int n_sy, int Hs) {
  using T = typename E::Real;
  using Row = StreamRow<E>;
  constexpr int C = E::C, NS = E::kStatePlanes;
  if (S->stopped || (lm_gate && S->done)) return;
  double alpha = 0.0, beta = 0.0;
  if (iter >= 0) {
    const double gam = reduce_partials(b.part_in, b.n_part_in);
    const double del = reduce_partials(b.part_in + kMaxBlocks, b.n_part_in);
    double den = del;
    if (iter > 0) {
      beta = gam / S->gam[(iter - 1) & 1];
      den = del - beta * gam / S->alpha[(iter - 1) & 1];
    }
    if (!(den > 0.0)) {
      if (is_block_leader()) S->stopped = 1;
      return;
    }
    alpha = gam / den;
    if (is_block_leader()) {
      S->gam[iter & 1] = gam;
      S->alpha[iter & 1] = alpha;
    }
  }
  const T aT = (T)alpha, bT = (T)beta;
  const bool read_pold = iter > 0, write_out = iter >= 0, damped = b.damp != nullptr;
  const int W = e.W, H = e.H, n = e.n;
  const int lane = threadIdx.x & 63;
  const int strip = unit_of_block(gridDim.x) * kWaves + (threadIdx.x >> 6);
  double g_acc = 0.0, d_acc = 0.0;

  if (strip < n_sx * n_sy) {
    const int sx = strip / n_sy, sy = strip % n_sy;
    const int col = sx * kStripCols - 2 + lane;
    const int y0 = sy * Hs, y1 = min(y0 + Hs, H);
    const bool colin = col >= 0 && col < W;
    const bool out_lane = colin && lane >= 2 && lane < 2 + kStripCols;
    const int K = (y1 - y0) + 4;  // rows y0-2 .. y1+1
    Row ring[4];
    // Raw loads of the rows 1..4 steps ahead: row y0-2+k is issued at step k-4
    // and finished at step k, so its memory latency overlaps four steps of work.
    Row pre[4];

    auto issue = [&](Row& R, int y) {
      const bool in = colin && y >= 0 && y < H && y <= y1 + 1;
      const int s = in ? y * W + col : 0;
      const bool prod = in && y >= y0 && y < y1;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * n + s;
        R.r[c] = in ? b.r_in[o] : T(0);
        R.m[c] = in ? b.minv[o] : T(0);
        R.p[c] = (in && read_pold) ? b.p_in[o] : T(0);
        R.x[c] = (prod && write_out) ? b.x[o] : T(0);
        R.dmp[c] = (in && damped) ? b.damp[o] : T(0);
      }
#pragma unroll
      for (int q = 0; q < NS; ++q) R.st[q] = in ? e.state_plane(q)[s] : T(0);
      R.f = in ? (uint32_t)e.flags[s] : 0u;
    };
    // p_i = M^-1 r_i + beta p_{i-1} (the staged p holds p_{i-1})
    auto finish = [&](Row& R, const Row& P) {
      R = P;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const T u = R.m[c] * R.r[c];
        R.p[c] = read_pold ? fma(bT, P.p[c], u) : u;
      }
    };
    auto selp = [](const Row& R, int c) { return R.p[c]; };
    auto selu = [](const Row& R, int c) { return R.m[c]; };

    auto step = [&](auto PH, int k) {
      constexpr int ph = decltype(PH)::value;
      Row& R0 = ring[ph];            // row y = y0 - 2 + k
      Row& R1 = ring[(ph + 3) & 3];  // y - 1
      Row& R2 = ring[(ph + 2) & 3];  // y - 2
      Row& R3 = ring[(ph + 1) & 3];  // y - 3
      const int y = y0 - 2 + k;
      finish(R0, pre[ph]);
      issue(pre[ph], y + 4);
      if (k >= 2) {
        // s = A p and r_{i+1}, u_{i+1} on row y - 1
        T g[C];
        stream_apply(e, R2, R1, R0, selp, col, y - 1, g);
        const bool act = R1.f & E::ACTIVE;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const T sv = damped ? fma(R1.dmp[c], R1.p[c], g[c]) : g[c];
          R1.r[c] = act ? fma(-aT, sv, R1.r[c]) : T(0);
          R1.m[c] = act ? R1.m[c] * R1.r[c] : T(0);
        }
      }
      if (k >= 4) {
        // w = A u_{i+1} on row y - 2; partials and outputs
        const int yo = y - 2;
        T wv[C];
        stream_apply(e, R3, R2, R1, selu, col, yo, wv);
        const bool act = R2.f & E::ACTIVE;
        if (out_lane && act) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const T ww = damped ? fma(R2.dmp[c], R2.m[c], wv[c]) : wv[c];
            g_acc += (double)R2.r[c] * (double)R2.m[c];
            d_acc += (double)ww * (double)R2.m[c];
          }
        }
        if (write_out && out_lane) {
          const int s = yo * W + col;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const size_t o = (size_t)c * n + s;
            const T pv = act ? R2.p[c] : T(0);
            if (act) b.x[o] = fma(aT, pv, R2.x[c]);
            b.r_out[o] = R2.r[c];
            b.p_out[o] = pv;
          }
        }
      }
    };
    issue(pre[0], y0 - 2);
    issue(pre[1], y0 - 1);
    issue(pre[2], y0);
    issue(pre[3], y0 + 1);
    for (int k = 0; k < K; k += 4) {
      step(std::integral_constant<int, 0>{}, k);
      if (k + 1 < K) step(std::integral_constant<int, 1>{}, k + 1);
      if (k + 2 < K) step(std::integral_constant<int, 2>{}, k + 2);
      if (k + 3 < K) step(std::integral_constant<int, 3>{}, k + 3);
    }
  }
  const double gs_ = block_sum(g_acc);
  const double ds_ = block_sum(d_acc);
  if (threadIdx.x == 0) {
    b.part_out[blockIdx.x] = gs_;
    b.part_out[kMaxBlocks + blockIdx.x] = ds_;
  }
}

// ---------------------------------------------------------------- updates
// GN: x += d on active sites.  LM: the same, only if the step was accepted.
template <class E>
__global__ void __launch_bounds__(kBlock)
k_apply_step(E e, typename E::Real* __restrict__ x, const typename E::Real* __restrict__ delta,
             const DevScalars* __restrict__ S, int lm_gate) {
  constexpr int C = E::C;
  if (lm_gate && !S->accepted) return;
  const int n = e.n;
  OPT_SITE_LOOP(s, n) {
    if (!(e.flags[s] & E::ACTIVE)) continue;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      x[o] = x[o] + delta[o];
    }
  }
}

// ---------------------------------------------------------------- cost
// FP64 cost partials at x (delta == nullptr) or at the trial point x + delta,
// rounded to the bulk type exactly as k_apply_step would store it.
template <class E>
__global__ void __launch_bounds__(kBlock)
k_cost(E e, const typename E::Real* __restrict__ x, const typename E::Real* __restrict__ delta,
       double* __restrict__ part, const DevScalars* __restrict__ S, int lm_gate) {
  using T = typename E::Real;
  if (lm_gate && S->done) return;
  const int n = e.n;
  auto X = [&](int c, int s) -> double {
    const size_t o = (size_t)c * n + s;
    if (delta == nullptr) return (double)x[o];
    return (double)(T)(x[o] + delta[o]);
  };
  double acc = 0.0;
  OPT_SITE_LOOP(s, n) acc += e.cost(X, s);
  block_store(acc, part);
}

// LM model partials: sum_r (J d)_r (2 F_r + (J d)_r) at x.
template <class E>
__global__ void __launch_bounds__(kBlock)
k_model(E e, const typename E::Real* __restrict__ x, const typename E::Real* __restrict__ delta,
        double* __restrict__ part, const DevScalars* __restrict__ S) {
  if (S->done) return;
  const int n = e.n;
  auto X = [&](int c, int s) -> double { return (double)x[(size_t)c * n + s]; };
  auto D = [&](int c, int s) -> double { return (double)delta[(size_t)c * n + s]; };
  double acc = 0.0;
  OPT_SITE_LOOP(s, n) acc += e.model(X, D, s);
  block_store(acc, part);
}

// ---------------------------------------------------------------- scalar kernels
struct LMConsts {
  double radius_min, radius_max, min_rel_decrease;
};

// Single block.  Sets up the scalars of a solve.
__global__ void k_setup(DevScalars* S, double lambda, double radius0, int lm) {
  if (threadIdx.x == 0) {
    S->rz[0] = S->rz[1] = 0.0;
    S->gam[0] = S->gam[1] = 0.0;
    S->alpha[0] = S->alpha[1] = 0.0;
    S->E0 = S->E1 = S->m = 0.0;
    S->radius = radius0;
    S->nu = 2.0;
    S->lambda = lm ? 1.0 / radius0 : lambda;
    S->E_final = 0.0;
    S->stopped = 0;
    S->accepted = 0;
    S->need_lin = 1;
    S->done = 0;
    S->n_accepted = 0;
    S->outer_done = 0;
    S->nonfinite = 0;
  }
}

// Single block.  LM step decision (gain ratio, Nielsen radius update).
__global__ void k_lm_decide(DevScalars* S, const double* __restrict__ m_part,
                            const double* __restrict__ c_part, int nb, LMConsts lc) {
  if (S->done) return;
  // the partials hold sum (J d)(2F + J d); the model decrease is its negation
  const double m = -reduce_partials(m_part, nb);
  const double E1 = reduce_partials(c_part, nb);
  if (threadIdx.x == 0) {
    S->m = m;
    S->E1 = E1;
    if (!finite_d(E1)) S->nonfinite = 1;
    const double rho = m != 0.0 ? (S->E0 - E1) / m : -INFINITY;
    if (m > 0.0 && rho > lc.min_rel_decrease) {
      const double t = 2.0 * rho - 1.0;
      const double f = fmax(1.0 / 3.0, 1.0 - t * t * t);
      S->radius = fmin(S->radius / f, lc.radius_max);
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
    if (S->radius < lc.radius_min) S->done = 1;
    S->lambda = 1.0 / S->radius;
  }
}

// Single block.  Finish a cost reduction into E_final (and optionally a trace slot).
__global__ void k_finish_cost(DevScalars* S, const double* __restrict__ part, int nb,
                              double* __restrict__ trace, int trace_idx) {
  const double E = reduce_partials(part, nb);
  if (threadIdx.x == 0) {
    S->E_final = E;
    if (!finite_d(E)) S->nonfinite = 1;
    if (trace) trace[trace_idx] = E;
  }
}

}  // namespace optmi
