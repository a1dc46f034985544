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
#include "common.h"

namespace optmi {

// Grid-stride loop over sites with a fixed per-thread order (the grid size
// depends only on n), so the partial sums are reproducible.
#define OPT_SITE_LOOP(s, n) \
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < (n); s += gridDim.x * kBlock)

// Views over global memory centred at site s = j*W + i of a W x H grid.
#define OPT_GRID_VIEWS(e, s)                                                          \
  const int vi_ = (s) % (e).W, vj_ = (s) / (e).W;                                     \
  auto Fg = [&](int di, int dj) -> uint32_t {                                         \
    const int ii = vi_ + di, jj = vj_ + dj;                                           \
    return (ii >= 0 && ii < (e).W && jj >= 0 && jj < (e).H) ? (e).flags[(s) + dj * (e).W + di] \
                                                            : 0u;                     \
  };                                                                                  \
  auto Sg = [&](int k, int di, int dj) { return (e).state_plane(k)[(s) + dj * (e).W + di]; };

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
    OPT_GRID_VIEWS(e, s)
    if (Fg(0, 0) & E::ACTIVE) {
      auto Xg = [&](int c, int di, int dj) { return x[(size_t)c * n + s + dj * e.W + di]; };
      e.jtf_diag(Xg, Sg, Fg, s, b, d);
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
  OPT_SITE_LOOP(s, n) {
    OPT_GRID_VIEWS(e, s)
    auto Pg = [&](int c, int di, int dj) -> T {
      const size_t o = (size_t)c * n + s + dj * e.W + di;
      if (MODE == 1) return b.pold[o];
      const T z = b.minv[o] * b.r[o];
      return k == 0 ? z : fma(beta, b.pold[o], z);
    };
    T g[C];
    const bool act = Fg(0, 0) & E::ACTIVE;
    if (act) e.apply(Pg, Sg, Fg, g);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      T pv = T(0), qv = T(0);
      if (act) {
        pv = Pg(c, 0, 0);
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

// Tile geometry: TW x TH sites per tile, halo 2*radius, one tile at a time per
// block; blocks stride over the tiles in an XCD-aware order.
template <class E, int TW, int TH>
struct FusedGeom {
  static constexpr int HALO = 2 * E::kRadius;
  static constexpr int RW = TW + 2 * HALO, RH = TH + 2 * HALO, N = RW * RH;
  static constexpr int R1 = HALO - E::kRadius;              // ring-1 offset in the region
  static constexpr int R1W = TW + 2 * E::kRadius, R1H = TH + 2 * E::kRadius;
};

// The k-th tile of this block.  Blocks are spread over the 8 XCDs round-robin;
// each XCD takes one contiguous run of tiles so neighbouring tiles share its L2.
__device__ __forceinline__ int tile_of(int k, int n_tiles) {
  const int G = gridDim.x;
  if (G % 8 != 0) return blockIdx.x + k * G;
  const int per = G / 8, xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int chunk = (n_tiles + 7) / 8;
  const int t = xcd * chunk + slot + k * per;
  return t < min((xcd + 1) * chunk, n_tiles) ? t : n_tiles;
}

template <class E, int TW, int TH>
__global__ void __launch_bounds__(kBlock, 2)
k_fused(E e, FusedBufs<typename E::Real> b, DevScalars* S, int iter, int lm_gate, int tiles_x,
        int n_tiles) {
  using T = typename E::Real;
  using G = FusedGeom<E, TW, TH>;
  constexpr int C = E::C, NS = E::kStatePlanes, N = G::N, RW = G::RW;
  __shared__ T sP[C * N], sR[C * N], sM[C * N], sS[NS * N];
  __shared__ uint8_t sF[N];

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
  const int W = e.W, H = e.H, n = e.n;
  double g_acc = 0.0, d_acc = 0.0;

  for (int k = 0;; ++k) {
    const int tile = tile_of(k, n_tiles);
    if (tile >= n_tiles) break;
    const int tx0 = (tile % tiles_x) * TW - G::HALO, ty0 = (tile / tiles_x) * TH - G::HALO;
    // phase 1: stage the region; p_i = M^-1 r_i + beta p_{i-1}
    for (int t = threadIdx.x; t < N; t += kBlock) {
      const int i = tx0 + t % RW, j = ty0 + t / RW;
      if (i >= 0 && i < W && j >= 0 && j < H) {
        const int s = j * W + i;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const size_t o = (size_t)c * n + s;
          const T r = b.r_in[o], m = b.minv[o];
          const T u = m * r;
          sP[c * N + t] = iter > 0 ? fma(bT, b.p_in[o], u) : u;
          sR[c * N + t] = r;
          sM[c * N + t] = m;
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) sS[q * N + t] = e.state_plane(q)[s];
        sF[t] = e.flags[s];
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          sP[c * N + t] = T(0);
          sR[c * N + t] = T(0);
          sM[c * N + t] = T(0);
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) sS[q * N + t] = T(0);
        sF[t] = 0;
      }
    }
    __syncthreads();
    // phase 2: s_i = A p_i and r_{i+1} = r_i - alpha s_i on the tile plus one radius
    for (int t = threadIdx.x; t < G::R1W * G::R1H; t += kBlock) {
      const int rx = G::R1 + t % G::R1W, ry = G::R1 + t / G::R1W;
      const int idx = ry * RW + rx;
      if (!(sF[idx] & E::ACTIVE)) continue;
      auto Pv = [&](int c, int di, int dj) { return sP[c * N + idx + dj * RW + di]; };
      auto Sv = [&](int q, int di, int dj) { return sS[q * N + idx + dj * RW + di]; };
      auto Fv = [&](int di, int dj) -> uint32_t { return sF[idx + dj * RW + di]; };
      T g[C];
      e.apply(Pv, Sv, Fv, g);
      if (b.damp) {
        const int s = (ty0 + ry) * W + (tx0 + rx);
#pragma unroll
        for (int c = 0; c < C; ++c) g[c] += b.damp[(size_t)c * n + s] * sP[c * N + idx];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) sR[c * N + idx] = fma(-aT, g[c], sR[c * N + idx]);
    }
    __syncthreads();
    // phase 3: w = A u_{i+1} on the tile; partials; d += alpha p_i; store r, p
    for (int t = threadIdx.x; t < TW * TH; t += kBlock) {
      const int rx = G::HALO + t % TW, ry = G::HALO + t / TW;
      const int i = tx0 + rx, j = ty0 + ry;
      if (i >= W || j >= H) continue;
      const int idx = ry * RW + rx, s = j * W + i;
      const bool act = sF[idx] & E::ACTIVE;
      if (act) {
        auto Uv = [&](int c, int di, int dj) {
          const int o = c * N + idx + dj * RW + di;
          return sM[o] * sR[o];
        };
        auto Sv = [&](int q, int di, int dj) { return sS[q * N + idx + dj * RW + di]; };
        auto Fv = [&](int di, int dj) -> uint32_t { return sF[idx + dj * RW + di]; };
        T w[C];
        e.apply(Uv, Sv, Fv, w);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const T uo = Uv(c, 0, 0);
          if (b.damp) w[c] += b.damp[(size_t)c * n + s] * uo;
          g_acc += (double)sR[c * N + idx] * (double)uo;
          d_acc += (double)w[c] * (double)uo;
        }
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * n + s;
        const T pv = act ? sP[c * N + idx] : T(0);
        if (iter >= 0 && act) b.x[o] = fma(aT, pv, b.x[o]);
        b.r_out[o] = sR[c * N + idx];
        b.p_out[o] = pv;
      }
    }
    __syncthreads();
  }
  const double gs = block_sum(g_acc);
  const double ds = block_sum(d_acc);
  if (threadIdx.x == 0) {
    b.part_out[blockIdx.x] = gs;
    b.part_out[kMaxBlocks + blockIdx.x] = ds;
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
