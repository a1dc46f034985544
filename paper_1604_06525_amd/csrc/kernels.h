// Kernels of one solve, generic over the energy.
//
// One PCG iteration (Sec. 4.1) is two kernels.  Kernel boundaries are the only
// grid-wide synchronisation: a scalar that needs a sum over the whole problem
// (p.q, r.z) is produced as per-block FP64 partials by one kernel and summed,
// in a fixed order, by every block of the next kernel, so no fence or atomic is
// needed and the result is the same on every run.
//
//   pcg_a(k):  beta = rz_k / rz_{k-1} (k > 0);  p_k = z_k + beta p_{k-1}, with
//              z = M^-1 r, evaluated on the fly for each site and for the
//              neighbours its product reads;  q = (J^T J + lambda D) p_k;
//              write p_k and q;  partials of p_k . q.
//   pcg_b(k):  alpha = rz_k / (p.q);  d += alpha p;  r -= alpha q;
//              z = M^-1 r;  partials of r . z = rz_{k+1}.
//
// If p.q is not positive the PCG stops (DevScalars::stopped) and every later
// iteration kernel returns at once, which leaves d as it was.
#pragma once
#include "common.h"

namespace optmi {

// Grid-stride loop over sites with a fixed per-thread order (the grid size
// depends only on n), so the partial sums are reproducible.
#define OPT_SITE_LOOP(s, n) \
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < (n); s += gridDim.x * kBlock)

// ---------------------------------------------------------------- linearize
template <class E>
__global__ void __launch_bounds__(kBlock)
k_linearize(E e, const typename E::Real* __restrict__ x, double* __restrict__ part,
            const DevScalars* __restrict__ S, int lm_gate) {
  using T = typename E::Real;
  if (lm_gate && (S->done || !S->need_lin)) return;
  double acc = 0.0;
  const int n = e.n;
  auto X = [&](int ch, int s) -> double { return (double)x[(size_t)ch * n + s]; };
  OPT_SITE_LOOP(s, n) {
    e.linearize(x, s);
    acc += e.cost(X, s);
  }
  block_store(acc, part);
  (void)sizeof(T);
}

// ---------------------------------------------------------------- init
// r = b = -J^T F, diag = diag(J^T J), d = 0, rz_0 partials; also finishes the
// cost of the linearisation (trace entry k) and resets the PCG state.
template <class E>
__global__ void __launch_bounds__(kBlock)
k_init(E e, const typename E::Real* __restrict__ x, typename E::Real* __restrict__ r,
       typename E::Real* __restrict__ diag, typename E::Real* __restrict__ delta,
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
    if (e.active(s)) {
      e.jtf_diag(x, s, b, d);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) { b[c] = T(0); d[c] = T(0); }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      r[o] = b[c];
      diag[o] = d[c];
      delta[o] = T(0);
      const T z = pc.minv(d[c]) * b[c];
      rz += (double)b[c] * (double)z;
    }
  }
  block_store(rz, rz_part);
}

// ---------------------------------------------------------------- pcg_a
// MODE 0: PCG iteration (p from r, the previous p and beta).
// MODE 1: plain product q = (J^T J + lambda D) p_in (p_in passed as `pold`).
template <class E, int MODE>
__global__ void __launch_bounds__(kBlock)
k_pcg_a(E e, int k, const typename E::Real* __restrict__ r, const typename E::Real* __restrict__ diag,
        const typename E::Real* __restrict__ pold, typename E::Real* __restrict__ pnew,
        typename E::Real* __restrict__ q, const double* __restrict__ rz_part, int n_rz,
        double* __restrict__ pq_part, DevScalars* S, Precond<typename E::Real> pc, int lm_gate) {
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
  if (lm_gate) pc.lam = (T)S->lambda;
  auto P = [&](int c, int s) -> T {
    const size_t o = (size_t)c * n + s;
    if (MODE == 1) return pold[o];
    const T z = pc.minv(diag[o]) * r[o];
    return k == 0 ? z : fma(beta, pold[o], z);
  };
  double pq = 0.0;
  OPT_SITE_LOOP(s, n) {
    T g[C];
    const bool act = e.active(s);
    if (act) e.jtjp(s, P, g);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      T pv = T(0), qv = T(0);
      if (act) {
        pv = P(c, s);
        qv = g[c];
        if (pc.lam != T(0)) qv += pc.damp(diag[o]) * pv;
      }
      if (MODE == 0) pnew[o] = pv;
      q[o] = qv;
      pq += (double)pv * (double)qv;
    }
  }
  if (MODE == 0) block_store(pq, pq_part);
}

// ---------------------------------------------------------------- pcg_b
template <typename T, int C>
__global__ void __launch_bounds__(kBlock)
k_pcg_b(int n, int k, const uint8_t* __restrict__ flags_unused, T* __restrict__ delta,
        T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
        const T* __restrict__ diag, const double* __restrict__ pq_part, int n_pq,
        double* __restrict__ rz_part, DevScalars* S, Precond<T> pc, int lm_gate) {
  if (S->stopped || (lm_gate && S->done)) return;
  const double pq = reduce_partials(pq_part, n_pq);
  if (!(pq > 0.0)) {
    if (is_block_leader()) S->stopped = 1;
    return;
  }
  if (lm_gate) pc.lam = (T)S->lambda;
  const T alpha = (T)(S->rz[k & 1] / pq);
  double rz = 0.0;
  OPT_SITE_LOOP(s, n) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = (size_t)c * n + s;
      const T pv = p[o];
      delta[o] = fma(alpha, pv, delta[o]);
      const T rv = fma(-alpha, q[o], r[o]);
      r[o] = rv;
      const T z = pc.minv(diag[o]) * rv;
      rz += (double)rv * (double)z;
    }
  }
  block_store(rz, rz_part);
  (void)flags_unused;
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
    if (!e.active(s)) continue;
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

// LM model decrease partials: sum_r (J d)_r (2 F_r + (J d)_r) at x.
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
