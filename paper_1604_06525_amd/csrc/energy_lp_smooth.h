// Edge-preserving image smoothing with an l_p regulariser, solved by
// iteratively reweighted least squares (Sec. 7, variants of GN/LM).
//
// One unknown per pixel; data A (1 plane); params w_fit, w_reg, p, eps.
//   fit   r = w_fit (X_p - A_p)                        (squared: l_2)
//   edge  f = w_reg (X(i,j) - X(i+1,j)), w_reg (X(i,j) - X(i,j+1)) where the
//         neighbour is on the grid, entering the objective as (f^2 + eps^2)^(p/2)
// Objective (the cost the solver reports): sum r^2 + sum_edges (f^2 + eps^2)^(p/2).
// Each linearisation freezes a weight per edge at the current x,
//   w = (p/2) (f^2 + eps^2)^((p-2)/2),
// and the PCG solves the least-squares problem sum r^2 + sum w f^2 with those
// weights fixed (no derivative of w): one IRLS iteration per Gauss-Newton step.
// The paper's weight f^(p-2) is for a sum of l_p terms alone; eps keeps it
// finite at f = 0, and the factor p/2 makes a fixed point of the iteration a
// stationary point of the objective when the l_2 data term is present.
// The weights are the per-pixel state: (w of the edge to the right, w of the edge
// below).  Products at pixel s with in-grid neighbours q, w_sq the edge weight:
//   (J^T J P)_s = w_fit^2 P_s + w_reg^2 sum_q w_sq (P_s - P_q)
//   b_s = -w_fit^2 (X_s - A_s) - w_reg^2 sum_q w_sq (X_s - X_q)
//   diag_s = w_fit^2 + w_reg^2 sum_q w_sq
// Levenberg-Marquardt is not offered for this energy (its step test would
// compare the objective with the model of the reweighted problem).
#pragma once
#include "common.h"

namespace optmi {

template <typename T>
struct LpSmoothGrid {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 1;
  static constexpr int kStatePlanes = 2;
  static constexpr int kOwnState = 2;
  static constexpr int kRadius = 1;
  // fused strip walk in FP32: three rows ahead and d loaded with its row (four
  // rows measured 4% slower, d a step ahead 4% slower, the peeled walk 13%)
  static constexpr int kFusedPrefetch = sizeof(T) == 4 ? 3 : 2;
  static constexpr int kFusedWalk = sizeof(T) == 4 ? 1 : 0;
  enum : uint32_t { ACTIVE = 1, INGRID = 2 };

  int W, H, n;
  const T* __restrict__ A;
  T* __restrict__ st;  // [n][2]: weight of the edge to the right, of the edge below (0 off the grid)
  uint8_t* __restrict__ flags;
  T wf2, wr2;                       // squared weights
  double wf_d, wr_d, p_d, eps2_d;   // weights, p and eps^2 (objective and weights in FP64)

  __device__ __forceinline__ T state_at(int k, int s) const { return st[(size_t)s * 2 + k]; }
  __device__ __forceinline__ const T* state_base() const { return st; }

  __device__ __forceinline__ double weight(double f) const {
    return 0.5 * p_d * pow(f * f + eps2_d, 0.5 * (p_d - 2.0));
  }
  __device__ __forceinline__ double smooth_term(double f) const { return pow(f * f + eps2_d, 0.5 * p_d); }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int s) const {
    const int i = s % W, j = s / W;
    const double r = wf_d * (X(0, s) - (double)A[s]);
    double e = r * r;
    if (i + 1 < W) e += smooth_term(wr_d * (X(0, s) - X(0, s + 1)));
    if (j + 1 < H) e += smooth_term(wr_d * (X(0, s) - X(0, s + W)));
    return e;
  }

  // Freeze the weights of the two edges anchored at s at the current x.
  __device__ __forceinline__ void linearize(const T* __restrict__ x, int s) const {
    const int i = s % W, j = s / W;
    const double xs = (double)x[s];
    st[(size_t)s * 2] = i + 1 < W ? (T)weight(wr_d * (xs - (double)x[s + 1])) : T(0);
    st[(size_t)s * 2 + 1] = j + 1 < H ? (T)weight(wr_d * (xs - (double)x[s + W])) : T(0);
    flags[s] = (uint8_t)(INGRID | ACTIVE);
  }

  // the weight of the edge from the centre to neighbour k (0: right, 1: left,
  // 2: below, 3: above), 0 where that neighbour is off the grid
  template <class SV, class FV>
  __device__ __forceinline__ T wedge(SV S, FV F, int k) const {
    const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
    if (!(F(di, dj) & INGRID)) return T(0);
    return k == 0 ? S(0, 0, 0) : k == 1 ? S(0, -1, 0) : k == 2 ? S(1, 0, 0) : S(1, 0, -1);
  }

  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV S, FV F, int s, int, int, T* b, T* d) const {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      acc = fma(wedge(S, F, k), X(0, 0, 0) - X(0, di, dj), acc);
    }
    b[0] = -wf2 * (X(0, 0, 0) - A[s]) - wr2 * acc;
    diag(S, F, d);
  }

  template <class SV, class FV>
  __device__ __forceinline__ void diag(SV S, FV F, T* d) const {
    const T ws = (wedge(S, F, 0) + wedge(S, F, 1)) + (wedge(S, F, 2) + wedge(S, F, 3));
    d[0] = fma(wr2, ws, wf2);
  }

  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV S, FV F, int, int, T* g) const {
    const T p0 = P(0, 0, 0);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      acc = fma(wedge(S, F, k), p0 - P(0, di, dj), acc);
    }
    g[0] = fma(wr2, acc, wf2 * p0);
  }

  // The centre's share of |J u|^2: its fit row plus half of each weighted
  // edge row it is an end of (symmetric in the four directions).
  template <class PV, class SV, class FV>
  __device__ __forceinline__ T jsq(PV U, SV S, FV F, int, int) const {
    const T u = U(0, 0, 0);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T e = u - U(0, di, dj);
      acc = fma(wedge(S, F, k) * e, e, acc);
    }
    return fma(T(0.5) * wr2, acc, wf2 * u * u);
  }

  // The model decrease of the reweighted problem (kept for completeness: the
  // solver does not run Levenberg-Marquardt on this energy).
  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    const int i = s % W, j = s / W;
    const double f = wf_d * (X(0, s) - (double)A[s]), jd = wf_d * Dl(0, s);
    double acc = jd * (2.0 * f + jd);
    auto edge = [&](int q, int k) {
      const double w = (double)st[(size_t)s * 2 + k];
      const double fe = wr_d * (X(0, s) - X(0, q)), je = wr_d * (Dl(0, s) - Dl(0, q));
      acc += w * je * (2.0 * fe + je);
    };
    if (i + 1 < W) edge(s + 1, 0);
    if (j + 1 < H) edge(s + W, 1);
    return acc;
  }
};

}  // namespace optmi
