// Intrinsic image decomposition (A.2.4, Fig. 33), solved by iteratively
// reweighted least squares (Sec. 7, variants of GN/LM).
//
// Unknowns per pixel: reflectance r (3 channels) and shading s, channels
// (r0, r1, r2, s).  Data I (3 planes, log domain); params w_fit, w_a, w_s, p, eps.
//   fit        w_fit (r_c + s - I_c), c = 0..2                         (squared)
//   reflectance, for each stencil neighbour q on the grid (+x, -x, +y, -y):
//              f = w_a (r - r_q), entering as (|f|^2 + eps^2)^(p/2)
//   shading, for the same neighbours: w_s (s - s_q)                   (squared)
// Each edge is a residual at both of its ends.  The cost the solver reports is
// sum fit^2 + sum_(pixel, q) [(|f|^2 + eps^2)^(p/2) + (w_s (s - s_q))^2].
// Each linearisation freezes one weight per edge at the current x,
//   w = (p/2) (|f|^2 + eps^2)^((p-2)/2)
// (the paper's |f|^(p-2), with eps keeping it finite and the factor p/2 making
// a fixed point stationary beside the l_2 fit), and the PCG solves the least-
// squares problem with the reflectance rows scaled by sqrt(w).  The weights are
// the per-pixel state: (w of the edge to the right, w of the edge below).  With
// w_k the weight towards neighbour k, m_k = 1 where it is on the grid:
//   (J^T J P)_rc = w_fit^2 (P_rc + P_s) + 2 w_a^2 sum_k w_k (P_rc - P_rc(q_k))
//   (J^T J P)_s  = w_fit^2 sum_c (P_rc + P_s) + 2 w_s^2 sum_k m_k (P_s - P_s(q_k))
//   diag_rc = w_fit^2 + 2 w_a^2 sum_k w_k,   diag_s = 3 w_fit^2 + 2 w_s^2 sum_k m_k
// (a uniform shift down of r and up of s changes nothing: the normal equations
// are semidefinite, and PCG from d = 0 keeps to their range).  Levenberg-
// Marquardt is not offered (its step test would compare the objective with the
// model of the reweighted problem).
#pragma once
#include "common.h"

namespace optmi {

template <typename T>
struct IntrinsicImage {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 4;
  static constexpr int kStatePlanes = 2;
  static constexpr int kOwnState = 2;
  static constexpr int kRadius = 1;
  static constexpr int kFusedWalk = sizeof(T) == 4 ? 1 : 0;  // FP32: d loaded with its row (the peeled walk was slower)
  enum : uint32_t { ACTIVE = 1, INGRID = 2 };

  int W, H, n;
  const T* __restrict__ I;  // [3][n]
  T* __restrict__ st;       // [n][2]: weight of the edge to the right, of the edge below (0 off the grid)
  uint8_t* __restrict__ flags;
  T wf2, wa2, ws2;                      // squared weights
  double wf_d, wa_d, ws_d, p_d, eps2_d;  // weights, p and eps^2 (objective and weights in FP64)

  __device__ __forceinline__ T state_at(int k, int s) const { return st[(size_t)s * 2 + k]; }
  __device__ __forceinline__ const T* state_base() const { return st; }

  __device__ __forceinline__ double weight(double f2) const {
    return 0.5 * p_d * pow(f2 + eps2_d, 0.5 * (p_d - 2.0));
  }

  // |f|^2 of the reflectance edge between sites s and q, x caller-facing planes
  template <class XA>
  __device__ __forceinline__ double f2_of(XA X, int s, int q) const {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double d = wa_d * (X(c, s) - X(c, q));
      a += d * d;
    }
    return a;
  }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int s) const {
    const int i = s % W, j = s / W;
    double e = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double f = wf_d * (X(c, s) + X(3, s) - (double)I[(size_t)c * n + s]);
      e += f * f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (i + di < 0 || i + di >= W || j + dj < 0 || j + dj >= H) continue;
      const int q = s + dj * W + di;
      e += pow(f2_of(X, s, q) + eps2_d, 0.5 * p_d);
      const double g = ws_d * (X(3, s) - X(3, q));
      e += g * g;
    }
    return e;
  }

  // Freeze the weights of the two edges anchored at s at the current x.
  __device__ __forceinline__ void linearize(const T* __restrict__ x, int s) const {
    const int i = s % W, j = s / W;
    auto X = [&](int c, int site) -> double { return (double)x[(size_t)c * n + site]; };
    st[(size_t)s * 2] = i + 1 < W ? (T)weight(f2_of(X, s, s + 1)) : T(0);
    st[(size_t)s * 2 + 1] = j + 1 < H ? (T)weight(f2_of(X, s, s + W)) : T(0);
    flags[s] = (uint8_t)(INGRID | ACTIVE);
  }

  // the weight of the reflectance edge from the centre to neighbour k (0:
  // right, 1: left, 2: below, 3: above), 0 where that neighbour is off the grid
  template <class SV, class FV>
  __device__ __forceinline__ T wedge(SV S, FV F, int k) const {
    const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
    if (!(F(di, dj) & INGRID)) return T(0);
    return k == 0 ? S(0, 0, 0) : k == 1 ? S(0, -1, 0) : k == 2 ? S(1, 0, 0) : S(1, 0, -1);
  }

  template <class SV, class FV>
  __device__ __forceinline__ void diag(SV S, FV F, T* d) const {
    T ws = T(0), cnt = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      ws += wedge(S, F, k);
      cnt += (F(di, dj) & INGRID) ? T(1) : T(0);
    }
    const T dr = fma(T(2) * wa2, ws, wf2);
    d[0] = d[1] = d[2] = dr;
    d[3] = fma(T(2) * ws2, cnt, T(3) * wf2);
  }

  // g = (J^T J) P at the centre, or (X for P) the gradient part of J^T F
  // without the data; shared by apply and jtf_diag
  template <class PV, class SV, class FV>
  __device__ __forceinline__ void jtj(PV P, SV S, FV F, T* g) const {
    T acc[4] = {};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = wedge(S, F, k);
      const T m = (F(di, dj) & INGRID) ? T(1) : T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = fma(w, P(c, 0, 0) - P(c, di, dj), acc[c]);
      acc[3] = fma(m, P(3, 0, 0) - P(3, di, dj), acc[3]);
    }
    const T ps = P(3, 0, 0);
    T sum = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T f = P(c, 0, 0) + ps;
      sum += f;
      g[c] = fma(T(2) * wa2, acc[c], wf2 * f);
    }
    g[3] = fma(T(2) * ws2, acc[3], wf2 * sum);
  }

  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV S, FV F, int s, int, int, T* b, T* d) const {
    // J^T F = (J^T J) X with the fit's data term moved out: fit rows are
    // w_fit (r_c + s - I_c), the others are linear in X with no constant
    T g[4];
    jtj(X, S, F, g);
    T isum = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T ic = I[(size_t)c * n + s];
      isum += ic;
      b[c] = -fma(-wf2, ic, g[c]);
    }
    b[3] = -fma(-wf2, isum, g[3]);
    diag(S, F, d);
  }

  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV S, FV F, int, int, T* g) const {
    jtj(P, S, F, g);
  }

  // The centre's share of |J u|^2: its three fit rows and the reflectance and
  // shading rows of its four outgoing edges (every row belongs to one pixel).
  template <class PV, class SV, class FV>
  __device__ __forceinline__ T jsq(PV U, SV S, FV F, int, int) const {
    const T us = U(3, 0, 0);
    T fit = T(0), refl = T(0), shad = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T f = U(c, 0, 0) + us;
      fit = fma(f, f, fit);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = wedge(S, F, k);
      const T m = (F(di, dj) & INGRID) ? T(1) : T(0);
      T e2 = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T e = U(c, 0, 0) - U(c, di, dj);
        e2 = fma(e, e, e2);
      }
      refl = fma(w, e2, refl);
      const T es = us - U(3, di, dj);
      shad = fma(m * es, es, shad);
    }
    return fma(wf2, fit, fma(wa2, refl, ws2 * shad));
  }

  // The model decrease of the reweighted problem (kept for completeness: the
  // solver does not run Levenberg-Marquardt on this energy).
  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    const int i = s % W, j = s / W;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double f = wf_d * (X(c, s) + X(3, s) - (double)I[(size_t)c * n + s]);
      const double jd = wf_d * (Dl(c, s) + Dl(3, s));
      acc += jd * (2.0 * f + jd);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (i + di < 0 || i + di >= W || j + dj < 0 || j + dj >= H) continue;
      const int q = s + dj * W + di;
      const int a = k == 1 ? q : (k == 3 ? q : s);  // the edge's anchor
      const double w = (double)st[(size_t)a * 2 + (k >= 2 ? 1 : 0)];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double fe = wa_d * (X(c, s) - X(c, q)), je = wa_d * (Dl(c, s) - Dl(c, q));
        acc += w * je * (2.0 * fe + je);
      }
      const double fs = ws_d * (X(3, s) - X(3, q)), js = ws_d * (Dl(3, s) - Dl(3, q));
      acc += js * (2.0 * fs + js);
    }
    return acc;
  }
};

}  // namespace optmi
