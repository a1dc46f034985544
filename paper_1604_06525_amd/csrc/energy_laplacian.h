// Laplacian smoothing: the paper's introductory energy (Fig. 3 on an image,
// Fig. 5 on a graph).
//
// Grid (one unknown per pixel): data A (1 plane), params w_fit, w_reg.
//   fit  r = w_fit (X_p - A_p)
//   h    r = w_reg (X(i,j) - X(i+1,j))   where (i+1, j) is on the grid
//   v    r = w_reg (X(i,j) - X(i,j+1))   where (i, j+1) is on the grid
// Graph (three unknowns per vertex, float3): data A (3 planes), params w_fit,
// w_reg.
//   fit  r = w_fit (X_v - A_v) per component
//   edge r = w_reg (X_v0 - X_v1) per component, once per listed edge
// Both are linear: J^T J = w_fit^2 I + w_reg^2 L with L the graph Laplacian of
// the pixel lattice or of the listed edges, so one Gauss-Newton step with an
// exact inner solve reaches the minimiser.
//
// Matrix-free products at a site p with neighbours q (the lattice's in-grid
// 4-neighbourhood, or the incidence list):
//   (J^T J P)_p = w_fit^2 P_p + w_reg^2 sum_q (P_p - P_q)
//   b_p = -w_fit^2 (X_p - A_p) - w_reg^2 sum_q (X_p - X_q)
//   diag_p = w_fit^2 + w_reg^2 * (number of q other than p itself)
#pragma once
#include "common.h"

namespace optmi {

template <typename T>
struct LaplacianGrid {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 1;
  static constexpr int kStatePlanes = 0;
  static constexpr int kOwnState = 0;
  static constexpr int kRadius = 1;
  static constexpr int kFusedWalk = sizeof(T) == 4 ? 1 : 0;  // fused strip walk in FP32: d loaded with its row
  static constexpr int kFusedPrefetch = sizeof(T) == 4 ? 3 : 2;  // rows ahead (four measured 7% slower in FP32)
  enum : uint32_t { ACTIVE = 1, INGRID = 2 };

  int W, H, n;
  const T* __restrict__ A;
  uint8_t* __restrict__ flags;
  T wf2, wr2;          // squared weights
  double wf_d, wr_d;   // weights (cost and model in FP64)

  __device__ __forceinline__ T state_at(int, int) const { return T(0); }
  __device__ __forceinline__ const T* state_base() const { return nullptr; }

  // residuals anchored at s (fit, h, v) in FP64
  template <class XA>
  __device__ __forceinline__ void anchored(XA X, int s, double* r, bool* on) const {
    const int i = s % W, j = s / W;
    r[0] = wf_d * (X(0, s) - (double)A[s]);
    on[0] = true;
    on[1] = i + 1 < W;
    on[2] = j + 1 < H;
    r[1] = on[1] ? wr_d * (X(0, s) - X(0, s + 1)) : 0.0;
    r[2] = on[2] ? wr_d * (X(0, s) - X(0, s + W)) : 0.0;
  }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int s) const {
    double r[3];
    bool on[3];
    anchored(X, s, r, on);
    return r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  }

  __device__ __forceinline__ void linearize(const T* __restrict__, int s) const {
    flags[s] = (uint8_t)(INGRID | ACTIVE);
  }

  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV, FV F, int s, int, int, T* b, T* d) const {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & INGRID)) continue;
      acc += X(0, 0, 0) - X(0, di, dj);
    }
    b[0] = -wf2 * (X(0, 0, 0) - A[s]) - wr2 * acc;
    diag(nullptr, F, d);
  }

  template <class SV, class FV>
  __device__ __forceinline__ void diag(SV, FV F, T* d) const {
    T cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      cnt += (F(di, dj) & INGRID) ? T(1) : T(0);
    }
    d[0] = wf2 + wr2 * cnt;
  }

  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV, FV F, int, int, T* g) const {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & INGRID)) continue;
      acc += P(0, 0, 0) - P(0, di, dj);
    }
    g[0] = wf2 * P(0, 0, 0) + wr2 * acc;
  }

  // The centre's share of |J u|^2: its fit residual squared plus half of each
  // squared difference to a neighbour on the grid (each lattice edge's
  // residual is shared by its two pixels).  Summed over all sites this is
  // |J u|^2.  Symmetric in the four directions, as the fused kernel needs (a
  // strip may walk its rows upwards, so "below" can be either neighbour).
  template <class PV, class SV, class FV>
  __device__ __forceinline__ T jsq(PV U, SV, FV F, int, int) const {
    const T u = U(0, 0, 0);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T e = (F(di, dj) & INGRID) ? u - U(0, di, dj) : T(0);
      acc += e * e;
    }
    return wf2 * u * u + T(0.5) * wr2 * acc;
  }

  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    double r[3];
    bool on[3];
    anchored(X, s, r, on);
    const double jd[3] = {wf_d * Dl(0, s), on[1] ? wr_d * (Dl(0, s) - Dl(0, s + 1)) : 0.0,
                          on[2] ? wr_d * (Dl(0, s) - Dl(0, s + W)) : 0.0};
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) acc += jd[k] * (2.0 * r[k] + jd[k]);
    return acc;
  }
};

template <typename T>
struct LaplacianGraph {
  using Real = T;
  static constexpr bool kGraph = true;
  static constexpr int C = 3;
  static constexpr int kStatePlanes = 0;
  static constexpr int kOwnState = 0;
  static constexpr int kRadius = 1;
  enum : uint32_t { ACTIVE = 1, INGRID = 2 };

  int n;
  const int* __restrict__ rp;   // [n+1] incidence offsets
  const int* __restrict__ nb;   // [2E] neighbour ids
  const T* __restrict__ A;      // [3][n]
  uint8_t* __restrict__ flags;
  T wf2, wr2;
  double wf_d, wr_d;

  // Each listed edge is counted once in the cost and the model: at the end
  // with the smaller id (a loop {v, v} has a zero residual).
  template <class XA>
  __device__ __forceinline__ double cost(XA X, int v) const {
    double e = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double f = wf_d * (X(c, v) - (double)A[(size_t)c * n + v]);
      e += f * f;
    }
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
      if (u <= v) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double f = wr_d * (X(c, v) - X(c, u));
        e += f * f;
      }
    }
    return e;
  }

  __device__ __forceinline__ void linearize(const T* __restrict__, int v) const {
    flags[v] = (uint8_t)(INGRID | ACTIVE);
  }

  template <class XA>
  __device__ __forceinline__ void jtf_diag_site(XA X, int v, T* b, T* dg) const {
    T acc[3] = {}, cnt = 0;
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
      if (u == v) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += X(c, v) - X(c, u);
      cnt += T(1);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      b[c] = -wf2 * (X(c, v) - A[(size_t)c * n + v]) - wr2 * acc[c];
      dg[c] = wf2 + wr2 * cnt;
    }
  }

  template <class PA>
  __device__ __forceinline__ void apply_site(PA P, int v, T* g) const {
    T acc[3] = {};
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += P(c, v) - P(c, u);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = wf2 * P(c, v) + wr2 * acc[c];
  }

  // Fused graph PCG hooks: the staged record of a vertex is its p, and a
  // neighbour's share of delta reads all three components of u.  A loop
  // {v, v} adds nothing to the product and is not counted in the diagonal.
  static constexpr bool kGraphFused = true;
  static constexpr int kRec = 3;
  static constexpr int kHalo = 3;
  struct GOwn {};
  using GRaw = Vals<T, 1>;
  __device__ __forceinline__ GRaw graw(int) const { return GRaw{}; }
  __device__ __forceinline__ GOwn gown_of(const GRaw&) const { return GOwn{}; }
  __device__ __forceinline__ void grec(const GOwn&, const T* p, T* r) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = p[c];
  }
  template <class RA, class NA>
  __device__ __forceinline__ void gapply_h(int sv, RA R, NA NB, int k0, int k1, uint32_t, T* g, T* dg) const {
    T acc[3] = {}, cnt = T(0);
    for (int k = k0; k < k1; ++k) {
      const int s = NB(k);
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += R(sv, c) - R(s, c);
      cnt += s != sv ? T(1) : T(0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[c] = fma(wr2, acc[c], wf2 * R(sv, c));
      dg[c] = wf2 + wr2 * cnt;
    }
  }
  template <class RA, class NA>
  __device__ __forceinline__ void gapply(const GOwn&, const T*, const T*, int sv, RA R, NA NB, int k0, int k1,
                                         uint32_t fl, T* g) const {
    T dg[3];
    gapply_h(sv, R, NB, k0, k1, fl, g, dg);
  }
  // the product and the diagonal (init's value, formed the same way)
  template <class RA, class NA>
  __device__ __forceinline__ void gapply_d(const GOwn&, const T*, const T*, int sv, RA R, NA NB, int k0, int k1,
                                           uint32_t fl, T* g, T* dg) const {
    gapply_h(sv, R, NB, k0, k1, fl, g, dg);
  }
  // w_fit^2 |u_v|^2 + half of w_reg^2 |u_v - u_s|^2 for each listed edge at v
  // (each edge's residual is shared by its two ends).
  template <class RA, class UA, class NA>
  __device__ __forceinline__ T gjsq(const GOwn&, const T* u, RA, UA UH, NA NB, int k0, int k1, uint32_t) const {
    T acc = T(0);
    for (int k = k0; k < k1; ++k) {
      const int s = NB(k);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T e = u[c] - UH(s, c);
        acc = fma(e, e, acc);
      }
    }
    const T uu = fma(u[2], u[2], fma(u[1], u[1], u[0] * u[0]));
    return fma(T(0.5) * wr2, acc, wf2 * uu);
  }

  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int v) const {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double f = wf_d * (X(c, v) - (double)A[(size_t)c * n + v]);
      const double jd = wf_d * Dl(c, v);
      acc += jd * (2.0 * f + jd);
    }
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
      if (u <= v) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double f = wr_d * (X(c, v) - X(c, u));
        const double jd = wr_d * (Dl(c, v) - Dl(c, u));
        acc += jd * (2.0 * f + jd);
      }
    }
    return acc;
  }
};

}  // namespace optmi
