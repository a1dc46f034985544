// Poisson image editing on a pixel grid (Fig. 27, Appendix A.1.4).
//
// Unknowns per pixel: X (4 planes, RGBA).  Data: T (4 planes), mask (uint8).
// For every stencil offset s with q = p + s on the grid, one residual per channel
//   r = (X_p - X_q) - (T_p - T_q),
// no weights.  Pixels with mask != 0 are excluded (constants).  The energy is
// linear, J holds only +1 and -1, so GN reaches the minimiser in one outer
// iteration with an exact inner solve (Sec. 8.1).
//
// Matrix-free products: the residuals reading X_p are p's own four and the four
// of its neighbours pointing back at p; both have derivative +-1 at p, so
//   (J^T J P)_p = 2 sum_{q on grid} (P_p - P_q),   b_p = -2 sum_q r_pq,
//   diag_p = 2 * (number of neighbours on the grid),
// where P_q is zero at excluded pixels (the PCG vectors vanish there).
#pragma once
#include "common.h"

namespace optmi {

template <typename T>
struct Poisson {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 4;
  static constexpr int kStatePlanes = 0;
  static constexpr int kOwnState = 0;
  static constexpr int kRadius = 1;
  enum : uint32_t { ACTIVE = 1, INGRID = 2 };

  int W, H, n;
  const T* __restrict__ Tg;   // [4][n]
  const uint8_t* __restrict__ mask;
  uint8_t* __restrict__ flags;

  __device__ __forceinline__ T state_at(int, int) const { return T(0); }
  __device__ __forceinline__ const T* state_base() const { return nullptr; }

  __device__ __forceinline__ int nbr(int i, int j, int s, int k) const {
    switch (k) {
      case 0: return i + 1 < W ? s + 1 : -1;
      case 1: return i > 0 ? s - 1 : -1;
      case 2: return j + 1 < H ? s + W : -1;
      default: return j > 0 ? s - W : -1;
    }
  }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int s) const {
    const int i = s % W, j = s / W;
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = nbr(i, j, s, k);
      if (q < 0) continue;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * n;
        const double r = (X(c, s) - X(c, q)) - ((double)Tg[o + s] - (double)Tg[o + q]);
        e += r * r;
      }
    }
    return e;
  }

  __device__ __forceinline__ void linearize(const T* __restrict__, int s) const {
    flags[s] = (uint8_t)(INGRID | (mask[s] == 0 ? ACTIVE : 0));
  }

  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV, FV F, int s, int, int, T* b, T* d) const {
    T acc[C] = {};
    T cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & INGRID)) continue;
      const int q = s + dj * W + di;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * n;
        acc[c] += (X(c, 0, 0) - X(c, di, dj)) - (Tg[o + s] - Tg[o + q]);
      }
      cnt += T(2);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) b[c] = T(-2) * acc[c];
    diag(nullptr, F, d);
  }

  // diag(J^T J) at an active centre: 2 per neighbour on the grid.
  template <class SV, class FV>
  __device__ __forceinline__ void diag(SV, FV F, T* d) const {
    T cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      cnt += (F(di, dj) & INGRID) ? T(2) : T(0);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) d[c] = cnt;
  }

  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV, FV F, int, int, T* g) const {
    T acc[C] = {};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & INGRID)) continue;
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] += P(c, 0, 0) - P(c, di, dj);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) g[c] = T(2) * acc[c];
  }

  // sum over the residuals anchored at the centre of (J u)_r^2 (u is zero at
  // excluded pixels); summed over all sites this is |J u|^2.
  template <class PV, class SV, class FV>
  __device__ __forceinline__ T jsq(PV U, SV, FV F, int, int) const {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = (F(di, dj) & INGRID) ? T(1) : T(0);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const T e = U(c, 0, 0) - U(c, di, dj);
        acc += w * e * e;
      }
    }
    return acc;
  }

  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    const int i = s % W, j = s / W;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = nbr(i, j, s, k);
      if (q < 0) continue;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = (size_t)c * n;
        const double r = (X(c, s) - X(c, q)) - ((double)Tg[o + s] - (double)Tg[o + q]);
        const double jd = Dl(c, s) - Dl(c, q);
        acc += jd * (2.0 * r + jd);
      }
    }
    return acc;
  }
};

}  // namespace optmi
