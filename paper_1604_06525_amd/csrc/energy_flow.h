// Dense optical flow on a pixel grid (Fig. 30, Appendix A.2.3).
//
// Unknowns per pixel: flow (u, v).  Data: I, I_hat and the derivative images
// dI_hat/dx, dI_hat/dy.  Residuals anchored at p = (i, j):
//   fit  r = w_fit (I(i,j) - S(I_hat; i+u, j+v))                         (1 row)
//   reg  r = w_reg (X_p - X_q) per channel, q = p + s on the grid          (2 rows each)
// S is the sampled-image operator of Sec. 7: a bilinear sample with texel
// centres at integer coordinates and clamp-to-edge addressing.  Its partial
// derivatives are, by definition, the same samples of the derivative images, so
// J_fit = -w_fit (S(dI/dx), S(dI/dy)) at the linearisation point.  Those two values
// are the per-pixel state (Sec. 7's precomputed arrays); everything else in J is
// constant.
//   (J^T J P)_p = J_fit^T (J_fit . P_p) + 2 w_reg^2 sum_{q on grid} (P_p - P_q)
#pragma once
#include "common.h"

namespace optmi {

// Bilinear clamp-to-edge sample of a W x H image at (x, y) in the precision R.
template <typename R, typename T>
__device__ __forceinline__ R sample_bilinear(const T* __restrict__ img, int W, int H, R x, R y) {
  const R x0 = floor(x), y0 = floor(y);
  const R fx = x - x0, fy = y - y0;
  // clamp before the conversion (also maps NaN to the edge); indices past the
  // border read the edge texel, as clamping each index does
  const int ix = (int)fmin(fmax(x0, R(-1)), R(W));
  const int iy = (int)fmin(fmax(y0, R(-1)), R(H));
  const int ix0 = min(max(ix, 0), W - 1), ix1 = min(max(ix + 1, 0), W - 1);
  const int iy0 = min(max(iy, 0), H - 1), iy1 = min(max(iy + 1, 0), H - 1);
  const R a = img[iy0 * W + ix0], b = img[iy0 * W + ix1];
  const R c = img[iy1 * W + ix0], d = img[iy1 * W + ix1];
  return (R(1) - fx) * (R(1) - fy) * a + fx * (R(1) - fy) * b + (R(1) - fx) * fy * c + fx * fy * d;
}

template <typename T>
struct OpticalFlow {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 2;
  static constexpr int kStatePlanes = 2;  // J_fit along u and along v
  static constexpr int kOwnState = 2;
  static constexpr int kRadius = 1;
  // fused strip walk in FP32: d loaded with its row, start-up peeled (in FP64
  // the registers they take cost more than the waits they save)
  static constexpr int kFusedWalk = sizeof(T) == 4 ? 3 : 0;
  enum : uint32_t { ACTIVE = 1, INGRID = 2 };

  int W, H, n;
  const T* __restrict__ I;
  const T* __restrict__ Ih;
  const T* __restrict__ Idx;
  const T* __restrict__ Idy;
  T* __restrict__ jf;          // [2][n]
  uint8_t* __restrict__ flags;
  T wf, wr;
  double wf_d, wr_d;

  __device__ __forceinline__ T state_at(int k, int site) const { return jf[(size_t)site * 2 + k]; }
  __device__ __forceinline__ const T* state_base() const { return jf; }

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
    const double u = X(0, s), v = X(1, s);
    const double f = wf_d * ((double)I[s] - sample_bilinear<double>(Ih, W, H, i + u, j + v));
    double e = f * f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = nbr(i, j, s, k);
      if (q < 0) continue;
      const double ru = wr_d * (u - X(0, q)), rv = wr_d * (v - X(1, q));
      e += ru * ru + rv * rv;
    }
    return e;
  }

  __device__ __forceinline__ void linearize(const T* __restrict__ x, int s) const {
    const int i = s % W, j = s / W;
    const double xs = i + (double)x[s], ys = j + (double)x[n + s];
    jf[(size_t)s * 2] = (T)(-wf_d * sample_bilinear<double>(Idx, W, H, xs, ys));
    jf[(size_t)s * 2 + 1] = (T)(-wf_d * sample_bilinear<double>(Idy, W, H, xs, ys));
    flags[s] = (uint8_t)(INGRID | ACTIVE);
  }

  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV S, FV F, int s, int, int, T* b, T* d) const {
    const int i = s % W, j = s / W;
    const T ju = S(0, 0, 0), jv = S(1, 0, 0);
    const T u = X(0, 0, 0), v = X(1, 0, 0);
    const T f = wf * (I[s] - sample_bilinear<T>(Ih, W, H, T(i) + u, T(j) + v));
    T su = 0, sv = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & INGRID)) continue;
      su += u - X(0, di, dj);
      sv += v - X(1, di, dj);
      cnt += T(1);
    }
    const T w2 = T(2) * wr * wr;
    b[0] = -ju * f - w2 * su;
    b[1] = -jv * f - w2 * sv;
    diag(S, F, d);
  }

  // diag(J^T J) at an active centre, from the state and flags alone.
  template <class SV, class FV>
  __device__ __forceinline__ void diag(SV S, FV F, T* d) const {
    const T ju = S(0, 0, 0), jv = S(1, 0, 0);
    T cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      cnt += (F(di, dj) & INGRID) ? T(1) : T(0);
    }
    const T w2 = T(2) * wr * wr;
    d[0] = ju * ju + w2 * cnt;
    d[1] = jv * jv + w2 * cnt;
  }

  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV S, FV F, int, int, T* g) const {
    const T ju = S(0, 0, 0), jv = S(1, 0, 0);
    const T pu = P(0, 0, 0), pv = P(1, 0, 0);
    T su = 0, sv = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & INGRID)) continue;
      su += pu - P(0, di, dj);
      sv += pv - P(1, di, dj);
    }
    const T jp = ju * pu + jv * pv;
    const T w2 = T(2) * wr * wr;
    g[0] = ju * jp + w2 * su;
    g[1] = jv * jp + w2 * sv;
  }

  // sum over the residuals anchored at the centre of (J u)_r^2; summed over all
  // sites this is |J u|^2.
  template <class PV, class SV, class FV>
  __device__ __forceinline__ T jsq(PV U, SV S, FV F, int, int) const {
    const T uu = U(0, 0, 0), uv = U(1, 0, 0);
    const T jp = S(0, 0, 0) * uu + S(1, 0, 0) * uv;
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = (F(di, dj) & INGRID) ? T(1) : T(0);
      const T eu = uu - U(0, di, dj), ev = uv - U(1, di, dj);
      acc += w * (eu * eu + ev * ev);
    }
    return jp * jp + wr * wr * acc;
  }

  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    const int i = s % W, j = s / W;
    const double u = X(0, s), v = X(1, s);
    const double xs = i + u, ys = j + v;
    const double f = wf_d * ((double)I[s] - sample_bilinear<double>(Ih, W, H, xs, ys));
    const double jd = -wf_d * (sample_bilinear<double>(Idx, W, H, xs, ys) * Dl(0, s) +
                               sample_bilinear<double>(Idy, W, H, xs, ys) * Dl(1, s));
    double acc = jd * (2.0 * f + jd);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = nbr(i, j, s, k);
      if (q < 0) continue;
      const double fu = wr_d * (u - X(0, q)), fv = wr_d * (v - X(1, q));
      const double ju = wr_d * (Dl(0, s) - Dl(0, q)), jv = wr_d * (Dl(1, s) - Dl(1, q));
      acc += ju * (2.0 * fu + ju) + jv * (2.0 * fv + jv);
    }
    return acc;
  }
};

}  // namespace optmi
