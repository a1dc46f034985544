// Shape from shading on a pixel grid (Fig. 26, Appendix A.1.3).
//
// Unknown per pixel: depth X.  Data: input depth D_i, intensity Im, edge masks
// eR, eC (uint8).  Params: w_p, w_s, w_g (energy weights; their square roots are
// applied), f_x, f_y, u_x, u_y, L1..L9.
//   position   p(a,b) = (k_x(a) X, k_y(b) X, X),  k_x(a) = (a-u_x)/f_x, k_y(b) = (b-u_y)/f_y (eq. 8)
//   normal     n_x = X(a,b-1)(X(a,b)-X(a-1,b))/f_y,  n_y = X(a-1,b)(X(a,b)-X(a,b-1))/f_x,
//              n_z = n_x(u_x-a)/f_x + n_y(u_y-b)/f_y - X(a-1,b)X(a,b-1)/(f_x f_y),
//              divided by its length when that is positive (eq. 10)
//   shading    B = L1 + L2 n_y + L3 n_z + L4 n_x + L5 n_x n_y + L6 n_y n_z
//                  + L7(-n_x^2 - n_y^2 + 2 n_z^2) + L8 n_z n_x + L9(n_x^2 - n_y^2)
//   B_I(a,b) = B - (Im(a,b)/2 + (Im(a-1,b) + Im(a,b-1))/4) where (a,b) is at least one
//              pixel inside the border (IBE) and D_i > 0 at (a-1,b), (a,b), (a,b-1); else 0
// Residuals at (i,j):
//   r_p  = sqrt(w_p)(X - D_i)                               if D_i(i,j) > 0
//   r_gh = sqrt(w_g) eR(i,j)(B_I(i,j) - B_I(i+1,j))         if IBE(i,j)
//   r_gv = sqrt(w_g) eC(i,j)(B_I(i,j) - B_I(i,j+1))         if IBE(i,j)
//   r_s  = sqrt(w_s)(4p(i,j) - p(i-1,j) - p(i,j-1) - p(i+1,j) - p(i,j+1))   (3 rows)
//          if D_i > 0 on the 5-point stencil, |X(i,j) - X(nbr)| < 0.01 for all four
//          neighbours, and IBE(i,j); this test is taken at the linearisation point
// Pixels with D_i <= 0 are excluded.
//
// Per-pixel state (the precomputed lighting of Sec. 8.3): B_I and its partial
// derivatives with respect to X(a,b), X(a-1,b), X(a,b-1), plus flags.  J^T J then
// reaches two pixels (the shading residuals read B_I one pixel away, and B_I
// reads three depths); it is formed as the sum over the residuals r that read
// x00 of (dr/dx00)(J p)_r, the residuals being found by shifting each residual
// template by the offsets of its unknowns (Sec. 5.3.1).
#pragma once
#include "common.h"

namespace optmi {

template <typename T>
struct ShapeFromShading {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 1;
  static constexpr int kStatePlanes = 4;  // B_I, dB/dX(a,b), dB/dX(a-1,b), dB/dX(a,b-1)
  static constexpr int kOwnState = 4;
  static constexpr int kRadius = 2;
  enum : uint32_t {
    ACTIVE = 1,    // D_i > 0
    INGRID = 2,
    IBE = 4,       // one pixel inside the border
    VS = 8,        // smoothness residual valid (at the linearisation point)
    ER = 16,       // edge mask eR
    EC = 32,       // edge mask eC
  };

  int W, H, n;
  const T* __restrict__ D;
  const T* __restrict__ Im;
  const uint8_t* __restrict__ eR;
  const uint8_t* __restrict__ eC;
  T* __restrict__ st;          // [4][n]
  uint8_t* __restrict__ flags;
  double sw_p, sw_s, sw_g, fx, fy, ux, uy;
  double L[9];
  T sw_pT, sw_sT, sw_gT;

  __device__ __forceinline__ T state_at(int k, int site) const { return st[(size_t)site * 4 + k]; }
  __device__ __forceinline__ const T* state_base() const { return st; }

  __device__ __forceinline__ bool ibe(int i, int j) const {
    return i >= 1 && i <= W - 2 && j >= 1 && j <= H - 2;
  }
  __device__ __forceinline__ bool dv(int i, int j) const {
    return i >= 0 && i < W && j >= 0 && j < H && D[j * W + i] > T(0);
  }

  // B_I at (a,b) and its partials with respect to X(a,b), X(a-1,b), X(a,b-1), in
  // the precision R; X(di, dj) reads the depth at (a+di, b+dj).
  template <typename R, class XA>
  __device__ __forceinline__ void shading(int a, int b, XA X, R* val, R* g0, R* gl, R* gu) const {
    *val = *g0 = *gl = *gu = R(0);
    if (!(ibe(a, b) && dv(a - 1, b) && dv(a, b) && dv(a, b - 1))) return;
    const R fxr = (R)fx, fyr = (R)fy, uxr = (R)ux, uyr = (R)uy;
    const R x0 = X(0, 0), xl = X(-1, 0), xu = X(0, -1);
    const R cx = (uxr - R(a)) / fxr, cy = (uyr - R(b)) / fyr;
    R n[3], dn[3][3];  // dn[k][v]: d n_k / d {X00, Xl, Xu}
    n[0] = xu * (x0 - xl) / fyr;
    n[1] = xl * (x0 - xu) / fxr;
    n[2] = n[0] * cx + n[1] * cy - xl * xu / (fxr * fyr);
    dn[0][0] = xu / fyr;  dn[0][1] = -xu / fyr;       dn[0][2] = (x0 - xl) / fyr;
    dn[1][0] = xl / fxr;  dn[1][1] = (x0 - xu) / fxr; dn[1][2] = -xl / fxr;
#pragma unroll
    for (int v = 0; v < 3; ++v) dn[2][v] = dn[0][v] * cx + dn[1][v] * cy;
    dn[2][1] -= xu / (fxr * fyr);
    dn[2][2] -= xl / (fxr * fyr);
    const R sq = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    R m[3], dm[3][3];
    if (sq > R(0)) {
      const R inv = R(1) / sqrt(sq);
#pragma unroll
      for (int k = 0; k < 3; ++k) m[k] = n[k] * inv;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const R md = m[0] * dn[0][v] + m[1] * dn[1][v] + m[2] * dn[2][v];
#pragma unroll
        for (int k = 0; k < 3; ++k) dm[k][v] = (dn[k][v] - m[k] * md) * inv;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        m[k] = n[k];
#pragma unroll
        for (int v = 0; v < 3; ++v) dm[k][v] = dn[k][v];
      }
    }
    const R L1 = (R)L[0], L2 = (R)L[1], L3 = (R)L[2], L4 = (R)L[3], L5 = (R)L[4], L6 = (R)L[5],
            L7 = (R)L[6], L8 = (R)L[7], L9 = (R)L[8];
    const R mx = m[0], my = m[1], mz = m[2];
    const R B = L1 + L2 * my + L3 * mz + L4 * mx + L5 * mx * my + L6 * my * mz +
                L7 * (-mx * mx - my * my + R(2) * mz * mz) + L8 * mz * mx + L9 * (mx * mx - my * my);
    const R bx = L4 + L5 * my - R(2) * L7 * mx + L8 * mz + R(2) * L9 * mx;
    const R by = L2 + L5 * mx + L6 * mz - R(2) * L7 * my - R(2) * L9 * my;
    const R bz = L3 + L6 * my + R(4) * L7 * mz + L8 * mx;
    const int s = b * W + a;
    const R I = R(0.5) * (R)Im[s] + R(0.25) * ((R)Im[s - 1] + (R)Im[s - W]);
    *val = B - I;
    *g0 = bx * dm[0][0] + by * dm[1][0] + bz * dm[2][0];
    *gl = bx * dm[0][1] + by * dm[1][1] + bz * dm[2][1];
    *gu = bx * dm[0][2] + by * dm[1][2] + bz * dm[2][2];
  }

  // Smoothness validity at (i,j) for depths read through X(di, dj).
  template <class XA>
  __device__ __forceinline__ bool smooth_valid(int i, int j, XA X) const {
    if (!(ibe(i, j) && dv(i, j) && dv(i - 1, j) && dv(i + 1, j) && dv(i, j - 1) && dv(i, j + 1)))
      return false;
    const double x0 = X(0, 0);
    return fabs(x0 - (double)X(1, 0)) < 0.01 && fabs(x0 - (double)X(-1, 0)) < 0.01 &&
           fabs(x0 - (double)X(0, 1)) < 0.01 && fabs(x0 - (double)X(0, -1)) < 0.01;
  }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int s) const {
    const int i = s % W, j = s / W;
    auto Xo = [&](int di, int dj) -> double { return X(0, s + dj * W + di); };
    double e = 0.0;
    if (dv(i, j)) {
      const double f = sw_p * (Xo(0, 0) - (double)D[s]);
      e += f * f;
    }
    if (ibe(i, j)) {
      double b0, b1, b2, t0, t1, t2;
      shading<double>(i, j, Xo, &b0, &t0, &t1, &t2);
      auto Xr = [&](int di, int dj) -> double { return Xo(di + 1, dj); };
      auto Xd = [&](int di, int dj) -> double { return Xo(di, dj + 1); };
      shading<double>(i + 1, j, Xr, &b1, &t0, &t1, &t2);
      shading<double>(i, j + 1, Xd, &b2, &t0, &t1, &t2);
      const double fh = sw_g * (eR[s] ? 1.0 : 0.0) * (b0 - b1);
      const double fv = sw_g * (eC[s] ? 1.0 : 0.0) * (b0 - b2);
      e += fh * fh + fv * fv;
    }
    if (smooth_valid(i, j, Xo)) {
      double sm[3];
      smooth_res(i, j, Xo, sm);
      e += sm[0] * sm[0] + sm[1] * sm[1] + sm[2] * sm[2];
    }
    return e;
  }

  // r_s at (i,j) (without the validity test), depths read through X(di, dj)
  template <class XA>
  __device__ __forceinline__ void smooth_res(int i, int j, XA X, double* r) const {
    auto kx = [&](int a) { return (a - ux) / fx; };
    auto ky = [&](int b) { return (b - uy) / fy; };
    const double x0 = X(0, 0), xl = X(-1, 0), xr = X(1, 0), xu = X(0, -1), xd = X(0, 1);
    r[0] = sw_s * (4 * kx(i) * x0 - kx(i - 1) * xl - kx(i) * xu - kx(i + 1) * xr - kx(i) * xd);
    r[1] = sw_s * (4 * ky(j) * x0 - ky(j) * xl - ky(j - 1) * xu - ky(j) * xr - ky(j + 1) * xd);
    r[2] = sw_s * (4 * x0 - xl - xu - xr - xd);
  }

  __device__ __forceinline__ void linearize(const T* __restrict__ x, int s) const {
    const int i = s % W, j = s / W;
    auto Xo = [&](int di, int dj) -> T { return x[s + dj * W + di]; };
    T v, g0, gl, gu;
    shading<T>(i, j, Xo, &v, &g0, &gl, &gu);
    T* q = st + (size_t)s * 4;
    q[0] = v;
    q[1] = g0;
    q[2] = gl;
    q[3] = gu;
    uint32_t f = INGRID;
    if (dv(i, j)) f |= ACTIVE;
    if (ibe(i, j)) f |= IBE;
    if (smooth_valid(i, j, Xo)) f |= VS;
    if (eR[s]) f |= ER;
    if (eC[s]) f |= EC;
    flags[s] = (uint8_t)f;
  }

  // Shading residual sites that read x00 and their derivative d r / d x00 / sqrt(w_g):
  // five horizontal (gh) and five vertical (gv) ones; S(q, di, dj) gives the state.
  template <class SV, class FV>
  __device__ __forceinline__ void shading_partials(SV S, FV F, T* dh, T* dv_) const {
    // dh: sites (0,0), (-1,0), (1,0), (0,1), (-1,1);  dv: (0,0), (0,-1), (1,0), (1,-1), (0,1)
    const T dB0 = S(1, 0, 0), dBlR = S(2, 1, 0), dBuD = S(3, 0, 1);
    auto eh = [&](int di, int dj) -> T {
      const uint32_t f = F(di, dj);
      return (f & IBE) && (f & ER) ? T(1) : T(0);
    };
    auto ev = [&](int di, int dj) -> T {
      const uint32_t f = F(di, dj);
      return (f & IBE) && (f & EC) ? T(1) : T(0);
    };
    dh[0] = eh(0, 0) * (dB0 - dBlR);
    dh[1] = -eh(-1, 0) * dB0;
    dh[2] = eh(1, 0) * dBlR;
    dh[3] = eh(0, 1) * dBuD;
    dh[4] = -eh(-1, 1) * dBuD;
    dv_[0] = ev(0, 0) * (dB0 - dBuD);
    dv_[1] = -ev(0, -1) * dB0;
    dv_[2] = ev(1, 0) * dBlR;
    dv_[3] = -ev(1, -1) * dBlR;
    dv_[4] = ev(0, 1) * dBuD;
  }

  // (J p) / sqrt(w_g) of the shading residual gh at (a,b) = (di,dj) from the centre,
  // without its edge-mask factor: dB at (a,b) and (a+1,b) dotted with p.
  template <class PV, class SV>
  __device__ __forceinline__ T jp_gh(PV P, SV S, int a, int b) const {
    return S(1, a, b) * P(0, a, b) + S(2, a, b) * P(0, a - 1, b) + S(3, a, b) * P(0, a, b - 1) -
           (S(1, a + 1, b) * P(0, a + 1, b) + S(2, a + 1, b) * P(0, a, b) +
            S(3, a + 1, b) * P(0, a + 1, b - 1));
  }
  template <class PV, class SV>
  __device__ __forceinline__ T jp_gv(PV P, SV S, int a, int b) const {
    return S(1, a, b) * P(0, a, b) + S(2, a, b) * P(0, a - 1, b) + S(3, a, b) * P(0, a, b - 1) -
           (S(1, a, b + 1) * P(0, a, b + 1) + S(2, a, b + 1) * P(0, a - 1, b + 1) +
            S(3, a, b + 1) * P(0, a, b));
  }
  // (J p) of the smoothness residual at (a,b) from the centre, per component,
  // without sqrt(w_s); (i, j) is the centre pixel.
  template <class PV>
  __device__ __forceinline__ void jp_s(PV P, int i, int j, int a, int b, T* out) const {
    const T kxa = T((i + a - ux) / fx), kxl = T((i + a - 1 - ux) / fx), kxr = T((i + a + 1 - ux) / fx);
    const T kyb = T((j + b - uy) / fy), kyu = T((j + b - 1 - uy) / fy), kyd = T((j + b + 1 - uy) / fy);
    const T p0 = P(0, a, b), pl = P(0, a - 1, b), pr = P(0, a + 1, b), pu = P(0, a, b - 1),
            pd = P(0, a, b + 1);
    out[0] = T(4) * kxa * p0 - kxl * pl - kxa * pu - kxr * pr - kxa * pd;
    out[1] = T(4) * kyb * p0 - kyb * pl - kyu * pu - kyb * pr - kyd * pd;
    out[2] = T(4) * p0 - pl - pu - pr - pd;
  }

  // b = -J^T F and diag(J^T J) at an active pixel (i,j) = site s.
  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV S, FV F, int s, int i, int j, T* b,
                                           T* d) const {
    T dh[5], dvv[5];
    shading_partials(S, F, dh, dvv);
    const int ho[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, 1}, {-1, 1}};
    const int vo[5][2] = {{0, 0}, {0, -1}, {1, 0}, {1, -1}, {0, 1}};
    const T wg2 = sw_gT * sw_gT;
    T acc = 0, dg = 0;
    // r_p
    const T rp = sw_pT * (X(0, 0, 0) - D[s]);
    acc += sw_pT * rp;
    dg += sw_pT * sw_pT;
    // shading: F = sqrt(w_g) e (B_I(a,b) - B_I(a+1,b)) and the vertical analogue
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int a = ho[k][0], c = ho[k][1];
      const T fh = F(a, c) & ER ? S(0, a, c) - S(0, a + 1, c) : T(0);
      acc += wg2 * dh[k] * fh;
      dg += wg2 * dh[k] * dh[k];
      const int a2 = vo[k][0], c2 = vo[k][1];
      const T fv = F(a2, c2) & EC ? S(0, a2, c2) - S(0, a2, c2 + 1) : T(0);
      acc += wg2 * dvv[k] * fv;
      dg += wg2 * dvv[k] * dvv[k];
    }
    // smoothness: centre coefficient 4 k(i,j), neighbours -k(i,j)
    const T kx = T((i - ux) / fx), ky = T((j - uy) / fy);
    const T kk = kx * kx + ky * ky + T(1);
    const int so[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int a = so[k][0], c = so[k][1];
      if (!(F(a, c) & VS)) continue;
      auto Xd = [&](int di, int dj) -> T { return X(0, a + di, c + dj); };
      const T coef = k == 0 ? T(4) : T(-1);
      // residual at (a,b) recomputed in the bulk type
      const T ka = T((i + a - ux) / fx), kl = T((i + a - 1 - ux) / fx), kr = T((i + a + 1 - ux) / fx);
      const T kb = T((j + c - uy) / fy), ku = T((j + c - 1 - uy) / fy), kd = T((j + c + 1 - uy) / fy);
      const T x0 = Xd(0, 0), xl = Xd(-1, 0), xr = Xd(1, 0), xu = Xd(0, -1), xd = Xd(0, 1);
      const T r0 = T(4) * ka * x0 - kl * xl - ka * xu - kr * xr - ka * xd;
      const T r1 = T(4) * kb * x0 - kb * xl - ku * xu - kb * xr - kd * xd;
      const T r2 = T(4) * x0 - xl - xu - xr - xd;
      const T ws2 = sw_sT * sw_sT;
      acc += ws2 * coef * (kx * r0 + ky * r1 + r2);
      dg += ws2 * coef * coef * kk;
    }
    b[0] = -acc;
    d[0] = dg;
  }

  // g = J^T J P at the active pixel (i,j).
  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV S, FV F, int i, int j, T* g) const {
    T dh[5], dvv[5];
    shading_partials(S, F, dh, dvv);
    const int ho[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, 1}, {-1, 1}};
    const int vo[5][2] = {{0, 0}, {0, -1}, {1, 0}, {1, -1}, {0, 1}};
    const T wg2 = sw_gT * sw_gT;
    T acc = sw_pT * sw_pT * P(0, 0, 0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      if (dh[k] != T(0)) acc += wg2 * dh[k] * jp_gh(P, S, ho[k][0], ho[k][1]);
      if (dvv[k] != T(0)) acc += wg2 * dvv[k] * jp_gv(P, S, vo[k][0], vo[k][1]);
    }
    const T kx = T((i - ux) / fx), ky = T((j - uy) / fy);
    const int so[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    const T ws2 = sw_sT * sw_sT;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int a = so[k][0], c = so[k][1];
      if (!(F(a, c) & VS)) continue;
      T jp[3];
      jp_s(P, i, j, a, c, jp);
      const T coef = k == 0 ? T(4) : T(-1);
      acc += ws2 * coef * (kx * jp[0] + ky * jp[1] + jp[2]);
    }
    g[0] = acc;
  }

  // Materialised Jacobian (evalJ, Sec. 7 and the fully materialised strategy
  // of Sec. 8.3): the rows anchored at pixel s, kJSlots entries each (column =
  // pixel, -1 for none, value 0 there): row 0 the depth prior, 1 and 2 the
  // shading differences gh and gv, 3..5 the three smoothness components.  Each
  // entry is d r / d X from the stored lighting partials, summed where a row
  // reads a pixel twice; columns of excluded pixels are dropped.  A row that
  // exists has all its pixels on the grid (IBE keeps them one pixel inside).
  static constexpr int kJRows = 6, kJSlots = 5, kJTSlots = 26;
  __device__ __forceinline__ void eval_j(int s, T* __restrict__ val, int* __restrict__ col) const {
    const int i = s % W, j = s / W;
    const uint32_t f = flags[s];
    auto B = [&](int site, int k) -> T { return st[(size_t)site * 4 + k]; };
    auto put = [&](int row, int slot, int site, bool on, T v) {
      const bool keep = on && (flags[site] & ACTIVE);
      col[row * kJSlots + slot] = keep ? site : -1;
      val[row * kJSlots + slot] = keep ? v : T(0);
    };
    for (int k = 0; k < kJRows * kJSlots; ++k) {
      col[k] = -1;
      val[k] = T(0);
    }
    put(0, 0, s, (f & ACTIVE) != 0, sw_pT);
    const bool rh = (f & IBE) && (f & ER), rv = (f & IBE) && (f & EC);
    if (rh) {
      put(1, 0, s, true, sw_gT * (B(s, 1) - B(s + 1, 2)));
      put(1, 1, s - 1, true, sw_gT * B(s, 2));
      put(1, 2, s - W, true, sw_gT * B(s, 3));
      put(1, 3, s + 1, true, -sw_gT * B(s + 1, 1));
      put(1, 4, s + 1 - W, true, -sw_gT * B(s + 1, 3));
    }
    if (rv) {
      put(2, 0, s, true, sw_gT * (B(s, 1) - B(s + W, 3)));
      put(2, 1, s - 1, true, sw_gT * B(s, 2));
      put(2, 2, s - W, true, sw_gT * B(s, 3));
      put(2, 3, s + W, true, -sw_gT * B(s + W, 1));
      put(2, 4, s + W - 1, true, -sw_gT * B(s + W, 2));
    }
    if (f & VS) {
      const T kxa = T((i - ux) / fx), kxl = T((i - 1 - ux) / fx), kxr = T((i + 1 - ux) / fx);
      const T kyb = T((j - uy) / fy), kyu = T((j - 1 - uy) / fy), kyd = T((j + 1 - uy) / fy);
      const T c0[5] = {T(4) * kxa, -kxl, -kxa, -kxr, -kxa};  // s, s-1, s-W, s+1, s+W
      const T c1[5] = {T(4) * kyb, -kyb, -kyu, -kyb, -kyd};
      const T c2[5] = {T(4), T(-1), T(-1), T(-1), T(-1)};
      const int at[5] = {s, s - 1, s - W, s + 1, s + W};
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        put(3, t, at[t], true, sw_sT * c0[t]);
        put(4, t, at[t], true, sw_sT * c1[t]);
        put(5, t, at[t], true, sw_sT * c2[t]);
      }
    }
  }

  // The entries of J's column s (kJTSlots indices into eval_j's entries, -1
  // for none): for each row type, the anchor pixels whose row reads s and the
  // slot s takes there (the slot tables of eval_j read backwards).  Anchors off
  // the grid are skipped; an anchor whose row is absent holds a 0 entry there.
  __device__ __forceinline__ void eval_jt(int s, int* __restrict__ jt) const {
    const int i = s % W, j = s / W;
    auto at = [](int site, int row, int slot) { return (site * kJRows + row) * kJSlots + slot; };
    int m = 0;
    auto add = [&](int di, int dj, int row, int slot) {
      const int a = i + di, b = j + dj;
      jt[m++] = (a >= 0 && a < W && b >= 0 && b < H) ? at(s + dj * W + di, row, slot) : -1;
    };
    add(0, 0, 0, 0);
    // gh anchored at s, s+1, s+W, s-1, s-1+W (slots 0..4)
    add(0, 0, 1, 0);
    add(1, 0, 1, 1);
    add(0, 1, 1, 2);
    add(-1, 0, 1, 3);
    add(-1, 1, 1, 4);
    // gv anchored at s, s+1, s+W, s-W, s+1-W
    add(0, 0, 2, 0);
    add(1, 0, 2, 1);
    add(0, 1, 2, 2);
    add(0, -1, 2, 3);
    add(1, -1, 2, 4);
    // smoothness anchored at s, s+1, s+W, s-1, s-W
#pragma unroll
    for (int row = 3; row < 6; ++row) {
      add(0, 0, row, 0);
      add(1, 0, row, 1);
      add(0, 1, row, 2);
      add(-1, 0, row, 3);
      add(0, -1, row, 4);
    }
  }

  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    const int i = s % W, j = s / W;
    auto Xo = [&](int di, int dj) -> double { return X(0, s + dj * W + di); };
    auto Do = [&](int di, int dj) -> double { return Dl(0, s + dj * W + di); };
    double acc = 0.0;
    if (dv(i, j)) {
      const double f = sw_p * (Xo(0, 0) - (double)D[s]);
      const double jd = sw_p * Do(0, 0);
      acc += jd * (2.0 * f + jd);
    }
    if (ibe(i, j)) {
      double b0, g0, gl, gu, b1, h0, hl, hu, b2, v0, vl, vu;
      shading<double>(i, j, Xo, &b0, &g0, &gl, &gu);
      auto Xr = [&](int di, int dj) -> double { return Xo(di + 1, dj); };
      auto Xd = [&](int di, int dj) -> double { return Xo(di, dj + 1); };
      shading<double>(i + 1, j, Xr, &b1, &h0, &hl, &hu);
      shading<double>(i, j + 1, Xd, &b2, &v0, &vl, &vu);
      const double jb0 = g0 * Do(0, 0) + gl * Do(-1, 0) + gu * Do(0, -1);
      const double jb1 = h0 * Do(1, 0) + hl * Do(0, 0) + hu * Do(1, -1);
      const double jb2 = v0 * Do(0, 1) + vl * Do(-1, 1) + vu * Do(0, 0);
      const double eh = eR[s] ? sw_g : 0.0, ev = eC[s] ? sw_g : 0.0;
      const double fh = eh * (b0 - b1), fv = ev * (b0 - b2);
      const double jh = eh * (jb0 - jb1), jv = ev * (jb0 - jb2);
      acc += jh * (2.0 * fh + jh) + jv * (2.0 * fv + jv);
    }
    if (smooth_valid(i, j, Xo)) {
      double f[3], jd[3];
      smooth_res(i, j, Xo, f);
      smooth_res(i, j, Do, jd);
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += jd[k] * (2.0 * f[k] + jd[k]);
    }
    return acc;
  }
};

// Shape from shading with nothing stored between linearisations but the
// depth: the fully matrix-free strategy of Sec. 8.3 (Fig. 17).  The product
// recomputes the lighting term's partials from the linearisation point xlin in
// every PCG iteration, at each of the eleven pixels whose partials the centre's
// J^T J p reads (the shading residuals of its two-pixel neighbourhood), with
// the same arithmetic as linearize, so the stored values are reproduced.  Only
// the product (the split form's pcg_a) uses it.
template <typename T>
struct ShapeFromShadingLit : ShapeFromShading<T> {
  using Base = ShapeFromShading<T>;
  const T* __restrict__ xlin;  // the linearisation point (caller-facing plane)

  // table slot of a pixel offset the product reads, -1 for one it does not
  static constexpr int slot_of(int di, int dj) {
    return dj == 0 ? (di == 0 ? 0 : di == -1 ? 1 : di == 1 ? 2 : di == 2 ? 3 : -1)
         : dj == -1 ? (di == 0 ? 4 : di == 1 ? 5 : -1)
         : dj == 1 ? (di == 0 ? 6 : di == -1 ? 7 : di == 1 ? 8 : -1)
         : dj == 2 ? (di == 0 ? 9 : -1) : -1;
  }
  static constexpr int kPix = 10;

  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV, FV F, int i, int j, T* g) const {
    const int W = this->W;
    const int s = j * W + i;
    T tab[kPix][4];
    constexpr int off[kPix][2] = {{0, 0}, {-1, 0}, {1, 0}, {2, 0}, {0, -1}, {1, -1}, {0, 1}, {-1, 1}, {1, 1}, {0, 2}};
#pragma unroll
    for (int t = 0; t < kPix; ++t) {
      const int a = i + off[t][0], b = j + off[t][1], q = s + off[t][1] * W + off[t][0];
      auto Xo = [&](int di, int dj) -> T { return xlin[q + dj * W + di]; };
      // shading() reads nothing for a pixel not one inside the border
      this->template shading<T>(a, b, Xo, &tab[t][0], &tab[t][1], &tab[t][2], &tab[t][3]);
    }
    auto Sl = [&](int k, int di, int dj) -> T {
      const int t = slot_of(di, dj);
      return t >= 0 ? tab[t][k] : T(0);
    };
    Base::apply(P, Sl, F, i, j, g);
  }
};

}  // namespace optmi
