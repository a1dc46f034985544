// As-rigid-as-possible image warping with explicit connectivity (Sec. 7, the
// comparison of Fig. 18): the residuals of energy_arap_warp.h, with the pixel
// neighbourhood given as an edge list instead of the implicit grid stencil.
//
// Unknowns per vertex: offset O (2 planes) and angle t (1 plane).  Data: rest
// positions U (2 planes), targets C (2 planes), mask (uint8).  For every listed
// edge {v, u}, both orientations, when both ends have mask 0:
//   r(v->u) = w_reg [ (O_v - O_u) - R(t_v)(U_v - U_u) ]      (2 rows)
// and per vertex the fit r = w_fit (O_v - C_v) when both components of C_v are
// >= 0.  With the 4-neighbour edges of a W x H lattice (each pair once) this is
// the grid energy term for term.  The edge list is turned into a per-vertex
// incidence list (CSR) at creation; each vertex gathers its own edges.
// Per-vertex state: cos t, sin t at the linearisation point, U_x, U_y.
#pragma once
#include "common.h"

namespace optmi {

template <typename T>
struct ArapWarpGraph {
  using Real = T;
  static constexpr bool kGraph = true;
  static constexpr int C = 3;
  static constexpr int kStatePlanes = 4;  // cos t, sin t, U_x, U_y
  static constexpr int kOwnState = 4;
  static constexpr int kRadius = 1;
  enum : uint32_t { ACTIVE = 1, INGRID = 2, FIT = 4 };
  // pcg_a could stage a vertex chunk and its halo in LDS (apply_staged), but on
  // pixel lattices the neighbours' reads already hit the caches, and staging
  // measured slower (69.0 vs 64.2 us per PCG iteration at 1024^2).
  static constexpr bool kStaged = false;
  static constexpr int kStageVals = 5;   // staged per vertex: cos t, sin t, U_x, U_y, active

  int n;
  const int* __restrict__ rp;  // [n+1] CSR offsets
  const int* __restrict__ nb;  // [2E] neighbour ids
  const T* __restrict__ U;     // [2][n]
  const T* __restrict__ Ct;    // [2][n]
  const uint8_t* __restrict__ mask;
  T* __restrict__ st;          // [n][4]
  uint8_t* __restrict__ flags;
  Halo halo;                   // pcg_a's staging lists
  T wf, wr;
  double wf_d, wr_d;

  __device__ __forceinline__ T state_at(int k, int v) const { return st[(size_t)v * 4 + k]; }
  __device__ __forceinline__ const T* state_base() const { return st; }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int v) const {
    double e = 0.0;
    const double Ox = X(0, v), Oy = X(1, v);
    if (mask[v] == 0) {
      double sn, c;
      sincos_t(X(2, v), &sn, &c);
      const double Ux = U[v], Uy = U[n + v];
      for (int k = rp[v]; k < rp[v + 1]; ++k) {
        const int u = nb[k];
        if (mask[u] != 0) continue;
        const double dx = Ux - (double)U[u], dy = Uy - (double)U[n + u];
        const double rx = wr_d * ((Ox - X(0, u)) - (c * dx - sn * dy));
        const double ry = wr_d * ((Oy - X(1, u)) - (sn * dx + c * dy));
        e += rx * rx + ry * ry;
      }
    }
    const double cx = Ct[v], cy = Ct[n + v];
    if (cx >= 0.0 && cy >= 0.0) {
      const double fx = wf_d * (Ox - cx), fy = wf_d * (Oy - cy);
      e += fx * fx + fy * fy;
    }
    return e;
  }

  __device__ __forceinline__ void linearize(const T* __restrict__ x, int v) const {
    T sn, c;
    sincos_t(x[2 * (size_t)n + v], &sn, &c);
    T* q = st + (size_t)v * 4;
    q[0] = c;
    q[1] = sn;
    q[2] = U[v];
    q[3] = U[n + v];
    const bool fit = Ct[v] >= T(0) && Ct[n + v] >= T(0);
    flags[v] = (uint8_t)(INGRID | (mask[v] == 0 ? ACTIVE : 0) | (fit ? FIT : 0));
  }

  // b = -J^T F and diag(J^T J) at an active vertex v.
  template <class XA>
  __device__ __forceinline__ void jtf_diag_site(XA X, int v, T* b, T* d) const {
    const T* sv = st + (size_t)v * 4;
    const T c = sv[0], sn = sv[1], Ux = sv[2], Uy = sv[3];
    const T Ox = X(0, v), Oy = X(1, v);
    T bx = 0, by = 0, bt = 0, nact = 0, dt = 0;
    const T wr2 = wr * wr;
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
      if (!(flags[u] & ACTIVE)) continue;
      const T* su = st + (size_t)u * 4;
      const T dx = Ux - su[2], dy = Uy - su[3];
      const T cq = su[0], sq = su[1];
      const T ex = Ox - X(0, u), ey = Oy - X(1, u);
      const T f1x = ex - (c * dx - sn * dy), f1y = ey - (sn * dx + c * dy);
      const T f2x = -ex + (cq * dx - sq * dy), f2y = -ey + (sq * dx + cq * dy);
      const T apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
      bx += wr2 * (f2x - f1x);
      by += wr2 * (f2y - f1y);
      bt += wr2 * (apx * f1x + apy * f1y);
      nact += T(1);
      dt += dx * dx + dy * dy;
    }
    const bool fit = flags[v] & FIT;
    if (fit) {
      const T wf2 = wf * wf;
      bx -= wf2 * (Ox - Ct[v]);
      by -= wf2 * (Oy - Ct[n + v]);
    }
    b[0] = bx;
    b[1] = by;
    b[2] = bt;
    const T dO = T(2) * wr2 * nact + (fit ? wf * wf : T(0));
    d[0] = dO;
    d[1] = dO;
    d[2] = wr2 * dt;
  }

  // g = J^T J P at an active vertex v; P(c, site) reads the direction.
  template <class PA>
  __device__ __forceinline__ void apply_site(PA P, int v, T* g) const {
    apply_staged(P, [&](int u) { return stage_vals(u); }, [&](int k) { return nb[k]; }, v, rp[v], rp[v + 1],
                 (uint32_t)flags[v], g);
  }

  // The staged values of vertex u: its state, then 1 when it is active, else 0.
  __device__ __forceinline__ Vals<T, 5> stage_vals(int u) const {
    Vals<T, 5> r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.v[k] = st[(size_t)u * 4 + k];
    r.v[4] = (flags[u] & ACTIVE) ? T(1) : T(0);
    return r;
  }

  // apply_site with every vertex named by a slot: vs for the vertex itself,
  // NB(k) for the neighbour of its incidence entries k0 <= k < k1; P(c, slot)
  // reads the direction, SA(slot) the staged values; fl is its flags byte.
  template <class PA, class SA, class NA>
  __device__ __forceinline__ void apply_staged(PA P, SA Sv, NA NB, int vs, int k0, int k1, uint32_t fl,
                                               T* g) const {
    const Vals<T, 5> sv = Sv(vs);
    const T c = sv.v[0], sn = sv.v[1], Ux = sv.v[2], Uy = sv.v[3];
    const T px = P(0, vs), py = P(1, vs), pt = P(2, vs);
    T gx = 0, gy = 0, gt = 0;
    const T wr2 = wr * wr;
    for (int k = k0; k < k1; ++k) {
      const int u = NB(k);
      const Vals<T, 5> su = Sv(u);
      const T w = su.v[4] * wr2;
      const T dx = Ux - su.v[2], dy = Uy - su.v[3];
      const T cq = su.v[0], sq = su.v[1];
      const T qx = P(0, u), qy = P(1, u), qt = P(2, u);
      const T apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
      const T aqx = sq * dx + cq * dy, aqy = -cq * dx + sq * dy;
      const T ex = px - qx, ey = py - qy;
      const T j1x = ex - apx * pt, j1y = ey - apy * pt;
      const T j2x = -ex - aqx * qt, j2y = -ey - aqy * qt;
      gx += w * (j1x - j2x);
      gy += w * (j1y - j2y);
      gt -= w * (apx * j1x + apy * j1y);
    }
    const T wfit = (fl & FIT) ? wf * wf : T(0);
    g[0] = fma(wfit, px, gx);
    g[1] = fma(wfit, py, gy);
    g[2] = gt;
  }

  // LM model term of the residuals anchored at v, in FP64.
  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int v) const {
    double acc = 0.0;
    const double Ox = X(0, v), Oy = X(1, v);
    const double dOx = Dl(0, v), dOy = Dl(1, v);
    if (mask[v] == 0) {
      double sn, c;
      sincos_t(X(2, v), &sn, &c);
      const double dt = Dl(2, v);
      const double Ux = U[v], Uy = U[n + v];
      for (int k = rp[v]; k < rp[v + 1]; ++k) {
        const int u = nb[k];
        if (mask[u] != 0) continue;
        const double dx = Ux - (double)U[u], dy = Uy - (double)U[n + u];
        const double fx = wr_d * ((Ox - X(0, u)) - (c * dx - sn * dy));
        const double fy = wr_d * ((Oy - X(1, u)) - (sn * dx + c * dy));
        const double apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
        const double jx = wr_d * ((dOx - Dl(0, u)) - apx * dt);
        const double jy = wr_d * ((dOy - Dl(1, u)) - apy * dt);
        acc += jx * (2.0 * fx + jx) + jy * (2.0 * fy + jy);
      }
    }
    const double cx = Ct[v], cy = Ct[n + v];
    if (cx >= 0.0 && cy >= 0.0) {
      const double fx = wf_d * (Ox - cx), fy = wf_d * (Oy - cy);
      const double jx = wf_d * dOx, jy = wf_d * dOy;
      acc += jx * (2.0 * fx + jx) + jy * (2.0 * fy + jy);
    }
    return acc;
  }
};

}  // namespace optmi
