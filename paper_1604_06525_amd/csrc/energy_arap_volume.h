// As-rigid-as-possible volumetric deformation on a 3D grid (Fig. 31, Appendix
// A.2.5): the ARAP energy of the mesh example with the voxel lattice as its
// implicit connectivity.
//
// Unknowns per voxel: offset O (3 planes) and Euler angles a (3 planes),
// R(a) = Rz(a_z) Ry(a_y) Rx(a_x).  Data: rest positions U (3 planes), targets C
// (3 planes; component k is used when C_k >= -999999.9).  Voxel v = (k*H + j)*W
// + i, i along the width.
// Residuals:
//   fit  r = w_fit (O_v - C_v), per valid component
//   reg  for every voxel v and each of its in-bounds neighbours u along +-x,
//        +-y, +-z (the 7-point stencil without its centre):
//        r(v->u) = w_reg [ (O_v - O_u) - R(a_v)(U_v - U_u) ]   (3 rows)
// Every lattice edge thus appears in both orientations, as in the mesh energy
// with both orientations of each listed edge, and each voxel gathers the terms
// of its own neighbourhood (no atomics; a fixed summation order).
// Per-voxel state: cos and sin of the three angles at the linearisation point
// and the rest position, one 36-byte record (what a neighbour's term reads).
#pragma once
#include "common.h"
#include "energy_arap_mesh.h"

namespace optmi {

template <typename T>
struct ArapVolume {
  using Real = T;
  // site-indexed accessors like a graph energy, with the neighbours computed
  // from the lattice instead of read from an incidence list
  static constexpr bool kGraph = true;
  static constexpr int C = 6;
  static constexpr int kStatePlanes = 9;
  static constexpr int kOwnState = 9;
  static constexpr int kRadius = 1;
  enum : uint32_t { ACTIVE = 1, INGRID = 2, FIT0 = 4 };  // FIT0 << k: component k

  int n, W, H, D;
  const T* __restrict__ U;   // [3][n]
  const T* __restrict__ Ct;  // [3][n]
  T* __restrict__ trig;      // [n][9]: cos/sin of a_x, a_y, a_z, then U
  uint8_t* __restrict__ flags;
  T wf, wr;
  double wf_d, wr_d;

  // The in-bounds lattice neighbours of v, in the order +x, -x, +y, -y, +z, -z;
  // returns their number.
  __device__ __forceinline__ int neighbours(int v, int* nb) const {
    const int i = v % W, j = (v / W) % H, k = v / (W * H);
    const int plane = W * H;
    int m = 0;
    if (i + 1 < W) nb[m++] = v + 1;
    if (i > 0) nb[m++] = v - 1;
    if (j + 1 < H) nb[m++] = v + W;
    if (j > 0) nb[m++] = v - W;
    if (k + 1 < D) nb[m++] = v + plane;
    if (k > 0) nb[m++] = v - plane;
    return m;
  }

  __device__ __forceinline__ T state_at(int k, int v) const { return trig[(size_t)v * 9 + k]; }
  __device__ __forceinline__ Vals<T, 9> rec(int v) const {
    Vals<T, 9> r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.v[k] = trig[(size_t)v * 9 + k];
    return r;
  }

  template <class XA>
  __device__ __forceinline__ EulerTrig<double> trig_d(XA X, int v) const {
    EulerTrig<double> t;
    sincos_t((double)X(3, v), &t.sx, &t.cx);
    sincos_t((double)X(4, v), &t.sy, &t.cy);
    sincos_t((double)X(5, v), &t.sz, &t.cz);
    return t;
  }

  template <class XA>
  __device__ __forceinline__ double cost(XA X, int v) const {
    double e = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double cv = Ct[(size_t)c * n + v];
      if (cv >= -999999.9) {
        const double f = wf_d * (X(c, v) - cv);
        e += f * f;
      }
    }
    const EulerTrig<double> t = trig_d(X, v);
    int nb[6];
    const int m = neighbours(v, nb);
    for (int q = 0; q < m; ++q) {
      const int u = nb[q];
      double d[3], Rd[3], G[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = (double)U[(size_t)c * n + v] - (double)U[(size_t)c * n + u];
      euler_rot_grad(t, d, Rd, G);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double f = wr_d * ((X(c, v) - X(c, u)) - Rd[c]);
        e += f * f;
      }
    }
    return e;
  }

  __device__ __forceinline__ void linearize(const T* __restrict__ x, int v) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T s, c;
      sincos_t(x[(size_t)(3 + k) * n + v], &s, &c);
      trig[(size_t)v * 9 + 2 * k] = c;
      trig[(size_t)v * 9 + 2 * k + 1] = s;
      trig[(size_t)v * 9 + 6 + k] = U[(size_t)k * n + v];
    }
    uint32_t f = ACTIVE | INGRID;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (Ct[(size_t)c * n + v] >= T(-999999.9)) f |= FIT0 << c;
    flags[v] = (uint8_t)f;
  }

  // b = -J^T F and diag(J^T J) at voxel v; X(c, site) reads the unknowns.
  template <class XA>
  __device__ __forceinline__ void jtf_diag_site(XA X, int v, T* b, T* dg) const {
    const EulerTrig<T> tv = ArapMesh<T>::trig_from(trig + (size_t)v * 9);
    T bO[3] = {}, ba[3] = {}, dO = 0, da[3] = {};
    const T wr2 = wr * wr;
    int nb[6];
    const int m = neighbours(v, nb);
    for (int q = 0; q < m; ++q) {
      const int u = nb[q];
      const EulerTrig<T> tu = ArapMesh<T>::trig_from(trig + (size_t)u * 9);
      T d[3], Rv[3], Gv[3][3], Ru[3], Gu[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = U[(size_t)c * n + v] - U[(size_t)c * n + u];
      euler_rot_grad(tv, d, Rv, Gv);
      euler_rot_grad(tu, d, Ru, Gu);
      T f1[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T e = X(c, v) - X(c, u);
        f1[c] = e - Rv[c];
        const T f2 = -e + Ru[c];
        bO[c] += wr2 * (f2 - f1[c]);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ba[k] += wr2 * (Gv[k][0] * f1[0] + Gv[k][1] * f1[1] + Gv[k][2] * f1[2]);
        da[k] += wr2 * (Gv[k][0] * Gv[k][0] + Gv[k][1] * Gv[k][1] + Gv[k][2] * Gv[k][2]);
      }
      dO += T(2) * wr2;
    }
    const uint32_t fl = flags[v];
    const T wf2 = wf * wf;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T dc = dO;
      if (fl & (FIT0 << c)) {
        bO[c] -= wf2 * (X(c, v) - Ct[(size_t)c * n + v]);
        dc += wf2;
      }
      b[c] = bO[c];
      dg[c] = dc;
      b[3 + c] = ba[c];
      dg[3 + c] = da[c];
    }
  }

  // g = J^T J P at voxel v; P(c, site) reads the direction.  Per neighbour u
  // the two residual blocks of the edge {v, u}: v->u (own) and u->v (back).
  template <class PA>
  __device__ __forceinline__ void apply_site(PA P, int v, T* g) const {
    const Vals<T, 9> sv = rec(v);
    const EulerTrig<T> tv = ArapMesh<T>::trig_from(sv.v);
    T pO[3], pa[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pO[c] = P(c, v);
      pa[c] = P(3 + c, v);
    }
    T gO[3] = {}, ga[3] = {};
    const T wr2 = wr * wr;
    int nb[6];
    const int m = neighbours(v, nb);
    for (int q = 0; q < m; ++q) {
      const int u = nb[q];
      const Vals<T, 9> su = rec(u);
      const EulerTrig<T> tu = ArapMesh<T>::trig_from(su.v);
      T d[3], Rv[3], Gv[3][3], Ru[3], Gu[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = sv.v[6 + c] - su.v[6 + c];
      euler_rot_grad(tv, d, Rv, Gv);
      euler_rot_grad(tu, d, Ru, Gu);
      T qa[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) qa[c] = P(3 + c, u);
      T j1[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T e = pO[c] - P(c, u);
        j1[c] = e - (Gv[0][c] * pa[0] + Gv[1][c] * pa[1] + Gv[2][c] * pa[2]);
        const T j2 = -e + (Gu[0][c] * qa[0] + Gu[1][c] * qa[1] + Gu[2][c] * qa[2]);
        gO[c] += wr2 * (j1[c] - j2);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) ga[k] -= wr2 * (Gv[k][0] * j1[0] + Gv[k][1] * j1[1] + Gv[k][2] * j1[2]);
    }
    const uint32_t fl = flags[v];
    const T wf2 = wf * wf;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[c] = (fl & (FIT0 << c)) ? gO[c] + wf2 * pO[c] : gO[c];
      g[3 + c] = ga[c];
    }
  }

  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int v) const {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double cv = Ct[(size_t)c * n + v];
      if (cv >= -999999.9) {
        const double f = wf_d * (X(c, v) - cv);
        const double jd = wf_d * Dl(c, v);
        acc += jd * (2.0 * f + jd);
      }
    }
    const EulerTrig<double> t = trig_d(X, v);
    int nb[6];
    const int m = neighbours(v, nb);
    for (int q = 0; q < m; ++q) {
      const int u = nb[q];
      double d[3], Rd[3], G[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = (double)U[(size_t)c * n + v] - (double)U[(size_t)c * n + u];
      euler_rot_grad(t, d, Rd, G);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double f = wr_d * ((X(c, v) - X(c, u)) - Rd[c]);
        const double jd = wr_d * ((Dl(c, v) - Dl(c, u)) -
                                  (G[0][c] * Dl(3, v) + G[1][c] * Dl(4, v) + G[2][c] * Dl(5, v)));
        acc += jd * (2.0 * f + jd);
      }
    }
    return acc;
  }
};

}  // namespace optmi
