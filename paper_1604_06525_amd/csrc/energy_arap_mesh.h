// As-rigid-as-possible mesh deformation on a graph (Fig. 25, Appendix A.1.2).
//
// Unknowns per vertex: offset O (3 planes) and Euler angles a (3 planes) with
// R(a) = Rz(a_z) Ry(a_y) Rx(a_x).  Data: rest positions U (3 planes), targets C
// (3 planes; component k is used when C_k >= -999999.9).
// Residuals:
//   fit   r = w_fit (O_v - C_v), per valid component
//   edge  for every listed edge {v0, v1}, both orientations (3 rows each):
//         r(v->u) = w_reg [ (O_v - O_u) - R(a_v)(U_v - U_u) ]
//
// The edge list is turned into a per-vertex incidence list (CSR, neighbours in
// edge-list order) when the problem is created, so each vertex gathers the terms
// of its own edges: no atomics, and every sum has a fixed order.  The paper
// scatters per edge with atomic adds instead (Sec. 4.1, graph residuals).
// With d = U_v - U_u and G_v(d) = [dR/da_x d, dR/da_y d, dR/da_z d] at a_v:
//   own   J p = w_reg [ (P^O_v - P^O_u) - G_v(d) P^a_v ]
//   back  J p = w_reg [ (P^O_u - P^O_v) + G_u(d) P^a_u ]
//   (J^T J P)^O_v += w_reg (own) - w_reg (back),  (J^T J P)^a_v += -w_reg G_v(d)^T (own)
// Per-vertex state: cos and sin of the three angles at the linearisation point.
#pragma once
#include "common.h"

namespace optmi {

template <typename R>
struct EulerTrig {
  R cx, sx, cy, sy, cz, sz;
};

// R d and G(d) (columns: d/da_x, d/da_y, d/da_z of R d) for R = Rz Ry Rx.
template <typename R>
__device__ __forceinline__ void euler_rot_grad(const EulerTrig<R>& t, const R* d, R* Rd, R (*G)[3]) {
  // x-rotation and its derivative
  const R v1[3] = {d[0], t.cx * d[1] - t.sx * d[2], t.sx * d[1] + t.cx * d[2]};
  const R v1x[3] = {R(0), -t.sx * d[1] - t.cx * d[2], t.cx * d[1] - t.sx * d[2]};
  auto ry = [&](const R* v, R* o) {
    o[0] = t.cy * v[0] + t.sy * v[2];
    o[1] = v[1];
    o[2] = -t.sy * v[0] + t.cy * v[2];
  };
  auto ry_d = [&](const R* v, R* o) {
    o[0] = -t.sy * v[0] + t.cy * v[2];
    o[1] = R(0);
    o[2] = -t.cy * v[0] - t.sy * v[2];
  };
  auto rz = [&](const R* v, R* o) {
    o[0] = t.cz * v[0] - t.sz * v[1];
    o[1] = t.sz * v[0] + t.cz * v[1];
    o[2] = v[2];
  };
  auto rz_d = [&](const R* v, R* o) {
    o[0] = -t.sz * v[0] - t.cz * v[1];
    o[1] = t.cz * v[0] - t.sz * v[1];
    o[2] = R(0);
  };
  R v2[3], v2x[3], v2y[3];
  ry(v1, v2);
  ry(v1x, v2x);
  ry_d(v1, v2y);
  rz(v2, Rd);
  rz(v2x, G[0]);
  rz(v2y, G[1]);
  rz_d(v2, G[2]);
}

template <typename T>
struct ArapMesh {
  using Real = T;
  static constexpr bool kGraph = true;
  static constexpr int C = 6;
  // per vertex: cos/sin of a_x, a_y, a_z, then U (copied at linearisation so
  // that everything a neighbour's product term reads is one 36-byte record)
  static constexpr int kStatePlanes = 9;
  static constexpr int kOwnState = 9;
  static constexpr int kRadius = 1;
  enum : uint32_t { ACTIVE = 1, INGRID = 2, FIT0 = 4 };  // FIT0 << k: component k
  static constexpr bool kStaged = true;  // pcg_a stages a vertex chunk in LDS (apply_staged)
  static constexpr int kStageVals = 9;   // staged per vertex: cos/sin of the angles, U

  int n;                         // vertices
  const int* __restrict__ rp;    // [n+1] CSR offsets
  const int* __restrict__ nb;    // [2E] neighbour ids
  Halo halo;                     // pcg_a's staging lists
  const T* __restrict__ U;       // [3][n]
  const T* __restrict__ Ct;      // [3][n]
  T* __restrict__ trig;          // [n][9]: per vertex cos/sin of the three angles, U
  uint8_t* __restrict__ flags;
  T wf, wr;
  double wf_d, wr_d;

  __device__ __forceinline__ T state_at(int k, int v) const { return trig[(size_t)v * 9 + k]; }

  __device__ __forceinline__ EulerTrig<T> trig_at(int v) const { return trig_from(trig + (size_t)v * 9); }
  // the six state values of a vertex (cos, sin of a_x, a_y, a_z) at q
  __device__ __forceinline__ static EulerTrig<T> trig_from(const T* q) {
    EulerTrig<T> t;
    t.cx = q[0];
    t.sx = q[1];
    t.cy = q[2];
    t.sy = q[3];
    t.cz = q[4];
    t.sz = q[5];
    return t;
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
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
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

  // b = -J^T F and diag(J^T J) at vertex v; X(c, site) reads the unknowns.
  template <class XA>
  __device__ __forceinline__ void jtf_diag_site(XA X, int v, T* b, T* dg) const {
    const EulerTrig<T> tv = trig_at(v);
    T bO[3] = {}, ba[3] = {}, Sdd[6] = {};
    const T wr2 = wr * wr;
    int cnt = 0;
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
      const EulerTrig<T> tu = trig_at(u);
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
      for (int q = 0; q < 3; ++q) ba[q] += wr2 * (Gv[q][0] * f1[0] + Gv[q][1] * f1[1] + Gv[q][2] * f1[2]);
      add_ddt(Sdd, d);
      ++cnt;
    }
    const uint32_t fl = flags[v];
    T G[3][3][3];
    unit_grads(tv, G);
    diag_from(G, Sdd, cnt, fl, dg);
    const T wf2 = wf * wf;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (fl & (FIT0 << c)) bO[c] -= wf2 * (X(c, v) - Ct[(size_t)c * n + v]);
      b[c] = bO[c];
      b[3 + c] = ba[c];
    }
  }

  // ---------------------------------------------- pieces of the diagonal
  // diag(J^T J) at a vertex: the offset entries are 2 w_reg^2 per incidence
  // entry (+ w_fit^2 on a fitted component); the angle entry q is
  // w_reg^2 sum_edges |R'_q d|^2 with R'_q = dR/da_q at the vertex's angles and
  // d = U_v - U_u.  That sum is written as <R'_q^T R'_q, S> with S = sum d d^T
  // (accumulated per edge, add_ddt), so the per-edge work does not depend on
  // the angles.  G[j][q] = R'_q e_j (unit_grads) holds the columns of R'_q.
  __device__ __forceinline__ static void add_ddt(T* S, const T* d) {
    S[0] = fma(d[0], d[0], S[0]);
    S[1] = fma(d[0], d[1], S[1]);
    S[2] = fma(d[0], d[2], S[2]);
    S[3] = fma(d[1], d[1], S[3]);
    S[4] = fma(d[1], d[2], S[4]);
    S[5] = fma(d[2], d[2], S[5]);
  }
  // The columns of R'_x = Rz Ry Rx', R'_y = Rz Ry' Rx and R'_z = Rz' Ry Rx in
  // closed form (A = Rz Ry by columns; Rz Ry' has columns -A_2, 0, A_0; C is
  // Rz' Ry, whose last row is zero), with the structural zeros written as such.
  __device__ __forceinline__ static void unit_grads(const EulerTrig<T>& t, T (*G)[3][3]) {
    const T cx = t.cx, sx = t.sx, cy = t.cy, sy = t.sy, cz = t.cz, sz = t.sz;
    const T A0[3] = {cz * cy, sz * cy, -sy};
    const T A2[3] = {cz * sy, sz * sy, cy};
    const T c0[2] = {-sz * cy, cz * cy};
    const T c2[2] = {-sz * sy, cz * sy};
    // R'_x: column 0 is zero; A_1 = (-sz, cz, 0)
    G[0][0][0] = G[0][0][1] = G[0][0][2] = T(0);
    G[1][0][0] = fma(cx, A2[0], sx * sz);
    G[1][0][1] = fma(cx, A2[1], -sx * cz);
    G[1][0][2] = cx * A2[2];
    G[2][0][0] = fma(-sx, A2[0], cx * sz);
    G[2][0][1] = fma(-sx, A2[1], -cx * cz);
    G[2][0][2] = -sx * A2[2];
    // R'_y
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      G[0][1][i] = -A2[i];
      G[1][1][i] = sx * A0[i];
      G[2][1][i] = cx * A0[i];
    }
    // R'_z: C_1 = (-cz, -sz, 0); row 2 is zero
    G[0][2][0] = c0[0];
    G[0][2][1] = c0[1];
    G[1][2][0] = fma(sx, c2[0], -cx * cz);
    G[1][2][1] = fma(sx, c2[1], -cx * sz);
    G[2][2][0] = fma(cx, c2[0], sx * cz);
    G[2][2][1] = fma(cx, c2[1], sx * sz);
    G[0][2][2] = G[1][2][2] = G[2][2][2] = T(0);
  }
  __device__ __forceinline__ T diag_o(int cnt, uint32_t fl, int c) const {
    const T d = T(2) * (wr * wr) * T(cnt);
    return (fl & (FIT0 << c)) ? d + wf * wf : d;
  }
  __device__ __forceinline__ void diag_from(const T (*G)[3][3], const T* S, int cnt, uint32_t fl, T* dg) const {
    const T wr2 = wr * wr;
#pragma unroll
    for (int c = 0; c < 3; ++c) dg[c] = diag_o(cnt, fl, c);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      // <R'_q^T R'_q, S>, S symmetric: the diagonal terms, then twice the upper ones
      auto gram = [&](int j, int k) {
        return fma(G[j][q][2], G[k][q][2], fma(G[j][q][1], G[k][q][1], G[j][q][0] * G[k][q][0]));
      };
      T acc = gram(0, 0) * S[0];
      acc = fma(gram(1, 1), S[3], acc);
      acc = fma(gram(2, 2), S[5], acc);
      const T off = fma(gram(1, 2), S[4], fma(gram(0, 2), S[2], gram(0, 1) * S[1]));
      dg[3 + q] = wr2 * fma(T(2), off, acc);
    }
  }

  // ---------------------------------------------- fused graph PCG hooks
  // The fused iteration stages a record per vertex: p^O, the 3 x 3 matrix
  // D = sum_q p^a_q R'_q (row-major; G_v(d) p^a = D d for any d, so an edge
  // term costs two 3 x 3 products instead of two evaluations of the rotation
  // chain) and U.  A neighbour's share of delta reads only the offset of u.
  static constexpr bool kGraphFused = true;
  static constexpr int kRec = 15;
  static constexpr int kHalo = 3;
  struct GOwn {
    T G[3][3][3];  // G[j][q] = R'_q e_j at the vertex's angles
    T U[3];
  };
  // a vertex's state as loaded (graw) and what the products use of it (gown_of)
  using GRaw = Vals<T, 9>;
  __device__ __forceinline__ GRaw graw(int v) const {
    const auto* q = gmem(trig) + (size_t)v * 9;
    GRaw r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.v[k] = q[k];
    return r;
  }
  __device__ __forceinline__ GOwn gown_of(const GRaw& r) const {
    GOwn o;
    unit_grads(trig_from(r.v), o.G);
#pragma unroll
    for (int c = 0; c < 3; ++c) o.U[c] = r.v[6 + c];
    return o;
  }
  __device__ __forceinline__ static void dmat(const GOwn& o, const T* pa, T* D) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        D[3 * i + j] = fma(pa[2], o.G[j][2][i], fma(pa[1], o.G[j][1][i], pa[0] * o.G[j][0][i]));
  }
  __device__ __forceinline__ static void mul_d(const T* D, const T* d, T* out) {
#pragma unroll
    for (int i = 0; i < 3; ++i) out[i] = fma(D[3 * i + 2], d[2], fma(D[3 * i + 1], d[1], D[3 * i] * d[0]));
  }
  __device__ __forceinline__ void grec(const GOwn& o, const T* p, T* r) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = p[c];
      r[12 + c] = o.U[c];
    }
    dmat(o, p + 3, r + 3);
  }
  // The offset part of edge v -> (slot s): d = U_v - U_u, the own residual's
  // J p (j1) and the back residual's (j2 = D_u d - (p^O_v - p^O_u)); adds
  // w_reg^2 (j1 - j2) to gO.  gapply and gapply_h both go through here, so a
  // vertex's offset product has the same bits wherever it is evaluated.
  template <class RA>
  __device__ __forceinline__ void edge_o(const T* pO, const T* D, const T* Uv, RA R, int s, T wr2, T* gO, T* d,
                                         T* j1) const {
    T Du[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Du[k] = R(s, 3 + k);
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = Uv[c] - R(s, 12 + c);
    T dv[3], du[3];
    mul_d(D, d, dv);
    mul_d(Du, d, du);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T e = pO[c] - R(s, c);
      j1[c] = e - dv[c];
      const T j2 = du[c] - e;
      gO[c] = fma(wr2, j1[c] - j2, gO[c]);
    }
  }
  // (J^T J p)_v at a vertex of the chunk: p its direction, rv its record,
  // R(slot, k) a staged record entry, NB(k) the slot of incidence entry k
  // (k0 <= k < k1).  (The kernel reads the diagonal init stored.)
  template <class RA, class NA>
  __device__ __forceinline__ void gapply(const GOwn& o, const T* p, const T* rv, int, RA R, NA NB, int k0, int k1,
                                         uint32_t fl, T* g) const {
    const T wr2 = wr * wr, wf2 = wf * wf;
    T gO[3] = {}, Mv[9] = {};
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      T d[3], j1[3];
      edge_o(p, rv + 3, o.U, R, NB(k), wr2, gO, d, j1);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Mv[3 * i + j] = fma(j1[i], d[j], Mv[3 * i + j]);
    }
    // angle q: -w_reg^2 sum_edges (R'_q d) . j1 = -w_reg^2 <R'_q, sum j1 d^T>
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc = fma(o.G[j][q][i], Mv[3 * i + j], acc);
      g[3 + q] = -wr2 * acc;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = (fl & (FIT0 << c)) ? fma(wf2, p[c], gO[c]) : gO[c];
  }
  // gapply and the vertex's diagonal, formed from the same edges (d d^T summed
  // in incidence order and diag_from: init's arithmetic, so the same bits
  // init stored, without reading them).
  template <class RA, class NA>
  __device__ __forceinline__ void gapply_d(const GOwn& o, const T* p, const T* rv, int, RA R, NA NB, int k0,
                                           int k1, uint32_t fl, T* g, T* dg) const {
    const T wr2 = wr * wr, wf2 = wf * wf;
    T gO[3] = {}, Mv[9] = {}, Sdd[6] = {};
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      T d[3], j1[3];
      edge_o(p, rv + 3, o.U, R, NB(k), wr2, gO, d, j1);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Mv[3 * i + j] = fma(j1[i], d[j], Mv[3 * i + j]);
      add_ddt(Sdd, d);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc = fma(o.G[j][q][i], Mv[3 * i + j], acc);
      g[3 + q] = -wr2 * acc;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = (fl & (FIT0 << c)) ? fma(wf2, p[c], gO[c]) : gO[c];
    diag_from(o.G, Sdd, k1 - k0, fl, dg);
  }
  // The offset part of gapply at the staged vertex in slot sv (R1 of a chunk),
  // and of the diagonal (as init's diag_from gives it).
  template <class RA, class NA>
  __device__ __forceinline__ void gapply_h(int sv, RA R, NA NB, int k0, int k1, uint32_t fl, T* g, T* dg) const {
    const T wr2 = wr * wr, wf2 = wf * wf;
    T pO[3], D[9], Uv[3], gO[3] = {};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pO[c] = R(sv, c);
      Uv[c] = R(sv, 12 + c);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) D[k] = R(sv, 3 + k);
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      T d[3], j1[3];
      edge_o(pO, D, Uv, R, NB(k), wr2, gO, d, j1);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[c] = (fl & (FIT0 << c)) ? fma(wf2, pO[c], gO[c]) : gO[c];
      dg[c] = diag_o(k1 - k0, fl, c);
    }
  }
  // The vertex's share of |J u|^2: its own edge residuals and its fit rows
  // (every residual row belongs to exactly one vertex); UH(slot, c) reads a
  // neighbour's offset of u.
  template <class RA, class UA, class NA>
  __device__ __forceinline__ T gjsq(const GOwn& o, const T* u, RA R, UA UH, NA NB, int k0, int k1,
                                    uint32_t fl) const {
    T Du[9];
    dmat(o, u + 3, Du);
    T acc = T(0);
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const int s = NB(k);
      T d[3], dd[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = o.U[c] - R(s, 12 + c);
      mul_d(Du, d, dd);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T r = (u[c] - UH(s, c)) - dd[c];
        acc = fma(r, r, acc);
      }
    }
    T f = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (fl & (FIT0 << c)) f = fma(u[c], u[c], f);
    return fma(wr * wr, acc, (wf * wf) * f);
  }

  // g = J^T J P at vertex v; P(c, site) reads the direction.
  template <class PA>
  __device__ __forceinline__ void apply_site(PA P, int v, T* g) const {
    apply_staged(P, [&](int u) { return stage_vals(u); }, [&](int k) { return nb[k]; }, v, rp[v], rp[v + 1],
                 (uint32_t)flags[v], g);
  }

  // The staged values of vertex u: its state record (cos/sin of its angles, U).
  __device__ __forceinline__ Vals<T, 9> stage_vals(int u) const {
    Vals<T, 9> r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.v[k] = trig[(size_t)u * 9 + k];
    return r;
  }

  // apply_site with every vertex named by a slot: vs for the vertex itself,
  // NB(k) for the neighbour of its incidence entries k0 <= k < k1; P(c, slot)
  // reads the direction, SA(slot) the staged values; fl is its flags byte.
  template <class PA, class SA, class NA>
  __device__ __forceinline__ void apply_staged(PA P, SA Sv, NA NB, int vs, int k0, int k1, uint32_t fl,
                                               T* g) const {
    const Vals<T, 9> sv = Sv(vs);
    const EulerTrig<T> tv = trig_from(sv.v);
    T pO[3], pa[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pO[c] = P(c, vs);
      pa[c] = P(3 + c, vs);
    }
    T gO[3] = {}, ga[3] = {};
    const T wr2 = wr * wr;
    for (int k = k0; k < k1; ++k) {
      const int u = NB(k);
      const Vals<T, 9> su = Sv(u);
      const EulerTrig<T> tu = trig_from(su.v);
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
      for (int q = 0; q < 3; ++q)
        ga[q] -= wr2 * (Gv[q][0] * j1[0] + Gv[q][1] * j1[1] + Gv[q][2] * j1[2]);
    }
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
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int u = nb[k];
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
