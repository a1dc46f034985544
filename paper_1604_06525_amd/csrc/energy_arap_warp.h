// As-rigid-as-possible image warping on a pixel grid (Fig. 24, Appendix A.1.1).
//
// Unknowns per pixel p: offset O_p (2 planes) and angle t_p (1 plane).  Data:
// rest positions U (2 planes), targets C (2 planes), mask (uint8).
// Residuals anchored at p:
//   for each stencil offset s, q = p + s, when q is on the grid and both p and q
//   have mask 0:  r = w_reg [ (O_p - O_q) - R(t_p) (U_p - U_q) ]       (2 rows)
//   when both components of C_p are >= 0:  r = w_fit (O_p - C_p)       (2 rows)
// with R(t) = [[cos t, -sin t], [sin t, cos t]].  Pixels with mask != 0 are
// excluded (Exclude in Fig. 24): constants that keep their terms.
//
// Matrix-free products (the template-shift view of Sec. 5.3.1): the residuals
// that read the unknowns of p are p's own four regularisers, the four
// regularisers anchored at its neighbours that point back at p, and p's fit.
// With d = U_p - U_q, a_p = R'(t_p) d and a_q = R'(t_q)(U_q - U_p):
//   own    J p = w_reg [ (P_p - P_q) - a_p P^t_p ]
//   back   J p = w_reg [ (P_q - P_p) - a_q P^t_q ]
//   (J^T J P)_O(p) += w_reg (own) - w_reg (back),  (J^T J P)_t(p) += -w_reg a_p . (own)
// R'(t) d is R(t) d turned by +90 degrees, so |a_p| = |d|.  J^T J couples a
// pixel to its four neighbours only (operator radius 1).
//
// Stencil functions read through views: P(c, di, dj) and S(k, di, dj) give
// unknown-vector channel c and state plane k at offset (di, dj) from the centre,
// F(di, dj) the flags there (0 off the grid).  State planes: cos t, sin t, U_x, U_y.
// In FP32 a site stores its angle instead of cos t and sin t (12 bytes instead
// of 16, read every PCG iteration); the two are formed where the record is read,
// by the branch-free sin and cos of angle_trig.h.  FP64 stores them.
#pragma once
#include "angle_trig.h"
#include "common.h"

namespace optmi {

template <typename T>
struct ArapWarp {
  using Real = T;
  static constexpr bool kGraph = false;
  static constexpr int C = 3;             // unknown channels
  static constexpr int kStatePlanes = 4;  // as the products read them: cos t, sin t, U_x, U_y
  // as stored per site: FP32 (t, U_x, U_y), FP64 (cos t, sin t, U_x, U_y); U is
  // copied beside the angle so that a site's state is one record
  static constexpr int kStateRec = sizeof(T) == 4 ? 3 : 4;
  static constexpr int kOwnState = 4;     // workspace planes per site (the wider record)
  static constexpr int kRadius = 1;       // stencil radius of J^T J
  enum : uint32_t { ACTIVE = 1, INGRID = 2, FIT = 4 };

  int W, H, n;
  const T* __restrict__ U;    // [2][n]
  const T* __restrict__ Ct;   // [2][n]
  const uint8_t* __restrict__ mask;
  T* __restrict__ st;         // [n][kStateRec]: the angle (or its cos, sin) at the linearisation point, U_x, U_y
  uint8_t* __restrict__ flags;
  T wf, wr;                   // w_fit, w_reg in the bulk type
  double wf_d, wr_d;          // and in double for the cost

  __device__ __forceinline__ T state_at(int k, int site) const {
    const T* r = st + (size_t)site * kStateRec;
    if constexpr (kStateRec == 4) {
      return r[k];
    } else {
      if (k >= 2) return r[k - 1];
      float sn, c;
      sincos_angle(r[0], &sn, &c);
      return k == 0 ? c : sn;
    }
  }
  __device__ __forceinline__ const T* state_base() const { return st; }
  // The four planes from a record loaded into their last kStateRec places.
  __device__ __forceinline__ static void expand_state(T* s) {
    if constexpr (kStateRec == 3) {
      float sn, c;
      sincos_angle(s[1], &sn, &c);
      s[0] = c;
      s[1] = sn;
    }
  }

  // Neighbour k of site (i, j) in the order (1,0), (-1,0), (0,1), (0,-1);
  // its id, or -1 off the grid.
  __device__ __forceinline__ int nbr(int i, int j, int s, int k) const {
    switch (k) {
      case 0: return i + 1 < W ? s + 1 : -1;
      case 1: return i > 0 ? s - 1 : -1;
      case 2: return j + 1 < H ? s + W : -1;
      default: return j > 0 ? s - W : -1;
    }
  }

  // FP64 sum of squares of the residuals anchored at s, unknowns read through
  // X(ch, site) (values of the bulk type, returned as double).
  template <class XA>
  __device__ __forceinline__ double cost(XA X, int s) const {
    const int i = s % W, j = s / W;
    const bool ap = mask[s] == 0;
    double sn, c;
    sincos_t(X(2, s), &sn, &c);
    const double Ox = X(0, s), Oy = X(1, s);
    const double Ux = U[s], Uy = U[n + s];
    double e = 0.0;
    if (ap) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = nbr(i, j, s, k);
        if (q < 0 || mask[q] != 0) continue;
        const double dx = Ux - (double)U[q], dy = Uy - (double)U[n + q];
        const double rx = wr_d * ((Ox - X(0, q)) - (c * dx - sn * dy));
        const double ry = wr_d * ((Oy - X(1, q)) - (sn * dx + c * dy));
        e += rx * rx + ry * ry;
      }
    }
    const double cx = Ct[s], cy = Ct[n + s];
    if (cx >= 0.0 && cy >= 0.0) {
      const double fx = wf_d * (Ox - cx), fy = wf_d * (Oy - cy);
      e += fx * fx + fy * fy;
    }
    return e;
  }

  // Per-site state for the products: the angle (or its cos/sin), U and the flags.
  __device__ __forceinline__ void linearize(const T* __restrict__ x, int s) const {
    const T t = x[2 * (size_t)n + s];
    T* q = st + (size_t)s * kStateRec;
    if constexpr (kStateRec == 4) {
      T sn, c;
      sincos_t(t, &sn, &c);
      q[0] = c;
      q[1] = sn;
    } else {
      q[0] = t;
    }
    q[kStateRec - 2] = U[s];
    q[kStateRec - 1] = U[n + s];
    const bool fit = Ct[s] >= T(0) && Ct[n + s] >= T(0);
    flags[s] = (uint8_t)(INGRID | (mask[s] == 0 ? ACTIVE : 0) | (fit ? FIT : 0));
  }

  // b = -J^T F and diag(J^T J) at an active site s (global index) at the
  // linearisation point; X views the unknowns.
  template <class XV, class SV, class FV>
  __device__ __forceinline__ void jtf_diag(XV X, SV S, FV F, int s, int, int, T* b, T* d) const {
    const T c = S(0, 0, 0), sn = S(1, 0, 0), Ux = S(2, 0, 0), Uy = S(3, 0, 0);
    const T Ox = X(0, 0, 0), Oy = X(1, 0, 0);
    T bx = 0, by = 0, bt = 0;
    const T wr2 = wr * wr;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      if (!(F(di, dj) & ACTIVE)) continue;
      const T dx = Ux - S(2, di, dj), dy = Uy - S(3, di, dj);
      const T cq = S(0, di, dj), sq = S(1, di, dj);
      const T ex = Ox - X(0, di, dj), ey = Oy - X(1, di, dj);
      // own residual / w_reg, and the back residual / w_reg
      const T f1x = ex - (c * dx - sn * dy), f1y = ey - (sn * dx + c * dy);
      const T f2x = -ex + (cq * dx - sq * dy), f2y = -ey + (sq * dx + cq * dy);
      const T apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
      bx += wr2 * (f2x - f1x);
      by += wr2 * (f2y - f1y);
      bt += wr2 * (apx * f1x + apy * f1y);
    }
    if (F(0, 0) & FIT) {
      const T wf2 = wf * wf;
      bx -= wf2 * (Ox - Ct[s]);
      by -= wf2 * (Oy - Ct[n + s]);
    }
    b[0] = bx; b[1] = by; b[2] = bt;
    diag(S, F, d);
  }

  // diag(J^T J) at an active centre, from the state and flags alone: 2 w_reg^2
  // per active neighbour (+ w_fit^2) for the offsets, w_reg^2 |U_p - U_q|^2 per
  // active neighbour for the angle (|R'(t) d| = |d|).
  template <class SV, class FV>
  __device__ __forceinline__ void diag(SV S, FV F, T* d) const {
    const T Ux = S(2, 0, 0), Uy = S(3, 0, 0);
    const T wr2 = wr * wr;
    T nact = 0, dt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = (F(di, dj) & ACTIVE) ? T(1) : T(0);
      const T dx = Ux - S(2, di, dj), dy = Uy - S(3, di, dj);
      nact += w;
      dt += w * (dx * dx + dy * dy);
    }
    const T dO = T(2) * wr2 * nact + ((F(0, 0) & FIT) ? wf * wf : T(0));
    d[0] = dO;
    d[1] = dO;
    d[2] = wr2 * dt;
  }

  // Materialised Jacobian (evalJ, Sec. 7): the rows anchored at site s, each
  // with kJSlots entries (column = internal vector index site*C + channel, -1
  // for no entry, value 0 there): rows 2k, 2k+1 are the x and y regulariser
  // towards neighbour k, rows 8, 9 the x and y fit.  Columns of excluded
  // unknowns are dropped (Exclude), so a row exists only where both of its
  // pixels are active.  An unknown appears in at most kJTSlots rows: an offset
  // in its fit, its four own regularisers and its four neighbours'; an angle in
  // its own eight regulariser rows.
  static constexpr int kJRows = 10, kJSlots = 3, kJTSlots = 9;
  __device__ __forceinline__ void eval_j(int s, T* __restrict__ val, int* __restrict__ col) const {
    const int i = s % W, j = s / W;
    const uint32_t fp = flags[s];
    const T c = state_at(0, s), sn = state_at(1, s), Ux = state_at(2, s), Uy = state_at(3, s);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = nbr(i, j, s, k);
      const bool on = (fp & ACTIVE) && q >= 0 && (flags[q] & ACTIVE);
      const T dx = on ? Ux - state_at(2, q) : T(0), dy = on ? Uy - state_at(3, q) : T(0);
      const T a[2] = {-sn * dx - c * dy, c * dx - sn * dy};  // R'(t_p)(U_p - U_q)
#pragma unroll
      for (int ch = 0; ch < 2; ++ch) {
        const int r = (2 * k + ch) * kJSlots;
        col[r] = on ? s * 3 + ch : -1;
        col[r + 1] = on ? q * 3 + ch : -1;
        col[r + 2] = on ? s * 3 + 2 : -1;
        val[r] = on ? wr : T(0);
        val[r + 1] = on ? -wr : T(0);
        val[r + 2] = on ? -wr * a[ch] : T(0);
      }
    }
    const bool fit = (fp & ACTIVE) && (fp & FIT);
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const int r = (8 + ch) * kJSlots;
      col[r] = fit ? s * 3 + ch : -1;
      col[r + 1] = -1;
      col[r + 2] = -1;
      val[r] = fit ? wf : T(0);
      val[r + 1] = T(0);
      val[r + 2] = T(0);
    }
  }

  // The column lists of J^T for the unknowns of site s (kJTSlots entries each,
  // indices into eval_j's entries, in row order of appearance below, -1 after
  // the last): the structure of eval_j read by column.  Offset channel c: its
  // fit row, its own four regularisers (slot 0), the neighbours' regularisers
  // pointing back at s (slot 1); angle: its own eight regulariser rows (slot 2).
  __device__ __forceinline__ void eval_jt(int s, int* __restrict__ jt) const {
    const int i = s % W, j = s / W;
    const bool act = flags[s] & ACTIVE;
    bool on[4];
    int q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[k] = nbr(i, j, s, k);
      on[k] = act && q[k] >= 0 && (flags[q[k]] & ACTIVE);
    }
    const bool fit = act && (flags[s] & FIT);
    auto at = [](int site, int row, int slot) { return (site * kJRows + row) * kJSlots + slot; };
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      int* o = jt + ch * kJTSlots;
      int m = 0;
      if (fit) o[m++] = at(s, 8 + ch, 0);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (on[k]) o[m++] = at(s, 2 * k + ch, 0);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (on[k]) o[m++] = at(q[k], 2 * (k ^ 1) + ch, 1);  // (k ^ 1): the opposite offset
      for (; m < kJTSlots; ++m) o[m] = -1;
    }
    int* o = jt + 2 * kJTSlots;
    int m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int ch = 0; ch < 2; ++ch)
        if (on[k]) o[m++] = at(s, 2 * k + ch, 2);
    for (; m < kJTSlots; ++m) o[m] = -1;
  }

  // Per-site edge geometry that apply computes and jsq reuses: for each
  // neighbour k, a_p = R'(t_p)(U_p - U_q).
  struct JCache {
    T ax[4], ay[4];
  };

  // g = J^T J P at an active centre site.
  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply(PV P, SV S, FV F, int i, int j, T* g) const {
    JCache jc;
    apply_c(P, S, F, i, j, g, jc);
  }

  // apply, also filling the edge geometry of the centre.
  template <class PV, class SV, class FV>
  __device__ __forceinline__ void apply_c(PV P, SV S, FV F, int, int, T* g, JCache& jc) const {
    const T c = S(0, 0, 0), sn = S(1, 0, 0), Ux = S(2, 0, 0), Uy = S(3, 0, 0);
    const T px = P(0, 0, 0), py = P(1, 0, 0), pt = P(2, 0, 0);
    T gx = 0, gy = 0, gt = 0;
    const T wr2 = wr * wr;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      // a neighbour that is excluded or off the grid contributes nothing; its
      // values are finite (zero off the grid), so weight instead of branching
      const T w = (F(di, dj) & ACTIVE) ? wr2 : T(0);
      const T dx = Ux - S(2, di, dj), dy = Uy - S(3, di, dj);
      const T cq = S(0, di, dj), sq = S(1, di, dj);
      const T qx = P(0, di, dj), qy = P(1, di, dj), qt = P(2, di, dj);
      const T apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
      const T aqx = sq * dx + cq * dy, aqy = -cq * dx + sq * dy;
      const T ex = px - qx, ey = py - qy;
      const T j1x = ex - apx * pt, j1y = ey - apy * pt;
      const T j2x = -ex - aqx * qt, j2y = -ey - aqy * qt;
      gx += w * (j1x - j2x);
      gy += w * (j1y - j2y);
      gt -= w * (apx * j1x + apy * j1y);
      jc.ax[k] = apx;
      jc.ay[k] = apy;
    }
    const T wfit = (F(0, 0) & FIT) ? wf * wf : T(0);
    g[0] = fma(wfit, px, gx);
    g[1] = fma(wfit, py, gy);
    g[2] = gt;
  }

  // sum over the residuals anchored at the centre of (J u)_r^2, u read through
  // the view U (zero at excluded sites); summed over all sites this is
  // |J u|^2 = u . (J^T J u).  An excluded centre anchors only constants.
  template <class PV, class SV, class FV>
  __device__ __forceinline__ T jsq(PV U, SV S, FV F, int, int) const {
    const uint32_t f0 = F(0, 0);
    const T c = S(0, 0, 0), sn = S(1, 0, 0), Ux = S(2, 0, 0), Uy = S(3, 0, 0);
    const T ux = U(0, 0, 0), uy = U(1, 0, 0), ut = U(2, 0, 0);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = (F(di, dj) & ACTIVE) ? T(1) : T(0);
      const T dx = Ux - S(2, di, dj), dy = Uy - S(3, di, dj);
      const T apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
      const T jx = (ux - U(0, di, dj)) - apx * ut, jy = (uy - U(1, di, dj)) - apy * ut;
      acc += w * (jx * jx + jy * jy);
    }
    const T wfit = (f0 & FIT) ? wf * wf : T(0);
    acc = fma(wr * wr, acc, wfit * (ux * ux + uy * uy));
    return (f0 & ACTIVE) ? acc : T(0);
  }

  // Streaming apply (the fused kernel walks rows in order).  Each regulariser
  // residual (J P)_r / w_reg is formed once, by its anchor, and handed to the
  // other end of its edge: across lanes by a lane shift, and from one row step
  // to the next through a Carry.  The sums are those of apply, term for term.
  struct Res {
    T jx, jy;  // (P_a - P_b) - a_a P^t_a, anchored at a toward b
    T ax, ay;  // a_a = R'(t_a)(U_a - U_b)
  };
  __device__ __forceinline__ static Res own_res(T c, T sn, T dx, T dy, T pax, T pay, T pat, T pbx, T pby) {
    Res r;
    r.ax = -sn * dx - c * dy;
    r.ay = c * dx - sn * dy;
    r.jx = (pax - pbx) - r.ax * pat;
    r.jy = (pay - pby) - r.ay * pat;
    return r;
  }
  // The two residuals of the edge between a row A and the row B after it in
  // the walk: A's toward B (with A's a) and B's toward A (with B's a).
  struct Carry {
    Res a, b;
  };
  template <class Row>
  __device__ __forceinline__ Carry edge_next(const Row& A, const Row& B) const {
    const T dx = A.st[2] - B.st[2], dy = A.st[3] - B.st[3];
    Carry e;
    e.a = own_res(A.st[0], A.st[1], dx, dy, A.p[0], A.p[1], A.p[2], B.p[0], B.p[1]);
    e.b = own_res(B.st[0], B.st[1], -dx, -dy, B.p[0], B.p[1], B.p[2], A.p[0], A.p[1]);
    return e;
  }
  // g = J^T J P at the centre row, from its horizontal edges (formed here; the
  // neighbours' halves arrive through Hs(v, di), the value v of lane +di) and
  // its vertical edges: prev (previous row in the walk, dj = -1 in the views)
  // and next (dj = +1).  Fills the edge geometry for jsq_c.
  template <class PV, class SV, class FV, class AV, class HS>
  __device__ __forceinline__ void apply_stream(PV P, SV S, FV F, AV A, HS Hs, const Carry& prev,
                                               const Carry& next, T* g, JCache& jc) const {
    const T c = S(0, 0, 0), sn = S(1, 0, 0), Ux = S(2, 0, 0), Uy = S(3, 0, 0);
    const T px = P(0, 0, 0), py = P(1, 0, 0), pt = P(2, 0, 0);
    const Res rp = own_res(c, sn, Ux - S(2, 1, 0), Uy - S(3, 1, 0), px, py, pt, P(0, 1, 0), P(1, 1, 0));
    const Res rm = own_res(c, sn, Ux - S(2, -1, 0), Uy - S(3, -1, 0), px, py, pt, P(0, -1, 0), P(1, -1, 0));
    // neighbour +x holds its residual toward -x (this site), and the reverse
    const T bpx = Hs(rm.jx, 1), bpy = Hs(rm.jy, 1);
    const T bmx = Hs(rp.jx, -1), bmy = Hs(rp.jy, -1);
    const Res own[4] = {rp, rm, next.a, prev.b};
    const T bx[4] = {bpx, bmx, next.b.jx, prev.a.jx};
    const T by[4] = {bpy, bmy, next.b.jy, prev.a.jy};
    T gx = 0, gy = 0, gt = 0;
    const T wr2 = wr * wr;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = wr2 * A(di, dj);
      gx += w * (own[k].jx - bx[k]);
      gy += w * (own[k].jy - by[k]);
      gt -= w * (own[k].ax * own[k].jx + own[k].ay * own[k].jy);
      jc.ax[k] = own[k].ax;
      jc.ay[k] = own[k].ay;
    }
    const T wfit = (F(0, 0) & FIT) ? wf * wf : T(0);
    g[0] = fma(wfit, px, gx);
    g[1] = fma(wfit, py, gy);
    g[2] = gt;
  }

  // diag as above, with the neighbours' activity as weights A (1 or 0).
  template <class SV, class FV, class AV>
  __device__ __forceinline__ void diag_stream(SV S, FV F, AV A, T* d) const {
    const T Ux = S(2, 0, 0), Uy = S(3, 0, 0);
    const T wr2 = wr * wr;
    T nact = 0, dt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = A(di, dj);
      const T dx = Ux - S(2, di, dj), dy = Uy - S(3, di, dj);
      nact += w;
      dt += w * (dx * dx + dy * dy);
    }
    const T dO = T(2) * wr2 * nact + ((F(0, 0) & FIT) ? wf * wf : T(0));
    d[0] = dO;
    d[1] = dO;
    d[2] = wr2 * dt;
  }

  // jsq from the edge geometry that apply_c left for this centre: only the
  // vector (through U), the centre's flags and the activity weights are read.
  template <class PV, class FV, class AV>
  __device__ __forceinline__ T jsq_c(PV U, FV F, AV A, const JCache& jc) const {
    const uint32_t f0 = F(0, 0);
    const T ux = U(0, 0, 0), uy = U(1, 0, 0), ut = U(2, 0, 0);
    T acc = (f0 & FIT) ? wf * wf * (ux * ux + uy * uy) : T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k == 0 ? 1 : (k == 1 ? -1 : 0), dj = k == 2 ? 1 : (k == 3 ? -1 : 0);
      const T w = wr * wr * A(di, dj);
      const T jx = (ux - U(0, di, dj)) - jc.ax[k] * ut, jy = (uy - U(1, di, dj)) - jc.ay[k] * ut;
      acc = fma(w, jx * jx + jy * jy, acc);
    }
    return (f0 & ACTIVE) ? acc : T(0);
  }

  // LM model term of the residuals anchored at s, in FP64:
  //   sum_r (J d)_r (2 F_r + (J d)_r), J and F at X, step Dl.
  template <class XA, class DA>
  __device__ __forceinline__ double model(XA X, DA Dl, int s) const {
    const int i = s % W, j = s / W;
    const bool ap = mask[s] == 0;
    double acc = 0.0;
    const double Ox = X(0, s), Oy = X(1, s);
    const double dOx = Dl(0, s), dOy = Dl(1, s);
    if (ap) {
      double sn, c;
      sincos_t(X(2, s), &sn, &c);
      const double dt = Dl(2, s);
      const double Ux = U[s], Uy = U[n + s];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = nbr(i, j, s, k);
        if (q < 0 || mask[q] != 0) continue;
        const double dx = Ux - (double)U[q], dy = Uy - (double)U[n + q];
        const double fx = wr_d * ((Ox - X(0, q)) - (c * dx - sn * dy));
        const double fy = wr_d * ((Oy - X(1, q)) - (sn * dx + c * dy));
        const double apx = -sn * dx - c * dy, apy = c * dx - sn * dy;
        const double jx = wr_d * ((dOx - Dl(0, q)) - apx * dt);
        const double jy = wr_d * ((dOy - Dl(1, q)) - apy * dt);
        acc += jx * (2.0 * fx + jx) + jy * (2.0 * fy + jy);
      }
    }
    const double cx = Ct[s], cy = Ct[n + s];
    if (cx >= 0.0 && cy >= 0.0) {
      const double fx = wf_d * (Ox - cx), fy = wf_d * (Oy - cy);
      const double jx = wf_d * dOx, jy = wf_d * dOy;
      acc += jx * (2.0 * fx + jx) + jy * (2.0 * fy + jy);
    }
    return acc;
  }
};

}  // namespace optmi
