// Fused PCG iteration for shape from shading (Sec. 8.3, Fig. 26): the same
// single-reduction u-form recurrences as the generic fused kernel, for an
// operator of radius 2.
//
// J^T J p is formed residual by residual instead of site by site.  With the
// shading partials dB0, dBl, dBu of B_I(a,b) with respect to X(a,b), X(a-1,b)
// and X(a,b-1) (the per-pixel state), the J p of the shading residuals are
//   JB(a,b) = dB0(a,b) p(a,b) + dBl(a,b) p(a-1,b) + dBu(a,b) p(a,b-1)
//   gh(a,b) = eh(a,b) (JB(a,b) - JB(a+1,b)),  gv(a,b) = ev(a,b) (JB(a,b) - JB(a,b+1))
// (eh, ev: the edge masks, 0 off the band one pixel inside the border), and J^T
// gathers them back through G(a,b) = gh(a,b) - gh(a-1,b) + gv(a,b) - gv(a,b-1):
//   q(x) = w_p p(x) + w_g [dB0(x) G(x) + dBl(x+e_x) G(x+e_x) + dBu(x+e_y) G(x+e_y)]
//        + w_s sum over the 5-point stencil n of x where the smoothness residual
//          is valid of c_n (k_x(x) s0(n) + k_y(x) s1(n) + s2(n)),
// c_n = 4 at x and -1 at its neighbours, s0..s2 the three components of that
// residual's J p.  Each residual's J p is thus formed once, by its anchor, and
// reaches the other pixels it touches by lane shifts (DPP) and the row ring.
// delta = |J u|^2 is summed over the residuals anchored at each pixel.
//
// A wave owns a strip of at most 58 produced columns (3 halo lanes each side)
// and walks it downwards: step k starts row y = y0 - 3 + k, forms p and JB
// there, the vertical shading terms, G and the smoothness J p one row up, q, the
// u update and the partial of gamma two rows up (where d, u, p are stored), and
// the partial of delta three rows up.  Loads cover rows y0-3 .. y1+2; d comes
// with its row, and the start-up steps are peeled off the loop (walk_steps).
// k_y of the walk's rows is formed once per 64 rows, lane i holding that of
// step i, and read back with a lane read per step.
#pragma once
#include "energy_sfs.h"
#include "kernels.h"

namespace optmi {

constexpr int kSfsCols = 58;  // produced columns per strip

template <typename T>
struct SfsRow {
  T u, p, po, x, dg;  // u_i then u_{i+1}; p_{i-1} then p_i; p_{i-1} kept; d; diag(J^T J)
  T dB0, dBl, dBu;    // shading partials of B_I at this pixel
  uint32_t f;
  T JB, gh, gv, G;    // shading terms along p
  T s0, s1, s2;       // smoothness J p (0 where that residual is not valid)
  T JBu;              // shading derivative along u_{i+1}
  T ky;               // k_y of this row
};

template <typename T, bool DAMP>
__device__ __forceinline__ void run(const FusedArgs<ShapeFromShading<T>, DAMP>& a, VG g, int iter) {
  using E = ShapeFromShading<T>;
  using Row = SfsRow<T>;
  // rows prefetched ahead: three in FP32 (four measured 4% slower: the extra
  // ring slot's registers cost more than the deeper prefetch gains), two in FP64
  constexpr int kPrefetch = sizeof(T) > 4 ? 2 : 3;
  constexpr int N = kPrefetch + 5;  // rows y-4 .. y in use, the rest in flight
  const E& e = a.e;
  DevScalars* S = a.S;
  if (iter >= a.L) return;
  const bool write_out = iter >= 0;
  // d is updated every second iteration, as in the generic fused kernel
  const bool xupd = write_out && ((iter & 1) || iter == a.L - 1);
  const bool xtwo = xupd && (iter & 1);
  const int W = e.W, H = e.H, n = e.n, sw = a.sw;
  const int lane = threadIdx.x & 63;
  const int strip = unit_of_block(g) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool has_strip = strip < a.n_sx * a.n_sy;
  const int sy = strip / a.n_sx, sx = strip % a.n_sx;
  const int col = sx * sw - 3 + lane;
  const int y0 = sy * a.rq + min(sy, a.rr), y1 = min(y0 + a.rq + (sy < a.rr ? 1 : 0), H);
  const int ylo = max(y0 - 3, 0), yhi = min(y1 + 2, H - 1);
  const bool colin = has_strip && col >= 0 && col < W;
  const bool out_lane = colin && lane >= 3 && lane < 3 + sw;
  const int K = (y1 - y0) + 6;
  constexpr unsigned VB = sizeof(T), SB = 4 * sizeof(T);
  const size_t vbytes = (size_t)n * VB;
  const Buf<T> Buin = Buf<T>::make(pick(a.b.u, iter < 0 ? 0 : (iter & 1)), vbytes);
  const Buf<T> Bpin = Buf<T>::make(pick(a.b.p, (iter + 1) & 1), iter > 0 ? vbytes : 0);
  const Buf<T> Bx = Buf<T>::make(a.b.x, xupd ? vbytes : 0);
  const Buf<T> Buout = Buf<T>::make(pick(a.b.u, (iter + 1) & 1), write_out ? vbytes : 0);
  const Buf<T> Bpout = Buf<T>::make(pick(a.b.p, iter & 1), write_out ? vbytes : 0);
  const Buf<T> Bdg = Buf<T>::make(a.b.diag, vbytes);
  const Buf<T> Bst = Buf<T>::make(e.state_base(), (size_t)n * SB);
  const Buf<uint8_t> Bf = Buf<uint8_t>::make(e.flags, (size_t)n);
  // byte offsets: per-lane column part + scalar row part (see the generic kernel)
  const unsigned lane_v = colin ? (unsigned)col * VB : kBufOutOfRange;
  const unsigned lane_s = colin ? (unsigned)col * SB + (unsigned)sizeof(T) : kBufOutOfRange;
  const unsigned lane_f = colin ? (unsigned)col : kBufOutOfRange;
  const unsigned lane_o = out_lane ? (unsigned)col * VB : kBufOutOfRange;
  Row ring[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    Row& R = ring[k];
    R.u = R.p = R.po = R.x = R.dg = R.dB0 = R.dBl = R.dBu = T(0);
    R.f = 0;
    R.JB = R.gh = R.gv = R.G = R.s0 = R.s1 = R.s2 = R.JBu = R.ky = T(0);
  }
  auto issue = [&](Row& R, int y) {
    const bool in = y >= ylo && y <= yhi;
    const unsigned rs = (unsigned)(y * W);
    const unsigned ov = lane_v + (in ? rs * VB : kBufOutOfRange);
    T st[3];
    buf_loadv<3>(Bst, lane_s + (in ? rs * SB : kBufOutOfRange), 0, st);
    R.dB0 = st[0];
    R.dBl = st[1];
    R.dBu = st[2];
    R.f = Bf.load(lane_f + (in ? rs : kBufOutOfRange), 0);
    R.u = Buin.load(ov, 0);
    R.p = Bpin.load(ov, 0);
    R.dg = Bdg.load(ov, 0);
    // d of a produced row, when this launch updates it
    const bool prod = y >= y0 && y < y1;
    R.x = Bx.load(lane_o + ((prod && xupd) ? rs * VB : kBufOutOfRange), 0);
  };
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) issue(ring[k], y0 - 3 + k);

  const int stopped_at = S->stopped;
  const int lm_done = a.lm_gate ? S->done : 0;
  const double gam_old = iter > 0 ? S->gam[(iter - 1) & 1] : 1.0;
  const double alpha_old = iter > 0 ? S->alpha[(iter - 1) & 1] : 1.0;
  const double lam_now = a.lm_gate ? S->lambda : 0.0;
  if ((stopped_at != 0 && stopped_at != iter + 1) || lm_done) return;
  const double* part_in = pick(a.b.part, (iter + 1) & 1);
  double* part_out = pick(a.b.part, iter & 1);
  double alpha = 0.0, beta = 0.0;
  const double alpha_prev = (iter & 1) ? alpha_old : 0.0;
  if (iter >= 0) {
    double gam, del;
    reduce_partials2(part_in, part_in + kMaxBlocks, a.n_part, &gam, &del);
    double den = del;
    if (iter > 0) {
      beta = gam / gam_old;
      den = del - beta * gam / alpha_old;
    }
    if (!(den > 0.0)) {
      if (is_block_leader(g)) S->stopped = iter + 1;
      if ((iter & 1) && out_lane) {
        // the update alpha_{i-1} p_{i-1} deferred from the previous iteration
        const T ap = (T)alpha_prev;
        for (int y = y0; y < y1; ++y) {
          const unsigned s = (unsigned)(y * W + col);
          if (!(Bf.load(s, 0) & E::ACTIVE)) continue;
          const T xv = fma(ap, Bpin.load(s * VB, 0), Bx.load(s * VB, 0));
          buf_storev<1, kFusedStoreAux<T>>(Bx, s * VB, 0, &xv);
        }
      }
      return;
    }
    alpha = gam / den;
    if (is_block_leader(g)) {
      S->gam[iter & 1] = gam;
      S->alpha[iter & 1] = alpha;
    }
  }
  const T aT = (T)alpha, bT = (T)beta, apT = (T)alpha_prev;
  Precond<T> pc = a.pc;
  if (a.lm_gate) pc.lam = (T)lam_now;
  const T wp2 = e.sw_pT * e.sw_pT, wg2 = e.sw_gT * e.sw_gT, ws2 = e.sw_sT * e.sw_sT;
  // k_x of this lane's column and its neighbours' (as the energy forms them)
  const T kxc = T((col - e.ux) / e.fx), kxl = T((col - 1 - e.ux) / e.fx), kxr = T((col + 1 - e.ux) / e.fx);
  auto kyT = [&](int row) { return T((row - e.uy) / e.fy); };
  double g_acc = 0.0, d_acc = 0.0;

  if (has_strip) {
    // k_y of step k's row is lane k % 64 of kyv (refreshed every 64 steps)
    T kyv = kyT(y0 - 3 + lane);
    auto step = [&](auto PH, int k, auto steady) {
      constexpr int ph = decltype(PH)::value;
      constexpr bool st = decltype(steady)::value;
      Row& R0 = ring[ph];                // row y = y0 - 3 + k
      Row& R1 = ring[(ph + N - 1) % N];  // y - 1
      Row& R2 = ring[(ph + N - 2) % N];  // y - 2
      Row& R3 = ring[(ph + N - 3) % N];  // y - 3
      Row& R4 = ring[(ph + N - 4) % N];  // y - 4
      const int y = y0 - 3 + k;
      issue(ring[(ph + kPrefetch) % N], y + kPrefetch);
      // Each part runs only on the rows the produced rows need (uniform tests).
      // row y: p_i = u_i + beta p_{i-1} (beta is 0 and p_{i-1} reads 0 at
      // iteration 0), JB and gh (rows y0-2 .. y1+2)
      R0.po = R0.p;
      R0.p = fma(bT, R0.p, R0.u);
      if (k > 0 && (k & 63) == 0) kyv = kyT(y + lane);  // uniform
      R0.ky = lane_value(kyv, k & 63);
      if (st || k >= 1) {
        R0.JB = fma(R0.dB0, R0.p, fma(R0.dBl, from_left(R0.p), R0.dBu * R1.p));
        const uint32_t f = R0.f;
        const T eh = ((f & E::IBE) && (f & E::ER)) ? T(1) : T(0);
        R0.gh = eh * (R0.JB - from_right(R0.JB));
      }
      if (st || k >= 2) {
        // row y - 1: gv, G, smoothness J p
        const uint32_t f = R1.f;
        const T ev = ((f & E::IBE) && (f & E::EC)) ? T(1) : T(0);
        R1.gv = ev * (R1.JB - R0.JB);
        R1.G = (R1.gh - from_left(R1.gh)) + (R1.gv - R2.gv);
        const T p0 = R1.p, pl = from_left(R1.p), pr = from_right(R1.p), pu = R2.p, pd = R0.p;
        const T kyb = R1.ky, kyu = R2.ky, kyd = R0.ky;
        const bool vs = f & E::VS;
        R1.s0 = vs ? T(4) * kxc * p0 - kxl * pl - kxc * pu - kxr * pr - kxc * pd : T(0);
        R1.s1 = vs ? T(4) * kyb * p0 - kyb * pl - kyu * pu - kyb * pr - kyd * pd : T(0);
        R1.s2 = vs ? T(4) * p0 - pl - pu - pr - pd : T(0);
      }
      if (st || k >= 4) {
        // row y - 2 (rows y0-1 .. y1): q = J^T J p (+ lambda D p), u_{i+1},
        // gamma, stores
        const int y2 = y - 2;
        const T ky = R2.ky;
        const T sh = fma(R2.dB0, R2.G, fma(R1.dBu, R1.G, from_right(R2.dBl * R2.G)));
        const T sl0 = from_left(R2.s0), sr0 = from_right(R2.s0);
        const T sl1 = from_left(R2.s1), sr1 = from_right(R2.s1);
        const T sl2 = from_left(R2.s2), sr2 = from_right(R2.s2);
        const T sc = T(4) * (kxc * R2.s0 + ky * R2.s1 + R2.s2) -
                     (kxc * (sl0 + sr0 + R1.s0 + R3.s0) + ky * (sl1 + sr1 + R1.s1 + R3.s1) +
                      (sl2 + sr2 + R1.s2 + R3.s2));
        T sv = fma(wp2, R2.p, fma(wg2, sh, ws2 * sc));
        T dmp = T(0);
        if constexpr (DAMP) {
          dmp = pc.lam != T(0) ? pc.damp(R2.dg) : T(0);
          sv = fma(dmp, R2.p, sv);
        }
        const T m = DAMP ? pc.den(R2.dg) : (pc.use ? R2.dg : T(1));
        const T rm = recip(m);
        const T mi = pc.use ? (m > T(0) ? rm : T(0)) : T(1);
        const bool act = R2.f & E::ACTIVE;
        R2.u = act ? fma(-aT, mi * sv, R2.u) : T(0);
        const bool prod = y2 >= y0 && y2 < y1;  // uniform
        g_acc += (double)((out_lane && prod) ? m * R2.u * R2.u : T(0));
        if constexpr (DAMP) d_acc += (double)((out_lane && prod) ? dmp * R2.u * R2.u : T(0));
        R2.JBu = fma(R2.dB0, R2.u, fma(R2.dBl, from_left(R2.u), R2.dBu * R3.u));
        const unsigned o = lane_o + (prod ? (unsigned)(y2 * W) * VB : kBufOutOfRange);
        const unsigned ox = (act && xupd) ? o : kBufOutOfRange;
        const T pv = act ? R2.p : T(0);
        const T xo = xtwo ? fma(apT, R2.po, R2.x) : R2.x;
        const T xv = fma(aT, pv, xo);
        buf_storev<1, kFusedStoreAux<T>>(Bx, ox, 0, &xv);
        buf_storev<1, kFusedStoreAux<T>>(Buout, o, 0, &R2.u);
        buf_storev<1, kFusedStoreAux<T>>(Bpout, o, 0, &pv);
      }
      if (st || k >= 6) {
        // row y - 3 (a produced row) is final: partial of delta = |J u|^2 over
        // its residuals
        const int y3 = y - 3;
        const bool prod = y3 >= y0 && y3 < y1;  // uniform
        const uint32_t f = R3.f;
        const T eh = ((f & E::IBE) && (f & E::ER)) ? T(1) : T(0);
        const T ev = ((f & E::IBE) && (f & E::EC)) ? T(1) : T(0);
        const T ghu = eh * (R3.JBu - from_right(R3.JBu));
        const T gvu = ev * (R3.JBu - R2.JBu);
        const T u0 = R3.u, ul = from_left(R3.u), ur = from_right(R3.u), uu = R4.u, ud = R2.u;
        const T kyb = R3.ky, kyu = R4.ky, kyd = R2.ky;
        const bool vs = f & E::VS;
        const T t0 = T(4) * kxc * u0 - kxl * ul - kxc * uu - kxr * ur - kxc * ud;
        const T t1 = T(4) * kyb * u0 - kyb * ul - kyu * uu - kyb * ur - kyd * ud;
        const T t2 = T(4) * u0 - ul - uu - ur - ud;
        const T sm = vs ? fma(t0, t0, fma(t1, t1, t2 * t2)) : T(0);
        const T ds = fma(wp2, u0 * u0, fma(wg2, fma(ghu, ghu, gvu * gvu), ws2 * sm));
        d_acc += (double)((out_lane && prod) ? ds : T(0));
      }
    };
    walk_steps<N, 6, true>(K, step);
  }
  double gs, ds;
  block_sum2(g_acc, d_acc, &gs, &ds);
  if (threadIdx.x == 0) {
    part_out[g.bid] = gs;
    part_out[kMaxBlocks + g.bid] = ds;
  }
}

}  // namespace optmi
