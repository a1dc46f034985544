// The fused PCG iteration on a graph: one kernel per iteration, the same
// single-reduction recurrence (Chronopoulos and Gear) as the grid kernels.
//
// Iteration i needs, at every vertex v of the problem,
//   p_i = u_i + beta_i p_{i-1},   s_i = (J^T J + lambda D) p_i,
//   u_{i+1} = u_i - alpha_i M^-1 s_i,   d += alpha_i p_i,
// and the partial sums of gamma_{i+1} = sum M u_{i+1}^2 and of
// delta_{i+1} = |J u_{i+1}|^2 + u_{i+1}.(lambda D) u_{i+1}.  |J u|^2 at v reads
// u_{i+1} at v's neighbours, and u_{i+1} at a neighbour reads p_i at its
// neighbours: a block that owns a chunk C of kBlock consecutive vertices
// therefore stages p_i for C, its one-ring R1 and its two-ring R2, forms s and
// u_{i+1} on C and (the components delta reads) on R1, and then delta's share
// of C.  The lists (R1 and R2 ids, the incidence of C and R1 in chunk-local
// slots) are built when the problem is created; a graph with a chunk past
// their caps runs the split form.
//
// u_{i+1} on R1 is recomputed by the neighbouring chunk with the same
// operations its owner uses (the energy's edge term is shared by gapply and
// gapply_h), so delta is the one of the stored u_{i+1}, bit for bit.
//
// Per chunk, three phases separated by barriers:
//   1. each thread loads its vertex of C (u_i, p_{i-1}, flags, state and d)
//      and the outside vertices t, t + kBlock, ... of R1 and R2, forms p_i and
//      the energy's record (kRec values) of each into LDS;
//   2. s, the diagonal M and u_{i+1} on its vertex of C (all components) and on
//      R1 vertex t (the kHalo components delta reads); the C vertex's p_i,
//      u_{i+1} and d are final and stored here.  The diagonal is formed from
//      the staged records with init's arithmetic (the bits init stored, which
//      are not read);
//   3. its vertex's share of |J u_{i+1}|^2 (energy gjsq).
// The energy provides: kGraphFused, kRec, kHalo (a record starts with p's first
// kHalo components), GOwn gown(v), grec(own, p, rec), gapply_d (the full
// product and the diagonal), gapply_h (the first kHalo components of both) and
// gjsq; the diagonals have the bits init stores.
#pragma once
#include "kernels.h"

namespace optmi {

template <class E, class = void>
struct GraphFusedOf : std::false_type {};
template <class E>
struct GraphFusedOf<E, std::void_t<decltype(E::kGraphFused)>> : std::bool_constant<E::kGraphFused> {};

// The graph's per-chunk lists (layout: opt_limits.h, kGfRow).
struct GraphLists {
  const int* __restrict__ rows;  // [chunks][kGfRow]
};

typedef int GfInt4 __attribute__((ext_vector_type(4)));

template <class E, bool DAMP>
struct GraphFusedArgs {
  E e;
  FusedBufs<typename E::Real> b;
  GraphLists gl;
  Precond<typename E::Real> pc;
  int n_part;  // blocks of this problem
  DevScalars* S;
  int lm_gate;
  int L;
};

// LDS of one block: the staged records (structure of arrays), u_{i+1}'s halo
// components on C and R1, and the chunk's lists.
template <typename T, int NR, int NH>
struct GraphFusedLds {
  static constexpr int kSlots = kBlock + kGfR1 + kGfR2;
  T rec[NR][kSlots];
  T uh[NH][kBlock + kGfR1];
  // the chunk's 16-bit slot lists, stored as the row's 16-byte blocks
  GfInt4 cs[kGfCs / 8];
  GfInt4 r1s[kGfRs / 8];
  GfInt4 r1o[kGfRoN];
};

template <class E, bool DAMP>
__device__ __forceinline__ void run(const GraphFusedArgs<E, DAMP>& a, VG g, int iter) {
  using T = typename E::Real;
  constexpr int C = E::C, NR = E::kRec, NH = E::kHalo;
  static_assert(NH <= C && NH <= NR, "a record starts with the halo components of p");
  __shared__ GraphFusedLds<T, NR, NH> sm;
  const E& e = a.e;
  DevScalars* S = a.S;
  if (iter >= a.L) return;
  const bool read_pold = iter > 0, write_out = iter >= 0;
  // d is updated every second iteration (as in the grid kernels): an odd
  // iteration adds alpha_{i-1} p_{i-1} and alpha_i p_i, an even one only the
  // last time.
  const bool xupd = write_out && ((iter & 1) || iter == a.L - 1);
  const bool xtwo = xupd && (iter & 1);
  const int n = e.n, nch = (n + kBlock - 1) / kBlock;
  // every array through a global pointer (see gmem)
  const auto* __restrict__ uin = gmem(pick(a.b.u, iter < 0 ? 0 : (iter & 1)));
  const auto* __restrict__ pin = gmem(pick(a.b.p, (iter + 1) & 1));
  auto* __restrict__ uout = gmem(pick(a.b.u, (iter + 1) & 1));
  auto* __restrict__ pout = gmem(pick(a.b.p, iter & 1));
  auto* __restrict__ x = gmem(a.b.x);
  const auto* __restrict__ flags = gmem(e.flags);
  const auto* __restrict__ rp = gmem(e.rp);
  const auto* __restrict__ rows = gmem(a.gl.rows);

  // scalars of earlier launches (S->stopped: 1 + the iteration that stopped)
  const int stopped_at = S->stopped;
  const int lm_done = a.lm_gate ? S->done : 0;
  const double gam_old = iter > 0 ? S->gam[(iter - 1) & 1] : 1.0;
  const double alpha_old = iter > 0 ? S->alpha[(iter - 1) & 1] : 1.0;
  const double lam_now = a.lm_gate ? S->lambda : 0.0;
  if ((stopped_at != 0 && stopped_at != iter + 1) || lm_done) return;
  const int t = threadIdx.x;
  // What a thread loads for one chunk, issued while the chunk before it is
  // computed: its vertex of C and the chunk's lists (stage A) and the data of
  // its outside slot t (stage B), whose id was loaded one chunk earlier still,
  // so that both stages go out together.  Outside slots t + kBlock, ... (rings
  // past kBlock vertices) are loaded when the chunk is staged, from ids loaded
  // with stage A.  A row's unused id entries are 0, so a stage-B load past the
  // rings reads vertex 0 and is not used.
  struct Pre {
    int n1, n2;     // ring sizes of the chunk
    int kb, r0, r1; // CSR offsets: the chunk's first vertex, this vertex and the next
    uint8_t fl;
    T u[C], po[C], xv[C];
    typename E::GRaw raw;
    int id0, id1;
    uint32_t f0;
    T u0[C], p0[C];
    typename E::GRaw raw0;
    GfInt4 cs, r1s, r1o;  // 16-byte blocks t of the row's slot lists
  };
  auto id_of = [&](int chunk, int j) { return rows[(size_t)chunk * kGfRow + kGfIds + j]; };
  // p_{i-1} and d are read from u_i's addresses when they are not needed (no
  // extra HBM traffic; the values are not used).
  const auto* __restrict__ pin_l = read_pold ? pin : uin;
  const auto* __restrict__ x_l = xupd ? x : uin;
  // Both stages are free of branches and of arithmetic on what they load: a
  // value used (or a path merged) while loads are in flight waits for all of
  // them.  A thread past the graph's end reads the chunk's first vertex (its
  // values are not used), p_{i-1} and d are read whether or not they are
  // needed (selected where they are used), and the raw CSR offsets are kept.
  auto load_a = [&](int chunk, Pre& P) {
    const int v0 = chunk * kBlock, v = v0 + t;
    const int vl = v < n ? v : v0;
    const auto* __restrict__ row = rows + (size_t)chunk * kGfRow;
    P.id1 = row[kGfIds + kBlock + t];
    P.n1 = row[0];
    P.n2 = row[1];
    P.kb = rp[v0];
    P.r0 = rp[vl];
    P.r1 = rp[vl + 1];
    P.fl = flags[vl];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = vix<C>(c, vl);
      P.u[c] = uin[o];
      P.po[c] = pin_l[o];
      P.xv[c] = x_l[o];
    }
    P.raw = e.graw(vl);
    using G4 = const __attribute__((address_space(1))) GfInt4;
    P.cs = ((G4*)(row + kGfCsI))[t];
    P.r1s = ((G4*)(row + kGfRsI))[t];
    P.r1o = ((G4*)(row + kGfRoI))[t < kGfRoN ? t : kGfRoN - 1];
  };
  auto load_b = [&](Pre& P) {
    const int id = P.id0;
    P.f0 = flags[id];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const size_t o = vix<C>(c, id);
      P.u0[c] = uin[o];
      P.p0[c] = pin_l[o];
    }
    P.raw0 = e.graw(id);
  };
  // The first chunk's loads do not depend on alpha and beta: they go out
  // before the previous launch's partial sums are reduced.
  // (Chunk numbers past the last are read as the last chunk, whose loads are
  // then not used: a graph has at least one vertex, so nch >= 1.)
  const int first = unit_of_block(g);
  const int last = nch - 1;
  Pre P;
  P.id0 = id_of(min(first, last), t);
  load_a(min(first, last), P);
  load_b(P);
  int id_next = id_of(min(first + g.nb, last), t);  // outside slot t of the chunk after P's
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
      if (iter & 1) {
        // the update alpha_{i-1} p_{i-1} deferred from the previous iteration
        const T ap = (T)alpha_prev;
        for (int chunk = unit_of_block(g); chunk < nch; chunk += g.nb) {
          const int v = chunk * kBlock + (int)threadIdx.x;
          if (v >= n || !(flags[v] & E::ACTIVE)) continue;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const size_t o = vix<C>(c, v);
            x[o] = fma(ap, pin[o], x[o]);
          }
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
  // the preconditioner entry M and its inverse, and the damping, of an
  // unknown with diagonal dg (as Precond gives them; lambda is 0 for GN)
  auto precond = [&](T dg, T* m, T* mi, T* dmp) {
    *dmp = (DAMP && pc.lam != T(0)) ? pc.damp(dg) : T(0);
    *m = DAMP ? pc.den(dg) : (pc.use ? dg : T(1));
    const T rm = recip(*m);
    *mi = pc.use ? (*m > T(0) ? rm : T(0)) : T(1);
  };
  auto R = [&](int s, int k) -> T { return sm.rec[k][s]; };
  auto UH = [&](int s, int c) -> T { return sm.uh[c][s]; };
  double g_acc = 0.0, d_acc = 0.0;

  // p and the record of an outside vertex into slot kBlock + j
  auto stage_out = [&](int j, uint32_t f, const T* u, const T* pold, const typename E::GRaw& raw) {
    T pj[C], r[NR];
#pragma unroll
    for (int c = 0; c < C; ++c) pj[c] = (f & E::ACTIVE) ? fma(bT, pold[c], u[c]) : T(0);
    e.grec(e.gown_of(raw), pj, r);
#pragma unroll
    for (int k = 0; k < NR; ++k) sm.rec[k][kBlock + j] = r[k];
  };

  int chunk = first;
  for (; chunk < nch; chunk += g.nb) {
    const int v0 = chunk * kBlock, v = v0 + t;
    const bool in = v < n;
    const auto* __restrict__ row = rows + (size_t)chunk * kGfRow;
    const int n1 = P.n1, n2 = P.n2;
    // ---- phase 1: records and lists into LDS
    T uw[NH];  // u_i of R1 vertex t
    uint32_t flw = 0;
    if (t < n1 + n2) {
      T p0[C];
#pragma unroll
      for (int c = 0; c < C; ++c) p0[c] = read_pold ? P.p0[c] : T(0);
      stage_out(t, P.f0, P.u0, p0, P.raw0);
      if (t < n1) {
        flw = P.f0;
#pragma unroll
        for (int c = 0; c < NH; ++c) uw[c] = P.u0[c];
      }
    }
    for (int j = t + kBlock; j < n1 + n2; j += kBlock) {
      const int id = j < 2 * kBlock ? P.id1 : row[kGfIds + j];
      const uint32_t f = flags[id];
      T u[C], pold[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = vix<C>(c, id);
        u[c] = uin[o];
        pold[c] = read_pold ? pin[o] : T(0);
      }
      stage_out(j, f, u, pold, e.graw(id));
    }
    sm.cs[t] = P.cs;
    sm.r1s[t] = P.r1s;
    if (t < kGfRoN) sm.r1o[t] = P.r1o;
    // the chunk's own vertex, out of the prefetch registers
    const int k0 = in ? P.r0 - P.kb : 0, k1 = in ? P.r1 - P.kb : 0;
    const uint32_t fl = in ? (uint32_t)P.fl : 0u;
    const bool act = in && (fl & E::ACTIVE);
    T uv[C], po[C], xv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      uv[c] = P.u[c];
      po[c] = read_pold ? P.po[c] : T(0);
      xv[c] = xupd ? P.xv[c] : T(0);
    }
    typename E::GOwn own{};
    if (in) own = e.gown_of(P.raw);
    T p[C], rv[NR];
#pragma unroll
    for (int c = 0; c < C; ++c) p[c] = act ? fma(bT, po[c], uv[c]) : T(0);
    if (in) {
      e.grec(own, p, rv);
#pragma unroll
      for (int k = 0; k < NR; ++k) sm.rec[k][t] = rv[k];
    }
    __syncthreads();
    // the next chunk's loads go out now, to arrive while this one computes
    const int next = chunk + g.nb;
    if (next < nch) {
      P.id0 = id_next;
      load_a(next, P);
      load_b(P);
      id_next = id_of(min(next + g.nb, last), t);
    }
    // ---- phase 2: s, M, u_{i+1} on C (all components) and on R1 (halo)
    // (vector types may alias any other type, so reading the blocks as 16-bit
    // entries is defined)
    const uint16_t* cs16 = (const uint16_t*)sm.cs;
    const uint16_t* r1s16 = (const uint16_t*)sm.r1s;
    const uint16_t* r1o16 = (const uint16_t*)sm.r1o;
    auto NBc = [&](int k) -> int { return cs16[k]; };
    T un[C];
    {
      T sv[C], dg[C];
      if (act) {
        e.gapply_d(own, p, rv, t, R, NBc, k0, k1, fl, sv, dg);
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) sv[c] = dg[c] = T(0);
      }
      T gs = T(0), dd = T(0);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        T m, mi, dmp;
        precond(dg[c], &m, &mi, &dmp);
        const T s = DAMP ? fma(dmp, p[c], sv[c]) : sv[c];
        un[c] = act ? fma(-aT, mi * s, uv[c]) : T(0);
        gs = fma(m * un[c], un[c], gs);
        if constexpr (DAMP) dd = fma(dmp * un[c], un[c], dd);
      }
      if (act) g_acc += (double)gs;
      if constexpr (DAMP) {
        if (act && (fl & E::INGRID)) d_acc += (double)dd;
      }
      if (in) {
#pragma unroll
        for (int c = 0; c < NH; ++c) sm.uh[c][t] = un[c];
      }
    }
    if (t < n1) {
      const int sw = kBlock + t;
      const int q0 = r1o16[t], q1 = r1o16[t + 1];
      auto NBr = [&](int k) -> int { return r1s16[k]; };
      const bool actw = flw & E::ACTIVE;
      T sv[NH], dg[NH];
      if (actw) {
        e.gapply_h(sw, R, NBr, q0, q1, flw, sv, dg);
      } else {
#pragma unroll
        for (int c = 0; c < NH; ++c) sv[c] = dg[c] = T(0);
      }
#pragma unroll
      for (int c = 0; c < NH; ++c) {
        T m, mi, dmp;
        precond(dg[c], &m, &mi, &dmp);
        const T s = DAMP ? fma(dmp, R(sw, c), sv[c]) : sv[c];
        sm.uh[c][sw] = actw ? fma(-aT, mi * s, uw[c]) : T(0);
      }
    }
    if (in && write_out) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const size_t o = vix<C>(c, v);
        pout[o] = p[c];
        uout[o] = un[c];
        if (xupd && act) {
          const T xo = xtwo ? fma(apT, po[c], xv[c]) : xv[c];
          x[o] = fma(aT, p[c], xo);
        }
      }
    }
    __syncthreads();
    // ---- phase 3: the vertex's share of |J u_{i+1}|^2
    if (in && (fl & E::INGRID)) d_acc += (double)e.gjsq(own, un, R, UH, NBc, k0, k1, fl);
    __syncthreads();  // the next chunk reuses the LDS
  }
  double gs, ds;
  block_sum2(g_acc, d_acc, &gs, &ds);
  if (threadIdx.x == 0) {
    part_out[g.bid] = gs;
    part_out[kMaxBlocks + g.bid] = ds;
  }
}

// FP32 rows: at most 256 VGPRs, so that the two blocks a CU holds (LDS-bound)
// are not limited by registers.
template <class E, bool DAMP>
struct MinWavesOf<GraphFusedArgs<E, DAMP>> {
  static constexpr int value = sizeof(typename E::Real) == 4 ? 2 : 1;
};

}  // namespace optmi
