// The graph lists the library builds on the host from an edge list, as one
// array of ints (no device code, so that a CPU test can build and check them
// under the sanitizers):
//   [row offsets (V+1) | neighbour ids (2E)]                    the CSR
//   [chunk-local slots (2E) | halo counts (chunks) | halo ids (chunks x cap)]
//                                                               the split form's staging
//   [rows (chunks x kGfRow)]                                    the fused form's rings (gfz only)
// Chunks are kBlock consecutive vertex ids.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "opt_limits.h"

namespace optmi {
namespace lists {

struct GraphShape {
  int V, E;
  int cap;   // halo ids listed per chunk (0: the energy is not staged)
  bool gfz;  // build the fused form's rows
};

inline size_t gfz_words(int V) { return ((size_t)V + kBlock - 1) / kBlock * (size_t)kGfRow; }

inline size_t words(const GraphShape& g) {
  const size_t V = (size_t)g.V, E = (size_t)g.E, nch = (V + kBlock - 1) / kBlock;
  return (V + 1) + 2 * E + 2 * E + nch + nch * (size_t)g.cap + (g.gfz ? gfz_words(g.V) : 0);
}

// The fused form's rows (layout: opt_limits.h, kGfRow).  R1 lists the chunk's
// outside neighbours in order of first reference (its vertices in id order,
// each vertex's incidence in order), R2 the neighbours of R1 outside the chunk
// and R1 in the same way; an R1 vertex's list keeps its incidence order, so its
// terms are summed as its own chunk sums them.  False if a chunk passes a cap.
inline bool build_gfz(int V, const int* rp, const int* nb, int* out) {
  const int nch = (V + kBlock - 1) / kBlock;
  int* rows = out;
  std::vector<int> mark((size_t)V, -1), slot((size_t)V, 0), ring;
  for (int c = 0; c < nch; ++c) {
    const int v0 = c * kBlock, v1 = std::min(V, v0 + kBlock);
    int* row = rows + (size_t)c * kGfRow;
    std::fill(row, row + kGfRow, 0);
    if (rp[v1] - rp[v0] > kGfCs) return false;
    ring.clear();
    auto local = [&](int u) { return u >= v0 && u < v1; };
    for (int v = v0; v < v1; ++v)
      for (int k = rp[v]; k < rp[v + 1]; ++k) {
        const int u = nb[k];
        if (local(u) || mark[(size_t)u] == c) continue;
        mark[(size_t)u] = c;
        slot[(size_t)u] = kBlock + (int)ring.size();
        ring.push_back(u);
      }
    const int n1 = (int)ring.size();
    if (n1 > kGfR1) return false;
    for (int j = 0; j < n1; ++j) {
      const int w = ring[(size_t)j];
      for (int k = rp[w]; k < rp[w + 1]; ++k) {
        const int u = nb[k];
        if (local(u) || mark[(size_t)u] == c) continue;
        mark[(size_t)u] = c;
        slot[(size_t)u] = kBlock + (int)ring.size();
        ring.push_back(u);
      }
      if ((int)ring.size() - n1 > kGfR2) return false;
    }
    const int n2 = (int)ring.size() - n1;
    auto slot_of = [&](int u) { return local(u) ? u - v0 : slot[(size_t)u]; };
    uint16_t* cs = (uint16_t*)(row + kGfCsI);
    uint16_t* r1s = (uint16_t*)(row + kGfRsI);
    uint16_t* r1o = (uint16_t*)(row + kGfRoI);
    for (int k = rp[v0]; k < rp[v1]; ++k) cs[k - rp[v0]] = (uint16_t)slot_of(nb[k]);
    int ne1 = 0;
    r1o[0] = 0;
    for (int j = 0; j < n1; ++j) {
      const int w = ring[(size_t)j];
      if (ne1 + (rp[w + 1] - rp[w]) > kGfRs) return false;
      for (int k = rp[w]; k < rp[w + 1]; ++k) r1s[ne1++] = (uint16_t)slot_of(nb[k]);
      r1o[j + 1] = (uint16_t)ne1;
    }
    row[0] = n1;
    row[1] = n2;
    row[2] = ne1;
    for (int j = 0; j < n1 + n2; ++j) row[kGfIds + j] = ring[(size_t)j];
  }
  return true;
}

// Build every list from the edge list ([E][2]).  The CSR is a stable counting
// sort: vertex v lists, in edge-list order, the other end of every edge that
// touches it, so the order of every per-vertex sum is fixed.  Returns -1, or
// the index of the first edge that names a vertex outside [0, V) (nothing is
// then built).  *gfused: the fused form's rows were built and fit their caps.
inline long long build(const GraphShape& g, const int* edges, int* out, bool* gfused) {
  *gfused = false;
  const int V = g.V, E = g.E, cap = g.cap;
  for (int e = 0; e < E; ++e) {
    const int a = edges[2 * (size_t)e], b = edges[2 * (size_t)e + 1];
    if (a < 0 || a >= V || b < 0 || b >= V) return e;
  }
  int* rp = out;
  int* nb = rp + V + 1;
  int* nbl = nb + 2 * (size_t)E;
  const int nch = (V + kBlock - 1) / kBlock;
  int* hcnt = nbl + 2 * (size_t)E;
  int* hid = hcnt + nch;
  std::fill(rp, rp + V + 1, 0);
  for (int e = 0; e < E; ++e) {
    rp[(size_t)edges[2 * (size_t)e] + 1]++;
    rp[(size_t)edges[2 * (size_t)e + 1] + 1]++;
  }
  for (int v = 0; v < V; ++v) rp[(size_t)v + 1] += rp[v];
  std::vector<int> pos(rp, rp + V);
  for (int e = 0; e < E; ++e) {
    const int a = edges[2 * (size_t)e], b = edges[2 * (size_t)e + 1];
    nb[(size_t)pos[(size_t)a]++] = b;
    nb[(size_t)pos[(size_t)b]++] = a;
  }
  // Per chunk: its outside neighbours in order of first reference, the first
  // cap of them staged.  nbl names a neighbour by its LDS slot: u - chunk start
  // inside the chunk, kBlock + halo index for a staged outside one, -(u + 1)
  // for one past the cap (read from global memory).  An energy that is not
  // staged gets cap 0 and every outside slot negative.
  std::fill(hcnt, hcnt + nch, 0);
  std::fill(hid, hid + (size_t)nch * cap, 0);
  std::vector<int> seen((size_t)V, -1), slot((size_t)V, -1);
  for (int c = 0; c < nch; ++c) {
    int nh = 0;
    for (int v = c * kBlock; v < std::min(V, (c + 1) * kBlock); ++v)
      for (int k = rp[v]; k < rp[(size_t)v + 1]; ++k) {
        const int u = nb[k];
        if (u / kBlock == c) {
          nbl[k] = u - c * kBlock;
          continue;
        }
        if (seen[(size_t)u] != c) {
          seen[(size_t)u] = c;
          slot[(size_t)u] = nh < cap ? nh : -1;
          if (nh < cap) hid[(size_t)c * cap + nh++] = u;
        }
        nbl[k] = slot[(size_t)u] >= 0 ? kBlock + slot[(size_t)u] : -(u + 1);
      }
    hcnt[c] = nh;
  }
  if (g.gfz) *gfused = build_gfz(V, rp, nb, hid + (size_t)nch * cap);
  return -1;
}

}  // namespace lists
}  // namespace optmi
