// CPU check of the graph lists the library builds on the host (graph_lists.h),
// meant to run under AddressSanitizer and UndefinedBehaviorSanitizer.  For each
// graph it rebuilds every list by brute force and compares:
//  * the CSR: vertex v lists, in edge-list order, the other end of each edge at v;
//  * the split form's staging: each chunk's halo (outside neighbours in order of
//    first reference, at most cap), and every incidence entry's slot names its
//    neighbour (inside the chunk, a staged halo vertex, or -(u + 1));
//  * the fused form's rows (when they fit): R1 and R2 are exactly the one- and
//    two-ring, every slot of C's and R1's lists names the right vertex, R1's
//    lists keep incidence order, and the caps hold; when they do not fit, a cap
//    is indeed passed.
// Graphs: random (several densities), a hub, chains and grids, self-loops,
// repeated edges, no edges, and edge files given on the command line ([V, E,
// then E pairs] as int32).  An edge naming a missing vertex must be refused.
//   usage: graph_lists_harness <seed> [edge files...]
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "graph_lists.h"

using namespace optmi;
using namespace optmi::lists;

#define CHECK(c, ...)                                 \
  do {                                                \
    if (!(c)) {                                       \
      std::printf("FAIL line %d: ", __LINE__);        \
      std::printf(__VA_ARGS__);                       \
      std::printf("\n");                              \
      std::exit(1);                                   \
    }                                                 \
  } while (0)

static int n_fused = 0, n_split_only = 0;

static void check_graph(int V, const std::vector<int>& edges, int cap, const char* name) {
  const int E = (int)edges.size() / 2;
  for (bool gfz : {false, true}) {
    const GraphShape g{V, E, cap, gfz};
    // one guard word past the end: the builders must not touch it
    std::vector<int> w(words(g) + 1, 0x5a5a5a5a);
    bool ok = false;
    CHECK(build(g, edges.data(), w.data(), &ok) == -1, "%s: valid edges refused", name);
    CHECK(w.back() == 0x5a5a5a5a, "%s: wrote past the end", name);
    const int* rp = w.data();
    const int* nb = rp + V + 1;
    const int* nbl = nb + 2 * (size_t)E;
    const int nch = (V + kBlock - 1) / kBlock;
    const int* hcnt = nbl + 2 * (size_t)E;
    const int* hid = hcnt + nch;
    const int* rows = hid + (size_t)nch * cap;
    // CSR
    std::vector<std::vector<int>> adj((size_t)V);
    for (int e = 0; e < E; ++e) {
      adj[(size_t)edges[2 * e]].push_back(edges[2 * e + 1]);
      adj[(size_t)edges[2 * e + 1]].push_back(edges[2 * e]);
    }
    CHECK(rp[0] == 0 && rp[V] == 2 * E, "%s: CSR ends", name);
    for (int v = 0; v < V; ++v) {
      CHECK(rp[v + 1] - rp[v] == (int)adj[(size_t)v].size(), "%s: degree of %d", name, v);
      for (int k = 0; k < (int)adj[(size_t)v].size(); ++k)
        CHECK(nb[rp[v] + k] == adj[(size_t)v][(size_t)k], "%s: neighbour %d of %d", name, k, v);
    }
    // split form staging
    for (int c = 0; c < nch; ++c) {
      const int v0 = c * kBlock, v1 = std::min(V, v0 + kBlock);
      std::vector<int> halo;
      std::set<int> seen;
      for (int v = v0; v < v1; ++v)
        for (int u : adj[(size_t)v])
          if ((u < v0 || u >= v1) && seen.insert(u).second) halo.push_back(u);
      const int nh = std::min((int)halo.size(), cap);
      CHECK(hcnt[c] == nh, "%s: chunk %d halo count %d, want %d", name, c, hcnt[c], nh);
      for (int j = 0; j < nh; ++j) CHECK(hid[(size_t)c * cap + j] == halo[(size_t)j], "%s: halo id", name);
      for (int v = v0; v < v1; ++v)
        for (int k = rp[v]; k < rp[v + 1]; ++k) {
          const int s = nbl[k], u = nb[k];
          if (s < 0) {
            CHECK(-(s + 1) == u, "%s: unstaged slot", name);
            int idx = -1;
            for (int j = 0; j < (int)halo.size(); ++j)
              if (halo[(size_t)j] == u) idx = j;
            CHECK(idx >= cap, "%s: a staged vertex read from global memory", name);
          } else if (s < kBlock) {
            CHECK(v0 + s == u, "%s: chunk slot", name);
          } else {
            CHECK(s - kBlock < nh && hid[(size_t)c * cap + s - kBlock] == u, "%s: halo slot", name);
          }
        }
    }
    if (!gfz) continue;
    // fused form rows: rebuild the rings and check (or check that a cap is passed)
    bool fits = true;
    for (int c = 0; c < nch; ++c) {
      const int v0 = c * kBlock, v1 = std::min(V, v0 + kBlock);
      std::vector<int> r1, r2;
      std::set<int> in;
      for (int v = v0; v < v1; ++v)
        for (int u : adj[(size_t)v])
          if ((u < v0 || u >= v1) && in.insert(u).second) r1.push_back(u);
      for (int x : r1)
        for (int u : adj[(size_t)x])
          if ((u < v0 || u >= v1) && in.insert(u).second) r2.push_back(u);
      int ne1 = 0;
      for (int x : r1) ne1 += (int)adj[(size_t)x].size();
      fits = fits && rp[v1] - rp[v0] <= kGfCs && (int)r1.size() <= kGfR1 && (int)r2.size() <= kGfR2 &&
             ne1 <= kGfRs;
      if (!fits || !ok) continue;
      const int* row = rows + (size_t)c * kGfRow;
      const int n1 = row[0], n2 = row[1];
      CHECK(n1 == (int)r1.size() && n2 == (int)r2.size() && row[2] == ne1, "%s: ring sizes", name);
      std::map<int, int> slot_of;
      for (int j = 0; j < n1 + n2; ++j) {
        const int id = row[kGfIds + j];
        CHECK(id == (j < n1 ? r1[(size_t)j] : r2[(size_t)(j - n1)]), "%s: ring order", name);
        slot_of[id] = kBlock + j;
      }
      for (int j = n1 + n2; j < kGfR1 + kGfR2; ++j) CHECK(row[kGfIds + j] == 0, "%s: unused ids not 0", name);
      auto vert = [&](int s) { return s < kBlock ? v0 + s : row[kGfIds + s - kBlock]; };
      const uint16_t* cs = (const uint16_t*)(row + kGfCsI);
      for (int k = rp[v0]; k < rp[v1]; ++k) {
        const int s = cs[k - rp[v0]];
        CHECK(s < kBlock + n1 && vert(s) == nb[k], "%s: C slot", name);
        CHECK(s >= kBlock || v0 + s < V, "%s: C slot past the graph", name);
      }
      const uint16_t* r1s = (const uint16_t*)(row + kGfRsI);
      const uint16_t* r1o = (const uint16_t*)(row + kGfRoI);
      CHECK(r1o[0] == 0 && r1o[n1] == ne1, "%s: R1 offsets", name);
      for (int j = 0; j < n1; ++j) {
        const int x = r1[(size_t)j];
        CHECK(r1o[j + 1] - r1o[j] == (int)adj[(size_t)x].size(), "%s: R1 degree", name);
        for (int q = 0; q < (int)adj[(size_t)x].size(); ++q) {
          const int s = r1s[r1o[j] + q];
          CHECK(s < kBlock + n1 + n2 && vert(s) == adj[(size_t)x][(size_t)q], "%s: R1 slot", name);
        }
      }
    }
    CHECK(ok == fits, "%s: fused lists %s but the caps %s", name, ok ? "built" : "refused", fits ? "hold" : "fail");
    (ok ? n_fused : n_split_only)++;
  }
  // an edge naming a vertex outside [0, V) is refused, and nothing past the array is touched
  if (V > 0) {
    std::vector<int> bad = edges;
    bad.push_back(0);
    bad.push_back(V);
    const GraphShape g{V, E + 1, cap, true};
    std::vector<int> w(words(g), 0);
    bool ok = true;
    CHECK(build(g, bad.data(), w.data(), &ok) == E, "%s: bad edge not reported", name);
    CHECK(!ok, "%s: fused lists from a refused edge list", name);
  }
}

static std::vector<int> grid_edges(int W, int H) {
  std::vector<int> e;
  for (int j = 0; j < H; ++j)
    for (int i = 0; i + 1 < W; ++i) e.insert(e.end(), {j * W + i, j * W + i + 1});
  for (int j = 0; j + 1 < H; ++j)
    for (int i = 0; i < W; ++i) e.insert(e.end(), {j * W + i, (j + 1) * W + i});
  return e;
}

int main(int argc, char** argv) {
  std::mt19937 rng(argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u);
  const int caps[] = {0, 64, 256};
  for (int cap : caps) {
    check_graph(1, {}, cap, "single vertex");
    check_graph(300, {}, cap, "no edges");
    check_graph(5, {0, 0, 1, 1, 2, 3, 2, 3, 2, 3}, cap, "loops and repeats");
    std::vector<int> hub;
    for (int k = 1; k < 700; ++k) hub.insert(hub.end(), {0, 3 * k % 700});
    check_graph(700, hub, cap, "hub");
    check_graph(64 * 40, grid_edges(64, 40), cap, "grid 64x40");
    check_graph(1000 * 3, grid_edges(1000, 3), cap, "grid 1000x3");
    for (int t = 0; t < 6; ++t) {
      const int V = 1 + (int)(rng() % 3000), E = (int)(rng() % (4 * V));
      std::vector<int> e;
      for (int k = 0; k < 2 * E; ++k) e.push_back((int)(rng() % (unsigned)V));
      check_graph(V, e, cap, "random");
      // locally connected: neighbours within a window, so rings are small
      std::vector<int> l;
      for (int v = 0; v < V; ++v)
        for (int k = 0; k < 3; ++k) l.insert(l.end(), {v, std::min(V - 1, v + 1 + (int)(rng() % 40))});
      check_graph(V, l, cap, "local");
    }
  }
  for (int a = 2; a < argc; ++a) {
    FILE* f = std::fopen(argv[a], "rb");
    CHECK(f, "cannot open %s", argv[a]);
    int V = 0, E = 0;
    CHECK(std::fread(&V, 4, 1, f) == 1 && std::fread(&E, 4, 1, f) == 1, "header of %s", argv[a]);
    std::vector<int> e(2 * (size_t)E);
    CHECK(std::fread(e.data(), 4, e.size(), f) == e.size(), "edges of %s", argv[a]);
    std::fclose(f);
    check_graph(V, e, 256, argv[a]);
  }
  std::printf("ok: %d graph builds with fused rows, %d past a cap\n", n_fused, n_split_only);
  return 0;
}
