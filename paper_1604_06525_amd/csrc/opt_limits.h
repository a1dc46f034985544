// Launch geometry and the sizes of the graph staging lists: plain constants
// shared by the device code and the host-side list builders (graph_lists.h).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace optmi {

constexpr int kBlock = 256;      // threads per block (4 waves of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 1024; // cap on the grid of every site kernel; also the
                                 // length of each partial-sum buffer

// Graph domain: the vertices are cut into chunks of kBlock consecutive ids, and
// for each chunk up to halo_cap distinct outside neighbours are listed so that
// pcg_a can stage them in LDS next to the chunk itself.  The cap fills an LDS
// budget (30 KiB for FP32, 45 KiB for FP64) with the chunk and its halo at
// `width` values per vertex (p plus the energy's staged values), a multiple of 32.
// Width 0: the energy is not staged and no halo is listed.
constexpr int halo_cap(size_t tsize, int width) {
  const int h = width > 0 ? (tsize > 4 ? 46080 : 30720) / (width * (int)tsize) - kBlock : 0;
  return h < 0 ? 0 : h / 32 * 32;
}
// ... and up to this many of the chunk's neighbour slots are staged as well.
constexpr int nbl_cap(size_t tsize) { return tsize > 4 ? 1024 : 1536; }

// The fused graph PCG kernel stages, per chunk C of kBlock vertices, the chunk,
// its one-ring R1 (outside vertices adjacent to C) and its two-ring R2 (vertices
// adjacent to R1 outside C and R1), and needs the incidence lists of C and R1 in
// chunk-local slots: caps on |R1|, |R2|, C's incidence entries and R1's.  A
// graph with any chunk past a cap runs the split form.  A chunk's row of lists
// holds kGfRow ints: [|R1|, |R2|, R1 entries, 0], the R1 then R2 vertex ids
// (kGfR1 + kGfR2 ints), then three blocks of 16-bit slots, each 16-byte aligned
// and read whole: C's incidence entries (kGfCs), R1's (kGfRs) and R1's list
// offsets (kGfR1 + 2, padded).  Slots: 0..kBlock-1 for C, kBlock + i for R1
// vertex i, kBlock + |R1| + i for R2 vertex i.
constexpr int kGfR1 = 256, kGfR2 = 320, kGfCs = 2048, kGfRs = 2048;
constexpr int kGfIds = 4;                                          // ints before the ids
constexpr int kGfCsI = (kGfIds + kGfR1 + kGfR2 + 3) / 4 * 4;       // int offset of C's slots
constexpr int kGfRsI = kGfCsI + kGfCs / 2;                         // ... of R1's slots
constexpr int kGfRoI = kGfRsI + kGfRs / 2;                         // ... of R1's offsets
constexpr int kGfRoN = ((kGfR1 + 2) / 2 + 3) / 4;                  // 16-byte blocks of the offsets
constexpr int kGfRow = kGfRoI + 4 * kGfRoN;
static_assert(kGfCs / 8 == 256 && kGfRs / 8 == 256, "one 16-byte block of each slot list per thread");

}  // namespace optmi
