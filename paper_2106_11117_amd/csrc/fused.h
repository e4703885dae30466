// Tiling of a level for the fused step kernel (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "host.h"

namespace lts {

constexpr int kFineThreads = 1024;                  // threads per workgroup
constexpr int kNPT = 4;                             // region nodes per thread
constexpr int kRegionCap = kFineThreads * kNPT;     // nodes of one fine-tile region
constexpr int kCoarseRows = 16;                     // rows of one coarse item (4 per wavefront)
constexpr int kRectW = 64;                          // rect mode: region columns (one per lane)
constexpr int kRectH = 4 * (kFineThreads / 64);     // rect mode: region rows (4 per lane)
constexpr int kBndRows = 2 * (kFineThreads / 64) + 2;   // rect mode: boundary rows + 2 zero rows
constexpr int kBndSlots = kBndRows * 64;                 // rect mode: slots of one buffer
constexpr int kLdsSlots = 2 * kBndSlots > kRegionCap + 1 ? 2 * kBndSlots : kRegionCap + 1;
constexpr int kCompactSlots = 2 * (kRegionCap + 1);   // compact mode: two q buffers with a zero slot
constexpr int kCoarseThreads = 256;                 // coarse workgroup: one item, 4 rows per wavefront
constexpr int kMaxAdjP = 64;                        // largest p supported by the adjoint
constexpr int kMaxJobs = 32;                        // jobs of one batched launch
static_assert(kCoarseRows == 4 * (kCoarseThreads / 64), "coarse item rows = 4 per wavefront");
static_assert(kCoarseRows <= 16, "coarse row mask is 16 bits");

struct TilingHost {
  int TX = 0, TY = 0;
  int ox = 0, oy = 0;               // origin of the tile grid
  bool rect = false;                // region handled as a zero-padded rectangle (lane = column)
  int pitch = 0;                    // rect mode: LDS row pitch (slots)
  int n_fine = 0, n_coarse = 0, wg_per_sample = 0;   // wg_per_sample: fine + coarse workgroups
  double halo_ratio = 1.0;          // region lanes / F+ nodes
  double wg_work = 0.0;             // mean region nodes x substeps of one fine workgroup
  int nt = kFineThreads;            // compact mode: threads of a fine workgroup (256, 512 or 1024),
                                    // the fewest whose kNPT nodes per lane hold the largest region
  std::vector<int4> ent;            // compact mode: region entries (see lts_fused.hip)
  std::vector<int4> tiles;          // compact mode: offset, length, interior columns, rows (packed)
  std::vector<int4> rtiles;         // rect mode: region rectangle and tile interior (packed)
  std::vector<int4> citems;         // coarse items: origin, column mask, row mask
};

// Tiling of a level: TX x TY tiles with grid origin (ox, oy), or with TX = TY
// = 0 the adaptive compact tiling.  Compact regions hold at most `cap` nodes;
// their radius is H.p.
std::string build_tiling(const HostLevel& H, int ld, int TX, int TY, int ox, int oy, bool rect,
                         TilingHost& T, int cap = kRegionCap);

}  // namespace lts
