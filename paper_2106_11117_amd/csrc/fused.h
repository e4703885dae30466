// Tiling of a level for the fused step kernel (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "host.h"

namespace lts {

constexpr int kFineThreads = 1024;                  // threads per workgroup
constexpr int kNPT = 5;                             // region nodes per thread
constexpr int kRegionCap = kFineThreads * kNPT;     // nodes of one fine-tile region
constexpr int kCoarseRows = 16;                     // rows walked by one coarse wavefront

struct TilingHost {
  int TX = 0, TY = 0;
  int n_fine = 0, n_coarse = 0, wg_per_sample = 0;
  double halo_ratio = 1.0;          // region nodes / F+ nodes
  std::vector<int4> ent;            // region entries (see lts_fused.hip)
  std::vector<int2> tiles;          // (offset, length)
  std::vector<int2> citems;         // (i0, j0)
};

std::string build_tiling(const HostLevel& H, int ld, int TX, int TY, TilingHost& T);

}  // namespace lts
