// Device-side layout of a level and the per-sample tables (internal).
//
// States are stored sample-major: sample s owns a full node grid of
// ny_nodes rows with a padded row pitch `ld` (doubles), node (i, j) at
// s*sstride + j*ld + i.  Boundary (Dirichlet) nodes hold 0 and are never
// written, so every stencil access of a DOF is in bounds without checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lts {

enum : uint8_t { F_DOF = 1, F_P = 2, F_FPLUS = 4 };

struct LevelView {
  int nxn, nyn, ld, p, nb;
  const double* __restrict__ hx;      // [nxn]  x[i+1]-x[i] (0 for the last node)
  const double* __restrict__ hy;      // [nyn]
  const double* __restrict__ inv2hx;  // [nxn]  1/(2 hx)
  const double* __restrict__ inv2hy;  // [nyn]
  const double* __restrict__ x;       // [nxn]
  const double* __restrict__ y;       // [nyn]
  const uint8_t* __restrict__ cblk;   // [nyn*ld] block of cell (a,b) at b*ld+a; 255 = none
  const uint8_t* __restrict__ flags;  // [nyn*ld] F_* bits
  // [nyn*ld] per node (i, j): F_* bits | block of cell (i, j) << 8 | block of
  // cell (i-1, j) << 16 (255: no cell), so one 32-bit read gives a node's flags
  // and the blocks of the two cells above-right and above-left of it
  const uint32_t* __restrict__ ninfo;
  const double* __restrict__ invm;    // [nyn*ld] 1/m for DOFs, 0 elsewhere
  const double* __restrict__ qoiw;    // [nyn*ld]
  const double* __restrict__ beta;    // [p] beta_k, k = 1..p-1
  const double* __restrict__ beta_half;
};

// Edge coefficients of the lumped P1 stiffness at DOF (i, j): K u at the
// node is sum_k c_k (u_ij - u_k) over the four axis neighbours (the
// hypotenuse couplings of right triangles vanish).  Horizontal edge
// (i,j)-(i+1,j) collects kappa hy/(2 hx) from the cell above and the cell
// below; vertical edges likewise with hx/(2 hy).
__device__ __forceinline__ void edge_coefs(const LevelView& L, const double* __restrict__ kap, int i,
                                           int j, double& cE, double& cW, double& cN, double& cS) {
  const size_t r = (size_t)j * L.ld, rm = (size_t)(j - 1) * L.ld;
  const double kNE = kap[L.cblk[r + i]], kNW = kap[L.cblk[r + i - 1]];
  const double kSW = kap[L.cblk[rm + i - 1]], kSE = kap[L.cblk[rm + i]];
  const double hxE = L.hx[i], hxW = L.hx[i - 1], hyN = L.hy[j], hyS = L.hy[j - 1];
  cE = (kNE * hyN + kSE * hyS) * L.inv2hx[i];
  cW = (kNW * hyN + kSW * hyS) * L.inv2hx[i - 1];
  cN = (kNE * hxE + kNW * hxW) * L.inv2hy[j];
  cS = (kSE * hxE + kSW * hxW) * L.inv2hy[j - 1];
}

// Value of the next / previous lane of the wavefront (DPP wavefront shift by
// one lane); the last / first lane reads 0.  All lanes must be active.
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

}  // namespace lts
