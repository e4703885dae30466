// Fused stabilized LF-LTS step: one launch advances every active sample by
// one coarse step dt (Algorithm 2 on increments; see lts_step.hip for the
// update formulas).
//
// Work decomposition, shared by all samples of a level (host-built tiling):
//  * coarse items: 64 grid columns x CR rows.  One wavefront per item, one
//    lane per column walking down the rows; it updates the DOFs outside F+
//    (no P neighbour there, so w = A_u u and u_n+1 = 2u_n - u_n-1 + 2 a_p w).
//  * fine tiles: a rectangle of the node grid; its "region" is every F+ node
//    of the rectangle grown by p nodes in each direction (compacted, row
//    major).  One workgroup runs all p substeps with the P-masked q = u + d of
//    the region in LDS and the per-node state (u, d_m, d_m-1, w and the four
//    scaled edge coefficients) in registers.  Values near the region border
//    are wrong after a few substeps (missing neighbours read 0) but the error
//    front moves one node per substep, so after p substeps the rectangle is
//    exact; only its nodes are written back.
// A workgroup is either one fine tile or 16 coarse items (16 wavefronts).
// Workgroup ids are remapped so that each of the 8 XCDs works through a
// contiguous range of (sample, work item): halo rows and the shared level
// arrays then stay in that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ctx.h"
#include "fused.h"

namespace lts {

namespace {

struct StepArgs {
  LevelView L;
  const int4* __restrict__ ent;      // region entries of all fine tiles
  const int2* __restrict__ tiles;    // (offset, length) per fine tile
  const int2* __restrict__ citems;   // (i0, j0) per coarse item
  int n_fine, n_coarse, wg_per_sample, per_xcd, active;
  const double* __restrict__ kappa;  // [S][nb] (sorted sample order)
  const double* __restrict__ coef;   // [S][p+1]
  const double* __restrict__ Ucur;   // u_n of sample s at Ucur + s*sstride
  double* __restrict__ Uold;         // u_n-1 in, u_n+1 out
  size_t sstride;
  int startup;
  int s0;                            // first sample of this launch
};

__device__ __forceinline__ void coarse_item(const StepArgs& a, const double* __restrict__ lk, int s,
                                            int item) {
  const LevelView& L = a.L;
  const int lane = threadIdx.x & 63;
  const int2 it = a.citems[item];
  const int i = it.x + lane;
  if (i < 1 || i > L.nxn - 2) return;
  const double* __restrict__ u = a.Ucur + (size_t)s * a.sstride;
  double* __restrict__ uo = a.Uold + (size_t)s * a.sstride;
  const double ap = a.coef[(size_t)s * (L.p + 1)];
  const int jend = min(it.y + kCoarseRows, L.nyn - 1);
  for (int j = max(it.y, 1); j < jend; ++j) {
    const size_t k = (size_t)j * L.ld + i;
    const uint8_t f = L.flags[k];
    if ((f & (F_DOF | F_FPLUS)) != F_DOF) continue;
    double cE, cW, cN, cS;
    edge_coefs(L, lk, i, j, cE, cW, cN, cS);
    const double uc = u[k];
    const double w = L.invm[k] * (cE * (uc - u[k + 1]) + cW * (uc - u[k - 1]) +
                                  cN * (uc - u[k + L.ld]) + cS * (uc - u[k - L.ld]));
    const double d = ap * w;
    uo[k] = a.startup ? (uc + d) : (2.0 * uc - uo[k] + 2.0 * d);
  }
}

__device__ __forceinline__ void fine_tile(const StepArgs& a, const double* __restrict__ lk,
                                          double* __restrict__ lq, int s, int tile) {
  const LevelView& L = a.L;
  const int2 tl = a.tiles[tile];
  const int len = tl.y;
  const double* __restrict__ u_g = a.Ucur + (size_t)s * a.sstride;
  double* __restrict__ uo_g = a.Uold + (size_t)s * a.sstride;
  const double* __restrict__ cf = a.coef + (size_t)s * (L.p + 1);

  double u[kNPT], d[kNPT], dp[kNPT], w[kNPT], aE[kNPT], aW[kNPT], aN[kNPT], aS[kNPT];
  int ew[kNPT], ns[kNPT], kk[kNPT];
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    const int e = threadIdx.x + r * kFineThreads;
    d[r] = 0.0;
    dp[r] = 0.0;
    u[r] = 0.0;
    w[r] = 0.0;
    aE[r] = aW[r] = aN[r] = aS[r] = 0.0;
    ew[r] = 0;
    ns[r] = 0;
    kk[r] = -1;
    if (e < len) {
      const int4 en = a.ent[tl.x + e];
      const size_t k = (size_t)en.x;
      const int i = en.w & 0xFFFF, j = en.w >> 16;
      kk[r] = en.x;
      ew[r] = en.y;
      ns[r] = en.z;
      double cE, cW, cN, cS;
      edge_coefs(L, lk, i, j, cE, cW, cN, cS);
      const double im = L.invm[k];
      aE[r] = im * cE;
      aW[r] = im * cW;
      aN[r] = im * cN;
      aS[r] = im * cS;
      const bool pi = (en.y >> 15) & 1;
      const double uc = u_g[k];
      u[r] = uc;
      // w = A_u (I - P) u_n
      const double vi = pi ? 0.0 : uc;
      const double vE = (L.flags[k + 1] & F_P) ? 0.0 : u_g[k + 1];
      const double vW = (L.flags[k - 1] & F_P) ? 0.0 : u_g[k - 1];
      const double vN = (L.flags[k + L.ld] & F_P) ? 0.0 : u_g[k + L.ld];
      const double vS = (L.flags[k - L.ld] & F_P) ? 0.0 : u_g[k - L.ld];
      w[r] = aE[r] * (vi - vE) + aW[r] * (vi - vW) + aN[r] * (vi - vN) + aS[r] * (vi - vS);
      lq[e] = pi ? uc : 0.0;
    }
  }
  if (threadIdx.x == 0) lq[len] = 0.0;   // slot read for absent / non-P neighbours
  __syncthreads();

  const int p = L.p;
  for (int m = 0; m < p; ++m) {
    const double c = cf[1 + m];   // c1 for m = 0, c2_m otherwise
    const double b = m > 0 ? L.beta[m] : 0.0;
#pragma unroll
    for (int r = 0; r < kNPT; ++r) {
      if (kk[r] < 0) continue;
      const bool pi = (ew[r] >> 15) & 1;
      const double qi = pi ? u[r] + d[r] : 0.0;
      const double qE = lq[ew[r] & 0x7FFF], qW = lq[(ew[r] >> 16) & 0x7FFF];
      const double qN = lq[ns[r] & 0x7FFF], qS = lq[(ns[r] >> 16) & 0x7FFF];
      const double apq = aE[r] * (qi - qE) + aW[r] * (qi - qW) + aN[r] * (qi - qN) + aS[r] * (qi - qS);
      const double rr = w[r] + apq;
      const double dn = (m == 0) ? -c * rr : (1.0 + b) * d[r] - b * dp[r] - c * rr;
      dp[r] = d[r];
      d[r] = dn;
    }
    if (m + 1 < p) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kNPT; ++r) {
        if (kk[r] < 0) continue;
        const int e = threadIdx.x + r * kFineThreads;
        lq[e] = ((ew[r] >> 15) & 1) ? u[r] + d[r] : 0.0;
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    if (kk[r] < 0 || !((unsigned)ew[r] >> 31)) continue;
    const size_t k = (size_t)kk[r];
    uo_g[k] = a.startup ? (u[r] + d[r]) : (2.0 * u[r] - uo_g[k] + 2.0 * d[r]);
  }
}

__global__ __launch_bounds__(kFineThreads) void k_step(StepArgs a) {
  __shared__ double lq[kRegionCap + 1];
  __shared__ double lk[256];
  const int G = a.wg_per_sample * a.active;
  const int L = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (L >= G) return;
  const int s = a.s0 + L / a.wg_per_sample;
  const int wi = L % a.wg_per_sample;
  for (int t = threadIdx.x; t < a.L.nb; t += kFineThreads) lk[t] = a.kappa[(size_t)s * a.L.nb + t];
  __syncthreads();
  if (wi < a.n_fine) {
    fine_tile(a, lk, lq, s, wi);
  } else {
    const int item = (wi - a.n_fine) * (kFineThreads / 64) + (int)(threadIdx.x >> 6);
    if (item < a.n_coarse) coarse_item(a, lk, s, item);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host: tiling of a level for a fine-tile rectangle of TX x TY nodes.

std::string build_tiling(const HostLevel& H, int ld, int TX, int TY, TilingHost& T) {
  T = TilingHost();
  T.TX = TX;
  T.TY = TY;
  const int nxn = H.nxn, nyn = H.nyn, p = H.p;
  auto fl = [&](int i, int j) -> uint8_t { return H.flags[(size_t)j * nxn + i]; };
  const int RX = TX + 2 * p, RY = TY + 2 * p;
  std::vector<int32_t> loc((size_t)RX * RY);
  size_t n_region = 0, n_fplus = 0;
  for (int ty = 0; ty < nyn; ty += TY)
    for (int tx = 0; tx < nxn; tx += TX) {
      bool any = false;
      for (int j = ty; j < std::min(ty + TY, nyn) && !any; ++j)
        for (int i = tx; i < std::min(tx + TX, nxn); ++i)
          if (fl(i, j) & LTS_NODE_FPLUS) {
            any = true;
            break;
          }
      if (!any) continue;
      const int x0 = tx - p, y0 = ty - p;
      std::fill(loc.begin(), loc.end(), -1);
      int len = 0;
      for (int j = std::max(y0, 0); j < std::min(y0 + RY, nyn); ++j)
        for (int i = std::max(x0, 0); i < std::min(x0 + RX, nxn); ++i)
          if (fl(i, j) & LTS_NODE_FPLUS) loc[(size_t)(j - y0) * RX + (i - x0)] = len++;
      if (len > kRegionCap) return "fine tile region exceeds the workgroup capacity";
      const int off = (int)T.ent.size();
      auto nb = [&](int i, int j) -> int {
        if (i < x0 || j < y0 || i >= x0 + RX || j >= y0 + RY || i < 0 || j < 0 || i >= nxn || j >= nyn)
          return len;
        const int l = loc[(size_t)(j - y0) * RX + (i - x0)];
        if (l < 0 || !(fl(i, j) & LTS_NODE_P)) return len;
        return l;
      };
      for (int j = std::max(y0, 0); j < std::min(y0 + RY, nyn); ++j)
        for (int i = std::max(x0, 0); i < std::min(x0 + RX, nxn); ++i) {
          if (!(fl(i, j) & LTS_NODE_FPLUS)) continue;
          const bool interior = i >= tx && i < tx + TX && j >= ty && j < ty + TY;
          const bool isP = fl(i, j) & LTS_NODE_P;
          int4 e;
          e.x = j * ld + i;
          e.y = nb(i + 1, j) | (isP ? 0x8000 : 0) | (nb(i - 1, j) << 16) | (interior ? (int)0x80000000u : 0);
          e.z = nb(i, j + 1) | (nb(i, j - 1) << 16);
          e.w = i | (j << 16);
          T.ent.push_back(e);
          if (interior) ++n_fplus;
        }
      T.tiles.push_back(make_int2(off, len));
      n_region += len;
    }
  for (int ty = 0; ty < nyn; ty += kCoarseRows)
    for (int tx = 0; tx < nxn; tx += 64) {
      bool any = false;
      for (int j = ty; j < std::min(ty + kCoarseRows, nyn) && !any; ++j)
        for (int i = tx; i < std::min(tx + 64, nxn); ++i)
          if ((fl(i, j) & (LTS_NODE_DOF | LTS_NODE_FPLUS)) == LTS_NODE_DOF) {
            any = true;
            break;
          }
      if (any) T.citems.push_back(make_int2(tx, ty));
    }
  T.n_fine = (int)T.tiles.size();
  T.n_coarse = (int)T.citems.size();
  T.wg_per_sample = T.n_fine + (T.n_coarse + kFineThreads / 64 - 1) / (kFineThreads / 64);
  T.halo_ratio = n_fplus ? (double)n_region / n_fplus : 1.0;
  return "";
}

lts_status upload_tiling(lts_ctx c, const TilingHost& T, TilingDev& D) {
  D.TX = T.TX;
  D.TY = T.TY;
  D.n_fine = T.n_fine;
  D.n_coarse = T.n_coarse;
  D.wg_per_sample = T.wg_per_sample;
  D.halo_ratio = T.halo_ratio;
  LTS_HIP(c, D.ent.ensure(std::max<size_t>(T.ent.size() * sizeof(int4), 16)));
  LTS_HIP(c, D.tiles.ensure(std::max<size_t>(T.tiles.size() * sizeof(int2), 8)));
  LTS_HIP(c, D.citems.ensure(std::max<size_t>(T.citems.size() * sizeof(int2), 8)));
  if (!T.ent.empty())
    LTS_HIP(c, hipMemcpy(D.ent.p, T.ent.data(), T.ent.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!T.tiles.empty())
    LTS_HIP(c, hipMemcpy(D.tiles.p, T.tiles.data(), T.tiles.size() * sizeof(int2), hipMemcpyHostToDevice));
  if (!T.citems.empty())
    LTS_HIP(c, hipMemcpy(D.citems.p, T.citems.data(), T.citems.size() * sizeof(int2), hipMemcpyHostToDevice));
  return LTS_OK;
}

const std::vector<std::pair<int, int>>& tile_candidates() {
  static const std::vector<std::pair<int, int>> v = {
      {64, 48}, {48, 64}, {56, 56}, {48, 48}, {80, 32}, {32, 80}, {128, 24}, {24, 128}, {40, 40},
      {32, 32}, {16, 256}, {256, 16}, {16, 128}, {128, 16}, {24, 24}, {16, 64}, {64, 16}, {16, 16},
      {8, 256}, {256, 8}, {8, 64}, {64, 8}, {8, 8}};
  return v;
}

lts_status default_tiling(lts_ctx c, DevLevel& lv) {
  TilingHost best;
  bool have = false;
  for (auto& tc : tile_candidates()) {
    TilingHost T;
    if (!build_tiling(lv.H, lv.ld, tc.first, tc.second, T).empty()) continue;
    if (!have || T.halo_ratio < best.halo_ratio - 1e-9) {
      best = std::move(T);
      have = true;
    }
  }
  if (!have) {
    c->err = "no fine-tile size fits the workgroup capacity for this level";
    return LTS_ERR_ARG;
  }
  return upload_tiling(c, best, lv.tiling);
}

lts_status launch_step(lts_ctx c, const DevLevel& lv, const TilingDev& T, const double* d_kappa,
                       const double* d_coef, const double* Ucur, double* Uold, size_t sstride, int s0,
                       int active, int startup, hipStream_t stream) {
  if (active <= 0) return LTS_OK;
  StepArgs a;
  a.L = lv.view();
  a.ent = T.ent.as<int4>();
  a.tiles = T.tiles.as<int2>();
  a.citems = T.citems.as<int2>();
  a.n_fine = T.n_fine;
  a.n_coarse = T.n_coarse;
  a.wg_per_sample = T.wg_per_sample;
  const long long G = (long long)T.wg_per_sample * active;
  a.per_xcd = (int)((G + 7) / 8);
  a.active = active;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.Ucur = Ucur;
  a.Uold = Uold;
  a.sstride = sstride;
  a.startup = startup;
  a.s0 = s0;
  k_step<<<dim3((unsigned)(8LL * a.per_xcd)), dim3(kFineThreads), 0, stream>>>(a);
  return LTS_OK;
}

}  // namespace lts
