// Fused stabilized LF-LTS step: one launch advances every active sample by
// one coarse step dt (Algorithm 2 on increments; see lts_step.hip for the
// update formulas).
//
// Work decomposition, shared by all samples of a level (host-built tiling):
//  * coarse items: 64 grid columns x CR rows.  One wavefront per item, one
//    lane per column walking down the rows; it updates the DOFs outside F+
//    (no P neighbour there, so w = A_u u and u_n+1 = 2u_n - u_n-1 + 2 a_p w).
//  * fine tiles: a rectangle of the node grid; its "region" is every F+ node
//    of the rectangle grown by p nodes in each direction.  One workgroup runs
//    all p substeps with the P-masked q = u + d of the region in LDS (double
//    buffered, one barrier per substep) and the per-node state (u, d_m,
//    d_m-1, w and the scaled edge coefficients) in registers; threads are
//    assigned to the region's F+ nodes only (compact list).  Rect mode keeps
//    the region in LDS as a zero-padded rectangle, so the four neighbours of
//    a node sit at fixed offsets (+-1, +-pitch) from its slot; compact mode
//    (used when the rectangle does not fit, e.g. large p) stores the region
//    compacted with per-node neighbour indices.  Values near the region
//    border are wrong after a few substeps (missing neighbours read 0) but the
//    error front moves one node per substep, so after p substeps the
//    rectangle is exact; only its nodes are written back.
// Coarse items and fine tiles are two kernels launched back to back on the
// stream (they write disjoint nodes and only read u_n): the coarse kernel uses
// no LDS beyond the sample's coefficient table, so it runs at high occupancy,
// and each fine workgroup owns a whole CU's LDS.  Workgroup ids are remapped
// so that each of the 8 XCDs works through a contiguous range of (sample,
// work item): halo rows and the shared level arrays stay in that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "fused.h"

namespace lts {

struct StepArgs {
  LevelView L;
  const int4* __restrict__ ent;      // region entries of all fine tiles
  const int2* __restrict__ tiles;    // (offset, length) per fine tile
  const int2* __restrict__ citems;   // (i0, j0) per coarse item
  int n_fine, n_coarse, wg_per_sample, per_xcd, active;
  int pitch, rect_slots;             // rect mode
  const double* __restrict__ kappa;  // [S][nb] (sorted sample order)
  const double* __restrict__ coef;   // [S][p+1]
  const double* __restrict__ Ucur;   // u_n of sample s at Ucur + s*sstride
  double* __restrict__ Uold;         // u_n-1 in, u_n+1 out
  size_t sstride;
  int startup;
  int s0;                            // first sample of this launch
  double* B0;                        // batched jobs: the two state buffers (step t reads B[t&1])
  double* B1;
};

// Launch-time data of a batched launch over several jobs (levels).
struct MultiArgs {
  const StepArgs* __restrict__ jobs;   // static per-job data (device table)
  int n_jobs, per_xcd, step;
  int wg_off[kMaxJobs + 1];            // prefix sums of the jobs' workgroup counts
};

namespace {

// One coarse item per wavefront: lane = grid column, walking down the rows
// with the north/centre/south values and the cell coefficients of the row
// below carried in registers.
__device__ __forceinline__ void coarse_body(const StepArgs& a, const double* __restrict__ lk, int s,
                                            int item) {
  const LevelView& L = a.L;
  if (item >= a.n_coarse) return;
  const int2 it = a.citems[item];
  const int i = it.x + (int)(threadIdx.x & 63);
  if (i < 1 || i > L.nxn - 2) return;
  const double* __restrict__ u = a.Ucur + (size_t)s * a.sstride;
  double* __restrict__ uo = a.Uold + (size_t)s * a.sstride;
  const double ap = a.coef[(size_t)s * (L.p + 1)];
  const int jb = max(it.y, 1), je = min(it.y + kCoarseRows, L.nyn - 1);
  if (jb >= je) return;
  const double hxE = L.hx[i], hxW = L.hx[i - 1], ihE = L.inv2hx[i], ihW = L.inv2hx[i - 1];
  size_t k = (size_t)jb * L.ld + i;
  double uS = u[k - L.ld], uC = u[k];
  double kSW = lk[L.cblk[k - L.ld - 1]], kSE = lk[L.cblk[k - L.ld]];
#pragma unroll 2
  for (int j = jb; j < je; ++j, k += L.ld) {
    const double uN = u[k + L.ld], uE = u[k + 1], uW = u[k - 1];
    const uint8_t f = L.flags[k];
    const double kNW = lk[L.cblk[k - 1]], kNE = lk[L.cblk[k]];
    if ((f & (F_DOF | F_FPLUS)) == F_DOF) {
      const double hyN = L.hy[j], hyS = L.hy[j - 1];
      const double cE = (kNE * hyN + kSE * hyS) * ihE;
      const double cW = (kNW * hyN + kSW * hyS) * ihW;
      const double cN = (kNE * hxE + kNW * hxW) * L.inv2hy[j];
      const double cS = (kSE * hxE + kSW * hxW) * L.inv2hy[j - 1];
      const double w = L.invm[k] * (cE * (uC - uE) + cW * (uC - uW) + cN * (uC - uN) + cS * (uC - uS));
      const double d = ap * w;
      uo[k] = a.startup ? (uC + d) : (2.0 * uC - uo[k] + 2.0 * d);
    }
    uS = uC;
    uC = uN;
    kSW = kNW;
    kSE = kNE;
  }
}

__device__ __forceinline__ void load_kappa(const StepArgs& a, int s, double* __restrict__ lk) {
  for (int t = threadIdx.x; t < a.L.nb; t += blockDim.x) lk[t] = a.kappa[(size_t)s * a.L.nb + t];
  __syncthreads();
}

__global__ __launch_bounds__(kCoarseThreads) void k_coarse(StepArgs a) {
  __shared__ double lk[256];
  const int wpc = (a.n_coarse + 3) / 4;
  const int G = wpc * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  const int s = a.s0 + Lid / wpc;
  load_kappa(a, s, lk);
  coarse_body(a, lk, s, (Lid % wpc) * 4 + (int)(threadIdx.x >> 6));
}

// Job of a batched launch: the job whose workgroup range holds Lid.
__device__ __forceinline__ int find_job(const MultiArgs& m, int Lid) {
  int j = 0;
  while (j + 1 < m.n_jobs && Lid >= m.wg_off[j + 1]) ++j;
  return j;
}

__device__ __forceinline__ StepArgs job_args(const MultiArgs& m, int j) {
  StepArgs a = m.jobs[j];
  const bool odd = m.step & 1;
  a.Ucur = odd ? a.B1 : a.B0;
  a.Uold = odd ? a.B0 : a.B1;
  a.startup = m.step == 0;
  return a;
}

__global__ __launch_bounds__(kCoarseThreads) void k_coarse_multi(MultiArgs m) {
  __shared__ double lk[256];
  const int Lid = (int)(blockIdx.x & 7) * m.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= m.wg_off[m.n_jobs]) return;
  const int j = find_job(m, Lid);
  const StepArgs a = job_args(m, j);
  const int wpc = (a.n_coarse + 3) / 4;
  const int local = Lid - m.wg_off[j];
  const int s = local / wpc;
  load_kappa(a, s, lk);
  coarse_body(a, lk, s, (local % wpc) * 4 + (int)(threadIdx.x >> 6));
}

__device__ __forceinline__ void fine_tile_compact(const StepArgs& a, const double* __restrict__ lk,
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


// Rect mode.  Entry of a region node: x = flat grid index, y = LDS slot in the
// padded rectangle (row pitch kPitch), z = bit 0: node in P, bit 1: node
// inside the tile, w = i | j << 16.  Buffer b of q starts at b * kRectCap, so
// every neighbour read of a node is its base address plus a compile-time
// offset (all within the 16-bit immediate of the LDS instructions).
__device__ __forceinline__ void fine_tile_rect(const StepArgs& a, const double* __restrict__ lk,
                                               double* __restrict__ lq, int s, int tile) {
  constexpr int P = kPitch;
  const LevelView& L = a.L;
  const int2 tl = a.tiles[tile];
  const int len = tl.y;
  const int nzero = a.rect_slots + 2 * P + 1;         // rectangle plus the dummy node's pad
  const int dummy = a.rect_slots + P;                 // slot of threads without a node
  const double* __restrict__ u_g = a.Ucur + (size_t)s * a.sstride;
  double* __restrict__ uo_g = a.Uold + (size_t)s * a.sstride;
  const double* __restrict__ cf = a.coef + (size_t)s * (L.p + 1);

  for (int t = threadIdx.x; t < nzero; t += kFineThreads) {
    lq[t] = 0.0;
    lq[kRectCap + t] = 0.0;
  }
  double u[kNPT], d[kNPT], dp[kNPT], w[kNPT];
  double aE[kNPT], aW[kNPT], aN[kNPT], aS[kNPT], aD[kNPT];
  int base[kNPT], fl[kNPT];
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    const int e = threadIdx.x + r * kFineThreads;
    d[r] = dp[r] = u[r] = w[r] = 0.0;
    aE[r] = aW[r] = aN[r] = aS[r] = aD[r] = 0.0;
    base[r] = dummy - P;
    fl[r] = 0;
    if (e < len) {
      const int4 en = a.ent[tl.x + e];
      const size_t k = (size_t)en.x;
      const int i = en.w & 0xFFFF, j = en.w >> 16;
      base[r] = en.y - P;
      fl[r] = en.z;
      double cE, cW, cN, cS;
      edge_coefs(L, lk, i, j, cE, cW, cN, cS);
      const double im = L.invm[k];
      aE[r] = im * cE;
      aW[r] = im * cW;
      aN[r] = im * cN;
      aS[r] = im * cS;
      aD[r] = (aE[r] + aW[r]) + (aN[r] + aS[r]);
      const bool pi = en.z & 1;
      const double uc = u_g[k];
      u[r] = uc;
      // w = A_u (I - P) u_n
      const double vi = pi ? 0.0 : uc;
      const double vE = (L.flags[k + 1] & F_P) ? 0.0 : u_g[k + 1];
      const double vW = (L.flags[k - 1] & F_P) ? 0.0 : u_g[k - 1];
      const double vN = (L.flags[k + L.ld] & F_P) ? 0.0 : u_g[k + L.ld];
      const double vS = (L.flags[k - L.ld] & F_P) ? 0.0 : u_g[k - L.ld];
      w[r] = aE[r] * (vi - vE) + aW[r] * (vi - vW) + aN[r] * (vi - vN) + aS[r] * (vi - vS);
    }
  }
  __syncthreads();   // zero fill done before the first values land
#pragma unroll
  for (int r = 0; r < kNPT; ++r) lq[base[r] + P] = (fl[r] & 1) ? u[r] : 0.0;
  __syncthreads();

  const int p = L.p;
  // substep m reads buffer B = m & 1 and writes buffer 1 - B
  auto substep = [&](int m, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    const double c = cf[1 + m];   // c1 for m = 0, c2_m otherwise
    const double b = m > 0 ? L.beta[m] : 0.0;
    const double b1 = 1.0 + b;
    double qn[kNPT];
#pragma unroll
    for (int r = 0; r < kNPT; ++r) {
      const double* q = lq + B * kRectCap + base[r];
      const double qS = q[0], qW = q[P - 1], qi = q[P];
      const double qE = q[P + 1], qN = q[2 * P];
      double acc = aD[r] * qi;
      acc -= aE[r] * qE;
      acc -= aW[r] * qW;
      acc -= aN[r] * qN;
      acc -= aS[r] * qS;
      const double rr = w[r] + acc;
      const double dn = b1 * d[r] - b * dp[r] - c * rr;
      dp[r] = d[r];
      d[r] = dn;
      qn[r] = (fl[r] & 1) ? u[r] + dn : 0.0;
    }
    if (m + 1 < p) {
#pragma unroll
      for (int r = 0; r < kNPT; ++r) lq[(1 - B) * kRectCap + base[r] + P] = qn[r];
      __syncthreads();
    }
  };
  for (int m = 0; m < p; m += 2) {
    substep(m, std::integral_constant<int, 0>{});
    if (m + 1 < p) substep(m + 1, std::integral_constant<int, 1>{});
  }
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    if (!(fl[r] & 2)) continue;
    const size_t k = (size_t)a.ent[tl.x + threadIdx.x + r * kFineThreads].x;
    uo_g[k] = a.startup ? (u[r] + d[r]) : (2.0 * u[r] - uo_g[k] + 2.0 * d[r]);
  }
}

template <bool RECT>
__global__ __launch_bounds__(kFineThreads) void k_fine(StepArgs a) {
  __shared__ double lq[2 * kRectCap];
  __shared__ double lk[256];
  const int G = a.n_fine * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  const int s = a.s0 + Lid / a.n_fine;
  load_kappa(a, s, lk);
  if (RECT)
    fine_tile_rect(a, lk, lq, s, Lid % a.n_fine);
  else
    fine_tile_compact(a, lk, lq, s, Lid % a.n_fine);
}

template <bool RECT>
__global__ __launch_bounds__(kFineThreads) void k_fine_multi(MultiArgs m) {
  __shared__ double lq[2 * kRectCap];
  __shared__ double lk[256];
  const int Lid = (int)(blockIdx.x & 7) * m.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= m.wg_off[m.n_jobs]) return;
  const int j = find_job(m, Lid);
  const StepArgs a = job_args(m, j);
  const int local = Lid - m.wg_off[j];
  const int s = local / a.n_fine;
  load_kappa(a, s, lk);
  if (RECT)
    fine_tile_rect(a, lk, lq, s, local % a.n_fine);
  else
    fine_tile_compact(a, lk, lq, s, local % a.n_fine);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host: tiling of a level for a fine-tile rectangle of TX x TY nodes.

std::string build_tiling(const HostLevel& H, int ld, int TX, int TY, int ox, int oy, bool rect,
                         TilingHost& T) {
  T = TilingHost();
  T.TX = TX;
  T.TY = TY;
  T.ox = ox;
  T.oy = oy;
  T.rect = rect;
  const int nxn = H.nxn, nyn = H.nyn, p = H.p;
  auto fl = [&](int i, int j) -> uint8_t { return H.flags[(size_t)j * nxn + i]; };
  const int RX = TX + 2 * p, RY = TY + 2 * p;
  if (rect) {
    T.pitch = kPitch;
    T.rect_slots = kPitch * (RY + 2);
    if (RX + 2 > kPitch || T.rect_slots + 2 * kPitch + 1 > kRectCap)
      return "region rectangle exceeds LDS capacity";
  }
  std::vector<int32_t> loc((size_t)RX * RY);
  size_t n_region = 0, n_fplus = 0;
  for (int ty = oy - ((oy + TY - 1) / TY) * TY; ty < nyn; ty += TY)
    for (int tx = ox - ((ox + TX - 1) / TX) * TX; tx < nxn; tx += TX) {
      bool any = false;
      for (int j = std::max(ty, 0); j < std::min(ty + TY, nyn) && !any; ++j)
        for (int i = std::max(tx, 0); i < std::min(tx + TX, nxn); ++i)
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
          if (rect) {
            e.y = (j - y0 + 1) * T.pitch + (i - x0 + 1);
            e.z = (isP ? 1 : 0) | (interior ? 2 : 0);
          } else {
            e.y = nb(i + 1, j) | (isP ? 0x8000 : 0) | (nb(i - 1, j) << 16) | (interior ? (int)0x80000000u : 0);
            e.z = nb(i, j + 1) | (nb(i, j - 1) << 16);
          }
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
  T.wg_per_sample = T.n_fine + (T.n_coarse + 3) / 4;
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
  D.rect = T.rect;
  D.pitch = T.pitch;
  D.rect_slots = T.rect_slots;
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

std::vector<std::pair<int, int>> tile_origins(const HostLevel& H, int TX, int TY) {
  int fx = H.nxn, fy = H.nyn;
  for (int j = 0; j < H.nyn; ++j)
    for (int i = 0; i < H.nxn; ++i)
      if (H.flags[(size_t)j * H.nxn + i] & LTS_NODE_FPLUS) {
        fx = std::min(fx, i);
        fy = std::min(fy, j);
      }
  if (fx >= H.nxn) return {{0, 0}};
  std::vector<std::pair<int, int>> o = {{0, 0}, {fx % TX, fy % TY}, {fx % TX, 0}, {0, fy % TY}};
  std::sort(o.begin(), o.end());
  o.erase(std::unique(o.begin(), o.end()), o.end());
  return o;
}

lts_status default_tiling(lts_ctx c, DevLevel& lv) {
  TilingHost best;
  bool have = false;
  for (int mode = 1; mode >= 0 && !have; --mode)
    for (auto& tc : tile_candidates())
      for (auto& org : tile_origins(lv.H, tc.first, tc.second)) {
        TilingHost T;
        if (!build_tiling(lv.H, lv.ld, tc.first, tc.second, org.first, org.second, mode == 1, T).empty())
          continue;
        // cost proxy: region nodes (fine work) plus a per-workgroup overhead
        const double cost = T.halo_ratio * lv.H.n_F * lv.H.p + 2048.0 * T.wg_per_sample;
        const double bcost = have ? best.halo_ratio * lv.H.n_F * lv.H.p + 2048.0 * best.wg_per_sample : 0;
        if (!have || cost < bcost) {
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
  a.pitch = T.pitch;
  a.rect_slots = T.rect_slots;
  a.wg_per_sample = T.wg_per_sample;
  a.active = active;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.Ucur = Ucur;
  a.Uold = Uold;
  a.sstride = sstride;
  a.startup = startup;
  a.s0 = s0;
  if (T.n_coarse > 0) {
    const long long G = (long long)((T.n_coarse + 3) / 4) * active;
    a.per_xcd = (int)((G + 7) / 8);
    k_coarse<<<dim3((unsigned)(8LL * a.per_xcd)), dim3(kCoarseThreads), 0, stream>>>(a);
  }
  if (T.n_fine > 0) {
    const long long G = (long long)T.n_fine * active;
    a.per_xcd = (int)((G + 7) / 8);
    if (T.rect)
      k_fine<true><<<dim3((unsigned)(8LL * a.per_xcd)), dim3(kFineThreads), 0, stream>>>(a);
    else
      k_fine<false><<<dim3((unsigned)(8LL * a.per_xcd)), dim3(kFineThreads), 0, stream>>>(a);
  }
  return LTS_OK;
}

lts_status launch_multi_step(lts_ctx c, const StepArgs* d_jobs, const std::vector<const TilingDev*>& T,
                             const std::vector<int>& active, int step, hipStream_t stream) {
  const int nj = (int)T.size();
  if (nj > kMaxJobs) {
    c->err = "too many jobs in one batch";
    return LTS_ERR_ARG;
  }
  MultiArgs m{};
  m.jobs = d_jobs;
  m.n_jobs = nj;
  m.step = step;
  auto go = [&](int kind) {
    m.wg_off[0] = 0;
    for (int j = 0; j < nj; ++j) {
      int w = 0;
      if (kind == 0) w = (T[j]->n_coarse + 3) / 4;
      else if (kind == 1) w = T[j]->rect ? T[j]->n_fine : 0;
      else w = T[j]->rect ? 0 : T[j]->n_fine;
      m.wg_off[j + 1] = m.wg_off[j] + w * active[j];
    }
    const int G = m.wg_off[nj];
    if (G == 0) return;
    m.per_xcd = (G + 7) / 8;
    const dim3 grid((unsigned)(8 * m.per_xcd));
    if (kind == 0)
      k_coarse_multi<<<grid, dim3(kCoarseThreads), 0, stream>>>(m);
    else if (kind == 1)
      k_fine_multi<true><<<grid, dim3(kFineThreads), 0, stream>>>(m);
    else
      k_fine_multi<false><<<grid, dim3(kFineThreads), 0, stream>>>(m);
  };
  go(0);
  go(1);
  go(2);
  return LTS_OK;
}

void job_record(const DevLevel& lv, const TilingDev& T, const double* d_kappa, const double* d_coef,
                double* B0, double* B1, size_t sstride, void* out) {
  StepArgs a{};
  a.L = lv.view();
  a.ent = T.ent.as<int4>();
  a.tiles = T.tiles.as<int2>();
  a.citems = T.citems.as<int2>();
  a.n_fine = T.n_fine;
  a.n_coarse = T.n_coarse;
  a.pitch = T.pitch;
  a.rect_slots = T.rect_slots;
  a.wg_per_sample = T.wg_per_sample;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.sstride = sstride;
  a.B0 = B0;
  a.B1 = B1;
  a.Ucur = B0;
  a.Uold = B1;
  std::memcpy(out, &a, sizeof(a));
}

size_t step_args_size() { return sizeof(StepArgs); }

}  // namespace lts
