// Fused stabilized LF-LTS step: one launch advances every active sample by
// one coarse step dt (Algorithm 2 on increments; see lts_step.hip for the
// update formulas).
//
// Work decomposition, shared by all samples of a level (host-built tiling):
//  * coarse items: 64 grid columns x 16 rows.  One workgroup of four
//    wavefronts per item, lane = column, wavefront v = rows 4v .. 4v+3; all
//    its reads are issued in one batch, east / west neighbours come by DPP.
//    It updates the DOFs outside F+ (no P neighbour there, so w = A_u u and
//    u_n+1 = 2u_n - u_n-1 + 2 a_p w).
//  * fine tiles: a rectangle of the node grid; its "region" is the rectangle
//    grown by p nodes in each direction, clipped to the grid and to the F+
//    bounding box grown by one.  One workgroup runs all p substeps of the
//    region.  Rect mode (regions up to 64 x 64, p <= 64): lane = column,
//    wavefront v = rows 4v .. 4v+3, the per-node state (P u_n, d_m, d_m-1, w,
//    q and the scaled edge coefficients) in registers, east / west neighbours
//    by DPP and only the rows at wavefront boundaries exchanged through LDS
//    (double buffered, one barrier per substep).  Compact mode (regions that
//    do not fit, large p, or sparse F+) assigns lanes to the region's F+ nodes
//    only and keeps them compacted in LDS with per-node neighbour slots; its
//    tiles are rectangles of a uniform grid or of the adaptive bisection of
//    F+, on 256-, 512- or 1024-thread workgroups (the fewest that hold the
//    largest region; small ones only while a launch has workgroups to spare).
//    Values near the region border are wrong after a few substeps (missing
//    neighbours read 0) but the error front moves one node per substep, so
//    after p substeps the tile is exact; only its nodes are written back.
// Coarse items and fine tiles are separate kernels launched back to back on
// the stream (they write disjoint nodes and only read u_n): the coarse kernel
// uses no LDS beyond the sample's coefficient table, so it runs at high
// occupancy, and a 1024-thread fine workgroup fills a CU's register file.
// Workgroup ids are remapped so that each of the 8 XCDs works through a
// contiguous range of (sample, work item) of a level (in a batched launch:
// of every job): halo rows and the shared level arrays stay in that XCD's L2.
// For coarse items that range is about one horizontal band of the level's
// items over all samples; for fine tiles, every tile of an eighth of the
// samples.
//
// The same tile and item bodies also run inside k_persist, the persistent
// form of the batched solve: one cooperative launch for all steps of all
// jobs, a device-wide barrier after each step (see the comment there).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "fused.h"

namespace lts {

struct StepArgs {
  LevelView L;
  const int4* __restrict__ ent;      // region entries of all fine tiles
  const int4* __restrict__ tiles;    // compact mode: offset, length, ix0 | ix1 << 16, iy0 | iy1 << 16
  const int4* __restrict__ rtiles;   // rect mode: packed region / interior per fine tile
  const int4* __restrict__ citems;   // per coarse item: origin, column mask, row mask
  int n_fine, n_coarse, wg_per_sample, per_xcd, active;
  const double* __restrict__ kappa;  // [S][nb] (sorted sample order)
  const double* __restrict__ coef;   // [S][p+1]
  const double* __restrict__ Ucur;   // u_n of sample s at Ucur + s*sstride
  double* __restrict__ Uold;         // u_n-1 in
  double* Unew;                      // u_n+1 out (Uold: in place)
  size_t sstride;
  int startup;
  int s0;                            // first sample of this launch
  double* B0;                        // batched jobs: the two state buffers (step t reads B[t&1])
  double* B1;
};

// What changes from step to step: the state buffers and the start-up flag.
// Kept apart from the job data so that the batched kernels read a job's
// record in place (a copy would hide that its pointers address global memory).
struct StepState {
  const double* Ucur;   // u_n of sample s at Ucur + s*sstride
  double* Uold;         // u_n-1 in
  double* Unew;         // u_n+1 out (Uold for the in-place update)
  int startup;
  double* Dout = nullptr;   // adjoint recompute: d_m+1 of sample s at Dout + m*dstride + s*sstride
  size_t dstride = 0;
};

// Launch-time data of a batched launch over several jobs (levels).  Each
// job's workgroups are split into 8 contiguous chunks, one per XCD, and every
// XCD runs its chunks of the jobs in the order given by `order`.
struct MultiArgs {
  const StepArgs* __restrict__ jobs;   // static per-job data (device table)
  int n_jobs, step;
  int order[kMaxJobs];                 // job at launch position q
  int wg_n[kMaxJobs];                  // workgroups of the job at position q
  int chunk_off[kMaxJobs + 1];         // prefix sums over positions of ceil(wg_n / 8)
};

namespace {

// One coarse item (64 grid columns x kCoarseRows rows) per workgroup: lane =
// column, wavefront v = rows 4v .. 4v+3 of the item.  Every global read of a
// wavefront is issued in one batch (u of its rows and the rows above and
// below, the two columns just outside the item, u_n-1, 1/m, the node words
// with flags and cell blocks), then the four rows are updated.  The
// item descriptor is x = i0 | j0 << 16, (y, z) = 64-bit mask of the columns
// holding a DOF outside F+, w = 16-bit mask of such rows; lanes and wavefronts
// without such a DOF return at once.
// tid: thread index within the item's 256 threads; on = false: the threads
// read in bounds (item and s must be valid) but write nothing, and meet the
// same workgroup barrier.
template <class T>
__device__ __forceinline__ void coarse_body(const StepArgs& a, const StepState& st, double* __restrict__ lk, int s,
                                            int item, int tid, bool on) {
  const LevelView& L = a.L;
  const int4 it = a.citems[item];
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t rows = ((uint32_t)it.w >> (4 * wv)) & 0xFu;
  const int lane = tid & 63;
  const uint64_t lm = (uint64_t)(uint32_t)it.y | (uint64_t)(uint32_t)it.z << 32;
  const bool live = on && rows != 0 && ((lm >> lane) & 1);
  // Lane = column x0 + lane.  Values are read at the column clamped into the
  // grid (a live lane's column holds a DOF, 1 <= i <= nxn - 2; the boundary
  // columns hold u = 0), so the east / west neighbours of a live lane are the
  // adjacent lanes' values (DPP), except past the item's first and last lane.
  const int i0 = it.x & 0xFFFF;
  const int iv = min(i0 + lane, L.nxn - 1);          // value column
  const int i = min(max(i0 + lane, 1), L.nxn - 2);   // geometry column
  const int j0 = (it.x >> 16) + 4 * wv;               // rows j0 .. j0 + 3
  const int ld = L.ld;
  const T* __restrict__ u = reinterpret_cast<const T*>(st.Ucur) + (size_t)s * a.sstride;
  T* __restrict__ uo = reinterpret_cast<T*>(st.Uold) + (size_t)s * a.sstride;
  T* un = reinterpret_cast<T*>(st.Unew) + (size_t)s * a.sstride;
  const T ap = (T)a.coef[(size_t)s * (L.p + 1)];
  const bool startup = st.startup;
  constexpr int R = 4;
  // ---- one batch of reads (with the sample's kappa table); rows off the grid
  //      are clamped and never used
  const double kv = tid < L.nb ? a.kappa[(size_t)s * L.nb + tid] : 0.0;
  const double hxE = L.hx[i], hxW = L.hx[i - 1], ihE = L.inv2hx[i], ihW = L.inv2hx[i - 1];
  T uc[R + 2], ued[R], uold[R];
  double im[R], hy[R + 1], ihy[R + 1];
  uint32_t ni[R + 1];                                  // node words of rows j0-1 .. j0+3
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    const int j = min(max(j0 - 1 + q, 0), L.nyn - 1);
    uc[q] = u[(size_t)j * ld + iv];
  }
#pragma unroll
  for (int q = 0; q <= R; ++q) {
    const int j = min(max(j0 - 1 + q, 0), L.nyn - 2);  // cell row below node row j0 + q
    hy[q] = L.hy[j];
    ihy[q] = L.inv2hy[j];
    ni[q] = L.ninfo[(size_t)min(max(j0 - 1 + q, 0), L.nyn - 1) * ld + i];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = min(j0 + r, L.nyn - 1);
    const size_t k = (size_t)j * ld + i;
    ued[r] = (T)0;
    if (lane == 0 || lane == 63) ued[r] = u[(size_t)j * ld + min(max(i0 + lane + (lane ? 1 : -1), 0), L.nxn - 1)];
    im[r] = L.invm[k];
    uold[r] = startup ? (T)0 : uo[k];
  }
  if (tid < L.nb) lk[tid] = kv;
  __syncthreads();
  // east / west values of rows j0 .. j0+3 (every lane still active for DPP)
  T ue[R], uw[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const T e = lane_next(uc[r + 1]), w = lane_prev(uc[r + 1]);
    ue[r] = lane == 63 ? ued[r] : e;
    uw[r] = lane == 0 ? ued[r] : w;
  }
  if (!live) return;
  // ---- update the rows' DOFs outside F+ (edge form)
  double kE[R + 1], kW[R + 1];
#pragma unroll
  for (int q = 0; q <= R; ++q) {
    kE[q] = lk[(ni[q] >> 8) & 0xFF];
    kW[q] = lk[(ni[q] >> 16) & 0xFF];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if ((ni[r + 1] & (F_DOF | F_FPLUS)) != F_DOF) continue;
    const T uS = uc[r], uC = uc[r + 1], uN = uc[r + 2];
    const double cEg = (kE[r + 1] * hy[r + 1] + kE[r] * hy[r]) * ihE;
    const double cWg = (kW[r + 1] * hy[r + 1] + kW[r] * hy[r]) * ihW;
    const double cNg = (kE[r + 1] * hxE + kW[r + 1] * hxW) * ihy[r + 1];
    const double cSg = (kE[r] * hxE + kW[r] * hxW) * ihy[r];
    const T w = (T)im[r] * ((T)cEg * (uC - ue[r]) + (T)cWg * (uC - uw[r]) + (T)cNg * (uC - uN) +
                            (T)cSg * (uC - uS));
    const T d = ap * w;
    un[(size_t)(j0 + r) * ld + i] = startup ? (uC + d) : ((T)2 * uC - uold[r] + (T)2 * d);
  }
}

__device__ __forceinline__ void load_kappa(const StepArgs& a, int s, double* __restrict__ lk) {
  for (int t = threadIdx.x; t < a.L.nb; t += blockDim.x) lk[t] = a.kappa[(size_t)s * a.L.nb + t];
  __syncthreads();
}

// Workgroup order over (item, sample): the items are cut into 8 bands of
// consecutive items (horizontal strips of the level, the last one ragged), and
// each band is walked sample-major, items fastest.  A launch hands each XCD a
// contiguous eighth of the order, so an XCD runs about one band: its workgroups
// stream one sample's strip row after row (contiguous HBM lines), the band's
// mesh arrays stay in that XCD's L2 for all samples, and the halo lines of an
// item's neighbours were loaded shortly before (one workgroup back
// horizontally, one item row vertically).  Every Lid < n_items * active maps to
// a distinct (item, s).
__device__ __forceinline__ void coarse_order(int Lid, int n_items, int active, int& item, int& s) {
  const int cb = (n_items + 7) / 8;                  // items per band
  const int b = Lid / (cb * active);
  const int nb = min(cb, n_items - b * cb);          // items in band b (>= 1)
  const int rem = Lid - b * cb * active;
  s = rem / nb;
  item = b * cb + (rem - s * nb);
}

template <class T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse(StepArgs a) {
  __shared__ double lk[256];
  const int G = a.n_coarse * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  int item, s;
  coarse_order(Lid, a.n_coarse, a.active, item, s);
  coarse_body<T>(a, StepState{a.Ucur, a.Uold, a.Unew, a.startup}, lk, a.s0 + s, item, (int)threadIdx.x, true);
}

// Job and job-local workgroup index of this workgroup in a batched launch;
// false for the workgroups past a job's count in its last chunk.  The hardware
// hands workgroup b to XCD b mod 8, so XCD x runs, for each launch position in
// turn, chunk x of that job: every XCD gets an equal share of every job (jobs
// differ in cost per workgroup by a large factor), and neighbouring tiles of a
// sample stay in one XCD's L2.
__device__ __forceinline__ bool multi_slot(const MultiArgs& m, int& j, int& local, int& n) {
  const int x = (int)(blockIdx.x & 7), k = (int)(blockIdx.x >> 3);
  int q = 0;
  while (q + 1 < m.n_jobs && k >= m.chunk_off[q + 1]) ++q;
  const int per = m.chunk_off[q + 1] - m.chunk_off[q];
  j = m.order[q];
  n = m.wg_n[q];
  local = x * per + (k - m.chunk_off[q]);
  return k < m.chunk_off[m.n_jobs] && local < n;
}

// A pointer field of a job record loaded as a global-address-space pointer.
// Copied as plain pointers out of device memory, the job's pointers would be
// addressed as flat pointers (slower accesses, 64-bit addresses in vector
// registers); loaded with the global type, the compiler keeps global accesses.
#define LTS_GPTR(f) \
  ((decltype(+(f)))(*(__attribute__((address_space(1))) std::remove_pointer_t<decltype(+(f))>* const*)(&(f))))

__device__ __forceinline__ StepArgs job_record(const StepArgs& a) {
  StepArgs b;
  b.L.nxn = a.L.nxn; b.L.nyn = a.L.nyn; b.L.ld = a.L.ld; b.L.p = a.L.p; b.L.nb = a.L.nb;
  b.L.hx = LTS_GPTR(a.L.hx); b.L.hy = LTS_GPTR(a.L.hy);
  b.L.inv2hx = LTS_GPTR(a.L.inv2hx); b.L.inv2hy = LTS_GPTR(a.L.inv2hy);
  b.L.x = LTS_GPTR(a.L.x); b.L.y = LTS_GPTR(a.L.y);
  b.L.cblk = LTS_GPTR(a.L.cblk); b.L.flags = LTS_GPTR(a.L.flags); b.L.ninfo = LTS_GPTR(a.L.ninfo);
  b.L.invm = LTS_GPTR(a.L.invm); b.L.qoiw = LTS_GPTR(a.L.qoiw);
  b.L.beta = LTS_GPTR(a.L.beta); b.L.beta_half = LTS_GPTR(a.L.beta_half);
  b.ent = LTS_GPTR(a.ent); b.tiles = LTS_GPTR(a.tiles); b.rtiles = LTS_GPTR(a.rtiles);
  b.citems = LTS_GPTR(a.citems);
  b.n_fine = a.n_fine; b.n_coarse = a.n_coarse; b.wg_per_sample = a.wg_per_sample;
  b.per_xcd = a.per_xcd; b.active = a.active;
  b.kappa = LTS_GPTR(a.kappa); b.coef = LTS_GPTR(a.coef);
  b.Ucur = nullptr; b.Uold = nullptr; b.Unew = nullptr;   // per step: StepState
  b.sstride = a.sstride; b.startup = 0; b.s0 = a.s0;
  b.B0 = LTS_GPTR(a.B0); b.B1 = LTS_GPTR(a.B1);
  return b;
}

__device__ __forceinline__ StepState job_state(const MultiArgs& m, const StepArgs& a) {
  const bool odd = m.step & 1;
  return StepState{odd ? a.B1 : a.B0, odd ? a.B0 : a.B1, odd ? a.B0 : a.B1, m.step == 0};
}

template <class T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_multi(MultiArgs m) {
  __shared__ double lk[256];
  int j, local, n;
  if (!multi_slot(m, j, local, n)) return;
  const StepArgs a = job_record(m.jobs[j]);
  const int act = n / a.n_coarse;                      // active samples of the job
  int item, s;
  coarse_order(local, a.n_coarse, act, item, s);
  coarse_body<T>(a, job_state(m, a), lk, s, item, (int)threadIdx.x, true);
}

// Compact mode.  The region's nodes (the F+ nodes within Manhattan distance p
// of the tile, ordered by that distance) are spread over the lanes, kNPT per
// lane; q lives in LDS in two buffers (substep m reads one and writes the
// other: one barrier per substep).  A node at distance D can influence the tile
// only after D more substeps, so substep m updates only the nodes within
// p - 1 - m: with the distance ordering those form a prefix of the entries and
// the wavefronts past it skip the substep.  An entry is x = grid index | P flag
// << 31, y = E | W << 16, z = N | S << 16 (neighbour slots; slot len holds 0
// for an absent or non-P neighbour), w = i | j << 16.  Each lane turns its
// neighbour slots into LDS byte addresses once; the substeps run in pairs so
// that the two buffers and the roles of the increment registers are fixed.
// tid: thread index within the tile's NT threads.  on = false: the threads
// touch no global memory and meet the same workgroup barriers (a persistent
// workgroup runs several tiles of one level side by side).
// ADJ (the adjoint's recompute of a step, FP64): every increment d_m+1 of the
// tile's own nodes of P goes to st.Dout, and u_n+1 is written only if
// st.Unew is given (the adjoint runs the step backward in time: Uold = y_n+1,
// Unew = y_n-1).
template <class T, int NT, bool ADJ = false>
__device__ __forceinline__ void fine_tile_compact(const StepArgs& a, const StepState& st, const double* __restrict__ lk,
                                                  T* __restrict__ lq, int s, int tile, int tid, bool on) {
  constexpr int kCap = NT * kNPT;      // region nodes this workgroup size holds
  const LevelView& L = a.L;
  const int4 tl = a.tiles[tile];
  const int len = on ? tl.y : 0;
  const int ix0 = tl.z & 0xFFFF, ix1 = tl.z >> 16, iy0 = tl.w & 0xFFFF, iy1 = tl.w >> 16;
  const int p = L.p;
  const T* __restrict__ u_g = reinterpret_cast<const T*>(st.Ucur) + (size_t)s * a.sstride;
  T* __restrict__ uo_g = reinterpret_cast<T*>(st.Uold) + (size_t)s * a.sstride;
  T* uw_g = reinterpret_cast<T*>(st.Unew) + (size_t)s * a.sstride;
  const double* __restrict__ cf = a.coef + (size_t)s * (L.p + 1);
  T* const q0 = lq;                    // q of the even substeps' inputs
  T* const q1 = lq + (kCap + 1);       // and of the odd ones'; slot len of each holds 0

  T u[kNPT], pm[kNPT], d0[kNPT], d1[kNPT], w[kNPT], aE[kNPT], aW[kNPT], aN[kNPT], aS[kNPT];
  uint32_t ad[kNPT][4];                // LDS byte offsets of the E, W, N, S neighbours
  int kk[kNPT], dd[kNPT];
  // The lane's entries are read in one batch (a lane past the region end reads
  // the last entry again and ignores it); then, node by node, everything an
  // entry indexes: u and 1/m of the node, u and the flags of its four
  // neighbours (an F+ node is an interior DOF, so they exist, and their values
  // are read with their flags and masked afterwards), the blocks of its four
  // cells and the cell sizes.
  int4 en[kNPT];
#pragma unroll
  for (int r = 0; r < kNPT; ++r) en[r] = on ? a.ent[tl.x + min(tid + r * NT, len - 1)] : make_int4(0, 0, 0, 0);
  const int ld = L.ld;
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    d0[r] = d1[r] = (T)0;
    u[r] = pm[r] = w[r] = (T)0;
    aE[r] = aW[r] = aN[r] = aS[r] = (T)0;
#pragma unroll
    for (int t = 0; t < 4; ++t) ad[r][t] = (uint32_t)(len * sizeof(T));
    kk[r] = 0;
    dd[r] = p;                         // never updated, never written
    const int e = tid + r * NT;
    if (e < len) {
      const size_t k = (size_t)(en[r].x & 0x7FFFFFFF);
      const bool pi = en[r].x < 0;
      const int i = en[r].w & 0xFFFF, j = en[r].w >> 16;
      kk[r] = (int)k;
      ad[r][0] = (uint32_t)(en[r].y & 0xFFFF) * sizeof(T);
      ad[r][1] = ((uint32_t)en[r].y >> 16) * sizeof(T);
      ad[r][2] = (uint32_t)(en[r].z & 0xFFFF) * sizeof(T);
      ad[r][3] = ((uint32_t)en[r].z >> 16) * sizeof(T);
      dd[r] = max(max(ix0 - i, i - (ix1 - 1)), 0) + max(max(iy0 - j, j - (iy1 - 1)), 0);
      const T uc = u_g[k];
      const T uE = u_g[k + 1], uW = u_g[k - 1], uN = u_g[k + ld], uS = u_g[k - ld];
      const uint8_t fE = L.flags[k + 1], fW = L.flags[k - 1], fN = L.flags[k + ld], fS = L.flags[k - ld];
      const double im = L.invm[k];
      double cE, cW, cN, cS;
      edge_coefs(L, lk, i, j, cE, cW, cN, cS);
      u[r] = uc;
      pm[r] = pi ? (T)1 : (T)0;
      q0[e] = pi ? uc : (T)0;
      // coefficients (zero for a node no substep updates) and w = A_u (I - P) u_n,
      // formed without a branch so that all of the node's reads go out together
      const double imu = dd[r] < p ? im : 0.0;
      aE[r] = (T)(imu * cE);
      aW[r] = (T)(imu * cW);
      aN[r] = (T)(imu * cN);
      aS[r] = (T)(imu * cS);
      const T vi = pi ? (T)0 : uc;
      const T vE = (fE & F_P) ? (T)0 : uE;
      const T vW = (fW & F_P) ? (T)0 : uW;
      const T vN = (fN & F_P) ? (T)0 : uN;
      const T vS = (fS & F_P) ? (T)0 : uS;
      w[r] = aE[r] * (vi - vE) + aW[r] * (vi - vW) + aN[r] * (vi - vN) + aS[r] * (vi - vS);
    }
  }
  if (tid == 0) q0[len] = q1[len] = (T)0;            // slot read for absent / non-P neighbours
  __syncthreads();

  // Substep m: d_m+1 = (1 + beta_m) d_m - beta_m d_m-1 - c_m (w + A_u q_m) with
  // d_0 = d_-1 = 0 and beta_0 = 0 (so m = 0 gives -c_0 (w + A_u q_0)), and
  // q_m+1 = P (u_n + d_m+1).  At even m, d0 holds d_m and d1 d_m-1 (overwritten
  // by d_m+1); at odd m the roles swap.
  auto substep = [&](int m, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    T* dc = B == 0 ? d0 : d1;          // d_m
    T* dq = B == 0 ? d1 : d0;          // d_m-1 in, d_m+1 out
    const T c = (T)cf[1 + m];          // c1 for m = 0, c2_m otherwise
    const T b = m > 0 ? (T)L.beta[m] : (T)0;
    const char* rq = reinterpret_cast<const char*>(B == 0 ? q0 : q1);
    T* wq = B == 0 ? q1 : q0;
    const int reach = p - 1 - m;
#pragma unroll
    for (int r = 0; r < kNPT; ++r) {
      if (dd[r] > reach) continue;
      const T qi = pm[r] * (u[r] + dc[r]);
      const T qE = *reinterpret_cast<const T*>(rq + ad[r][0]);
      const T qW = *reinterpret_cast<const T*>(rq + ad[r][1]);
      const T qN = *reinterpret_cast<const T*>(rq + ad[r][2]);
      const T qS = *reinterpret_cast<const T*>(rq + ad[r][3]);
      const T apq = aE[r] * (qi - qE) + aW[r] * (qi - qW) + aN[r] * (qi - qN) + aS[r] * (qi - qS);
      const T rr = w[r] + apq;
      const T dn = ((T)1 + b) * dc[r] - b * dq[r] - c * rr;
      dq[r] = dn;
      if (m + 1 < p) wq[tid + r * NT] = pm[r] * (u[r] + dn);
      if (ADJ && dd[r] == 0 && pm[r] != (T)0)
        st.Dout[(size_t)m * st.dstride + (size_t)s * a.sstride + (size_t)kk[r]] = (double)dn;
    }
    if (m + 1 < p) __syncthreads();
  };
  int m = 0;
  for (; m + 1 < p; m += 2) {
    substep(m, std::integral_constant<int, 0>{});
    substep(m + 1, std::integral_constant<int, 1>{});
  }
  if (m < p) substep(m, std::integral_constant<int, 0>{});
  if (ADJ && st.Unew == nullptr) return;
  const T* dfin = (p & 1) ? d1 : d0;   // d_p
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    if (dd[r] != 0) continue;          // written back by the tile that owns the node
    const size_t k = (size_t)kk[r];
    uw_g[k] = st.startup ? (u[r] + dfin[r]) : ((T)2 * u[r] - uo_g[k] + (T)2 * dfin[r]);
  }
}

// Reverse sweep of the adjoint on one compact tile (FP64).  For y = u_n and
// mu = mu_n+1 with Lambda_p = f M mu, Lambda_p+1 = 0:
//   Lambda_m = (1 + beta_m) Lambda_m+1 - c2_m P K (Lambda_m+1 / m) - beta_m+1 Lambda_m+2
// at the nodes of P (m = p-1 .. 1), and lw = -c1 Lambda_1 - sum_{m=1}^{p-1} c2_m Lambda_m+1.
// Off P no stencil acts, so Lambda_m / m = rho_m f mu there: a neighbour that is
// not in P is read as rho_m+1 f mu from global memory (loaded once), a
// neighbour in P from LDS (two buffers of Lambda / m).  Lambda_m at a node at
// distance D is exact when D <= m (it reads Lambda_m+1 within D + 1 <= p), so
// step m updates the distance prefix D <= m, and the tile's own nodes of P
// store Lambda_1 .. Lambda_p-1 and lw.
struct AdjRevArgs {
  const double* __restrict__ MU;     // mu_n+1 of sample s at MU + s*sstride
  double* __restrict__ Lam1;         // Lambda_m of sample s at Lam1 + (m-1)*astride + s*sstride
  double* __restrict__ LW;
  const double* __restrict__ rho;    // rho_m, m = 1..p
  size_t astride;
  double f;
};

template <int NT>
__device__ __forceinline__ void adj_rev_compact(const StepArgs& a, const AdjRevArgs& x, const double* __restrict__ lk,
                                                double* __restrict__ lq, int s, int tile) {
  constexpr int kCap = NT * kNPT;
  const int tid = threadIdx.x;
  const LevelView& L = a.L;
  const int4 tl = a.tiles[tile];
  const int len = tl.y;
  const int ix0 = tl.z & 0xFFFF, ix1 = tl.z >> 16, iy0 = tl.w & 0xFFFF, iy1 = tl.w >> 16;
  const int p = L.p;
  const size_t so = (size_t)s * a.sstride;
  const double* __restrict__ mu = x.MU + so;
  const double* __restrict__ cf = a.coef + (size_t)s * (p + 1);
  double* const t0 = lq;                // Lambda / m of the even steps' inputs (m + 1 = p, p - 2, ...)
  double* const t1 = lq + (kCap + 1);   // and of the odd ones'; slot len of each holds 0
  double l1[kNPT], l2[kNPT], im[kNPT], lw[kNPT], cE[kNPT], cW[kNPT], cN[kNPT], cS[kNPT];
  uint32_t pmask = 0;                  // bit r: region node r of this lane is in P
  double co[kNPT];                     // sum over the neighbours off P of c_k f mu_k (rho-free)
  uint32_t ad[kNPT][4];
  int kk[kNPT], dd[kNPT];
  int4 en[kNPT];
#pragma unroll
  for (int r = 0; r < kNPT; ++r) en[r] = a.ent[tl.x + min(tid + r * NT, len - 1)];
  const int ld = L.ld;
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    l1[r] = l2[r] = im[r] = lw[r] = 0.0;
    cE[r] = cW[r] = cN[r] = cS[r] = co[r] = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) ad[r][t] = (uint32_t)(len * sizeof(double));
    kk[r] = 0;
    dd[r] = p + 1;                     // never updated, never written
    const int e = tid + r * NT;
    if (e < len) {
      const size_t k = (size_t)(en[r].x & 0x7FFFFFFF);
      const bool pi = en[r].x < 0;
      const int i = en[r].w & 0xFFFF, j = en[r].w >> 16;
      kk[r] = (int)k;
      ad[r][0] = (uint32_t)(en[r].y & 0xFFFF) * sizeof(double);
      ad[r][1] = ((uint32_t)en[r].y >> 16) * sizeof(double);
      ad[r][2] = (uint32_t)(en[r].z & 0xFFFF) * sizeof(double);
      ad[r][3] = ((uint32_t)en[r].z >> 16) * sizeof(double);
      dd[r] = max(max(ix0 - i, i - (ix1 - 1)), 0) + max(max(iy0 - j, j - (iy1 - 1)), 0);
      const uint8_t fE = L.flags[k + 1], fW = L.flags[k - 1], fN = L.flags[k + ld], fS = L.flags[k - ld];
      const double mk = mu[k], mE = mu[k + 1], mW = mu[k - 1], mN = mu[k + ld], mS = mu[k - ld];
      double ce, cw, cn, cs;
      edge_coefs(L, lk, i, j, ce, cw, cn, cs);
      cE[r] = ce;
      cW[r] = cw;
      cN[r] = cn;
      cS[r] = cs;
      co[r] = ce * ((fE & F_P) ? 0.0 : x.f * mE) + cw * ((fW & F_P) ? 0.0 : x.f * mW) +
              cn * ((fN & F_P) ? 0.0 : x.f * mN) + cs * ((fS & F_P) ? 0.0 : x.f * mS);
      im[r] = L.invm[k];
      if (pi) pmask |= 1u << r;
      l1[r] = pi && im[r] != 0.0 ? x.f * mk / im[r] : 0.0;   // Lambda_p
      t0[e] = pi ? x.f * mk : 0.0;                            // Lambda_p / m
    }
  }
  if (tid == 0) t0[len] = t1[len] = 0.0;
  __syncthreads();
  // Step m (m = p-1 .. 1): Lambda_m from Lambda_m+1 (l1 in, out) and
  // Lambda_m+2 (l2), reading Lambda_m+1 / m of the neighbours in P from
  // buffer B and writing Lambda_m / m to the other.  The roles of l1 / l2 and
  // of the buffers alternate, fixed per call.
  auto step = [&](int m, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    double* lc = B == 0 ? l1 : l2;     // Lambda_m+1
    double* lo = B == 0 ? l2 : l1;     // Lambda_m+2 in, Lambda_m out
    const char* rq = reinterpret_cast<const char*>(B == 0 ? t0 : t1);
    double* wq = B == 0 ? t1 : t0;
    const double c2 = cf[1 + m];
    const double bm = L.beta[m];
    const double bm1 = m + 1 < p ? L.beta[m + 1] : 0.0;
    const double r1 = x.rho[m + 1];
#pragma unroll
    for (int r = 0; r < kNPT; ++r) {
      if (dd[r] > m || !(pmask & (1u << r))) continue;
      const double lam = lc[r];
      lw[r] -= c2 * lam;
      const double ti = lam * im[r];
      // neighbours in P from LDS (0 for the others), those off P through co
      const double tE = *reinterpret_cast<const double*>(rq + ad[r][0]);
      const double tW = *reinterpret_cast<const double*>(rq + ad[r][1]);
      const double tN = *reinterpret_cast<const double*>(rq + ad[r][2]);
      const double tS = *reinterpret_cast<const double*>(rq + ad[r][3]);
      const double kt = cE[r] * (ti - tE) + cW[r] * (ti - tW) + cN[r] * (ti - tN) + cS[r] * (ti - tS) - r1 * co[r];
      const double ln = (1.0 + bm) * lam - c2 * kt - bm1 * lo[r];
      lo[r] = ln;
      if (m > 1) wq[tid + r * NT] = ln * im[r];
      if (dd[r] == 0) x.Lam1[(size_t)(m - 1) * x.astride + so + (size_t)kk[r]] = ln;
    }
    if (m > 1) __syncthreads();
  };
  int m = p - 1;
  for (; m >= 2; m -= 2) {
    step(m, std::integral_constant<int, 0>{});
    step(m - 1, std::integral_constant<int, 1>{});
  }
  if (m == 1) step(1, std::integral_constant<int, 0>{});
  // Lambda_1 is in l2 when p - 1 is odd (p even), else in l1
  const bool in_l2 = ((p - 1) & 1) != 0;
  const double c1 = cf[1];
#pragma unroll
  for (int r = 0; r < kNPT; ++r) {
    if (dd[r] != 0 || !(pmask & (1u << r))) continue;
    const double lam1 = p == 1 ? l1[r] : (in_l2 ? l2[r] : l1[r]);
    x.LW[so + (size_t)kk[r]] = lw[r] - c1 * lam1;
  }
}


// Rect mode.  A tile's region is a rectangle of RX x RY <= 64 x 64 grid nodes
// (the tile grown by p, clipped to the grid and to the bounding box of its F+
// nodes grown by one).  Lane x of wavefront v owns column x and the four
// vertically adjacent rows 4v .. 4v+3, all in registers: east / west
// neighbours come from the adjacent lanes by DPP wavefront shifts (lanes 0 and
// 63 read 0, the zero ring of the region), north / south neighbours inside the
// four rows from the lane's own registers, and only the rows next to another
// wavefront's go through LDS, where each wavefront publishes its top and
// bottom row (two buffers: substep m reads buffer m & 1 and writes the other;
// zero rows above wavefront 0 and below the last).  Lanes and rows outside the
// rectangle hold zeros.  The tile descriptor is x = x0 | y0 << 16 (region
// origin), y = RX | RY << 16, z = ix0 | ix1 << 16, w = iy0 | iy1 << 16 (tile
// interior [ix0, ix1) x [iy0, iy1)).  All global reads of a tile are issued in
// one batch before the first barrier.  w = A_u (I - P) u_n is formed from
// v = (I - P) u_n the same way.  A node next to the region border sees zeros
// beyond it instead of the true values of v and q: the same one-node-per-
// substep error front as for q alone, so the tile interior (at distance >= p
// from the border) stays exact.
// UNROLL = false: the substep loop is never unrolled and no substep scalar is
// preloaded (fewer scalar registers; the persistent kernel's choice).
template <class T, bool UNROLL = true>
__device__ __forceinline__ void fine_tile_rect(const StepArgs& a, const StepState& st, double* __restrict__ lk,
                                               T* __restrict__ lq, T* __restrict__ ls, int s, int tile,
                                               int tid_in = -1) {
  constexpr int R = 4;                                  // rows per lane
  constexpr int W = 64;                                 // boundary-row buffer pitch
  const LevelView& L = a.L;
  const int4 td = a.rtiles[tile];
  const int x0 = td.x & 0xFFFF, y0 = td.x >> 16;
  const int RX = td.y & 0xFFFF, RY = td.y >> 16;
  const int ix0 = td.z & 0xFFFF, ix1 = td.z >> 16, iy0 = td.w & 0xFFFF, iy1 = td.w >> 16;
  const int tid = tid_in < 0 ? (int)threadIdx.x : tid_in;
  const int x = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int yb = 4 * wv;                                // first row of this wavefront
  const bool wave_on = yb < RY;                         // wavefront holds region rows
  const int gx = x0 + x;
  const bool col_on = x < RX && gx < L.nxn;
  const T* __restrict__ u_g = reinterpret_cast<const T*>(st.Ucur) + (size_t)s * a.sstride;
  T* __restrict__ uo_g = reinterpret_cast<T*>(st.Uold) + (size_t)s * a.sstride;
  T* uw_g = reinterpret_cast<T*>(st.Unew) + (size_t)s * a.sstride;
  const double* __restrict__ cf = a.coef + (size_t)s * (L.p + 1);
  const bool startup = st.startup;
  const int ld = L.ld;
  const int p = L.p;                                    // <= 64 in rect mode

  // ---- the substep scalars of the unrolled refinement ratios (p = 4, 8),
  //      read before anything else: the substeps then wait on LDS only
  constexpr int kPre = 8;
  double c_pre[kPre], b_pre[kPre];
  if (UNROLL && (p == 4 || p == 8)) {
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
      c_pre[m] = m < p ? cf[1 + m] : 0.0;
      b_pre[m] = m > 0 && m < p ? L.beta[m] : 0.0;
    }
  }
  // ---- one batch of global reads (nothing read here decides another read)
  const double kv = tid < L.nb ? a.kappa[(size_t)s * L.nb + tid] : 0.0;
  const int gxc = min(gx, L.nxn - 1);                  // column, in bounds off the grid
  const int gxw = max(gxc - 1, 0);
  const double hxE = L.hx[gxc], hxW = L.hx[gxw];
  const double ihE = L.inv2hx[gxc];
  const int gyb = y0 + yb;
  double hyv[R + 1], ihy[R + 1];                       // rows gy-1 .. gy+3 (wavefront-uniform)
  uint32_t ni[R + 1];                                  // node words of rows gy-1 .. gy+3
#pragma unroll
  for (int q = 0; q <= R; ++q) {
    const int g = min(max(gyb - 1 + q, 0), L.nyn - 1);
    hyv[q] = L.hy[g];
    ihy[q] = L.inv2hy[g];
    ni[q] = L.ninfo[g * ld + gxc];
  }
  // u_n-1 enters only the update of the written-back nodes: it is read at the
  // tile interior only (the halo is 43 % of a 64 x 64 region at p = 8)
  const bool col_in = gx >= ix0 && gx < ix1;
  T u[R], uo[R];
  double im[R];
  uint32_t f[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool ok = wave_on && col_on && yb + r < RY && gyb + r < L.nyn;
    const int k = ok ? (gyb + r) * ld + gx : ld + 1;
    u[r] = ok ? u_g[k] : (T)0;
    im[r] = L.invm[k];
    const bool in = ok && col_in && gyb + r >= iy0 && gyb + r < iy1;
    uo[r] = (startup || !in) ? (T)0 : uo_g[k];
    f[r] = ok ? ni[r + 1] & 0xFFu : 0u;
  }
  // ---- LDS: kappa table (zero past the last block, so that the missing cells
  //      off the grid read 0), boundary rows of q_0 = P u (buffer 0) and of
  //      v = (I - P) u (buffer 1), the zero rows
  T* const lb0 = lq;
  T* const lb1 = lq + kBndSlots;
  const int top = (2 * wv + 1) * W + x, bot = (2 * wv + 2) * W + x;   // this wavefront's rows
  const int below = 2 * wv * W + x, above = (2 * wv + 3) * W + x;     // neighbours' rows
  if (tid < 256) lk[tid] = kv;
  T up[R], pm[R], v[R + 2];                            // v of rows gy-1 .. gy+4
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool pi = f[r] & F_P;
    up[r] = pi ? u[r] : (T)0;
    pm[r] = pi ? (T)1 : (T)0;
    v[r + 1] = u[r] - up[r];
  }
  lb0[top] = up[0];
  lb0[bot] = up[R - 1];
  lb1[top] = v[1];
  lb1[bot] = v[R];
  if (tid < 4 * W) {                                   // zero rows 0 and kBndRows - 1
    const int z = (tid & (2 * W - 1)) < W ? (tid & (W - 1)) : (kBndRows - 1) * W + (tid & (W - 1));
    (tid < 2 * W ? lb0 : lb1)[z] = (T)0;
  }
  __syncthreads();

  // ---- scaled edge coefficients and w = A_u (I - P) u_n
  T aE[R], aW[R], aN[R], aS[R], w[R], q[R];
  uint32_t wmask = 0;                                  // bit r: row r is written back
  {
    double kE[R + 1], kW[R + 1];                       // kappa of the cells east / west of the node
#pragma unroll
    for (int c = 0; c <= R; ++c) {
      kE[c] = lk[(ni[c] >> 8) & 0xFFu];
      kW[c] = lk[(ni[c] >> 16) & 0xFFu];
    }
    // vertical edges: row r's south edge is row r-1's north edge (same value)
    double cV[R + 1];
#pragma unroll
    for (int c = 0; c <= R; ++c) cV[c] = (kE[c] * hxE + kW[c] * hxW) * ihy[c];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool fp = f[r] & F_FPLUS;
      const double imf = fp ? im[r] : 0.0;             // coefficients vanish off F+
      // a node's west edge is its west neighbour's east edge (same value)
      const double cE = (kE[r + 1] * hyv[r + 1] + kE[r] * hyv[r]) * ihE;
      const double cW = lane_prev(cE);
      aE[r] = (T)(imf * cE);
      aW[r] = (T)(imf * cW);
      aN[r] = (T)(imf * cV[r + 1]);
      aS[r] = (T)(imf * cV[r]);
      if (fp && col_in && gyb + r >= iy0 && gyb + r < iy1) wmask |= 1u << r;
      q[r] = up[r];
      ls[r * kFineThreads + tid] = startup ? u[r] : (T)2 * u[r] - uo[r];   // this lane's own slots
    }
    v[0] = lb1[below];
    v[R + 1] = lb1[above];
    T dN[R + 1];                                       // dN[c] = v of row c-1 minus v of row c
#pragma unroll
    for (int c = 0; c <= R; ++c) dN[c] = v[c] - v[c + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T dE = v[r + 1] - lane_next(v[r + 1]);
      const T dWn = lane_prev(dE);
      w[r] = aS[r] * -dN[r] + (aN[r] * dN[r + 1] + (aW[r] * -dWn + aE[r] * dE));
    }
  }
  __syncthreads();   // buffer 1 is overwritten by the first substep

  // Substep m reads buffer B = m & 1 and writes buffer 1 - B.  The increments
  // d_m+1 and d_m-1 share a register: at even m, d0 holds d_m and d1 d_m-1
  // (overwritten by d_m+1); at odd m the roles swap, so no copies are needed.
  T d0[R], d1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) d0[r] = d1[r] = (T)0;
  auto substep = [&](int m, auto Bc, auto Pc) {
    constexpr int B = decltype(Bc)::value;
    constexpr bool PRE = decltype(Pc)::value;
    T* dc = B == 0 ? d0 : d1;       // d_m
    T* dq = B == 0 ? d1 : d0;       // d_m-1 in, d_m+1 out
    // c1 for m = 0, c2_m otherwise, and beta_m (preloaded, or scalar loads)
    const T c = PRE ? (T)c_pre[m] : (T)cf[1 + m];
    const T b = PRE ? (T)b_pre[m] : m > 0 ? (T)L.beta[m] : (T)0;
    // d_m+1 is needed only within distance p-1-m of the tile interior (it
    // reaches the interior through p-1-m more stencil applications); a
    // wavefront whose rows all lie farther out skips the substep.  Rows it
    // leaves stale are read only by rows that are themselves outside the next
    // band, so stale values never reach the interior.
    const int reach = p - 1 - m;
    if (wave_on && gyb + R > iy0 - reach && gyb < iy1 + reach) {
      const T* rb = B == 0 ? lb0 : lb1;
      T* wb = B == 0 ? lb1 : lb0;
      // edge form: K q at a node is the sum of c_k (q_i - q_k), so constants
      // are annihilated exactly.  Each difference is formed once: the west
      // difference of a node is minus the east difference of its west
      // neighbour (one DPP shift), the south one minus the north one of the
      // row below.
      T dN[R + 1];                                     // dN[r + 1] = q_r - q_r+1, dN[0] = q_-1 - q_0
      const T qb = rb[below], qa = rb[above];          // LDS: the neighbouring wavefronts' rows
      __builtin_amdgcn_sched_barrier(0);               // issue the LDS read before the inner rows
#pragma unroll
      for (int r = 0; r + 1 < R; ++r) dN[r + 1] = q[r] - q[r + 1];
      T qn[R];
      // the inner rows first: they need no LDS value, so the LDS read of the
      // boundary rows completes behind their arithmetic
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int r = k + 1 < R - 1 ? k + 1 : (k == R - 2 ? 0 : R - 1);   // 1, 2, .., R-2, 0, R-1
        if (k == R - 2) __builtin_amdgcn_sched_barrier(0);   // the LDS values are used from here on
        if (r == 0) dN[0] = qb - q[0];
        if (r == R - 1) dN[R] = q[R - 1] - qa;
        const T dE = q[r] - lane_next(q[r]);
        const T dWn = lane_prev(dE);                   // q_x-1 - q_x
        const T rr = aS[r] * -dN[r] + (aN[r] * dN[r + 1] + (aW[r] * -dWn + (aE[r] * dE + w[r])));
        const T dn = (dc[r] + b * (dc[r] - dq[r])) - c * rr;
        dq[r] = dn;
        qn[r] = pm[r] * dn + up[r];          // P (u_n + d_m+1): u_n + d exactly on P, 0 elsewhere
      }
#pragma unroll
      for (int r = 0; r < R; ++r) q[r] = qn[r];
      if (m + 1 < p) {
        wb[top] = q[0];
        wb[bot] = q[R - 1];
      }
    }
    if (m + 1 < p) __syncthreads();
  };
  // fully unrolled for the common refinement ratios (constant substep index:
  // no loop control, scheduling across substeps), a loop otherwise
  auto unrolled = [&](auto Pc) {
    constexpr int PP = decltype(Pc)::value;
    static_assert(PP <= kPre, "preloaded scalars");
#pragma unroll
    for (int m = 0; m < PP; m += 2) {
      substep(m, std::integral_constant<int, 0>{}, std::true_type{});
      substep(m + 1, std::integral_constant<int, 1>{}, std::true_type{});
    }
  };
  if (UNROLL && p == 8) {
    unrolled(std::integral_constant<int, 8>{});
  } else if (UNROLL && p == 4) {
    unrolled(std::integral_constant<int, 4>{});
  } else {
    for (int m = 0; m < p; m += 2) {
      substep(m, std::integral_constant<int, 0>{}, std::false_type{});
      if (m + 1 < p) substep(m + 1, std::integral_constant<int, 1>{}, std::false_type{});
    }
  }
  T d[R];
#pragma unroll
  for (int r = 0; r < R; ++r) d[r] = (p & 1) ? d1[r] : d0[r];   // d_p
  const T ds = startup ? (T)1 : (T)2;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (wmask & (1u << r)) uw_g[(gyb + r) * ld + gx] = ls[r * kFineThreads + tid] + ds * d[r];
}

template <bool RECT, class T>
__global__ __launch_bounds__(kFineThreads) void k_fine(StepArgs a) {
  __shared__ T lq[RECT ? kLdsSlots : kCompactSlots];
  __shared__ T ls[RECT ? 4 * kFineThreads : 1];   // rect mode: final-update term per node
  __shared__ double lk[256];
  const int G = a.n_fine * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  const int s = a.s0 + Lid / a.n_fine;
  if (RECT) {
    fine_tile_rect<T>(a, StepState{a.Ucur, a.Uold, a.Unew, a.startup}, lk, lq, ls, s, Lid % a.n_fine);
  } else {
    load_kappa(a, s, lk);
    fine_tile_compact<T, kFineThreads>(a, StepState{a.Ucur, a.Uold, a.Unew, a.startup}, lk, lq, s,
                                       Lid % a.n_fine, (int)threadIdx.x, true);
  }
}

// Coarse items and rect-mode fine tiles of one step in one launch of
// 1024-thread workgroups: n_fw fine workgroups (tile, sample) and n_cw coarse
// workgroups of four items each, interleaved evenly over the launch order, so
// that the coarse items' HBM stream runs while other CUs do the fine tiles'
// substeps (back to back, the coarse launch leaves the VALUs idle and the fine
// launch leaves HBM idle).  Each XCD takes a contiguous part of the order, as
// in the separate launches.
template <class T>
__global__ __launch_bounds__(kFineThreads) void k_step_mix(StepArgs a, int n_fw, int n_cw) {
  __shared__ T lq[kLdsSlots];
  __shared__ T ls[4 * kFineThreads];
  __shared__ double lk[4 * 256];
  const int N = n_fw + n_cw;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= N) return;
  const long long c0 = (long long)Lid * n_cw / N, c1 = (long long)(Lid + 1) * n_cw / N;
  const StepState st{a.Ucur, a.Uold, a.Unew, a.startup};
  const int tid = (int)threadIdx.x;
  if (c1 > c0) {
    // coarse workgroup c0: slots 4 c0 .. 4 c0 + 3 of the (item, sample) order
    const int gi = __builtin_amdgcn_readfirstlane(tid >> 8), slot = 4 * (int)c0 + gi;   // whole wavefronts
    const bool on = slot < a.n_coarse * a.active;
    int item = 0, s = 0;
    if (on) coarse_order(slot, a.n_coarse, a.active, item, s);
    coarse_body<T>(a, st, lk + 256 * gi, a.s0 + s, item, tid & 255, on);
  } else {
    const int f = Lid - (int)c0;                       // fine workgroup: sample-major (sample, tile)
    const int s = f / a.n_fine;
    fine_tile_rect<T>(a, st, lk, lq, ls, a.s0 + s, f - s * a.n_fine);
  }
}

// Compact tiles whose regions fit NT * kNPT < kRegionCap nodes: smaller
// workgroups, several per CU.
template <class T, int NT>
__global__ __launch_bounds__(NT) void k_fine_small(StepArgs a) {
  __shared__ T lq[2 * (NT * kNPT + 1)];
  __shared__ double lk[256];
  const int G = a.n_fine * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  const int s = a.s0 + Lid / a.n_fine;
  load_kappa(a, s, lk);
  fine_tile_compact<T, NT>(a, StepState{a.Ucur, a.Uold, a.Unew, a.startup}, lk, lq, s, Lid % a.n_fine,
                           (int)threadIdx.x, true);
}

template <bool RECT, class T>
__global__ __launch_bounds__(kFineThreads) void k_fine_multi(MultiArgs m) {
  __shared__ T lq[RECT ? kLdsSlots : kCompactSlots];
  __shared__ T ls[RECT ? 4 * kFineThreads : 1];
  __shared__ double lk[256];
  int j, local, n;
  if (!multi_slot(m, j, local, n)) return;
  const StepArgs a = job_record(m.jobs[j]);
  const StepState st = job_state(m, a);
  const int s = local / a.n_fine;
  if (RECT) {
    fine_tile_rect<T>(a, st, lk, lq, ls, s, local % a.n_fine);
  } else {
    load_kappa(a, s, lk);
    fine_tile_compact<T, kFineThreads>(a, st, lk, lq, s, local % a.n_fine, (int)threadIdx.x, true);
  }
}

template <class T, int NT>
__global__ __launch_bounds__(NT) void k_fine_small_multi(MultiArgs m) {
  __shared__ T lq[2 * (NT * kNPT + 1)];
  __shared__ double lk[256];
  int j, local, n;
  if (!multi_slot(m, j, local, n)) return;
  const StepArgs a = job_record(m.jobs[j]);
  const int s = local / a.n_fine;
  load_kappa(a, s, lk);
  fine_tile_compact<T, NT>(a, job_state(m, a), lk, lq, s, local % a.n_fine, (int)threadIdx.x, true);
}

// The thread index as a value the compiler cannot see through: everything a
// loop iteration derives from it is recomputed there instead of being hoisted
// out of the persistent loops and kept in registers across every unit.
__device__ __forceinline__ int opaque_tid() {
  int v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "v"((int)threadIdx.x));
  return v;
}

// The adjoint's two substep sweeps of one backward step on compact tiles:
// the forward recompute (the increments d_1 .. d_p at the nodes of P) and the
// reverse sweep (Lambda_1 .. Lambda_p-1 and lw at the nodes of P).  One
// workgroup per (sample, tile); each tile writes its own nodes of P.
template <int NT>
__global__ __launch_bounds__(NT) void k_adj_fsweep(StepArgs a, StepState st) {
  __shared__ double lq[2 * (NT * kNPT + 1)];
  __shared__ double lk[256];
  const int G = a.n_fine * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  const int s = Lid / a.n_fine;
  load_kappa(a, s, lk);
  fine_tile_compact<double, NT, true>(a, st, lk, lq, s, Lid % a.n_fine, (int)threadIdx.x, true);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_adj_rsweep(StepArgs a, AdjRevArgs x) {
  __shared__ double lq[2 * (NT * kNPT + 1)];
  __shared__ double lk[256];
  const int G = a.n_fine * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  const int s = Lid / a.n_fine;
  load_kappa(a, s, lk);
  adj_rev_compact<NT>(a, x, lk, lq, s, Lid % a.n_fine);
}

// ---------------------------------------------------------------------------
// Persistent form: one cooperative launch of one 1024-thread workgroup per CU
// advances every job through steps t0 .. t1-1, with a grid-wide barrier after
// each step (the fine tiles of step t+1 read the halo that other workgroups
// wrote in step t).
//
// Work of a step.  A unit is one workgroup's share: a rect-mode fine tile of
// one sample; S_b = 1024 / nt compact tiles (nt = 256, 512 or 1024 threads
// each) of one tile position for S_b consecutive samples, side by side in the
// workgroup's thread groups; or four coarse items.  The workgroups form ng
// groups (one per XCD: the hardware hands workgroup b to XCD b mod 8); each
// group works through its own eighth of every job's units (the fine units of
// the jobs in order of cost, then the coarse ones), as the per-step launches
// split them, so that neighbouring tiles stay in one L2.  Inside a group the
// units are handed out by an atomic counter: a workgroup takes the next index
// before starting a unit.  An index past the end of step t belongs to a later
// step; the workgroup keeps it across the barrier, so no index is lost and the
// counter never needs a reset within the launch.
//
// The barrier counts arrivals in two levels: per group, and the last arrival
// of a group at its k-th barrier of the launch (the k x group size-th) bumps a
// global counter that every workgroup waits on (k x ng), so that no counter
// takes more than one group's atomics.  Each workgroup makes its own stores
// visible with a release fence at device scope before it arrives and acquires
// after the wait.  The wait is bounded: a workgroup that waits longer than
// spin_ticks of the constant wall clock (or kSpinMax polls) sets the abort
// word, and every workgroup leaves at its next barrier, so the launch always
// ends; the host then reports the abort.
constexpr int kCtlUnit = 0, kCtlGroup = 256, kCtlGlobal = 512, kCtlAbort = 528, kCtlWords = 544;
struct PersistArgs {
  const StepArgs* __restrict__ jobs;
  const int* __restrict__ act;       // [t][n_jobs]: active samples of job j at step t
  unsigned* ctl;                     // words kCtlUnit + 16 x: unit counter of group x; kCtlGroup + 16 x:
                                     // its barrier arrivals; kCtlGlobal: groups arrived; kCtlAbort
  long long spin_ticks;
  int n_jobs, t0, t1, ng;
  int order[kMaxJobs];               // job at segment position q
  int sb[kMaxJobs];                  // per job: 0 rect mode, else S_b (compact, 1024 / S_b threads per tile)
  int nf[kMaxJobs], nc[kMaxJobs];    // per job: fine tiles and coarse items per sample
};

constexpr int kPersistThreads = 1024;
constexpr unsigned kSpinMax = 1u << 24;
constexpr int kPersistLds = 4 * (256 + 2 * (256 * kNPT + 1));   // doubles: the largest carve (4 x nt = 256)
static_assert(kPersistLds >= 256 + kLdsSlots + 4 * kFineThreads, "rect mode carve");
static_assert(kPersistLds >= 256 + kCompactSlots, "compact 1024 carve");
static_assert(kPersistLds >= 2 * (256 + 2 * (512 * kNPT + 1)), "compact 512 carve");

// k-th barrier of the launch for a workgroup of group x (ng groups; per_group
// workgroups in group x).
__device__ __forceinline__ bool step_barrier(unsigned* ctl, int x, unsigned per_group, unsigned ng, unsigned k,
                                             long long spin_ticks, int* s_ok) {
  // every wavefront's stores have reached the L2 before the workgroup barrier;
  // one release fence then writes the L2 back for the other XCDs (a fence per
  // wavefront would repeat that write-back sixteen times)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* glob = ctl + kCtlGlobal;
    unsigned* abort_w = ctl + kCtlAbort;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned old = __hip_atomic_fetch_add(ctl + kCtlGroup + 16 * x, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u == k * per_group) __hip_atomic_fetch_add(glob, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = k * ng;
    const long long t_start = wall_clock64();
    int ok = 1;
    for (unsigned n = 0;; ++n) {
      if (__hip_atomic_load(glob, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = 0;
        break;
      }
      if (wall_clock64() - t_start > spin_ticks || n >= kSpinMax) {
        __hip_atomic_store(abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the other workgroups' stores after it
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

template <class T, int NT>
__device__ __forceinline__ void persist_compact(const StepArgs& a, const StepState& st, double* __restrict__ smem,
                                                int act, int idx, int tid) {
  constexpr int G = kPersistThreads / NT;               // S_b: samples side by side
  constexpr int per = 256 + (2 * (NT * kNPT + 1) * (int)sizeof(T) + 7) / 8;   // doubles per thread group
  const int gi = __builtin_amdgcn_readfirstlane(tid / NT), gt = tid % NT;   // groups are whole wavefronts
  const int sg = idx / a.n_fine, tile = idx - sg * a.n_fine;
  const int s = sg * G + gi;
  const bool on = s < act;
  const int sv = on ? s : sg * G;                        // a valid sample for the idle groups' scalars
  double* lk = smem + gi * per;
  T* lq = reinterpret_cast<T*>(lk + 256);
  if (on)
    for (int t = gt; t < a.L.nb; t += NT) lk[t] = a.kappa[(size_t)s * a.L.nb + t];
  __syncthreads();
  fine_tile_compact<T, NT>(a, st, lk, lq, sv, tile, gt, on);
}

template <class T>
__global__ __launch_bounds__(kPersistThreads) void k_persist(PersistArgs pa) {
  __shared__ double smem[kPersistLds];
  __shared__ int seg_end[2 * kMaxJobs], seg_lo[2 * kMaxJobs], seg_act[2 * kMaxJobs];
  __shared__ unsigned s_idx;
  __shared__ int s_ok;
  const int nj = pa.n_jobs, nseg = 2 * nj;
  const int x = (int)(blockIdx.x % (unsigned)pa.ng);
  const unsigned per_group = (gridDim.x - (unsigned)x + (unsigned)pa.ng - 1u) / (unsigned)pa.ng;
  unsigned* cnt = pa.ctl + kCtlUnit + 16 * x;
  if (threadIdx.x == 0) s_idx = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned base = 0;
  // active samples of this lane's segment job at the current step (wavefront
  // 0; the next step's are read before each barrier)
  int a_cur = 0;
  if (threadIdx.x < (unsigned)nseg) {
    const int l = threadIdx.x;
    a_cur = pa.act[(size_t)pa.t0 * nj + pa.order[l < nj ? l : l - nj]];
  }
  for (int t = pa.t0; t < pa.t1; ++t) {
    const int tid = opaque_tid();
    // segments of this step for group x: position q < nj the fine units of
    // job order[q], q >= nj the coarse ones; units split into ng chunks
    if (tid < 64) {
      int len = 0, lo = 0, a = 0;
      if (tid < nseg) {
        const int q = tid < nj ? tid : tid - nj;
        const int j = pa.order[q];
        a = a_cur;
        int units;
        if (tid < nj) {
          const int g = pa.sb[j] > 0 ? pa.sb[j] : 1;
          units = pa.nf[j] * ((a + g - 1) / g);
        } else {
          units = (pa.nc[j] * a + 3) / 4;
        }
        const int ch = (units + pa.ng - 1) / pa.ng;
        lo = min(x * ch, units);
        len = min(lo + ch, units) - lo;
      }
      int v = len;                                      // inclusive scan over the wavefront
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int w = __builtin_amdgcn_ds_bpermute((tid - o) << 2, v);   // lane tid - o (wraps; masked)
        if (tid >= o) v += w;
      }
      if (tid < nseg) {
        seg_end[tid] = v;
        seg_lo[tid] = lo;
        seg_act[tid] = a;
      }
    }
    __syncthreads();
    const unsigned U = (unsigned)__builtin_amdgcn_readfirstlane(seg_end[nseg - 1]);
    unsigned g = __builtin_amdgcn_readfirstlane(s_idx);
    while (g - base < U && g >= base) {
      const int tid = opaque_tid();
      const int u = (int)(g - base);
      __syncthreads();                                   // everyone has read s_idx
      unsigned nxt = 0;
      if (tid == 0) nxt = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int k0 = 0, k1 = nseg - 1;                         // first segment with seg_end > u
      while (k0 < k1) {
        const int mid = (k0 + k1) >> 1;
        if (seg_end[mid] > u) k1 = mid;
        else k0 = mid + 1;
      }
      const int k = __builtin_amdgcn_readfirstlane(k0);
      // uniform over the workgroup: scalar registers and scalar address arithmetic
      const int idx = __builtin_amdgcn_readfirstlane(seg_lo[k] + u - (k > 0 ? seg_end[k - 1] : 0));
      const int act = __builtin_amdgcn_readfirstlane(seg_act[k]);
      const int j = pa.order[k < nj ? k : k - nj];
      const StepArgs a = job_record(pa.jobs[j]);
      const bool odd = t & 1;
      const StepState st{odd ? a.B1 : a.B0, odd ? a.B0 : a.B1, odd ? a.B0 : a.B1, t == 0};
      if (k >= nj) {
        // four coarse items: slots 4 idx .. 4 idx + 3 of the job's (item, sample) order
        const int gi = __builtin_amdgcn_readfirstlane(tid >> 8), slot = 4 * idx + gi;   // whole wavefronts
        const bool on = slot < a.n_coarse * act;
        int item = 0, s = 0;
        if (on) coarse_order(slot, a.n_coarse, act, item, s);
        coarse_body<T>(a, st, smem + 256 * gi, s, item, tid & 255, on);
      } else if (pa.sb[j] == 0) {
        const int s = idx / a.n_fine;
        fine_tile_rect<T, false>(a, st, smem, reinterpret_cast<T*>(smem + 256),
                                 reinterpret_cast<T*>(smem + 256) + kLdsSlots, s, idx - s * a.n_fine, tid);
      } else if (pa.sb[j] == 4) {
        persist_compact<T, 256>(a, st, smem, act, idx, tid);
      } else if (pa.sb[j] == 2) {
        persist_compact<T, 512>(a, st, smem, act, idx, tid);
      } else {
        persist_compact<T, 1024>(a, st, smem, act, idx, tid);
      }
      __syncthreads();                                   // LDS free for the next unit
      if (tid == 0) s_idx = nxt;
      __syncthreads();
      g = __builtin_amdgcn_readfirstlane(s_idx);
    }
    base += U;
    if (t + 1 < pa.t1) {
      if (threadIdx.x < (unsigned)nseg) {
        const int l = threadIdx.x;
        a_cur = pa.act[(size_t)(t + 1) * nj + pa.order[l < nj ? l : l - nj]];
      }
      if (!step_barrier(pa.ctl, x, per_group, (unsigned)pa.ng, (unsigned)(t - pa.t0 + 1), pa.spin_ticks, &s_ok))
        return;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host: tiling of a level for a fine-tile rectangle of TX x TY nodes.

std::string build_tiling(const HostLevel& H, int ld, int TX, int TY, int ox, int oy, bool rect,
                         TilingHost& T, int cap) {
  T = TilingHost();
  T.TX = TX;
  T.TY = TY;
  T.ox = ox;
  T.oy = oy;
  T.rect = rect;
  const int nxn = H.nxn, nyn = H.nyn, p = H.p;
  if (nxn > 0xFFFF || nyn > 0xFFFF) return "grid too large for the fine-tile descriptors";
  auto fl = [&](int i, int j) -> uint8_t { return H.flags[(size_t)j * nxn + i]; };
  const int RX = TX + 2 * p, RY = TY + 2 * p;
  std::vector<int32_t> loc;
  if (rect) T.pitch = kRectW;
  size_t n_region = 0, n_fplus = 0;
  // Compact mode, one tile with interior [ix0, ix1) x [iy0, iy1): its region
  // is the F+ nodes at Manhattan distance <= p from the interior (an error made
  // at the region border moves one node per substep, so farther nodes cannot
  // reach the interior), ordered by that distance: the nodes a substep still
  // needs are then a prefix, and whole wavefronts drop out.
  auto dist_to = [](int i, int j, int ix0, int ix1, int iy0, int iy1) {
    return std::max(std::max(ix0 - i, i - (ix1 - 1)), 0) + std::max(std::max(iy0 - j, j - (iy1 - 1)), 0);
  };
  auto add_compact = [&](int ix0, int ix1, int iy0, int iy1) -> std::string {
    const int x0 = ix0 - p, y0 = iy0 - p, RX = ix1 - ix0 + 2 * p, RY = iy1 - iy0 + 2 * p;
    std::vector<std::array<int, 3>> nodes;   // (distance, j, i), row-major within a distance
    for (int j = std::max(y0, 0); j < std::min(y0 + RY, nyn); ++j)
      for (int i = std::max(x0, 0); i < std::min(x0 + RX, nxn); ++i) {
        const int d = dist_to(i, j, ix0, ix1, iy0, iy1);
        if ((fl(i, j) & LTS_NODE_FPLUS) && d <= p) nodes.push_back({d, j, i});
      }
    std::stable_sort(nodes.begin(), nodes.end(),
                     [](const std::array<int, 3>& a, const std::array<int, 3>& b) { return a[0] < b[0]; });
    const int len = (int)nodes.size();
    if (len > cap) return "fine tile region exceeds the workgroup capacity";
    loc.assign((size_t)RX * RY, -1);
    for (int l = 0; l < len; ++l) loc[(size_t)(nodes[l][1] - y0) * RX + (nodes[l][2] - x0)] = l;
    const int off = (int)T.ent.size();
    auto nb = [&](int i, int j) -> int {
      if (i < x0 || j < y0 || i >= x0 + RX || j >= y0 + RY || i < 0 || j < 0 || i >= nxn || j >= nyn)
        return len;
      const int l = loc[(size_t)(j - y0) * RX + (i - x0)];
      if (l < 0 || !(fl(i, j) & LTS_NODE_P)) return len;
      return l;
    };
    for (const auto& nd : nodes) {
      const int j = nd[1], i = nd[2];
      const bool interior = nd[0] == 0;
      const bool isP = fl(i, j) & LTS_NODE_P;
      int4 e;
      e.x = (j * ld + i) | (isP ? (int)0x80000000u : 0);
      e.y = nb(i + 1, j) | (nb(i - 1, j) << 16);
      e.z = nb(i, j + 1) | (nb(i, j - 1) << 16);
      e.w = i | (j << 16);
      T.ent.push_back(e);
      if (interior) ++n_fplus;
    }
    T.tiles.push_back(make_int4(off, len, ix0 | ix1 << 16, iy0 | iy1 << 16));
    n_region += len;
    return "";
  };
  // Adaptive tiling (compact mode, TX = TY = 0): the grid is bisected
  // recursively, each box shrunk to the bounding box of its F+ nodes, until the
  // region of a box fits one workgroup.  A cut is chosen among 16 positions per
  // axis (F+ quantiles and even spacing) by the total region of the tiles that
  // plain median bisection would then make of the two halves; this keeps the
  // cuts across thin bands of F+, whose tiles end up long along the band.
  // Region sizes come from per-row prefix counts of F+ (O(rows) per box).
  const bool adaptive = TX == 0 && TY == 0;
  std::vector<int> rpre, cpre;                                   // F+ prefix counts per row / column
  auto rcount = [&](int j, int a, int b) { return rpre[(size_t)j * (nxn + 1) + b] - rpre[(size_t)j * (nxn + 1) + a]; };
  auto ccount = [&](int i, int a, int b) { return cpre[(size_t)i * (nyn + 1) + b] - cpre[(size_t)i * (nyn + 1) + a]; };
  if (adaptive) {
    rpre.assign((size_t)nyn * (nxn + 1), 0);
    cpre.assign((size_t)nxn * (nyn + 1), 0);
    for (int j = 0; j < nyn; ++j)
      for (int i = 0; i < nxn; ++i) {
        const int f = (fl(i, j) & LTS_NODE_FPLUS) ? 1 : 0;
        rpre[(size_t)j * (nxn + 1) + i + 1] = rpre[(size_t)j * (nxn + 1) + i] + f;
        cpre[(size_t)i * (nyn + 1) + j + 1] = cpre[(size_t)i * (nyn + 1) + j] + f;
      }
  }
  struct Box { int x0, x1, y0, y1; };
  auto shrink = [&](Box b, Box& out) {                           // F+ bounding box inside b
    int y0 = b.y0, y1 = b.y1, x0 = b.x0, x1 = b.x1;
    while (y0 < y1 && rcount(y0, b.x0, b.x1) == 0) ++y0;
    while (y1 > y0 && rcount(y1 - 1, b.x0, b.x1) == 0) --y1;
    if (y0 >= y1) return false;
    while (x0 < x1 && ccount(x0, y0, y1) == 0) ++x0;
    while (x1 > x0 && ccount(x1 - 1, y0, y1) == 0) --x1;
    out = Box{x0, x1, y0, y1};
    return true;
  };
  auto fast_region = [&](const Box& b) {                         // F+ within Manhattan distance p
    size_t n = 0;
    for (int j = std::max(b.y0 - p, 0); j < std::min(b.y1 + p, nyn); ++j) {
      const int dy = std::max(std::max(b.y0 - j, j - (b.y1 - 1)), 0);
      n += rcount(j, std::max(b.x0 - (p - dy), 0), std::min(b.x1 + (p - dy), nxn));
    }
    return n;
  };
  constexpr size_t kNoFit = size_t(1) << 40;
  auto halves = [](const Box& b, int axis, int c, Box& A, Box& B) {
    A = b;
    B = b;
    if (axis == 0) A.x1 = B.x0 = c;
    else A.y1 = B.y0 = c;
  };
  auto line_counts = [&](const Box& b, int axis) {               // F+ per column (axis 0) or row
    std::vector<int> v;
    if (axis == 0)
      for (int i = b.x0; i < b.x1; ++i) v.push_back(ccount(i, b.y0, b.y1));
    else
      for (int j = b.y0; j < b.y1; ++j) v.push_back(rcount(j, b.x0, b.x1));
    return v;
  };
  auto quantile_cut = [](const std::vector<int>& cnt, int lo, double f) {   // in [lo + 1, lo + n - 1]
    const int n = (int)cnt.size();
    long long tot = 0;
    for (int v : cnt) tot += v;
    long long acc = cnt[0];
    int c = lo + 1;                                              // halves [lo, c) and [c, lo + n)
    while (c < lo + n - 1 && (double)acc < f * (double)tot) acc += cnt[++c - lo - 1];
    return c;
  };
  // total region of the tiles that median bisection makes of box b
  std::function<size_t(const Box&)> median_total = [&](const Box& b0) -> size_t {
    Box b;
    if (!shrink(b0, b)) return 0;
    const size_t r = fast_region(b);
    if (r <= (size_t)cap) return r;
    size_t best = kNoFit;
    Box bA{}, bB{};
    for (int axis = 0; axis < 2; ++axis) {
      const int lo = axis == 0 ? b.x0 : b.y0, hi = axis == 0 ? b.x1 : b.y1;
      if (hi - lo < 2) continue;
      Box A, B, sA, sB;
      halves(b, axis, quantile_cut(line_counts(b, axis), lo, 0.5), A, B);
      const size_t cost = (shrink(A, sA) ? fast_region(sA) : 0) + (shrink(B, sB) ? fast_region(sB) : 0);
      if (cost < best) {
        best = cost;
        bA = A;
        bB = B;
      }
    }
    if (best == kNoFit) return kNoFit;
    const size_t ta = median_total(bA), tb = median_total(bB);
    return ta >= kNoFit || tb >= kNoFit ? kNoFit : ta + tb;
  };
  std::function<std::string(const Box&)> bisect = [&](const Box& b0) -> std::string {
    Box b;
    if (!shrink(b0, b)) return "";
    if (fast_region(b) <= (size_t)cap) return add_compact(b.x0, b.x1, b.y0, b.y1);
    size_t best = kNoFit;
    Box bA{}, bB{};
    for (int axis = 0; axis < 2; ++axis) {
      const int lo = axis == 0 ? b.x0 : b.y0, hi = axis == 0 ? b.x1 : b.y1;
      if (hi - lo < 2) continue;
      const std::vector<int> cnt = line_counts(b, axis);
      std::vector<int> cuts;
      for (int k = 1; k <= 8; ++k) {
        cuts.push_back(quantile_cut(cnt, lo, k / 9.0));
        cuts.push_back(std::min(std::max(lo + (hi - lo) * k / 9, lo + 1), hi - 1));
      }
      std::sort(cuts.begin(), cuts.end());
      cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
      for (int c : cuts) {
        Box A, B;
        halves(b, axis, c, A, B);
        const size_t ta = median_total(A), tb = median_total(B);
        const size_t cost = ta >= kNoFit || tb >= kNoFit ? kNoFit : ta + tb;
        if (cost < best) {
          best = cost;
          bA = A;
          bB = B;
        }
      }
    }
    if (best == kNoFit) return "fine tile region exceeds the workgroup capacity";
    std::string e = bisect(bA);
    if (!e.empty()) return e;
    return bisect(bB);
  };
  if (adaptive && rect) return "the adaptive tiling is compact mode only";
  if (!adaptive && (TX < 1 || TY < 1)) return "tile size out of range";
  if (!adaptive)
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
      if (rect) {
        // rectangle: F+ bounding box inside the grown tile, grown by one node (the
        // v = (I - P) u neighbours of its F+ nodes), clipped to the grown tile
        const int gx0 = std::max(x0, 0), gx1 = std::min(x0 + RX, nxn);
        const int gy0 = std::max(y0, 0), gy1 = std::min(y0 + RY, nyn);
        int bx0 = gx1, bx1 = gx0, by0 = gy1, by1 = gy0;
        for (int j = gy0; j < gy1; ++j)
          for (int i = gx0; i < gx1; ++i)
            if (fl(i, j) & LTS_NODE_FPLUS) {
              bx0 = std::min(bx0, i);
              bx1 = std::max(bx1, i + 1);
              by0 = std::min(by0, j);
              by1 = std::max(by1, j + 1);
            }
        bx0 = std::max(bx0 - 1, gx0);
        bx1 = std::min(bx1 + 1, gx1);
        by0 = std::max(by0 - 1, gy0);
        by1 = std::min(by1 + 1, gy1);
        const int rx = bx1 - bx0, ry = by1 - by0;
        if (rx > kRectW || ry > kRectH) return "region rectangle exceeds 64 x 64 nodes";
        if (p > 64) return "rect mode needs p <= 64";
        const int ix0 = std::max(tx, 0), ix1 = std::min(tx + TX, nxn);
        const int iy0 = std::max(ty, 0), iy1 = std::min(ty + TY, nyn);
        T.rtiles.push_back(make_int4(bx0 | by0 << 16, rx | ry << 16, ix0 | ix1 << 16, iy0 | iy1 << 16));
        for (int j = iy0; j < iy1; ++j)
          for (int i = ix0; i < ix1; ++i)
            if (fl(i, j) & LTS_NODE_FPLUS) ++n_fplus;
        n_region += (size_t)rx * ry;
        continue;
      }
      const std::string e = add_compact(std::max(tx, 0), std::min(tx + TX, nxn), std::max(ty, 0),
                                        std::min(ty + TY, nyn));
      if (!e.empty()) return e;
    }
  if (adaptive) {
    const std::string e = bisect(Box{0, nxn, 0, nyn});
    if (!e.empty()) return e;
  }
  // coarse items: 64 columns x kCoarseRows rows holding a DOF outside F+, with
  // the masks of such columns and rows
  for (int ty = 0; ty < nyn; ty += kCoarseRows)
    for (int tx = 0; tx < nxn; tx += 64) {
      uint64_t cm = 0;
      uint32_t rm = 0;
      for (int j = ty; j < std::min(ty + kCoarseRows, nyn); ++j)
        for (int i = tx; i < std::min(tx + 64, nxn); ++i)
          if ((fl(i, j) & (LTS_NODE_DOF | LTS_NODE_FPLUS)) == LTS_NODE_DOF) {
            cm |= 1ull << (i - tx);
            rm |= 1u << (j - ty);
          }
      if (cm) T.citems.push_back(make_int4(tx | ty << 16, (int)(uint32_t)cm, (int)(uint32_t)(cm >> 32), (int)rm));
    }
  T.n_fine = (int)(rect ? T.rtiles.size() : T.tiles.size());
  if (!rect) {
    int max_len = 0;
    for (const int4& t : T.tiles) max_len = std::max(max_len, t.y);
    T.nt = max_len <= 256 * kNPT ? 256 : max_len <= 512 * kNPT ? 512 : kFineThreads;
  }
  T.n_coarse = (int)T.citems.size();
  T.wg_per_sample = T.n_fine + T.n_coarse;
  T.halo_ratio = n_fplus ? (double)n_region / n_fplus : 1.0;
  T.wg_work = T.n_fine ? (double)n_region / T.n_fine * p : 0.0;
  return "";
}

lts_status upload_tiling(lts_ctx c, const TilingHost& T, TilingDev& D) {
  D.TX = T.TX;
  D.TY = T.TY;
  D.n_fine = T.n_fine;
  D.n_coarse = T.n_coarse;
  D.wg_per_sample = T.wg_per_sample;
  D.halo_ratio = T.halo_ratio;
  D.wg_work = T.wg_work;
  D.nt = T.nt;
  D.rect = T.rect;
  D.mix = false;
  D.pitch = T.pitch;
  static uint64_t gen_counter = 0;
  D.gen = ++gen_counter;
  LTS_HIP(c, D.ent.ensure(std::max<size_t>(T.ent.size() * sizeof(int4), 16)));
  LTS_HIP(c, D.tiles.ensure(std::max<size_t>(T.tiles.size() * sizeof(int4), 16)));
  LTS_HIP(c, D.rtiles.ensure(std::max<size_t>(T.rtiles.size() * sizeof(int4), 16)));
  LTS_HIP(c, D.citems.ensure(std::max<size_t>(T.citems.size() * sizeof(int4), 16)));
  if (!T.ent.empty())
    LTS_HIP(c, hipMemcpy(D.ent.p, T.ent.data(), T.ent.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!T.tiles.empty())
    LTS_HIP(c, hipMemcpy(D.tiles.p, T.tiles.data(), T.tiles.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!T.rtiles.empty())
    LTS_HIP(c, hipMemcpy(D.rtiles.p, T.rtiles.data(), T.rtiles.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!T.citems.empty())
    LTS_HIP(c, hipMemcpy(D.citems.p, T.citems.data(), T.citems.size() * sizeof(int4), hipMemcpyHostToDevice));
  return LTS_OK;
}

const std::vector<std::pair<int, int>>& tile_candidates() {
  static const std::vector<std::pair<int, int>> v = {
      {64, 48}, {48, 64}, {56, 56}, {48, 48}, {80, 32}, {32, 80}, {128, 24}, {24, 128}, {40, 40},
      {32, 32}, {16, 256}, {256, 16}, {16, 128}, {128, 16}, {24, 24}, {16, 64}, {64, 16}, {16, 16},
      {8, 256}, {256, 8}, {8, 64}, {64, 8}, {8, 8}};
  return v;
}

std::vector<std::pair<int, int>> level_tile_candidates(const HostLevel& H) {
  // first one tile over the whole level: where the level's F+ fits one
  // workgroup it has no halo at all (compact mode; small levels with large p);
  // then the adaptive tiling (0, 0: compact mode only)
  std::vector<std::pair<int, int>> v{{H.nxn, H.nyn}, {0, 0}};
  for (const auto& t : tile_candidates()) v.push_back(t);
  return v;
}

std::vector<std::pair<int, int>> tile_origins(const HostLevel& H, int TX, int TY) {
  if (TX < 1 || TY < 1) return {{0, 0}};              // adaptive tiling: no grid origin
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
    for (auto& tc : level_tile_candidates(lv.H))
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
                       int active, int startup, hipStream_t stream, bool fp32, double* Unew) {
  if (active <= 0) return LTS_OK;
  StepArgs a;
  a.L = lv.view();
  a.ent = T.ent.as<int4>();
  a.tiles = T.tiles.as<int4>();
  a.citems = T.citems.as<int4>();
  a.n_fine = T.n_fine;
  a.n_coarse = T.n_coarse;
  a.rtiles = T.rtiles.as<int4>();
  a.wg_per_sample = T.wg_per_sample;
  a.active = active;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.Ucur = Ucur;
  a.Uold = Uold;
  a.Unew = Unew ? Unew : Uold;
  a.sstride = sstride;
  a.startup = startup;
  a.s0 = s0;
  if (T.mix && T.rect && T.n_fine > 0) {
    // coarse items and fine tiles in one launch
    const int n_fw = T.n_fine * active, n_cw = (T.n_coarse * active + 3) / 4;
    a.per_xcd = (n_fw + n_cw + 7) / 8;
    const dim3 grid((unsigned)(8LL * a.per_xcd));
    if (fp32)
      k_step_mix<float><<<grid, dim3(kFineThreads), 0, stream>>>(a, n_fw, n_cw);
    else
      k_step_mix<double><<<grid, dim3(kFineThreads), 0, stream>>>(a, n_fw, n_cw);
    return LTS_OK;
  }
  if (T.n_coarse > 0) {
    const long long G = (long long)T.n_coarse * active;
    a.per_xcd = (int)((G + 7) / 8);
    const dim3 grid((unsigned)(8LL * a.per_xcd));
    if (fp32)
      k_coarse<float><<<grid, dim3(kCoarseThreads), 0, stream>>>(a);
    else
      k_coarse<double><<<grid, dim3(kCoarseThreads), 0, stream>>>(a);
  }
  if (T.n_fine > 0) {
    const long long G = (long long)T.n_fine * active;
    a.per_xcd = (int)((G + 7) / 8);
    const dim3 grid((unsigned)(8LL * a.per_xcd));
    const int nt = T.rect ? kFineThreads : compact_threads(T, active, c->n_cu);
    if (T.rect && fp32)
      k_fine<true, float><<<grid, dim3(kFineThreads), 0, stream>>>(a);
    else if (T.rect)
      k_fine<true, double><<<grid, dim3(kFineThreads), 0, stream>>>(a);
    else if (nt == 256 && fp32)
      k_fine_small<float, 256><<<grid, dim3(256), 0, stream>>>(a);
    else if (nt == 256)
      k_fine_small<double, 256><<<grid, dim3(256), 0, stream>>>(a);
    else if (nt == 512 && fp32)
      k_fine_small<float, 512><<<grid, dim3(512), 0, stream>>>(a);
    else if (nt == 512)
      k_fine_small<double, 512><<<grid, dim3(512), 0, stream>>>(a);
    else if (fp32)
      k_fine<false, float><<<grid, dim3(kFineThreads), 0, stream>>>(a);
    else
      k_fine<false, double><<<grid, dim3(kFineThreads), 0, stream>>>(a);
  }
  return LTS_OK;
}

lts_status launch_coarse(lts_ctx c, const DevLevel& lv, const TilingDev& T, const double* d_kappa,
                         const double* d_coef, const double* Ucur, double* Uold, size_t sstride, int active,
                         int startup, hipStream_t stream, bool fp32, double* Unew) {
  if (active <= 0 || T.n_coarse <= 0) return LTS_OK;
  StepArgs a{};
  a.L = lv.view();
  a.citems = T.citems.as<int4>();
  a.n_coarse = T.n_coarse;
  a.active = active;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.Ucur = Ucur;
  a.Uold = Uold;
  a.Unew = Unew ? Unew : Uold;
  a.sstride = sstride;
  a.startup = startup;
  const long long G = (long long)T.n_coarse * active;
  a.per_xcd = (int)((G + 7) / 8);
  if (fp32)
    k_coarse<float><<<dim3((unsigned)(8LL * a.per_xcd)), dim3(kCoarseThreads), 0, stream>>>(a);
  else
    k_coarse<double><<<dim3((unsigned)(8LL * a.per_xcd)), dim3(kCoarseThreads), 0, stream>>>(a);
  return LTS_OK;
}

lts_status launch_multi_step(lts_ctx c, const StepArgs* d_jobs, const std::vector<const TilingDev*>& T,
                             const std::vector<int>& active, int step, hipStream_t stream, bool fp32, int kinds) {
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
    // fine launches: the jobs with the costliest workgroups first, so that
    // the cheap ones fill in at the end
    int pos[kMaxJobs];                                 // job at launch position q
    for (int j = 0; j < nj; ++j) pos[j] = j;
    if (kind > 0)
      std::stable_sort(pos, pos + nj, [&](int x, int y) { return T[x]->wg_work > T[y]->wg_work; });
    m.chunk_off[0] = 0;
    for (int q = 0; q < nj; ++q) {
      const int j = pos[q];
      m.order[q] = j;
      int w = 0;
      if (kind == 0) w = T[j]->n_coarse;
      else if (kind == 1) w = T[j]->rect ? T[j]->n_fine : 0;
      else if (!T[j]->rect && compact_threads(*T[j], active[j], c->n_cu) == (kind == 2 ? kFineThreads : kind == 3 ? 512 : 256))
        w = T[j]->n_fine;
      m.wg_n[q] = w * active[j];
      m.chunk_off[q + 1] = m.chunk_off[q] + (m.wg_n[q] + 7) / 8;
    }
    if (m.chunk_off[nj] == 0) return;
    const dim3 grid((unsigned)(8 * m.chunk_off[nj]));
    if (fp32) {
      if (kind == 0)
        k_coarse_multi<float><<<grid, dim3(kCoarseThreads), 0, stream>>>(m);
      else if (kind == 1)
        k_fine_multi<true, float><<<grid, dim3(kFineThreads), 0, stream>>>(m);
      else if (kind == 2)
        k_fine_multi<false, float><<<grid, dim3(kFineThreads), 0, stream>>>(m);
      else if (kind == 3)
        k_fine_small_multi<float, 512><<<grid, dim3(512), 0, stream>>>(m);
      else
        k_fine_small_multi<float, 256><<<grid, dim3(256), 0, stream>>>(m);
    } else {
      if (kind == 0)
        k_coarse_multi<double><<<grid, dim3(kCoarseThreads), 0, stream>>>(m);
      else if (kind == 1)
        k_fine_multi<true, double><<<grid, dim3(kFineThreads), 0, stream>>>(m);
      else if (kind == 2)
        k_fine_multi<false, double><<<grid, dim3(kFineThreads), 0, stream>>>(m);
      else if (kind == 3)
        k_fine_small_multi<double, 512><<<grid, dim3(512), 0, stream>>>(m);
      else
        k_fine_small_multi<double, 256><<<grid, dim3(256), 0, stream>>>(m);
    }
  };
  for (int kind = 0; kind < std::min(kinds, 5); ++kind) go(kind);
  return LTS_OK;
}

namespace {

// Clear the persistent launch's counters; all: the abort word too.
__global__ void k_persist_reset(unsigned* ctl, int all) {
  for (int t = threadIdx.x; t < kCtlWords; t += blockDim.x)
    if (t != kCtlAbort || all) ctl[t] = 0u;
}

}  // namespace

lts_status launch_persist(lts_ctx c, const StepArgs* d_jobs, const std::vector<const TilingDev*>& T,
                          const std::vector<int>& act_host, const int* d_act, int n_steps, const std::vector<int>& sb,
                          hipStream_t stream, bool fp32) {
  const int nj = (int)T.size();
  if (nj < 1 || nj > kMaxJobs || (int)sb.size() != nj || (int)act_host.size() < n_steps * nj) {
    c->err = "persistent launch: bad job table";
    return LTS_ERR_ARG;
  }
  if (n_steps <= 0) return LTS_OK;
  int coop = 0;
  LTS_HIP(c, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device));
  if (!coop) {
    c->err = "persistent launch: the device has no cooperative launch";
    return LTS_ERR_STATE;
  }
  const void* fn = fp32 ? reinterpret_cast<const void*>(&k_persist<float>)
                        : reinterpret_cast<const void*>(&k_persist<double>);
  int per_cu = 0;
  LTS_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistThreads, 0));
  if (per_cu < 1) {
    c->err = "persistent launch: the kernel does not fit a compute unit";
    return LTS_ERR_STATE;
  }
  const int grid = per_cu * c->n_cu;
  PersistArgs pa{};
  pa.jobs = d_jobs;
  pa.act = d_act;
  LTS_HIP(c, c->p_ctl.ensure(kCtlWords * sizeof(unsigned)));
  pa.ctl = c->p_ctl.as<unsigned>();
  pa.spin_ticks = (long long)(c->barrier_ms * (double)c->wall_khz);
  pa.n_jobs = nj;
  pa.ng = std::min(8, grid);
  // fine segments: the costliest workgroups first, so that the cheap ones fill in at the end
  for (int j = 0; j < nj; ++j) pa.order[j] = j;
  std::stable_sort(pa.order, pa.order + nj, [&](int x, int y) { return T[x]->wg_work > T[y]->wg_work; });
  for (int j = 0; j < nj; ++j) {
    if (sb[j] != 0 && (T[j]->rect || (sb[j] != 1 && sb[j] != 2 && sb[j] != 4) || sb[j] > persist_sb_max(*T[j]))) {
      c->err = "persistent launch: S_b does not fit the tiling";
      return LTS_ERR_ARG;
    }
    if (sb[j] == 0 && !T[j]->rect && T[j]->n_fine > 0) {
      c->err = "persistent launch: compact tiling needs S_b >= 1";
      return LTS_ERR_ARG;
    }
    pa.sb[j] = sb[j];
    pa.nf[j] = T[j]->n_fine;
    pa.nc[j] = T[j]->n_coarse;
  }
  k_persist_reset<<<1, 256, 0, stream>>>(pa.ctl, 1);
  // launches of consecutive steps whose units keep every group counter below 2^30
  int t0 = 0;
  while (t0 < n_steps) {
    long long units = 0;
    int t1 = t0;
    while (t1 < n_steps) {
      long long u = 0;
      for (int j = 0; j < nj; ++j) {
        const long long a = act_host[(size_t)t1 * nj + j];
        const int g = sb[j] > 0 ? sb[j] : 1;
        u += (long long)T[j]->n_fine * ((a + g - 1) / g) + ((long long)T[j]->n_coarse * a + 3) / 4 + pa.ng;
      }
      if (t1 > t0 && units + u >= (1LL << 30)) break;
      units += u;
      ++t1;
    }
    if (t0 > 0) k_persist_reset<<<1, 256, 0, stream>>>(pa.ctl, 0);
    pa.t0 = t0;
    pa.t1 = t1;
    void* args[] = {&pa};
    LTS_HIP(c, hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(kPersistThreads), args, 0, stream));
    t0 = t1;
  }
  unsigned abort_w = 0;
  LTS_HIP(c, hipMemcpyAsync(&abort_w, pa.ctl + kCtlAbort, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
  LTS_HIP(c, hipStreamSynchronize(stream));
  if (abort_w != 0u) {
    c->err = "persistent launch: a workgroup waited longer than the barrier limit; results are invalid";
    return LTS_ERR_STATE;
  }
  return LTS_OK;
}

lts_status launch_adj_compact(lts_ctx c, const DevLevel& lv, const TilingDev& T, const double* d_kappa,
                              const double* d_coef, const double* Y, const double* MU, double* D1, double* Lam1,
                              double* LW, const double* rho, size_t astride, size_t sstride, int active, double f,
                              bool reverse, hipStream_t stream, const double* Yold, double* Ynew) {
  if (active <= 0 || T.n_fine == 0) return LTS_OK;
  if (T.rect) {
    c->err = "compact adjoint sweep on a rect tiling";
    return LTS_ERR_STATE;
  }
  StepArgs a{};
  a.L = lv.view();
  a.ent = T.ent.as<int4>();
  a.tiles = T.tiles.as<int4>();
  a.citems = T.citems.as<int4>();
  a.rtiles = T.rtiles.as<int4>();
  a.n_fine = T.n_fine;
  a.n_coarse = T.n_coarse;
  a.wg_per_sample = T.wg_per_sample;
  a.active = active;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.Ucur = Y;
  a.Uold = D1;
  a.Unew = D1;
  a.sstride = sstride;
  a.startup = 0;
  a.s0 = 0;
  const long long G = (long long)T.n_fine * active;
  a.per_xcd = (int)((G + 7) / 8);
  const dim3 grid((unsigned)(8LL * a.per_xcd));
  if (!reverse) {
    StepState st{Y, Yold ? const_cast<double*>(Yold) : D1, Ynew, 0};
    st.Dout = D1;
    st.dstride = astride;
    if (T.nt == 256) k_adj_fsweep<256><<<grid, dim3(256), 0, stream>>>(a, st);
    else if (T.nt == 512) k_adj_fsweep<512><<<grid, dim3(512), 0, stream>>>(a, st);
    else k_adj_fsweep<1024><<<grid, dim3(1024), 0, stream>>>(a, st);
  } else {
    AdjRevArgs x;
    x.MU = MU;
    x.Lam1 = Lam1;
    x.LW = LW;
    x.rho = rho;
    x.astride = astride;
    x.f = f;
    if (T.nt == 256) k_adj_rsweep<256><<<grid, dim3(256), 0, stream>>>(a, x);
    else if (T.nt == 512) k_adj_rsweep<512><<<grid, dim3(512), 0, stream>>>(a, x);
    else k_adj_rsweep<1024><<<grid, dim3(1024), 0, stream>>>(a, x);
  }
  return LTS_OK;
}

void job_record(const DevLevel& lv, const TilingDev& T, const double* d_kappa, const double* d_coef,
                double* B0, double* B1, size_t sstride, void* out) {
  StepArgs a{};
  a.L = lv.view();
  a.ent = T.ent.as<int4>();
  a.tiles = T.tiles.as<int4>();
  a.citems = T.citems.as<int4>();
  a.n_fine = T.n_fine;
  a.n_coarse = T.n_coarse;
  a.rtiles = T.rtiles.as<int4>();
  a.wg_per_sample = T.wg_per_sample;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.sstride = sstride;
  a.B0 = B0;
  a.B1 = B1;
  a.Ucur = B0;
  a.Uold = B1;
  a.Unew = B1;
  std::memcpy(out, &a, sizeof(a));
}

size_t step_args_size() { return sizeof(StepArgs); }

}  // namespace lts
