// Multi-level local time stepping on rectilinear levels (Sec. 3.5, closing
// remark): the fine region is split into tiers of ever smaller elements and
// Algorithm 2 is nested once per tier, so that each tier takes its own step.
//
// Tier j (0-based here) has the projector P_j (DOFs that are vertices of a
// cell of tier >= j) and the ratio p_j.  In increment form, for a force F
// held over the tier's time,
//   e_0 = e_-1 = 0,  Phi_m = F + A P_j e_m,
//   e_m+1 = (1 + beta_m)(e_m + h_m) - beta_m e_m-1,   beta_0 = 0,
// where h_m is the leapfrog half step from rest under Phi_m over the inner
// time sigma_j+1: for the innermost tier h_m = -c0 Phi_m, otherwise h_m is the
// increment of tier j+1 run with F = Phi_m.  (Algorithm 2's stage coefficients
// satisfy c_m = (1 + beta_m) c_0 because T_m+1 + T_m-1 = 2 delta T_m, which is
// what makes every stage's half step the same and lets the inner tier take
// it.)  One coarse step: u_n+1 = 2 u_n - u_n-1 + 2 e with e tier 0's increment
// for F = A u_n; only the innermost half-step coefficient c0 depends on the
// sample (through dt).
//
// Work decomposition: the DOFs outside F+ take the plain leapfrog update in
// the coarse kernel of the single-tier step.  The F+ DOFs run in compact
// fine tiles (lts_fused.hip's tiling, built here with region radius K, the
// number of stages whose force reads neighbours: sum_j (p_0 .. p_j-1)(p_j - 1);
// stage 0 of every tier starts from e = 0 and tier 0's F = A u_n is read from
// global memory).  One workgroup per (sample, tile) keeps every tier's
// (F, e_m, e_m-1) of its two nodes per lane in registers and exchanges P_j e_m
// through LDS, one barrier per reading stage, alternating two buffers.  Each
// reading stage moves the border error of the region in by one node, so the
// stage with `reach` r recomputes only the nodes within r of the tile (a
// prefix of the distance-ordered region); after the K reading stages the
// tile's own nodes are exact and are written back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ctx.h"
#include "fused.h"

namespace lts {

namespace {

constexpr int kMT = LTS_MLTS_MAX_TIERS;
constexpr int kMP = LTS_MLTS_MAX_P;
constexpr int kMNPT = 2;                      // region nodes per lane
constexpr int kMCap = kFineThreads * kMNPT;   // largest region
constexpr int kMPitch = 8;                    // row pitch multiple of the device arrays

// A job's record in device memory: level, tiling, tiers, the samples' tables
// and the two state buffers (step t reads B[t & 1], writes B[(t + 1) & 1]).
struct MltsJob {
  LevelView L;
  const int4* ent;
  const int4* tiles;
  const uint8_t* ptier;               // [nyn*ld] largest j + 1 with the node in P_j, 0 off P
  const double* kappa;                // [S][nb] (sorted sample order)
  const double* c0;                   // [S] innermost half-step coefficient
  double* B0;
  double* B1;
  size_t sstride;
  int n_fine, T, K, pad;
  int p[kMT];
  double beta[kMT][kMP];              // beta_m of tier j, beta[j][0] = 0
};

// One launch over the fine tiles of several jobs: job `order[q]` owns the
// workgroups of launch position q, wg_n[q] of them, split into 8 contiguous
// chunks (one per XCD) of ceil(wg_n / 8); chunk_off holds their prefix sums.
struct MltsLaunch {
  const MltsJob* jobs;
  int n_jobs, step;
  int order[kMaxJobs], wg_n[kMaxJobs], chunk_off[kMaxJobs + 1];
};

// A pointer field of a job record loaded as a global-address-space pointer, so
// that the accesses through it stay global loads (a plain copy out of device
// memory would be addressed as a flat pointer).
#define MLTS_GPTR(f) \
  ((decltype(+(f)))(*(__attribute__((address_space(1))) std::remove_pointer_t<decltype(+(f))>* const*)(&(f))))

// What a workgroup uses of its job's record, in registers.
struct MltsView {
  LevelView L;
  const int4* ent;
  const int4* tiles;
  const uint8_t* ptier;
  const double* kappa;
  const double* c0;
  double* B0;
  double* B1;
  size_t sstride;
  int n_fine, T, K;
  int p[kMT];
  const double* beta;                 // beta_m of tier j at beta[j * kMP + m] (the workgroup's LDS copy)
};

__device__ __forceinline__ MltsView job_view(const MltsJob& x) {
  MltsView v;
  v.L.nxn = x.L.nxn; v.L.nyn = x.L.nyn; v.L.ld = x.L.ld; v.L.p = x.L.p; v.L.nb = x.L.nb;
  v.L.hx = MLTS_GPTR(x.L.hx); v.L.hy = MLTS_GPTR(x.L.hy);
  v.L.inv2hx = MLTS_GPTR(x.L.inv2hx); v.L.inv2hy = MLTS_GPTR(x.L.inv2hy);
  v.L.x = MLTS_GPTR(x.L.x); v.L.y = MLTS_GPTR(x.L.y);
  v.L.cblk = MLTS_GPTR(x.L.cblk); v.L.flags = MLTS_GPTR(x.L.flags); v.L.ninfo = MLTS_GPTR(x.L.ninfo);
  v.L.invm = MLTS_GPTR(x.L.invm); v.L.qoiw = MLTS_GPTR(x.L.qoiw);
  v.L.beta = MLTS_GPTR(x.L.beta); v.L.beta_half = MLTS_GPTR(x.L.beta_half);
  v.ent = MLTS_GPTR(x.ent); v.tiles = MLTS_GPTR(x.tiles); v.ptier = MLTS_GPTR(x.ptier);
  v.kappa = MLTS_GPTR(x.kappa); v.c0 = MLTS_GPTR(x.c0);
  v.B0 = MLTS_GPTR(x.B0); v.B1 = MLTS_GPTR(x.B1);
  v.sstride = x.sstride;
  v.n_fine = x.n_fine; v.T = x.T; v.K = x.K;
#pragma unroll
  for (int j = 0; j < kMT; ++j) v.p[j] = x.p[j];
  v.beta = &x.beta[0][0];
  return v;
}

// The state of a lane's region nodes (T = double, or float for FP32 stepping).
template <class T>
struct MLane {
  T F[kMT][kMNPT], e[kMT][kMNPT], ep[kMT][kMNPT];
  T aE[kMNPT], aW[kMNPT], aN[kMNPT], aS[kMNPT];
  uint32_t ad[kMNPT][4];                // LDS byte offsets of the E, W, N, S neighbours
  int dd[kMNPT], tp[kMNPT];             // distance to the tile, tier of P
};

// Tier J over the force S.F[J]: leaves its increment in S.e[J].
template <class T, int NT, int J>
__device__ __forceinline__ void tier_run(const MltsView& x, MLane<T>& S, T* __restrict__ lq, int& ph,
                                         int& reach, T c0, int tid) {
  constexpr int kCap = NT * kMNPT;
  const int p = x.p[J];
#pragma unroll
  for (int r = 0; r < kMNPT; ++r) S.e[J][r] = S.ep[J][r] = (T)0;
  for (int m = 0; m < p; ++m) {
    T Phi[kMNPT];
#pragma unroll
    for (int r = 0; r < kMNPT; ++r) Phi[r] = S.F[J][r];
    if (m > 0) {
      // publish P_J e_m of the nodes the next reach still reads, then read the
      // neighbours' values
      T* buf = lq + (ph & 1) * (kCap + 1);
#pragma unroll
      for (int r = 0; r < kMNPT; ++r)
        if (S.dd[r] <= reach) buf[tid + r * NT] = S.tp[r] > J ? S.e[J][r] : (T)0;
      __syncthreads();
      --reach;
      const char* rb = reinterpret_cast<const char*>(buf);
#pragma unroll
      for (int r = 0; r < kMNPT; ++r) {
        if (S.dd[r] > reach) continue;
        const T qi = S.tp[r] > J ? S.e[J][r] : (T)0;
        const T qE = *reinterpret_cast<const T*>(rb + S.ad[r][0]);
        const T qW = *reinterpret_cast<const T*>(rb + S.ad[r][1]);
        const T qN = *reinterpret_cast<const T*>(rb + S.ad[r][2]);
        const T qS = *reinterpret_cast<const T*>(rb + S.ad[r][3]);
        Phi[r] += S.aE[r] * (qi - qE) + S.aW[r] * (qi - qW) + S.aN[r] * (qi - qN) + S.aS[r] * (qi - qS);
      }
      ++ph;
    }
    // the stage's half step: the inner tier, or -c0 Phi in the innermost one
    bool inner = false;
    if constexpr (J + 1 < kMT) {
      if (J + 1 < x.T) {
        inner = true;
#pragma unroll
        for (int r = 0; r < kMNPT; ++r) S.F[J + 1][r] = Phi[r];
        tier_run<T, NT, J + 1>(x, S, lq, ph, reach, c0, tid);
#pragma unroll
        for (int r = 0; r < kMNPT; ++r) Phi[r] = S.e[J + 1][r];
      }
    }
    if (!inner) {
#pragma unroll
      for (int r = 0; r < kMNPT; ++r) Phi[r] = -c0 * Phi[r];
    }
    const T b = (T)x.beta[J * kMP + m];
#pragma unroll
    for (int r = 0; r < kMNPT; ++r) {
      const T en = ((T)1 + b) * (S.e[J][r] + Phi[r]) - b * S.ep[J][r];
      S.ep[J][r] = S.e[J][r];
      S.e[J][r] = en;
    }
  }
}

// The job and job-local workgroup of this workgroup; false past a job's count.
// XCD x runs chunk x of every job in launch order, so neighbouring tiles of a
// sample share that XCD's L2.
__device__ __forceinline__ bool mlts_slot(const MltsLaunch& m, int& j, int& local) {
  const int x = (int)(blockIdx.x & 7), k = (int)(blockIdx.x >> 3);
  int q = 0;
  while (q + 1 < m.n_jobs && k >= m.chunk_off[q + 1]) ++q;
  const int per = m.chunk_off[q + 1] - m.chunk_off[q];
  j = m.order[q];
  local = x * per + (k - m.chunk_off[q]);
  return k < m.chunk_off[m.n_jobs] && local < m.wg_n[q];
}

// One workgroup per (job, sample, fine tile); the tile's region nodes (F+
// nodes within Manhattan distance K of the tile, by increasing distance) two
// per lane.  Region entries as in the single-tier compact tiles.  T: the type
// of the states and of the stepping arithmetic (the edge coefficients are
// formed in FP64 and rounded once).
// OCC: at most 64 VGPRs (8 wavefronts per SIMD), so that two 1024-thread
// workgroups share a CU (FP32 only: it spills a few values, which pays only
// when a launch has more workgroups than CUs).
template <class T, int NT, bool OCC = false>
__global__ __launch_bounds__(NT, OCC ? 8 : 1) void k_mlts(MltsLaunch m) {
  constexpr int kCap = NT * kMNPT;
  __shared__ T lq[2 * (kCap + 1)];
  __shared__ double lk[256];
  __shared__ double lbeta[kMT * kMP];
  int jb, local;
  if (!mlts_slot(m, jb, local)) return;
  MltsView x = job_view(m.jobs[jb]);
  for (int t = (int)threadIdx.x; t < kMT * kMP; t += NT) lbeta[t] = x.beta[t];
  x.beta = lbeta;
  const int s = local / x.n_fine, tile = local - s * x.n_fine;
  const LevelView& L = x.L;
  const int tid = (int)threadIdx.x;
  for (int t = tid; t < L.nb; t += NT) lk[t] = x.kappa[(size_t)s * L.nb + t];
  const int4 tl = x.tiles[tile];
  const int len = tl.y;
  const int ix0 = tl.z & 0xFFFF, ix1 = tl.z >> 16, iy0 = tl.w & 0xFFFF, iy1 = tl.w >> 16;
  const bool odd = m.step & 1, startup = m.step == 0;
  const T* __restrict__ u = reinterpret_cast<const T*>(odd ? x.B1 : x.B0) + (size_t)s * x.sstride;
  T* uo = reinterpret_cast<T*>(odd ? x.B0 : x.B1) + (size_t)s * x.sstride;
  const int ld = L.ld;
  int4 en[kMNPT];
#pragma unroll
  for (int r = 0; r < kMNPT; ++r) en[r] = x.ent[tl.x + min(tid + r * NT, len - 1)];
  __syncthreads();                     // lk
  MLane<T> S;
  T u0[kMNPT];
  int kk[kMNPT];
#pragma unroll
  for (int r = 0; r < kMNPT; ++r) {
#pragma unroll
    for (int j = 0; j < kMT; ++j) S.F[j][r] = S.e[j][r] = S.ep[j][r] = (T)0;
    S.aE[r] = S.aW[r] = S.aN[r] = S.aS[r] = (T)0;
#pragma unroll
    for (int t = 0; t < 4; ++t) S.ad[r][t] = (uint32_t)(len * sizeof(T));
    S.dd[r] = 1 << 30;                 // a lane past the region end: never within reach
    S.tp[r] = 0;
    u0[r] = (T)0;
    kk[r] = 0;
    const int e = tid + r * NT;
    if (e >= len) continue;
    const size_t k = (size_t)(en[r].x & 0x7FFFFFFF);
    const int i = en[r].w & 0xFFFF, j = en[r].w >> 16;
    kk[r] = (int)k;
    S.ad[r][0] = (uint32_t)(en[r].y & 0xFFFF) * sizeof(T);
    S.ad[r][1] = ((uint32_t)en[r].y >> 16) * sizeof(T);
    S.ad[r][2] = (uint32_t)(en[r].z & 0xFFFF) * sizeof(T);
    S.ad[r][3] = ((uint32_t)en[r].z >> 16) * sizeof(T);
    S.dd[r] = max(max(ix0 - i, i - (ix1 - 1)), 0) + max(max(iy0 - j, j - (iy1 - 1)), 0);
    S.tp[r] = x.ptier[k];
    double cE, cW, cN, cS;
    edge_coefs(L, lk, i, j, cE, cW, cN, cS);
    const double im = L.invm[k];
    S.aE[r] = (T)(im * cE);
    S.aW[r] = (T)(im * cW);
    S.aN[r] = (T)(im * cN);
    S.aS[r] = (T)(im * cS);
    // tier 0's force A u_n from global memory (a neighbour off the DOFs holds 0)
    const T uc = u[k];
    S.F[0][r] = S.aE[r] * (uc - u[k + 1]) + S.aW[r] * (uc - u[k - 1]) + S.aN[r] * (uc - u[k + ld]) +
                S.aS[r] * (uc - u[k - ld]);
    u0[r] = uc;
  }
  if (tid == 0) lq[len] = lq[kCap + 1 + len] = (T)0;   // slot of absent and non-P neighbours
  int ph = 0, reach = x.K;
  tier_run<T, NT, 0>(x, S, lq, ph, reach, (T)x.c0[s], tid);
#pragma unroll
  for (int r = 0; r < kMNPT; ++r) {
    if (S.dd[r] != 0) continue;        // written back by the tile that owns the node
    const size_t k = (size_t)kk[r];
    uo[k] = startup ? u0[r] + S.e[0][r] : (T)2 * u0[r] - uo[k] + (T)2 * S.e[0][r];
  }
}

// Host build of the tiers of a level.
struct MltsHost {
  int T = 0, K = 0, nt = kFineThreads, max_region = 0;
  int p[kMT] = {}, nP[kMT] = {};
  double updates = 0.0, omega[kMT] = {}, delta[kMT] = {}, beta[kMT][kMP] = {};
  std::vector<uint8_t> node_tier;     // [nyn*nxn]
  TilingHost tiling;
};

std::string build_mlts(const HostLevel& H, int ld, const lts_mlts_desc& d, MltsHost& M) {
  M = MltsHost();
  if (d.n_tiers < 1 || d.n_tiers > kMT) return "n_tiers must be in 1..LTS_MLTS_MAX_TIERS";
  M.T = d.n_tiers;
  long long span = 1, K = 0;
  for (int j = 0; j < M.T; ++j) {
    if (d.p[j] < 1 || d.p[j] > kMP) return "every p must be in 1..LTS_MLTS_MAX_P";
    M.p[j] = d.p[j];
    K += span * (d.p[j] - 1);
    span *= d.p[j];
  }
  if (K > 0xFFFF) return "too many reading stages per step";
  M.K = (int)K;
  const int nxc = H.nxc, nyc = H.nyc, nxn = H.nxn;
  std::vector<uint8_t> ct((size_t)nxc * nyc, 0);
  for (int b = 0; b < nyc; ++b)
    for (int a = 0; a < nxc; ++a) {
      const size_t c = (size_t)b * nxc + a;
      const bool fine = H.active[c] && H.fine[c];
      if (d.cell_tier) {
        const int v = d.cell_tier[c];
        if (v > M.T) return "cell_tier beyond n_tiers";
        if ((v >= 1) != fine) return "cell_tier must be >= 1 exactly on the active fine cells";
        ct[c] = (uint8_t)v;
      } else if (fine) {
        const double leg = std::min(H.x[a + 1] - H.x[a], H.y[b + 1] - H.y[b]);
        int t = 1;
        for (int j = 2; j <= M.T; ++j)
          if (leg < std::ldexp(H.h, -j)) ++t;
        ct[c] = (uint8_t)t;
      }
    }
  // a DOF's tier: the largest tier of its (up to four) cells
  M.node_tier.assign((size_t)nxn * H.nyn, 0);
  for (int j = 0; j < H.nyn; ++j)
    for (int i = 0; i < nxn; ++i) {
      const size_t k = (size_t)j * nxn + i;
      if (!(H.flags[k] & LTS_NODE_DOF)) continue;
      int t = 0;
      for (int b = j - 1; b <= j; ++b)
        for (int a = i - 1; a <= i; ++a)
          if (a >= 0 && b >= 0 && a < nxc && b < nyc) t = std::max(t, (int)ct[(size_t)b * nxc + a]);
      if ((t >= 1) != ((H.flags[k] & LTS_NODE_P) != 0)) return "internal: tier 1 differs from P";
      M.node_tier[k] = (uint8_t)t;
      for (int q = 0; q < t; ++q) ++M.nP[q];
    }
  M.updates = (double)(H.n_dof - M.nP[0]);
  long long rate = 1;
  for (int j = 0; j < M.T; ++j) {
    rate *= M.p[j];
    M.updates += (double)rate * (M.nP[j] - (j + 1 < M.T ? M.nP[j + 1] : 0));
    std::vector<double> b, bh;
    cheb_constants(M.p[j], H.nu, M.delta[j], M.omega[j], b, bh);
    for (int m = 1; m < M.p[j]; ++m) M.beta[j][m] = b[m];
  }
  const int cap = d.max_region == 0 ? kMCap : d.max_region;
  if (cap != 512 && cap != 1024 && cap != kMCap) return "max_region must be 0, 512, 1024 or 2048";
  HostLevel Hr = H;
  Hr.p = std::max(M.K, 1);
  std::string e = build_tiling(Hr, ld, 0, 0, 0, 0, false, M.tiling, cap);
  if (!e.empty()) return e;
  for (const int4& t : M.tiling.tiles) M.max_region = std::max(M.max_region, t.y);
  M.nt = M.max_region <= 256 * kMNPT ? 256 : M.max_region <= 512 * kMNPT ? 512 : kFineThreads;
  return "";
}

void fill_info(const MltsHost& M, lts_mlts_info* o) {
  *o = lts_mlts_info{};
  o->n_tiers = M.T;
  for (int j = 0; j < M.T; ++j) {
    o->p[j] = M.p[j];
    o->n_P[j] = M.nP[j];
  }
  o->phases = M.K;
  o->n_tiles = M.tiling.n_fine;
  o->max_region = M.max_region;
  o->threads = M.nt;
  o->halo_ratio = M.tiling.halo_ratio;
  o->updates_per_step = M.updates;
}

int pitch_of(int nxn) { return (nxn + kMPitch - 1) / kMPitch * kMPitch; }

lts_status mlts_solve(lts_ctx c, const DevLevel& lv, const Staged& st, const StagedDev& d, double width, bool fp32) {
  MltsDev& M = *lv.mlts;
  const int n = st.n;
  const size_t sstride = lv.nodes;
  const size_t es = fp32 ? sizeof(float) : sizeof(double);   // bytes per state value
  LTS_HIP(c, c->st0.ensure((size_t)n * sstride * es));
  LTS_HIP(c, c->st1.ensure((size_t)n * sstride * es));
  double* B[2] = {c->st0.as<double>(), c->st1.as<double>()};
  hipStream_t q = c->stream;
  M.c0_host.resize(n);
  mlts_c0(M, st.dt.data(), n, M.c0_host.data());
  LTS_HIP(c, M.c0.ensure((size_t)n * 8));
  LTS_HIP(c, M.rec.ensure(mlts_record_size()));
  std::vector<char> rec(mlts_record_size());
  mlts_record(lv, d.kappa, M.c0.as<double>(), B[0], B[1], rec.data());
  LTS_HIP(c, hipMemcpyAsync(M.c0.p, M.c0_host.data(), (size_t)n * 8, hipMemcpyHostToDevice, q));
  LTS_HIP(c, hipMemcpyAsync(M.rec.p, rec.data(), rec.size(), hipMemcpyHostToDevice, q));
  LTS_HIP(c, hipStreamSynchronize(q));               // the host copies may be released
  lts_status r = init_states(c, lv, n, d.x0, width, B[0], B[1], fp32);
  if (r != LTS_OK) return r;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    while (c->ev_pool.size() < 2) {
      hipEvent_t e;
      LTS_HIP(c, hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
    e0 = c->ev_pool[0];
    e1 = c->ev_pool[1];
    LTS_HIP(c, hipEventRecord(e0, q));
  }
  const std::vector<const MltsDev*> Mv = {&M};
  std::vector<int> act = {n};
  int64_t launches = 0;
  const int maxT = st.nsteps[0];
  for (int t = 0; t < maxT; ++t) {
    while (act[0] > 0 && st.nsteps[act[0] - 1] <= t) --act[0];
    if ((r = launch_coarse(c, lv, M.tiling, d.kappa, d.coef, B[t & 1], B[(t + 1) & 1], sstride, act[0], t == 0,
                           q, fp32)) != LTS_OK)
      return r;
    if ((r = launch_mlts(c, M.rec.p, Mv, act, t, q, fp32)) != LTS_OK) return r;
    ++launches;
  }
  LTS_HIP(c, hipGetLastError());
  c->last = lts_timing{};
  if (c->timing) {
    LTS_HIP(c, hipEventRecord(e1, q));
    LTS_HIP(c, hipEventSynchronize(e1));
    float ms = 0;
    LTS_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    c->last.step_kernel_ms = ms;
  }
  double dofu = 0.0;
  for (int s = 0; s < n; ++s) dofu += (double)st.nsteps[s] * M.updates;
  c->last.dof_updates = dofu;
  c->last.alg_bytes = 0.0;
  c->last.step_launches = launches;
  return qoi_device(c, lv, n, d.nsteps, B[0], B[1], c->Qd.as<double>(), fp32);
}

}  // namespace

size_t mlts_record_size() { return sizeof(MltsJob); }

void mlts_record(const DevLevel& lv, const double* d_kappa, const double* d_c0, double* B0, double* B1, void* out) {
  const MltsDev& M = *lv.mlts;
  MltsJob x{};
  x.L = lv.view();
  x.ent = M.tiling.ent.as<int4>();
  x.tiles = M.tiling.tiles.as<int4>();
  x.ptier = M.ptier.as<uint8_t>();
  x.kappa = d_kappa;
  x.c0 = d_c0;
  x.B0 = B0;
  x.B1 = B1;
  x.sstride = lv.nodes;
  x.n_fine = M.tiling.n_fine;
  x.T = M.T;
  x.K = M.K;
  for (int j = 0; j < M.T; ++j) {
    x.p[j] = M.p[j];
    for (int m = 0; m < kMP; ++m) x.beta[j][m] = M.beta[j][m];
  }
  std::memcpy(out, &x, sizeof x);
}

// The innermost half-step coefficient for steps dt: c0 = sigma_T^2 / (omega_T
// delta_T) with sigma_1 = dt, sigma_j+1^2 = sigma_j^2 2 / (omega_j delta_j).
void mlts_c0(const MltsDev& M, const double* dt, int n, double* c0) {
  long double f = 1.0L / ((long double)M.omega[M.T - 1] * M.delta[M.T - 1]);
  for (int j = 0; j + 1 < M.T; ++j) f *= 2.0L / ((long double)M.omega[j] * M.delta[j]);
  for (int s = 0; s < n; ++s) c0[s] = (double)((long double)dt[s] * dt[s] * f);
}

lts_status launch_mlts(lts_ctx c, const void* d_jobs, const std::vector<const MltsDev*>& M,
                       const std::vector<int>& active, int step, hipStream_t stream, bool fp32) {
  const int nj = (int)M.size();
  if (nj > kMaxJobs) {
    c->err = "too many jobs in one batch";
    return LTS_ERR_ARG;
  }
  // one launch per workgroup size; within it the costliest workgroups first
  for (int nt : {kFineThreads, 512, 256}) {
    MltsLaunch m{};
    m.jobs = static_cast<const MltsJob*>(d_jobs);
    m.step = step;
    int pos[kMaxJobs], n = 0;
    for (int j = 0; j < nj; ++j)
      if (M[j]->nt == nt && M[j]->tiling.n_fine > 0 && active[j] > 0) pos[n++] = j;
    if (n == 0) continue;
    std::stable_sort(pos, pos + n, [&](int a, int b) { return M[a]->max_region * M[a]->K > M[b]->max_region * M[b]->K; });
    m.n_jobs = n;
    m.chunk_off[0] = 0;
    for (int q = 0; q < n; ++q) {
      m.order[q] = pos[q];
      m.wg_n[q] = M[pos[q]]->tiling.n_fine * active[pos[q]];
      m.chunk_off[q + 1] = m.chunk_off[q] + (m.wg_n[q] + 7) / 8;
    }
    const dim3 g((unsigned)(8 * m.chunk_off[n]));
    if (fp32) {
      long long wgs = 0;
      for (int q = 0; q < n; ++q) wgs += m.wg_n[q];
      if (nt == 256) k_mlts<float, 256><<<g, 256, 0, stream>>>(m);
      else if (nt == 512) k_mlts<float, 512><<<g, 512, 0, stream>>>(m);
      else if (wgs > c->n_cu) k_mlts<float, kFineThreads, true><<<g, kFineThreads, 0, stream>>>(m);
      else k_mlts<float, kFineThreads><<<g, kFineThreads, 0, stream>>>(m);
    } else {
      if (nt == 256) k_mlts<double, 256><<<g, 256, 0, stream>>>(m);
      else if (nt == 512) k_mlts<double, 512><<<g, 512, 0, stream>>>(m);
      else k_mlts<double, kFineThreads><<<g, kFineThreads, 0, stream>>>(m);
    }
  }
  return LTS_OK;
}

}  // namespace lts

using namespace lts;

extern "C" {

lts_status lts_set_mlts(lts_ctx c, int32_t level, const lts_mlts_desc* d) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!d) return arg_fail(c, "desc is NULL");
  if (level < 0 || level >= (int32_t)c->levels.size()) return arg_fail(c, "no such level");
  DevLevel& lv = *c->levels[level];
  MltsHost M;
  std::string e = build_mlts(lv.H, lv.ld, *d, M);
  if (!e.empty()) return arg_fail(c, e);
  LTS_HIP(c, hipSetDevice(c->device));
  auto D = std::make_unique<MltsDev>();
  D->T = M.T;
  D->K = M.K;
  D->max_region = M.max_region;
  D->nt = M.nt;
  D->updates = M.updates;
  for (int j = 0; j < M.T; ++j) {
    D->p[j] = M.p[j];
    D->nP[j] = M.nP[j];
    D->omega[j] = M.omega[j];
    D->delta[j] = M.delta[j];
    for (int m = 0; m < kMP; ++m) D->beta[j][m] = M.beta[j][m];
  }
  lts_status r = upload_tiling(c, M.tiling, D->tiling);
  if (r != LTS_OK) return r;
  // the node tiers in the level's padded layout (row pitch ld)
  std::vector<uint8_t> pt((size_t)lv.ld * lv.H.nyn, 0);
  for (int j = 0; j < lv.H.nyn; ++j)
    std::memcpy(&pt[(size_t)j * lv.ld], &M.node_tier[(size_t)j * lv.H.nxn], (size_t)lv.H.nxn);
  LTS_HIP(c, D->ptier.ensure(pt.size()));
  LTS_HIP(c, hipMemcpy(D->ptier.p, pt.data(), pt.size(), hipMemcpyHostToDevice));
  lv.mlts = std::move(D);
  return LTS_OK;
}

lts_status lts_mlts_info_get(lts_ctx c, int32_t level, lts_mlts_info* out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!out) return arg_fail(c, "out is NULL");
  if (level < 0 || level >= (int32_t)c->levels.size()) return arg_fail(c, "no such level");
  const DevLevel& lv = *c->levels[level];
  if (!lv.mlts) {
    c->err = "no tiers attached to this level (lts_set_mlts)";
    return LTS_ERR_STATE;
  }
  const MltsDev& M = *lv.mlts;
  *out = lts_mlts_info{};
  out->n_tiers = M.T;
  for (int j = 0; j < M.T; ++j) {
    out->p[j] = M.p[j];
    out->n_P[j] = M.nP[j];
  }
  out->phases = M.K;
  out->n_tiles = M.tiling.n_fine;
  out->max_region = M.max_region;
  out->threads = M.nt;
  out->halo_ratio = M.tiling.halo_ratio;
  out->updates_per_step = M.updates;
  return LTS_OK;
}

lts_status lts_mlts_host(const lts_rect_rule* rule, const lts_mlts_desc* d, lts_mlts_info* info,
                         uint8_t* node_tier) {
  if (!rule || !d || !info) return LTS_ERR_ARG;
  std::vector<double> xs, ys;
  std::vector<uint8_t> act, fine, qoi;
  std::vector<int32_t> blk;
  double h = 0;
  int p = 0, nb = 0;
  if (!build_rect_desc(*rule, xs, ys, act, blk, fine, qoi, h, p, nb).empty()) return LTS_ERR_ARG;
  lts_grid_desc g{};
  g.nx_cells = (int32_t)xs.size() - 1;
  g.ny_cells = (int32_t)ys.size() - 1;
  g.x = xs.data(); g.y = ys.data();
  g.cell_active = act.data(); g.cell_block = blk.data(); g.cell_fine = fine.data(); g.cell_qoi = qoi.data();
  g.n_blocks = nb; g.h = h; g.p = p; g.nu = rule->nu;
  HostLevel H;
  if (!build_level_from_desc(g, H).empty()) return LTS_ERR_ARG;
  MltsHost M;
  if (!build_mlts(H, pitch_of(H.nxn), *d, M).empty()) return LTS_ERR_ARG;
  fill_info(M, info);
  if (node_tier) std::memcpy(node_tier, M.node_tier.data(), M.node_tier.size());
  return LTS_OK;
}

lts_status lts_mlts_forward(lts_ctx c, int32_t level, const lts_samples* S, int32_t precision, double* Q_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (level < 0 || level >= (int32_t)c->levels.size()) return arg_fail(c, "no such level");
  const DevLevel& lv = *c->levels[level];
  if (!lv.mlts) {
    c->err = "no tiers attached to this level (lts_set_mlts)";
    return LTS_ERR_STATE;
  }
  if (precision != LTS_FP64 && precision != LTS_FP32_STEP) return arg_fail(c, "bad precision");
  if (S && S->n > 0 && !Q_out) return arg_fail(c, "Q_out is NULL");
  Staged st;
  lts_status r = stage_samples(c, lv, S, st);
  if (r != LTS_OK) return r;
  if (st.n == 0) return LTS_OK;
  LTS_HIP(c, hipSetDevice(c->device));
  StagedDev d;
  if ((r = ctx_staging(c, lv, st.n, d)) != LTS_OK) return r;
  if ((r = upload_staged(c, lv, st, S, d)) != LTS_OK) return r;
  if ((r = mlts_solve(c, lv, st, d, S->width, precision == LTS_FP32_STEP)) != LTS_OK) return r;
  return finish_Q(c, st, c->Qd.as<double>(), d, Q_out);
}

}  // extern "C"
