// Context and device-level structures of the library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "device.h"
#include "fused.h"
#include "host.h"

namespace lts {

// Device buffer owned by a context: grows on demand, freed by release() or
// with the context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct TilingDev {
  int TX = 0, TY = 0, n_fine = 0, n_coarse = 0, wg_per_sample = 0;
  bool rect = false;
  int pitch = 0;
  double halo_ratio = 1.0;
  double wg_work = 0.0;  // mean region nodes x substeps of one fine workgroup
  int nt = kFineThreads; // compact mode: threads of a fine workgroup
  bool mix = false;     // rect mode: coarse items and fine tiles in one launch (k_step_mix)
  uint64_t gen = 0;     // distinct for every upload (keys captured graphs)
  DevBuf ent, tiles, rtiles, citems;
};

// Tiers of the multi-level step attached to a level (lts_set_mlts; see
// lts_mlts.hip).
struct MltsDev {
  int T = 0, K = 0;                        // tiers, exchange phases per step (= region radius)
  int p[LTS_MLTS_MAX_TIERS] = {};
  int nP[LTS_MLTS_MAX_TIERS] = {};         // |P_j|
  int max_region = 0, nt = 1024;
  double updates = 0.0;                    // DOF updates of one step of one sample
  double omega[LTS_MLTS_MAX_TIERS] = {}, delta[LTS_MLTS_MAX_TIERS] = {};
  double beta[LTS_MLTS_MAX_TIERS][LTS_MLTS_MAX_P] = {};   // beta_m of tier j, beta_0 = 0
  TilingDev tiling;                        // compact tiles, regions of radius K
  DevBuf ptier;                            // per node: largest j with the node in P_j (0 off P_1)
  DevBuf c0;                               // per sample of a solve: the innermost half-step coefficient
  std::vector<double> c0_host;             // its host copy
  DevBuf rec;                              // the job record of a single-level solve
};

struct DevLevel {
  HostLevel H;
  TilingDev tiling;     // fused-step tiling in use
  bool tuned = false;   // tiling chosen by measurement (autotuner)
  bool pinned = false;  // tiling set by the caller (lts_set_tiling); not re-tuned
  double tuned_ms = 0;  // measured step time of the chosen tiling
  int ld = 0;           // row pitch (elements) of node/cell arrays and states
  size_t nodes = 0;     // nyn * ld
  DevBuf hx, hy, inv2hx, inv2hy, x, y, cblk, flags, ninfo, invm, qoiw, beta, beta_half;
  std::unique_ptr<MltsDev> mlts;   // tiers of the multi-level step, if attached
  // compact lists of DOFs (flat padded index), used by reductions
  LevelView view() const {
    LevelView v;
    v.nxn = H.nxn; v.nyn = H.nyn; v.ld = ld; v.p = H.p; v.nb = H.n_blocks;
    v.hx = hx.as<double>(); v.hy = hy.as<double>();
    v.inv2hx = inv2hx.as<double>(); v.inv2hy = inv2hy.as<double>();
    v.x = x.as<double>(); v.y = y.as<double>();
    v.cblk = cblk.as<uint8_t>(); v.flags = flags.as<uint8_t>(); v.ninfo = ninfo.as<uint32_t>();
    v.invm = invm.as<double>(); v.qoiw = qoiw.as<double>();
    v.beta = beta.as<double>(); v.beta_half = beta_half.as<double>();
    return v;
  }
};

// A one-dimensional level on the device (Sec. 4.1, 4.2).
struct LineDev {
  LineHost H;
  DevBuf x, invh, invm, pflag, beta;
};

// A triangle-mesh level on the device (Sec. 3.1 on a triangulation).
struct TriDev {
  TriHost H;
  DevLevel shell;        // the header the sample staging reads (n_blocks, p, Chebyshev constants)
  size_t ld = 0;         // state stride per sample (elements): n_dof + 1 rounded up
  DevBuf dx, dy, invm, qoiw, dflag, rp, col, eblk, ewa, ewb, coarse, tiles, ent, tslot, beta;
};

struct lts_error {
  lts_status code;
  std::string msg;
};

}  // namespace lts

struct lts_ctx_s {
  int device = 0;
  int n_cu = 256;                 // compute units of the device
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<std::unique_ptr<lts::DevLevel>> levels;
  std::vector<std::unique_ptr<lts::LineDev>> lines;       // one-dimensional levels
  std::vector<std::unique_ptr<lts::TriDev>> meshes;       // triangle-mesh levels
  lts::DevBuf l_kap, l_coef, l_ns, l_U, l_Uc, l_pa, l_pt, l_mass, l_mean, l_dev;   // their workspace
  // workspace
  lts::DevBuf kappa, coef, nsteps, x0, Qd, perm, flag, st0, st1, wbuf, qa, qb, red, adj, adjscr, dldq, gout, adjlist;
  // batched form: per-job tables, states, job records, captured graph
  lts::DevBuf b_tab, b_states, b_jobs, b_Q, b_mjobs;
  // persistent form: active-sample table, control words (unit counters,
  // barrier arrivals, abort word), barrier wait bound and the wall-clock rate
  lts::DevBuf b_act, p_ctl;
  double barrier_ms = 2000.0;
  int wall_khz = 100000;
  std::map<std::vector<uint64_t>, std::pair<int, int>> batch_forms;   // LTS_BATCH_AUTO: form, S_b cap
  hipGraphExec_t graph = nullptr;
  std::vector<uint64_t> graph_key;
  bool timing = false;
  lts_timing last{};
  std::vector<hipEvent_t> ev_pool;
};

namespace lts {

// Map a HIP error to LTS_ERR_HIP (or LTS_ERR_OOM) with a message.
inline lts_status hip_fail(lts_ctx c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? LTS_ERR_OOM : LTS_ERR_HIP;
}

#define LTS_HIP(ctx, call)                                           \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) return ::lts::hip_fail((ctx), e_, #call); \
  } while (0)

inline lts_status arg_fail(lts_ctx c, const std::string& m) {
  c->err = m;
  return LTS_ERR_ARG;
}

// A sample batch staged for the device.  The host keeps what plans the
// launches: the step counts and steps dt, sorted by decreasing step count
// (stable), the permutation (sorted position -> caller index) and the
// per-sample step coefficients (formed on the host: a_p comes from an
// extended-precision recurrence).  For host arrays it also keeps sorted copies
// of kappa (or g) and x0; device arrays are gathered on the device.
struct Staged {
  int n = 0;
  int ptr_kind = LTS_PTR_HOST;
  bool g_mode = false;                 // the caller passed g = log c, kappa = exp(2 g) on the device
  std::vector<double> kappa, x0;       // host path only (kappa holds g in g_mode)
  std::vector<double> dt, coef;
  std::vector<int> nsteps;
  std::vector<int> perm;               // sorted position -> caller index
};
// Device destinations of a staged batch (sorted order) and the device scratch
// the staging uses (perm: n ints; flag: one int).
struct StagedDev {
  double* kappa;   // [n][nb]
  double* x0;      // [n][2]
  double* coef;    // [n][p+1]
  int* nsteps;     // [n]
  int* perm;       // [n]
  int* flag;       // [1]
};
lts_status stage_samples(lts_ctx c, const DevLevel& lv, const lts_samples* S, Staged& st);
// Writes the staged batch to `d` on the context stream; device kappa / g / x0
// are gathered there by a kernel that also checks them (LTS_ERR_ARG if a value
// is invalid; no step has been launched then).
lts_status upload_staged(lts_ctx c, const DevLevel& lv, const Staged& st, const lts_samples* S,
                         const StagedDev& d);
// The context's own staging buffers for n samples (allocates on demand).
lts_status ctx_staging(lts_ctx c, const DevLevel& lv, int n, StagedDev& d);
// Q of the sorted batch at d_Q into the caller's Q_out (ptr_kind of the
// batch): device outputs are scattered by a kernel, host outputs unpermuted on
// the host.  LTS_ERR_UNSTABLE if a QoI is not finite.
lts_status finish_Q(lts_ctx c, const Staged& st, const double* d_Q, const StagedDev& d, double* Q_out);

// Forward solve of `n` samples on level `lv` (device arrays already staged):
// implemented in the step source.
struct StepPlan;
lts_status forward_device(lts_ctx c, const DevLevel& lv, int n, const double* d_kappa,
                          const double* d_coef, const int* d_nsteps, const double* d_x0,
                          double width, const std::vector<int>& h_nsteps, int precision,
                          bool per_sample, double* d_Q);

// The same solve on caller-provided state buffers B0, B1 (n * lv.nodes values
// each, binary64 or, under LTS_FP32_STEP, binary32); allocates nothing on the
// device (HIP events only when `timing`).
lts_status forward_device_states(lts_ctx c, const DevLevel& lv, int n, const double* d_kappa,
                                 const double* d_coef, const int* d_nsteps, const double* d_x0, double width,
                                 const std::vector<int>& h_nsteps, int precision, bool per_sample, double* d_Q,
                                 double* B0, double* B1, bool timing);

lts_status moments_device(lts_ctx c, const double* d_x, int n, double* d_out3);
// (n, mean, M2) of each column b of the row-major [n][nb] array into d_out[3 b .. 3 b + 2].
lts_status moments_cols_device(lts_ctx c, const double* d_x, int n, int nb, double* d_out);

// Takes the device address of the no-allocation scratch array on `device`
// (current) once per device (see lts_noalloc.hip).
lts_status noalloc_attach(lts_ctx c, int device);

// u_0 (pulse) into B0 and zeros into B1 for samples 0..n-1.
lts_status init_states(lts_ctx c, const DevLevel& lv, int n, const double* d_x0, double width, double* B0,
                       double* B1, bool fp32 = false);

// Q[s] = w^T u_{n_steps[s]} with the final state in B[n_steps[s] % 2].
lts_status qoi_device(lts_ctx c, const DevLevel& lv, int n, const int* d_nsteps, const double* B0,
                      const double* B1, double* d_Q, bool fp32 = false);

// Checkpointed discrete adjoint for one sub-batch (see lts_adjoint.hip).
lts_status adjoint_device(lts_ctx c, const DevLevel& lv, int n, const double* d_kappa,
                          const double* d_coef, const int* d_nsteps, const double* d_x0, double width,
                          const std::vector<int>& h_nsteps, int K, const double* d_dldq, double* d_Q,
                          double* d_out, int s_base);

lts_status upload_tiling(lts_ctx c, const TilingHost& T, TilingDev& D);

// Threads of the compact fine workgroups of a launch with `active` samples on
// tiling T.  A small workgroup (T.nt < 1024) shares its CU with others: more
// throughput when the launch has workgroups to spare, a longer step when it
// has at most one or two per CU.  Every size gives the same results.
inline int compact_threads(const TilingDev& T, int active, int n_cu) {
  const long long w = (long long)active * T.n_fine;
  if (w <= n_cu) return kFineThreads;
  if (w <= 2LL * n_cu) return std::max(T.nt, 512);
  return T.nt;
}

// Tile-size candidates (TX, TY) tried for the fused step, in order.
const std::vector<std::pair<int, int>>& tile_candidates();
// The same for one level, led by one tile over the whole level.
std::vector<std::pair<int, int>> level_tile_candidates(const HostLevel& H);

// Grid origins tried for a tile size (0 and aligned to the F+ bounding box).
std::vector<std::pair<int, int>> tile_origins(const HostLevel& H, int TX, int TY);

// Choose and upload a default tiling (smallest region overhead that fits).
lts_status default_tiling(lts_ctx c, DevLevel& lv);

// Choose the tiling of a level by timing candidate tilings (cached per level shape).
lts_status autotune_level(lts_ctx c, DevLevel& lv);

// One batched step launch over several jobs (see lts_fused.hip).
struct StepArgs;
// With fp32 the jobs' state buffers hold binary32 values.
// kinds = 1: the coarse-item launch only.
lts_status launch_multi_step(lts_ctx c, const StepArgs* d_jobs, const std::vector<const TilingDev*>& T,
                             const std::vector<int>& active, int step, hipStream_t stream, bool fp32 = false,
                             int kinds = 5);
// Multi-level LTS jobs (lts_mlts.hip): the size of a job's device record, a
// record for samples 0 .. n-1 (sorted order) of level lv with their tables at
// d_kappa, d_c0 and states B0, B1 (written to out), the innermost half-step
// coefficients c0 of steps dt, and one fine-tile launch of every job for step
// `step` (active[j] samples of job j; M[j] its tiers).
size_t mlts_record_size();
void mlts_record(const DevLevel& lv, const double* d_kappa, const double* d_c0, double* B0, double* B1, void* out);
void mlts_c0(const MltsDev& M, const double* dt, int n, double* c0);
lts_status launch_mlts(lts_ctx c, const void* d_jobs, const std::vector<const MltsDev*>& M,
                       const std::vector<int>& active, int step, hipStream_t stream, bool fp32 = false);
// The persistent form: steps 0 .. n_steps-1 of every job in cooperative
// launches of one workgroup per CU with a grid barrier after each step
// (see lts_fused.hip).  act_host[t * n_jobs + j] = active samples of job j at
// step t (its copy d_act on the device); sb[j] = 0 for a rect-mode job, else
// S_b in {1, 2, 4}, the samples a workgroup runs side by side (compact tiles
// of at most 1024 / S_b threads).  Waits for the launches; LTS_ERR_STATE if a
// workgroup gave up at a barrier (c->barrier_ms).
lts_status launch_persist(lts_ctx c, const StepArgs* d_jobs, const std::vector<const TilingDev*>& T,
                          const std::vector<int>& act_host, const int* d_act, int n_steps, const std::vector<int>& sb,
                          hipStream_t stream, bool fp32);
// The adjoint's substep sweeps of one backward step on a compact tiling (FP64;
// samples 0 .. active-1): reverse = false recomputes d_1 .. d_p of y = Y at
// the nodes of P into D1 + (m-1)*astride; reverse = true runs the reverse
// sweep from Lambda_p = f M mu (mu = MU; rho_m as in lts_adjoint.hip) and
// writes Lambda_1 .. Lambda_p-1 into Lam1 + (m-1)*astride and lw into LW, at
// the nodes of P (per sample at + s*sstride).  With Ynew, the recompute also
// writes y_n-1 = 2 R y - y_n+1 (y_n+1 = Yold) at the tiles' own F+ nodes.
lts_status launch_adj_compact(lts_ctx c, const DevLevel& lv, const TilingDev& T, const double* d_kappa,
                              const double* d_coef, const double* Y, const double* MU, double* D1, double* Lam1,
                              double* LW, const double* rho, size_t astride, size_t sstride, int active, double f,
                              bool reverse, hipStream_t stream, const double* Yold = nullptr,
                              double* Ynew = nullptr);
// Largest S_b of a tiling: 0 in rect mode, else 1024 / (fewest threads holding its largest region).
inline int persist_sb_max(const TilingDev& T) { return T.rect ? 0 : kFineThreads / T.nt; }
// Writes the static step record of one job (step_args_size() bytes) to `out`.
void job_record(const DevLevel& lv, const TilingDev& T, const double* d_kappa, const double* d_coef,
                double* B0, double* B1, size_t sstride, void* out);
size_t step_args_size();

// One fused step launch for samples s0 .. s0+active-1 (sorted order): reads
// u_n from Ucur and u_n-1 from Uold, writes u_n+1 to Unew (NULL: into Uold).
// With fp32 the state buffers hold binary32 values (stride sstride elements).
lts_status launch_step(lts_ctx c, const DevLevel& lv, const TilingDev& T, const double* d_kappa,
                       const double* d_coef, const double* Ucur, double* Uold, size_t sstride, int s0,
                       int active, int startup, hipStream_t stream, bool fp32 = false, double* Unew = nullptr);
// The coarse-item launch of launch_step alone: the DOFs outside F+ (FP32
// states when fp32, the buffers then holding floats).
lts_status launch_coarse(lts_ctx c, const DevLevel& lv, const TilingDev& T, const double* d_kappa,
                         const double* d_coef, const double* Ucur, double* Uold, size_t sstride, int active,
                         int startup, hipStream_t stream, bool fp32 = false, double* Unew = nullptr);

}  // namespace lts
