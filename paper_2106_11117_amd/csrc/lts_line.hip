// One-dimensional workloads (Sec. 4.1, 4.2): stabilized LF-LTS on an interval
// with Neumann data, u(T) as the L^2(D)-valued QoI, and Algorithm 1 with the
// level variances and the bias in the L^2 norm.
//
// A 1D level has a few thousand nodes, so one workgroup of one wavefront per
// sample keeps the whole state in LDS and runs every time step of the sample in
// one launch (a barrier per step, no HBM traffic until u(T) is written).  Per
// step the nodes outside F+ take the single update u_n+1 = 2 u_n - u_n-1 +
// 2 a_p w (lanes strided over the nodes); the F+ nodes (contiguous, at most
// 64) sit one per lane for the p substeps, east / west neighbours by DPP lane
// shifts, with zero beyond F+ (no P node there).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

namespace lts {

namespace {

constexpr int kLineMaxNodes = 4096;   // 4 arrays of doubles in LDS: 128 KiB

struct LineArgs {
  int n, f0, nf, p;
  const double* __restrict__ x;
  const double* __restrict__ invh;      // [n-1] 1 / |cell|
  const double* __restrict__ invm;      // [n]
  const uint8_t* __restrict__ pflag;    // [n] node in P
  const double* __restrict__ beta;      // [p] beta_m (index 0 unused)
  const double* __restrict__ kappa;     // [S][n-1]
  const double* __restrict__ coef;      // [S][p+1]: a_p, c_1, c_2,1 .. c_2,p-1
  const int* __restrict__ nsteps;       // [S]
  double px, pw2;
  double* __restrict__ U;               // [S][n] u(T)
};

__global__ __launch_bounds__(64) void k_line(LineArgs a) {
  extern __shared__ double sh[];
  const int s = blockIdx.x, lane = threadIdx.x, n = a.n;
  double* u0 = sh;                      // the two time levels
  double* u1 = sh + n;
  double* ce = sh + 2 * n;              // kappa / |cell| per cell
  double* im = sh + 3 * n;              // 1 / m per node
  const double* __restrict__ kap = a.kappa + (size_t)s * (n - 1);
  for (int i = lane; i < n; i += 64) {
    im[i] = a.invm[i];
    const double dx = a.x[i] - a.px;
    u0[i] = exp(-(dx * dx) / a.pw2);
    u1[i] = 0.0;
    if (i < n - 1) ce[i] = kap[i] * a.invh[i];
  }
  __syncthreads();
  const double* __restrict__ cf = a.coef + (size_t)s * (a.p + 1);
  const double ap = cf[0];
  const int ns = a.nsteps[s];
  const bool fl = lane < a.nf;
  const int fi = a.f0 + lane;
  double aE = 0.0, aW = 0.0, pm = 0.0;
  bool pE = false, pW = false;
  if (fl) {
    aE = fi < n - 1 ? im[fi] * ce[fi] : 0.0;
    aW = fi > 0 ? im[fi] * ce[fi - 1] : 0.0;
    pm = a.pflag[fi] ? 1.0 : 0.0;
    pE = fi < n - 1 && a.pflag[fi + 1];
    pW = fi > 0 && a.pflag[fi - 1];
  }
  for (int t = 0; t < ns; ++t) {
    const double* cur = (t & 1) ? u1 : u0;
    double* nw = (t & 1) ? u0 : u1;     // u_n-1 in, u_n+1 out
    const bool st = t == 0;
    for (int i = lane; i < n; i += 64) {
      if (i >= a.f0 && i < a.f0 + a.nf) continue;
      const double v = cur[i];          // no P node next to i: (I - P) u = u here
      double k = 0.0;
      if (i > 0) k += ce[i - 1] * (v - cur[i - 1]);
      if (i < n - 1) k += ce[i] * (v - cur[i + 1]);
      const double d = ap * (im[i] * k);
      nw[i] = st ? v + d : 2.0 * v - nw[i] + 2.0 * d;
    }
    if (a.nf > 0) {
      double uc = 0.0, w = 0.0;
      if (fl) {
        uc = cur[fi];
        const double uE = fi < n - 1 ? cur[fi + 1] : 0.0, uW = fi > 0 ? cur[fi - 1] : 0.0;
        const double vi = pm != 0.0 ? 0.0 : uc, vE = pE ? 0.0 : uE, vW = pW ? 0.0 : uW;
        w = aE * (vi - vE) + aW * (vi - vW);             // A_u (I - P) u_n
      }
      double dc = 0.0, dq = 0.0, q = pm * uc;
      for (int m = 0; m < a.p; ++m) {
        const double c = cf[1 + m];
        const double b = m > 0 ? a.beta[m] : 0.0;
        const double qE = lane_next(q), qW = lane_prev(q);
        const double r = w + (aE * (q - qE) + aW * (q - qW));
        const double dn = (dc + b * (dc - dq)) - c * r;
        dq = dc;
        dc = dn;
        q = pm * (uc + dn);
      }
      if (fl) nw[fi] = st ? uc + dc : 2.0 * uc - nw[fi] + 2.0 * dc;
    }
    __syncthreads();
  }
  const double* fin = (ns & 1) ? u1 : u0;
  for (int i = lane; i < n; i += 64) a.U[(size_t)s * n + i] = fin[i];
}

// D[s][j] = Uf[s][j] - (I Uc[s])_j, I the nodal interpolation from the coarse
// mesh: (I v)_j = v[a_j] + t_j (v[a_j + 1] - v[a_j]); no coarse term if Uc is null.
__global__ __launch_bounds__(256) void k_line_delta(const double* __restrict__ Uf, int nfn,
                                                    const double* __restrict__ Uc, int ncn,
                                                    const int* __restrict__ pa, const double* __restrict__ pt,
                                                    int rows, double* __restrict__ D) {
  const long long tot = (long long)rows * nfn;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(e / nfn), j = (int)(e - (long long)s * nfn);
    double v = Uf[e];
    if (Uc) {
      const double* c = Uc + (size_t)s * ncn;
      const int k = pa[j];
      v -= c[k] + pt[j] * (c[k + 1] - c[k]);
    }
    D[e] = v;
  }
}

// mean[j] = sum_s D[s][j] / rows, rows summed in order.
__global__ __launch_bounds__(256) void k_col_mean(const double* __restrict__ D, int rows, int cols,
                                                  double* __restrict__ mean) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double acc = 0.0;
  for (int s = 0; s < rows; ++s) acc += D[(size_t)s * cols + j];
  mean[j] = acc / (double)rows;
}

// dev[s] = sum_j m_j (D[s][j] - mean_j)^2: one workgroup per row, fixed order.
__global__ __launch_bounds__(256) void k_row_dev(const double* __restrict__ D, int cols, const double* __restrict__ mean,
                                                 const double* __restrict__ m, double* __restrict__ dev) {
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int j = threadIdx.x; j < cols; j += blockDim.x) {
    const double d = D[(size_t)s * cols + j] - mean[j];
    acc += m[j] * (d * d);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) dev[s] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ void k_nonfinite(const double* __restrict__ v, long long n, int* __restrict__ bad) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    if (!isfinite(v[e])) atomicOr(bad, 1);
}

int grid_of(long long work) { return (int)std::max(1LL, std::min((work + 255) / 256, 4096LL)); }

const LineDev* get_line(lts_ctx c, int32_t id) {
  return id >= 0 && id < (int32_t)c->lines.size() ? c->lines[id].get() : nullptr;
}

// One line solve of n samples already on the device: kappa [n][n-1], coefficient
// tables [n][p+1], n_steps [n]; u(T) into U [n][nodes].
lts_status line_solve_device(lts_ctx c, const LineDev& L, int n, const double* d_kap, const double* d_coef,
                             const int* d_ns, const lts_line_sample_rule& rule, double* d_U) {
  if (n == 0) return LTS_OK;
  LineArgs a;
  a.n = (int)L.H.x.size();
  a.f0 = L.H.f0;
  a.nf = L.H.nf;
  a.p = L.H.p;
  a.x = L.x.as<double>();
  a.invh = L.invh.as<double>();
  a.invm = L.invm.as<double>();
  a.pflag = L.pflag.as<uint8_t>();
  a.beta = L.beta.as<double>();
  a.kappa = d_kap;
  a.coef = d_coef;
  a.nsteps = d_ns;
  a.px = rule.pulse_x;
  a.pw2 = rule.pulse_w2;
  a.U = d_U;
  const size_t lds = 4 * (size_t)a.n * sizeof(double);
  LTS_HIP(c, hipFuncSetAttribute((const void*)k_line, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  k_line<<<n, 64, lds, c->stream>>>(a);
  LTS_HIP(c, hipGetLastError());
  return LTS_OK;
}

std::string check_sample_rule(const lts_line_sample_rule* r) {
  if (!r) return "NULL sample rule";
  if (r->kind != LTS_LINE_KL && r->kind != LTS_LINE_JUMP) return "unknown line sample kind";
  if (!(r->pulse_w2 > 0.0) || !(r->T > 0.0) || !(r->cfl > 0.0)) return "pulse_w2, T and cfl must be > 0";
  return "";
}

// Per-sample step coefficient tables of a batch on the level.
std::vector<double> line_coefs(const LineHost& L, const double* dt, int n) {
  HostLevel h;
  h.p = L.p;
  h.nu = L.nu;
  h.delta = L.delta;
  h.omega = L.omega;
  h.beta = L.beta;
  h.beta_half = L.beta_half;
  std::vector<double> cf((size_t)n * (L.p + 1));
  for (int s = 0; s < n; ++s) step_coefficients(h, dt[s], &cf[(size_t)s * (L.p + 1)]);
  return cf;
}

double line_cost(const LineHost& L, const lts_line_sample_rule& rule) {
  long long nP = 0;
  for (uint8_t v : L.P) nP += v;
  const double n = (double)L.x.size();
  return std::ceil(rule.T / (rule.cfl * L.H)) * ((n - (double)nP) + (double)L.p * (double)nP);
}

// Nodal interpolation data from `coarse` to the nodes of `fine` (nested meshes).
void prolong_table(const LineHost& coarse, const LineHost& fine, std::vector<int>& pa, std::vector<double>& pt) {
  const int nc = (int)coarse.x.size(), nf = (int)fine.x.size();
  pa.resize(nf);
  pt.resize(nf);
  for (int j = 0; j < nf; ++j) {
    int k = (int)(std::upper_bound(coarse.x.begin(), coarse.x.end(), fine.x[j]) - coarse.x.begin()) - 1;
    k = std::min(std::max(k, 0), nc - 2);
    pa[j] = k;
    pt[j] = (fine.x[j] - coarse.x[k]) / (coarse.x[k + 1] - coarse.x[k]);
  }
}

}  // namespace

}  // namespace lts

using namespace lts;

extern "C" {

lts_status lts_line_level_host(const lts_line_rule* r, lts_line_info* info, double* x, double* mass, uint8_t* P) {
  if (!r || !info) return LTS_ERR_ARG;
  LineHost L;
  if (!build_line_level(*r, L).empty()) return LTS_ERR_ARG;
  info->n_nodes = (int32_t)L.x.size();
  int nP = 0;
  for (uint8_t v : L.P) nP += v;
  info->n_P = nP;
  info->p = L.p;
  info->f0 = L.f0;
  info->n_fplus = L.nf;
  info->H = L.H;
  info->nu = L.nu;
  if (x) std::memcpy(x, L.x.data(), L.x.size() * 8);
  if (mass) std::memcpy(mass, L.mass.data(), L.mass.size() * 8);
  if (P) std::memcpy(P, L.P.data(), L.P.size());
  return LTS_OK;
}

lts_status lts_gen_line_samples(uint64_t seed, int32_t sample_level, int64_t first, int32_t n,
                                const lts_line_sample_rule* rule, const lts_line_rule* mesh, double* kappa,
                                int32_t* n_steps, double* dt) {
  if (!rule || !mesh || !check_sample_rule(rule).empty()) return LTS_ERR_ARG;
  LineHost L;
  if (!build_line_level(*mesh, L).empty()) return LTS_ERR_ARG;
  return gen_line_samples(seed, sample_level, first, n, *rule, L, kappa, n_steps, dt).empty() ? LTS_OK : LTS_ERR_ARG;
}

lts_status lts_build_line_level(lts_ctx c, const lts_line_rule* r, int32_t* id) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!r || !id) return arg_fail(c, "NULL argument");
  auto D = std::make_unique<LineDev>();
  std::string e = build_line_level(*r, D->H);
  if (!e.empty()) return arg_fail(c, e);
  const LineHost& H = D->H;
  const int n = (int)H.x.size();
  if (n > kLineMaxNodes) return arg_fail(c, "line level: more than 4096 nodes (the state lives in LDS)");
  std::vector<double> invh(n - 1), invm(n), beta(std::max(H.p, 1), 0.0);
  for (int i = 0; i + 1 < n; ++i) invh[i] = 1.0 / (H.x[i + 1] - H.x[i]);
  for (int i = 0; i < n; ++i) invm[i] = 1.0 / H.mass[i];
  for (int k = 1; k < H.p; ++k) beta[k] = H.beta[k];
  LTS_HIP(c, hipSetDevice(c->device));
  auto put = [&](DevBuf& b, const void* src, size_t bytes) -> hipError_t {
    hipError_t er = b.ensure(std::max<size_t>(bytes, 8));
    return er != hipSuccess ? er : hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t er;
  if ((er = put(D->x, H.x.data(), n * 8)) != hipSuccess || (er = put(D->invh, invh.data(), (n - 1) * 8)) != hipSuccess ||
      (er = put(D->invm, invm.data(), n * 8)) != hipSuccess || (er = put(D->pflag, H.P.data(), n)) != hipSuccess ||
      (er = put(D->beta, beta.data(), beta.size() * 8)) != hipSuccess)
    return hip_fail(c, er, "upload line level");
  *id = (int32_t)c->lines.size();
  c->lines.push_back(std::move(D));
  return LTS_OK;
}

lts_status lts_line_forward(lts_ctx c, int32_t line_id, int32_t n, int32_t ptr_kind, const double* kappa,
                            const int32_t* n_steps, const double* dt, const lts_line_sample_rule* rule,
                            double* U_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  const LineDev* L = get_line(c, line_id);
  if (!L) return arg_fail(c, "no such line level");
  std::string e = check_sample_rule(rule);
  if (!e.empty()) return arg_fail(c, e);
  if (n < 0) return arg_fail(c, "n must be >= 0");
  if (ptr_kind != LTS_PTR_HOST && ptr_kind != LTS_PTR_DEVICE) return arg_fail(c, "bad ptr_kind");
  if (n == 0) return LTS_OK;
  if (!kappa || !n_steps || !dt || !U_out) return arg_fail(c, "NULL array");
  const int nodes = (int)L->H.x.size(), cells = nodes - 1;
  const bool dev = ptr_kind == LTS_PTR_DEVICE;
  LTS_HIP(c, hipSetDevice(c->device));
  // dt and the step counts plan the coefficient tables on the host
  std::vector<double> hdt(n);
  std::vector<int32_t> hns(n);
  const hipMemcpyKind k = dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  LTS_HIP(c, hipMemcpyAsync(hdt.data(), dt, (size_t)n * 8, k, c->stream));
  LTS_HIP(c, hipMemcpyAsync(hns.data(), n_steps, (size_t)n * 4, k, c->stream));
  LTS_HIP(c, hipStreamSynchronize(c->stream));
  for (int s = 0; s < n; ++s)
    if (!(hdt[s] > 0.0) || !std::isfinite(hdt[s]) || hns[s] < 1) return arg_fail(c, "dt > 0 and n_steps >= 1 required");
  if (!dev) {
    for (size_t q = 0; q < (size_t)n * cells; ++q)
      if (!(kappa[q] > 0.0) || !std::isfinite(kappa[q])) return arg_fail(c, "kappa must be finite and > 0");
  }
  std::vector<double> cf = line_coefs(L->H, hdt.data(), n);
  LTS_HIP(c, c->l_coef.ensure(cf.size() * 8));
  LTS_HIP(c, c->l_ns.ensure((size_t)n * 4));
  LTS_HIP(c, c->flag.ensure(256));
  LTS_HIP(c, hipMemcpyAsync(c->l_coef.p, cf.data(), cf.size() * 8, hipMemcpyHostToDevice, c->stream));
  LTS_HIP(c, hipMemcpyAsync(c->l_ns.p, hns.data(), (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  const double* d_kap = kappa;
  double* d_U = U_out;
  if (!dev) {
    LTS_HIP(c, c->l_kap.ensure((size_t)n * cells * 8));
    LTS_HIP(c, c->l_U.ensure((size_t)n * nodes * 8));
    LTS_HIP(c, hipMemcpyAsync(c->l_kap.p, kappa, (size_t)n * cells * 8, hipMemcpyHostToDevice, c->stream));
    d_kap = c->l_kap.as<double>();
    d_U = c->l_U.as<double>();
  }
  lts_status r = line_solve_device(c, *L, n, d_kap, c->l_coef.as<double>(), c->l_ns.as<int>(), *rule, d_U);
  if (r != LTS_OK) return r;
  int bad = 0;
  LTS_HIP(c, hipMemsetAsync(c->flag.p, 0, 4, c->stream));
  k_nonfinite<<<grid_of((long long)n * nodes), 256, 0, c->stream>>>(d_U, (long long)n * nodes, c->flag.as<int>());
  LTS_HIP(c, hipGetLastError());
  LTS_HIP(c, hipMemcpyAsync(&bad, c->flag.p, 4, hipMemcpyDeviceToHost, c->stream));
  if (!dev) LTS_HIP(c, hipMemcpyAsync(U_out, d_U, (size_t)n * nodes * 8, hipMemcpyDeviceToHost, c->stream));
  LTS_HIP(c, hipStreamSynchronize(c->stream));
  if (bad) {
    c->err = "non-finite u(T) (unstable sample)";
    return LTS_ERR_UNSTABLE;
  }
  return LTS_OK;
}

lts_status lts_line_mlmc(lts_ctx c, const lts_line_mlmc_opts* op, lts_line_mlmc_result* out, double* estimate) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!op || !out || !estimate) return arg_fail(c, "NULL argument");
  const lts_line_mlmc_opts& o = *op;
  if (o.n_levels < 1 || o.n_levels > LTS_MAX_LEVELS) return arg_fail(c, "n_levels out of range");
  std::vector<const LineDev*> lv(o.n_levels);
  for (int l = 0; l < o.n_levels; ++l) {
    if (!(lv[l] = get_line(c, o.line_ids[l]))) return arg_fail(c, "bad line level id");
    if (o.N_init[l] < 2) return arg_fail(c, "N_init must be >= 2");
  }
  std::string e = check_sample_rule(&o.rule);
  if (!e.empty()) return arg_fail(c, e);
  if (!(o.eps > 0.0) || !(o.alpha > 0.0)) return arg_fail(c, "eps and alpha must be > 0");
  LTS_HIP(c, hipSetDevice(c->device));
  const int Lmax = o.n_levels - 1;
  int L = std::min(std::max(o.L_start, 0), Lmax);
  std::vector<double> C(o.n_levels);
  for (int l = 0; l < o.n_levels; ++l)
    C[l] = line_cost(lv[l]->H, o.rule) + (l > 0 ? line_cost(lv[l - 1]->H, o.rule) : 0.0);
  // per level: Delta Q rows on the device (grown as N_l grows)
  std::vector<DevBuf> rows(o.n_levels);
  std::vector<int64_t> have(o.n_levels, 0), N(o.n_levels, 0);
  for (int l = 0; l <= L; ++l) N[l] = o.N_init[l];
  std::vector<double> var(o.n_levels, 0.0), mnorm(o.n_levels, 0.0);
  std::vector<std::vector<double>> mean(o.n_levels);
  auto t0 = std::chrono::steady_clock::now();
  lts_status r;
  // solve new samples [have, N) of level l, append their Delta Q rows
  auto extend = [&](int l) -> lts_status {
    const int add = (int)(N[l] - have[l]);
    if (add <= 0) return LTS_OK;
    const LineHost& F = lv[l]->H;
    const int nfn = (int)F.x.size();
    // grow the row buffer (keep the old rows)
    const size_t need = (size_t)N[l] * nfn * 8;
    if (rows[l].bytes < need) {
      DevBuf nb;
      LTS_HIP(c, nb.ensure(std::max(need, rows[l].bytes * 2)));
      if (have[l] > 0)
        LTS_HIP(c, hipMemcpyAsync(nb.p, rows[l].p, (size_t)have[l] * nfn * 8, hipMemcpyDeviceToDevice, c->stream));
      LTS_HIP(c, hipStreamSynchronize(c->stream));
      std::swap(rows[l].p, nb.p);
      std::swap(rows[l].bytes, nb.bytes);
    }
    double* Uc = nullptr;
    int ncn = 0;
    std::vector<double> kap, dtv, cf;
    std::vector<int32_t> ns;
    for (int side = 0; side < (l > 0 ? 2 : 1); ++side) {
      const LineHost& M = side == 0 ? F : lv[l - 1]->H;
      const int nodes = (int)M.x.size(), cells = nodes - 1;
      kap.resize((size_t)add * cells);
      dtv.resize(add);
      ns.resize(add);
      std::string ge = gen_line_samples(o.seed, l, have[l], add, o.rule, M, kap.data(), ns.data(), dtv.data());
      if (!ge.empty()) return arg_fail(c, ge);
      cf = line_coefs(M, dtv.data(), add);
      LTS_HIP(c, c->l_kap.ensure(kap.size() * 8));
      LTS_HIP(c, c->l_coef.ensure(cf.size() * 8));
      LTS_HIP(c, c->l_ns.ensure((size_t)add * 4));
      DevBuf& ub = side == 0 ? c->l_U : c->l_Uc;
      LTS_HIP(c, ub.ensure((size_t)add * nodes * 8));
      LTS_HIP(c, hipMemcpyAsync(c->l_kap.p, kap.data(), kap.size() * 8, hipMemcpyHostToDevice, c->stream));
      LTS_HIP(c, hipMemcpyAsync(c->l_coef.p, cf.data(), cf.size() * 8, hipMemcpyHostToDevice, c->stream));
      LTS_HIP(c, hipMemcpyAsync(c->l_ns.p, ns.data(), (size_t)add * 4, hipMemcpyHostToDevice, c->stream));
      lts_status rr = line_solve_device(c, side == 0 ? *lv[l] : *lv[l - 1], add, c->l_kap.as<double>(),
                                        c->l_coef.as<double>(), c->l_ns.as<int>(), o.rule, ub.as<double>());
      if (rr != LTS_OK) return rr;
      LTS_HIP(c, hipStreamSynchronize(c->stream));   // host tables are reused by the other side
      if (side == 1) {
        Uc = c->l_Uc.as<double>();
        ncn = nodes;
      }
    }
    const int* pa = nullptr;
    const double* pt = nullptr;
    if (l > 0) {
      std::vector<int> ha;
      std::vector<double> ht;
      prolong_table(lv[l - 1]->H, F, ha, ht);
      LTS_HIP(c, c->l_pa.ensure((size_t)nfn * 4));
      LTS_HIP(c, c->l_pt.ensure((size_t)nfn * 8));
      LTS_HIP(c, hipMemcpyAsync(c->l_pa.p, ha.data(), (size_t)nfn * 4, hipMemcpyHostToDevice, c->stream));
      LTS_HIP(c, hipMemcpyAsync(c->l_pt.p, ht.data(), (size_t)nfn * 8, hipMemcpyHostToDevice, c->stream));
      pa = c->l_pa.as<int>();
      pt = c->l_pt.as<double>();
    }
    k_line_delta<<<grid_of((long long)add * nfn), 256, 0, c->stream>>>(
        c->l_U.as<double>(), nfn, Uc, ncn, pa, pt, add, rows[l].as<double>() + (size_t)have[l] * nfn);
    LTS_HIP(c, hipGetLastError());
    LTS_HIP(c, hipStreamSynchronize(c->stream));
    have[l] = N[l];
    return LTS_OK;
  };
  // mean vector and V_l of level l's N_l rows
  auto moments = [&](int l) -> lts_status {
    const LineHost& F = lv[l]->H;
    const int nfn = (int)F.x.size();
    const int nr = (int)N[l];
    LTS_HIP(c, c->l_mean.ensure((size_t)nfn * 8));
    LTS_HIP(c, c->l_mass.ensure((size_t)nfn * 8));
    LTS_HIP(c, c->l_dev.ensure((size_t)nr * 8));
    LTS_HIP(c, hipMemcpyAsync(c->l_mass.p, F.mass.data(), (size_t)nfn * 8, hipMemcpyHostToDevice, c->stream));
    k_col_mean<<<(nfn + 255) / 256, 256, 0, c->stream>>>(rows[l].as<double>(), nr, nfn, c->l_mean.as<double>());
    k_row_dev<<<nr, 256, 0, c->stream>>>(rows[l].as<double>(), nfn, c->l_mean.as<double>(), c->l_mass.as<double>(),
                                         c->l_dev.as<double>());
    LTS_HIP(c, hipGetLastError());
    std::vector<double> dev(nr);
    mean[l].resize(nfn);
    LTS_HIP(c, hipMemcpyAsync(mean[l].data(), c->l_mean.p, (size_t)nfn * 8, hipMemcpyDeviceToHost, c->stream));
    LTS_HIP(c, hipMemcpyAsync(dev.data(), c->l_dev.p, (size_t)nr * 8, hipMemcpyDeviceToHost, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));
    double sdev = 0.0, sm = 0.0;
    for (double v : dev) sdev += v;
    for (int j = 0; j < nfn; ++j) sm += F.mass[j] * (mean[l][j] * mean[l][j]);
    if (!std::isfinite(sdev) || !std::isfinite(sm)) {
      c->err = "non-finite u(T) (unstable sample)";
      return LTS_ERR_UNSTABLE;
    }
    var[l] = nr > 1 ? sdev / (double)(nr - 1) : 0.0;
    mnorm[l] = std::sqrt(sm);
    return LTS_OK;
  };
  bool grew = true;
  while (grew) {
    for (int l = 0; l <= L; ++l)
      if ((r = extend(l)) != LTS_OK) return r;
    for (int l = 0; l <= L; ++l)
      if ((r = moments(l)) != LTS_OK) return r;
    double ssum = 0.0;
    for (int l = 0; l <= L; ++l) ssum += std::sqrt(var[l] * C[l]);
    grew = false;
    for (int l = 0; l <= L; ++l) {
      const double nl = std::ceil(2.0 / (o.eps * o.eps) * std::sqrt(var[l] / C[l]) * ssum);
      if (nl > (double)N[l]) {
        N[l] = (int64_t)nl;
        grew = true;
      }
    }
    const double bias = mnorm[L] / (std::pow(2.0, o.alpha) - 1.0);
    if (bias * bias >= 0.5 * o.eps * o.eps && L < Lmax) {
      ++L;
      N[L] = o.N_init[L];
      grew = true;
    }
  }
  *out = lts_line_mlmc_result{};
  double vsum = 0.0;
  for (int l = 0; l <= L; ++l) {
    out->N[l] = (int32_t)N[l];
    out->var[l] = var[l];
    out->mean_norm[l] = mnorm[l];
    out->cost[l] = C[l];
    vsum += var[l] / (double)N[l];
  }
  const double bias = mnorm[L] / (std::pow(2.0, o.alpha) - 1.0);
  out->L = L;
  out->bias = bias;
  out->rmse = std::sqrt(vsum + bias * bias);
  out->converged = bias * bias < 0.5 * o.eps * o.eps;
  out->n_nodes = (int32_t)lv[L]->H.x.size();
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // estimate: sum_l I mean_l on the finest mesh used
  std::vector<double> est = mean[0];
  for (int l = 1; l <= L; ++l) {
    std::vector<int> pa;
    std::vector<double> pt;
    prolong_table(lv[l - 1]->H, lv[l]->H, pa, pt);
    std::vector<double> nx(lv[l]->H.x.size());
    for (size_t j = 0; j < nx.size(); ++j)
      nx[j] = (est[pa[j]] + pt[j] * (est[pa[j] + 1] - est[pa[j]])) + mean[l][j];
    est.swap(nx);
  }
  std::memcpy(estimate, est.data(), est.size() * 8);
  return LTS_OK;
}

}  // extern "C"
