// C ABI of the library: contexts, levels, samples, forward solves, moments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

using namespace lts;

namespace lts {

namespace {

// Sorted copies of a device batch: row t of the outputs is caller sample
// perm[t].  kappa = exp(2 g) when the caller passed g (kappa NULL).  Invalid
// values set bit 1 (coefficient) or bit 2 (pulse centre) of *bad.
__global__ __launch_bounds__(256) void k_gather_samples(const double* __restrict__ kappa,
                                                        const double* __restrict__ g,
                                                        const double* __restrict__ x0,
                                                        const int* __restrict__ perm, int n, int nb,
                                                        double* __restrict__ kout, double* __restrict__ xout,
                                                        int* __restrict__ bad) {
  const long long tot = (long long)n * (nb + 2);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / (nb + 2)), b = (int)(e - (long long)t * (nb + 2));
    const size_t s = (size_t)perm[t];
    if (b < nb) {
      const double k = kappa ? kappa[s * nb + b] : exp(2.0 * g[s * nb + b]);
      if (!(k > 0.0) || !isfinite(k)) atomicOr(bad, 1);
      kout[(size_t)t * nb + b] = k;
    } else {
      const double v = x0[2 * s + (b - nb)];
      if (!isfinite(v)) atomicOr(bad, 2);
      xout[2 * (size_t)t + (b - nb)] = v;
    }
  }
}

// kappa = exp(2 g) in place (host batches given as g, already sorted).
__global__ __launch_bounds__(256) void k_exp2(double* __restrict__ v, long long n, int* __restrict__ bad) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const double k = exp(2.0 * v[e]);
    if (!(k > 0.0) || !isfinite(k)) atomicOr(bad, 1);
    v[e] = k;
  }
}

// out[perm[t]] = Q[t]; bit 1 of *bad for a non-finite value.
__global__ __launch_bounds__(256) void k_scatter_q(const double* __restrict__ Q, const int* __restrict__ perm, int n,
                                                   double* __restrict__ out, int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double q = Q[t];
  out[perm[t]] = q;
  if (!isfinite(q)) atomicOr(bad, 1);
}

// out[perm[t]][b] = rows[t][b]; bit 1 of *bad for a non-finite value.
__global__ __launch_bounds__(256) void k_scatter_rows(const double* __restrict__ rows, const int* __restrict__ perm,
                                                      int n, int nb, double* __restrict__ out, int* __restrict__ bad) {
  const long long tot = (long long)n * nb;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / nb), b = (int)(e - (long long)t * nb);
    const double v = rows[e];
    out[(size_t)perm[t] * nb + b] = v;
    if (!isfinite(v)) atomicOr(bad, 1);
  }
}

// out[t] = x[perm[t]].
__global__ __launch_bounds__(256) void k_gather_vec(const double* __restrict__ x, const int* __restrict__ perm, int n,
                                                    double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = x[perm[t]];
}

// d = a - b (the coupled difference of Sec. 2.2), optionally copying a and b.
__global__ __launch_bounds__(256) void k_coupled_diff(const double* __restrict__ a, const double* __restrict__ b, int n,
                                                      double* __restrict__ qa, double* __restrict__ qb,
                                                      double* __restrict__ d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (qa) qa[t] = a[t];
  if (qb) qb[t] = b[t];
  if (d) d[t] = a[t] - b[t];
}

__global__ void k_zero_flag(int* __restrict__ f) { *f = 0; }

int grid_for(long long work) { return (int)std::max(1LL, std::min((work + 255) / 256, 4096LL)); }

}  // namespace

// Reads a value of a possibly device-resident caller array to the host on
// the context stream.
static lts_status read_in(lts_ctx c, void* dst, const void* src, size_t bytes, int ptr_kind) {
  if (bytes == 0) return LTS_OK;
  if (ptr_kind == LTS_PTR_DEVICE) {
    LTS_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));
  } else {
    std::memcpy(dst, src, bytes);
  }
  return LTS_OK;
}

lts_status stage_samples(lts_ctx c, const DevLevel& lv, const lts_samples* S, Staged& st) {
  if (!S) return arg_fail(c, "samples is NULL");
  if (S->n < 0) return arg_fail(c, "samples.n must be >= 0");
  if (S->ptr_kind != LTS_PTR_HOST && S->ptr_kind != LTS_PTR_DEVICE)
    return arg_fail(c, "samples.ptr_kind must be LTS_PTR_HOST or LTS_PTR_DEVICE");
  if (!(S->width > 0.0) || !std::isfinite(S->width)) return arg_fail(c, "samples.width must be > 0");
  const int n = S->n, nb = lv.H.n_blocks, p = lv.H.p;
  st = Staged();
  st.n = n;
  st.ptr_kind = S->ptr_kind;
  st.g_mode = S->kappa == nullptr;
  if (n == 0) return LTS_OK;
  if ((!S->kappa && !S->g) || !S->x0 || !S->n_steps || !S->dt) return arg_fail(c, "NULL sample array");
  LTS_HIP(c, hipSetDevice(c->device));
  std::vector<double> dt(n);
  std::vector<int> ns(n);
  lts_status r;
  if ((r = read_in(c, ns.data(), S->n_steps, (size_t)n * 4, S->ptr_kind)) != LTS_OK) return r;
  if ((r = read_in(c, dt.data(), S->dt, (size_t)n * 8, S->ptr_kind)) != LTS_OK) return r;
  for (int s = 0; s < n; ++s) {
    if (!(dt[s] > 0.0) || !std::isfinite(dt[s])) return arg_fail(c, "dt must be finite and > 0");
    if (ns[s] < 1) return arg_fail(c, "n_steps must be >= 1");
  }
  // sort by decreasing step count (stable): running samples form a prefix
  st.perm.resize(n);
  for (int s = 0; s < n; ++s) st.perm[s] = s;
  std::stable_sort(st.perm.begin(), st.perm.end(), [&](int a, int b) { return ns[a] > ns[b]; });
  st.dt.resize(n);
  st.nsteps.resize(n);
  for (int t = 0; t < n; ++t) {
    st.dt[t] = dt[st.perm[t]];
    st.nsteps[t] = ns[st.perm[t]];
  }
  st.coef.resize((size_t)n * (p + 1));
  for (int t = 0; t < n; ++t) step_coefficients(lv.H, st.dt[t], &st.coef[(size_t)t * (p + 1)]);
  if (S->ptr_kind == LTS_PTR_HOST) {
    const double* kin = st.g_mode ? S->g : S->kappa;
    st.kappa.resize((size_t)n * nb);
    st.x0.resize((size_t)n * 2);
    for (int t = 0; t < n; ++t) {
      const int s = st.perm[t];
      for (int b = 0; b < nb; ++b) {
        const double k = kin[(size_t)s * nb + b];
        if (st.g_mode ? !std::isfinite(k) : (!(k > 0.0) || !std::isfinite(k)))
          return arg_fail(c, st.g_mode ? "g must be finite" : "kappa must be finite and > 0");
        st.kappa[(size_t)t * nb + b] = k;
      }
      st.x0[2 * t] = S->x0[2 * s];
      st.x0[2 * t + 1] = S->x0[2 * s + 1];
      if (!std::isfinite(st.x0[2 * t]) || !std::isfinite(st.x0[2 * t + 1])) return arg_fail(c, "x0 must be finite");
    }
  }
  return LTS_OK;
}

lts_status upload_staged(lts_ctx c, const DevLevel& lv, const Staged& st, const lts_samples* S,
                         const StagedDev& d) {
  const int n = st.n, nb = lv.H.n_blocks, p1 = lv.H.p + 1;
  if (n == 0) return LTS_OK;
  hipStream_t q = c->stream;
  LTS_HIP(c, hipMemcpyAsync(d.coef, st.coef.data(), (size_t)n * p1 * 8, hipMemcpyHostToDevice, q));
  LTS_HIP(c, hipMemcpyAsync(d.nsteps, st.nsteps.data(), (size_t)n * 4, hipMemcpyHostToDevice, q));
  const bool dev = st.ptr_kind == LTS_PTR_DEVICE;
  if (!dev && !st.g_mode) {
    // host batch with kappa: checked on the host, no device check needed
    LTS_HIP(c, hipMemcpyAsync(d.kappa, st.kappa.data(), st.kappa.size() * 8, hipMemcpyHostToDevice, q));
    LTS_HIP(c, hipMemcpyAsync(d.x0, st.x0.data(), st.x0.size() * 8, hipMemcpyHostToDevice, q));
    return LTS_OK;
  }
  k_zero_flag<<<1, 1, 0, q>>>(d.flag);
  if (dev) {
    LTS_HIP(c, hipMemcpyAsync(d.perm, st.perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, q));
    k_gather_samples<<<grid_for((long long)n * (nb + 2)), 256, 0, q>>>(S->kappa, S->kappa ? nullptr : S->g, S->x0,
                                                                     d.perm, n, nb, d.kappa, d.x0, d.flag);
  } else {
    LTS_HIP(c, hipMemcpyAsync(d.kappa, st.kappa.data(), st.kappa.size() * 8, hipMemcpyHostToDevice, q));
    LTS_HIP(c, hipMemcpyAsync(d.x0, st.x0.data(), st.x0.size() * 8, hipMemcpyHostToDevice, q));
    k_exp2<<<grid_for((long long)n * nb), 256, 0, q>>>(d.kappa, (long long)n * nb, d.flag);
  }
  LTS_HIP(c, hipGetLastError());
  int bad = 0;
  LTS_HIP(c, hipMemcpyAsync(&bad, d.flag, 4, hipMemcpyDeviceToHost, q));
  LTS_HIP(c, hipStreamSynchronize(q));
  if (bad & 1) return arg_fail(c, st.g_mode ? "g must be finite (and exp(2 g) finite)" : "kappa must be finite and > 0");
  if (bad & 2) return arg_fail(c, "x0 must be finite");
  return LTS_OK;
}

lts_status ctx_staging(lts_ctx c, const DevLevel& lv, int n, StagedDev& d) {
  const size_t m = std::max(n, 1);
  LTS_HIP(c, c->kappa.ensure(m * lv.H.n_blocks * 8));
  LTS_HIP(c, c->coef.ensure(m * (lv.H.p + 1) * 8));
  LTS_HIP(c, c->nsteps.ensure(m * 4));
  LTS_HIP(c, c->x0.ensure(m * 16));
  LTS_HIP(c, c->Qd.ensure(m * 8));
  LTS_HIP(c, c->perm.ensure(m * 4));
  LTS_HIP(c, c->flag.ensure(256));
  d = StagedDev{c->kappa.as<double>(), c->x0.as<double>(), c->coef.as<double>(), c->nsteps.as<int>(),
                c->perm.as<int>(), c->flag.as<int>()};
  return LTS_OK;
}

lts_status finish_Q(lts_ctx c, const Staged& st, const double* d_Q, const StagedDev& d, double* Q_out) {
  const int n = st.n;
  if (n == 0) return LTS_OK;
  hipStream_t q = c->stream;
  bool finite = true;
  if (st.ptr_kind == LTS_PTR_DEVICE) {
    k_zero_flag<<<1, 1, 0, q>>>(d.flag);
    k_scatter_q<<<(n + 255) / 256, 256, 0, q>>>(d_Q, d.perm, n, Q_out, d.flag);
    LTS_HIP(c, hipGetLastError());
    int bad = 0;
    LTS_HIP(c, hipMemcpyAsync(&bad, d.flag, 4, hipMemcpyDeviceToHost, q));
    LTS_HIP(c, hipStreamSynchronize(q));
    finite = bad == 0;
  } else {
    std::vector<double> qs(n);
    LTS_HIP(c, hipMemcpyAsync(qs.data(), d_Q, (size_t)n * 8, hipMemcpyDeviceToHost, q));
    LTS_HIP(c, hipStreamSynchronize(q));
    for (int t = 0; t < n; ++t) {
      Q_out[st.perm[t]] = qs[t];
      finite = finite && std::isfinite(qs[t]);
    }
  }
  if (!finite) {
    c->err = "non-finite QoI (unstable sample)";
    return LTS_ERR_UNSTABLE;
  }
  return LTS_OK;
}

}  // namespace lts

namespace {

constexpr int kPitchAlign = 8;  // row pitch multiple (doubles): 64-byte rows

lts_status upload_level(lts_ctx c, DevLevel& D) {
  const HostLevel& H = D.H;
  D.ld = (H.nxn + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
  D.nodes = (size_t)H.nyn * D.ld;
  std::vector<double> hx(H.nxn, 0.0), hy(H.nyn, 0.0), ihx(H.nxn, 0.0), ihy(H.nyn, 0.0);
  for (int i = 0; i + 1 < H.nxn; ++i) {
    hx[i] = H.x[i + 1] - H.x[i];
    ihx[i] = 1.0 / (2.0 * hx[i]);
  }
  for (int j = 0; j + 1 < H.nyn; ++j) {
    hy[j] = H.y[j + 1] - H.y[j];
    ihy[j] = 1.0 / (2.0 * hy[j]);
  }
  std::vector<uint8_t> cb(D.nodes, 255), fl(D.nodes, 0);
  std::vector<double> im(D.nodes, 0.0), qw(D.nodes, 0.0);
  for (int b = 0; b < H.nyc; ++b)
    for (int a = 0; a < H.nxc; ++a) {
      const int32_t blk = H.block[(size_t)b * H.nxc + a];
      cb[(size_t)b * D.ld + a] = blk < 0 ? 255 : (uint8_t)blk;
    }
  for (int j = 0; j < H.nyn; ++j)
    for (int i = 0; i < H.nxn; ++i) {
      const size_t k = (size_t)j * H.nxn + i, kd = (size_t)j * D.ld + i;
      fl[kd] = H.flags[k];
      if (H.flags[k] & LTS_NODE_DOF) im[kd] = 1.0 / H.mass[k];
      qw[kd] = H.qoiw[k];
    }
  // packed node word: flags | block of cell (i, j) << 8 | block of cell (i-1, j) << 16
  std::vector<uint32_t> ni(D.nodes, 0);
  for (int j = 0; j < H.nyn; ++j)
    for (int i = 0; i < (int)D.ld; ++i) {
      const size_t kd = (size_t)j * D.ld + i;
      const uint32_t ne = i < H.nxc && j < H.nyc ? cb[kd] : 255u;
      const uint32_t nw = i >= 1 && i - 1 < H.nxc && j < H.nyc ? cb[kd - 1] : 255u;
      ni[kd] = (uint32_t)fl[kd] | ne << 8 | nw << 16;
    }
  std::vector<double> bt(std::max(1, H.p), 0.0), bh(std::max(1, H.p), 0.0);
  for (int k = 1; k < H.p; ++k) {
    bt[k] = H.beta[k];
    bh[k] = H.beta_half[k];
  }
  auto put = [&](DevBuf& b, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = b.ensure(std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return e;
    return hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e;
  if ((e = put(D.hx, hx.data(), hx.size() * 8)) != hipSuccess ||
      (e = put(D.hy, hy.data(), hy.size() * 8)) != hipSuccess ||
      (e = put(D.inv2hx, ihx.data(), ihx.size() * 8)) != hipSuccess ||
      (e = put(D.inv2hy, ihy.data(), ihy.size() * 8)) != hipSuccess ||
      (e = put(D.x, H.x.data(), H.x.size() * 8)) != hipSuccess ||
      (e = put(D.y, H.y.data(), H.y.size() * 8)) != hipSuccess ||
      (e = put(D.cblk, cb.data(), cb.size())) != hipSuccess ||
      (e = put(D.flags, fl.data(), fl.size())) != hipSuccess ||
      (e = put(D.ninfo, ni.data(), ni.size() * 4)) != hipSuccess ||
      (e = put(D.invm, im.data(), im.size() * 8)) != hipSuccess ||
      (e = put(D.qoiw, qw.data(), qw.size() * 8)) != hipSuccess ||
      (e = put(D.beta, bt.data(), bt.size() * 8)) != hipSuccess ||
      (e = put(D.beta_half, bh.data(), bh.size() * 8)) != hipSuccess)
    return hip_fail(c, e, "upload level");
  return LTS_OK;
}

const DevLevel* get_level(lts_ctx c, int32_t level) {
  if (!c || level < 0 || level >= (int32_t)c->levels.size()) return nullptr;
  return c->levels[level].get();
}

lts_status forward_impl(lts_ctx c, int32_t level, const lts_samples* S, int32_t precision,
                        double* Q_out, bool per_sample) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  const DevLevel* lv = get_level(c, level);
  if (!lv) return arg_fail(c, "no such level");
  if (precision != LTS_FP64 && precision != LTS_FP32_STEP) return arg_fail(c, "bad precision");
  if (S && S->n > 0 && !Q_out) return arg_fail(c, "Q_out is NULL");
  Staged st;
  lts_status r = stage_samples(c, *lv, S, st);
  if (r != LTS_OK) return r;
  if (st.n == 0) return LTS_OK;
  LTS_HIP(c, hipSetDevice(c->device));
  StagedDev d;
  if ((r = ctx_staging(c, *lv, st.n, d)) != LTS_OK) return r;
  if ((r = upload_staged(c, *lv, st, S, d)) != LTS_OK) return r;
  r = forward_device(c, *lv, st.n, d.kappa, d.coef, d.nsteps, d.x0, S->width, st.nsteps, precision, per_sample,
                     c->Qd.as<double>());
  if (r != LTS_OK) return r;
  return finish_Q(c, st, c->Qd.as<double>(), d, Q_out);
}

}  // namespace

extern "C" {

lts_status lts_create(lts_ctx* out, int32_t hip_device, void* hip_stream) {
  if (!out) return LTS_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return LTS_ERR_ARG;
  lts_ctx c = new (std::nothrow) lts_ctx_s();
  if (!c) return LTS_ERR_OOM;
  c->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) {
    delete c;
    return LTS_ERR_HIP;
  }
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && n_cu > 0)
    c->n_cu = n_cu;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device) == hipSuccess && khz > 0)
    c->wall_khz = khz;
  if (noalloc_attach(c, hip_device) != LTS_OK) {
    delete c;
    return LTS_ERR_HIP;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return LTS_ERR_HIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return LTS_OK;
}

lts_status lts_destroy(lts_ctx c) {
  if (!c) return LTS_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return LTS_OK;
}

const char* lts_last_error(lts_ctx c) { return c ? c->err.c_str() : "NULL context"; }

lts_status lts_add_level(lts_ctx c, const lts_grid_desc* d, int32_t* id_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!d || !id_out) return arg_fail(c, "NULL argument");
  auto D = std::make_unique<DevLevel>();
  std::string e = build_level_from_desc(*d, D->H);
  if (!e.empty()) return arg_fail(c, e);
  // the step kernels index a sample's nodes with 32-bit row * pitch + column
  const size_t pitch = ((size_t)D->H.nxn + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
  if (pitch * (size_t)D->H.nyn >= ((size_t)1 << 31))
    return arg_fail(c, "grid too large: padded nodes per sample must stay below 2^31");
  LTS_HIP(c, hipSetDevice(c->device));
  lts_status r = upload_level(c, *D);
  if (r != LTS_OK) return r;
  if ((r = default_tiling(c, *D)) != LTS_OK) return r;
  *id_out = (int32_t)c->levels.size();
  c->levels.push_back(std::move(D));
  return LTS_OK;
}

lts_status lts_build_rect_level(lts_ctx c, const lts_rect_rule* r, int32_t* id_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!r || !id_out) return arg_fail(c, "NULL argument");
  std::vector<double> x, y;
  std::vector<uint8_t> act, fine, qoi;
  std::vector<int32_t> blk;
  double h = 0;
  int p = 0, nb = 0;
  std::string e = build_rect_desc(*r, x, y, act, blk, fine, qoi, h, p, nb);
  if (!e.empty()) return arg_fail(c, e);
  lts_grid_desc d{};
  d.nx_cells = (int32_t)x.size() - 1;
  d.ny_cells = (int32_t)y.size() - 1;
  d.x = x.data();
  d.y = y.data();
  d.cell_active = act.data();
  d.cell_block = blk.data();
  d.cell_fine = fine.data();
  d.cell_qoi = qoi.data();
  d.n_blocks = nb;
  d.h = h;
  d.p = p;
  d.nu = r->nu;
  return lts_add_level(c, &d, id_out);
}

lts_status lts_level_info_get(lts_ctx c, int32_t level, lts_level_info* out) {
  if (!c) return LTS_ERR_ARG;
  const DevLevel* lv = get_level(c, level);
  if (!lv || !out) return arg_fail(c, "no such level / NULL out");
  const HostLevel& H = lv->H;
  out->nx_nodes = H.nxn;
  out->ny_nodes = H.nyn;
  out->n_dof = H.n_dof;
  out->n_P = H.n_P;
  out->n_Fplus = H.n_F;
  out->p = H.p;
  out->n_blocks = H.n_blocks;
  out->h = H.h;
  out->nu = H.nu;
  out->delta = H.delta;
  out->omega = H.omega;
  out->tile_x = lv->tiling.TX;
  out->tile_y = lv->tiling.TY;
  out->tile_rect = lv->tiling.rect ? (lv->tiling.mix ? 2 : 1) : 0;
  out->tuned = lv->tuned ? 1 : 0;
  out->halo_ratio = lv->tiling.halo_ratio;
  out->tuned_ms = lv->tuned_ms;
  return LTS_OK;
}

lts_status lts_level_arrays(lts_ctx c, int32_t level, double* x, double* y, uint8_t* flags,
                            double* mass, double* qoi_w, int32_t* cell_block) {
  if (!c) return LTS_ERR_ARG;
  const DevLevel* lv = get_level(c, level);
  if (!lv) return arg_fail(c, "no such level");
  const HostLevel& H = lv->H;
  if (x) std::memcpy(x, H.x.data(), H.x.size() * 8);
  if (y) std::memcpy(y, H.y.data(), H.y.size() * 8);
  if (flags) std::memcpy(flags, H.flags.data(), H.flags.size());
  if (mass) std::memcpy(mass, H.mass.data(), H.mass.size() * 8);
  if (qoi_w) std::memcpy(qoi_w, H.qoiw.data(), H.qoiw.size() * 8);
  if (cell_block) std::memcpy(cell_block, H.block.data(), H.block.size() * 4);
  return LTS_OK;
}

// The host level of a rule (no device involved); "" on success.
static std::string host_level_of_rule(const lts_rect_rule& r, HostLevel& H) {
  std::vector<double> xs, ys;
  std::vector<uint8_t> act, fine, qoi;
  std::vector<int32_t> blk;
  double h = 0;
  int p = 0, nb = 0;
  std::string e = build_rect_desc(r, xs, ys, act, blk, fine, qoi, h, p, nb);
  if (!e.empty()) return e;
  lts_grid_desc d{};
  d.nx_cells = (int32_t)xs.size() - 1;
  d.ny_cells = (int32_t)ys.size() - 1;
  d.x = xs.data(); d.y = ys.data();
  d.cell_active = act.data(); d.cell_block = blk.data(); d.cell_fine = fine.data(); d.cell_qoi = qoi.data();
  d.n_blocks = nb; d.h = h; d.p = p; d.nu = r.nu;
  return build_level_from_desc(d, H);
}

lts_status lts_rect_level_host(const lts_rect_rule* r, lts_level_info* info, double* x, double* y,
                               uint8_t* flags, double* mass, double* qoi_w, int32_t* cell_block) {
  if (!r || !info) return LTS_ERR_ARG;
  HostLevel H;
  if (!host_level_of_rule(*r, H).empty()) return LTS_ERR_ARG;
  info->nx_nodes = H.nxn; info->ny_nodes = H.nyn; info->n_dof = H.n_dof; info->n_P = H.n_P;
  info->n_Fplus = H.n_F; info->p = H.p; info->n_blocks = H.n_blocks; info->h = H.h; info->nu = H.nu;
  info->delta = H.delta; info->omega = H.omega;
  info->tile_x = info->tile_y = info->tile_rect = info->tuned = 0;
  info->halo_ratio = info->tuned_ms = 0.0;
  if (x) std::memcpy(x, H.x.data(), H.x.size() * 8);
  if (y) std::memcpy(y, H.y.data(), H.y.size() * 8);
  if (flags) std::memcpy(flags, H.flags.data(), H.flags.size());
  if (mass) std::memcpy(mass, H.mass.data(), H.mass.size() * 8);
  if (qoi_w) std::memcpy(qoi_w, H.qoiw.data(), H.qoiw.size() * 8);
  if (cell_block) std::memcpy(cell_block, H.block.data(), H.block.size() * 4);
  return LTS_OK;
}

lts_status lts_tiling_host(const lts_rect_rule* r, int32_t tile_x, int32_t tile_y, int32_t rect,
                           lts_tiling_info* info, int32_t* owner) {
  if (!r || !info) return LTS_ERR_ARG;
  const bool adaptive = tile_x == 0 && tile_y == 0 && rect == 0;
  if (!adaptive && (tile_x < 1 || tile_y < 1 || tile_x > 4096 || tile_y > 4096)) return LTS_ERR_ARG;
  if (rect != 0 && rect != 1) return LTS_ERR_ARG;
  HostLevel H;
  if (!host_level_of_rule(*r, H).empty()) return LTS_ERR_ARG;
  const int p = H.p;
  const int ld = (H.nxn + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
  // the origin lts_set_tiling would take
  TilingHost T;
  bool have = false;
  for (auto& org : tile_origins(H, tile_x, tile_y)) {
    TilingHost C;
    if (!build_tiling(H, ld, tile_x, tile_y, org.first, org.second, rect == 1, C).empty()) continue;
    if (!have || C.halo_ratio * C.n_fine < T.halo_ratio * T.n_fine) {
      T = std::move(C);
      have = true;
    }
  }
  if (!have) return LTS_ERR_ARG;
  const int nx = H.nxn, ny = H.nyn;
  auto fplus = [&](int i, int j) { return (H.flags[(size_t)j * nx + i] & LTS_NODE_FPLUS) != 0; };
  auto dist = [](int i, int j, int x0, int x1, int y0, int y1) {
    return std::max(std::max(x0 - i, i - (x1 - 1)), 0) + std::max(std::max(y0 - j, j - (y1 - 1)), 0);
  };
  std::vector<int32_t> own((size_t)nx * ny, -1);
  auto claim = [&](int i, int j, int t) {
    int32_t& o = own[(size_t)j * nx + i];
    o = o == -1 ? t : -2;
  };
  bool exact = true;
  int max_region = 0;
  if (T.rect) {
    for (int t = 0; t < T.n_fine; ++t) {
      const int4 q = T.rtiles[t];
      const int rx0 = q.x & 0xFFFF, ry0 = q.x >> 16, rx1 = rx0 + (q.y & 0xFFFF), ry1 = ry0 + (q.y >> 16);
      const int x0 = q.z & 0xFFFF, x1 = q.z >> 16, y0 = q.w & 0xFFFF, y1 = q.w >> 16;
      max_region = std::max(max_region, (rx1 - rx0) * (ry1 - ry0));
      for (int j = std::max(y0 - p, 0); j < std::min(y1 + p, ny); ++j)
        for (int i = std::max(x0 - p, 0); i < std::min(x1 + p, nx); ++i) {
          if (!fplus(i, j)) continue;
          const int dd = dist(i, j, x0, x1, y0, y1);
          if (dd <= p && (i < rx0 || i >= rx1 || j < ry0 || j >= ry1)) exact = false;
          if (dd == 0) claim(i, j, t);
        }
    }
  } else {
    std::vector<int32_t> mark((size_t)nx * ny, -1);
    for (int t = 0; t < T.n_fine; ++t) {
      const int4 q = T.tiles[t];
      const int x0 = q.z & 0xFFFF, x1 = q.z >> 16, y0 = q.w & 0xFFFF, y1 = q.w >> 16;
      max_region = std::max(max_region, q.y);
      int want = 0;
      for (int j = std::max(y0 - p, 0); j < std::min(y1 + p, ny); ++j)
        for (int i = std::max(x0 - p, 0); i < std::min(x1 + p, nx); ++i)
          if (fplus(i, j) && dist(i, j, x0, x1, y0, y1) <= p) ++want;
      if (want != q.y) exact = false;
      for (int e = 0; e < q.y; ++e) {
        const int4 en = T.ent[(size_t)q.x + e];
        const int i = en.w & 0xFFFF, j = en.w >> 16;
        if (!fplus(i, j) || dist(i, j, x0, x1, y0, y1) > p || mark[(size_t)j * nx + i] == t) exact = false;
        mark[(size_t)j * nx + i] = t;
        if (dist(i, j, x0, x1, y0, y1) == 0) claim(i, j, t);
      }
    }
  }
  info->n_fine = T.n_fine;
  info->n_coarse = T.n_coarse;
  info->tile_x = T.TX;
  info->tile_y = T.TY;
  info->tile_rect = T.rect ? 1 : 0;
  info->max_region = max_region;
  info->regions_exact = exact ? 1 : 0;
  info->threads = T.rect ? kFineThreads : T.nt;
  info->halo_ratio = T.halo_ratio;
  if (owner) std::memcpy(owner, own.data(), own.size() * sizeof(int32_t));
  return LTS_OK;
}

lts_status lts_cheb_constants(int32_t p, double nu, double dt, double* delta, double* omega,
                              double* beta, double* beta_half, double* coef) {
  if (p < 1 || p > 256 || !(nu >= 0.0 && nu <= 1.0)) return LTS_ERR_ARG;
  HostLevel H;
  H.p = p;
  H.nu = nu;
  cheb_constants(p, nu, H.delta, H.omega, H.beta, H.beta_half);
  if (delta) *delta = H.delta;
  if (omega) *omega = H.omega;
  for (int k = 0; k < p; ++k) {
    if (beta) beta[k] = H.beta[k];
    if (beta_half) beta_half[k] = H.beta_half[k];
  }
  if (coef) step_coefficients(H, dt, coef);
  return LTS_OK;
}

lts_status lts_gen_samples(uint64_t seed, int32_t sample_level, int64_t first_index, int32_t n,
                           const lts_sample_rule* rule, double h_mesh, double* g, double* kappa,
                           double* x0, int32_t* n_steps, double* dt) {
  if (!rule) return LTS_ERR_ARG;
  std::string e = gen_samples(seed, sample_level, first_index, n, *rule, h_mesh, g, kappa, x0, n_steps, dt);
  return e.empty() ? LTS_OK : LTS_ERR_ARG;
}

lts_status lts_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  if (!ctr || !key || !out) return LTS_ERR_ARG;
  philox4x64_10(ctr, key, out);
  return LTS_OK;
}

lts_status lts_forward(lts_ctx c, int32_t level, const lts_samples* S, int32_t precision, double* Q) {
  return forward_impl(c, level, S, precision, Q, false);
}

lts_status lts_forward_plain(lts_ctx c, int32_t level, const lts_samples* S, int32_t precision, double* Q) {
  return forward_impl(c, level, S, precision, Q, true);
}

lts_status lts_forward_coupled(lts_ctx c, int32_t lf, int32_t lc, const lts_samples* F,
                               const lts_samples* C, int32_t precision, double* Qf, double* Qc,
                               double* dQ) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!F || !C) return arg_fail(c, "NULL samples");
  if (F->n != C->n || F->ptr_kind != C->ptr_kind) return arg_fail(c, "fine and coarse batches differ in n/ptr_kind");
  const int n = F->n;
  const bool dev = F->ptr_kind == LTS_PTR_DEVICE;
  std::vector<double> hf(n), hc(n);
  double *tf = nullptr, *tc = nullptr;
  lts_status r;
  if (dev) {
    LTS_HIP(c, hipSetDevice(c->device));
    LTS_HIP(c, c->red.ensure(std::max<size_t>(16 * (size_t)n, 16)));
    tf = c->red.as<double>();
    tc = tf + n;
  } else {
    tf = hf.data();
    tc = hc.data();
  }
  if ((r = lts_forward(c, lf, F, precision, tf)) != LTS_OK) return r;
  if ((r = lts_forward(c, lc, C, precision, tc)) != LTS_OK) return r;
  if (n == 0) return LTS_OK;
  if (dev) {
    k_coupled_diff<<<(n + 255) / 256, 256, 0, c->stream>>>(tf, tc, n, Qf, Qc, dQ);
    LTS_HIP(c, hipGetLastError());
    LTS_HIP(c, hipStreamSynchronize(c->stream));
  } else {
    for (int s = 0; s < n; ++s) {
      if (Qf) Qf[s] = hf[s];
      if (Qc) Qc[s] = hc[s];
      if (dQ) dQ[s] = hf[s] - hc[s];
    }
  }
  return LTS_OK;
}

lts_status lts_backward(lts_ctx c, int32_t level, const lts_samples* S, const double* dLdQ, int32_t K,
                        double* Q_out, double* dQ_dg_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  const DevLevel* lv = get_level(c, level);
  if (!lv) return arg_fail(c, "no such level");
  if (K < 1 || K > 4096) return arg_fail(c, "K_ckpt must be in 1..4096");
  if (lv->H.p > kMaxAdjP) return arg_fail(c, "p too large for the adjoint");
  if (S && S->n > 0 && (!dLdQ || !dQ_dg_out)) return arg_fail(c, "NULL dLdQ / output");
  Staged st;
  lts_status r = stage_samples(c, *lv, S, st);
  if (r != LTS_OK) return r;
  const int n = st.n, nb = lv->H.n_blocks;
  if (n == 0) return LTS_OK;
  LTS_HIP(c, hipSetDevice(c->device));
  StagedDev d;
  if ((r = ctx_staging(c, *lv, n, d)) != LTS_OK) return r;
  if ((r = upload_staged(c, *lv, st, S, d)) != LTS_OK) return r;
  LTS_HIP(c, c->dldq.ensure((size_t)n * 8));
  LTS_HIP(c, c->gout.ensure((size_t)n * nb * 8));
  if (st.ptr_kind == LTS_PTR_DEVICE) {
    k_gather_vec<<<(n + 255) / 256, 256, 0, c->stream>>>(dLdQ, d.perm, n, c->dldq.as<double>());
    LTS_HIP(c, hipGetLastError());
  } else {
    std::vector<double> dls(n);
    for (int t = 0; t < n; ++t) dls[t] = dLdQ[st.perm[t]];
    LTS_HIP(c, hipMemcpyAsync(c->dldq.p, dls.data(), (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));   // dls is released at the end of this scope
  }
  // Sub-batches sized to the device: the checkpoints, the segment and the
  // fused scratch of one sub-batch take at most 60 % of the free memory (this
  // context's own adjoint buffers counted as free), in equal sub-batches.
  // Fewer sub-batches mean fewer, fuller launches.
  const int n_ck = (st.nsteps[0] + K - 1) / K;
  const double per_sample = (2.0 * n_ck + K + 2.0 * lv->H.p + 8.0) * (double)lv->nodes * 8.0 +
                            (lv->tiling.rect ? (double)lv->tiling.n_fine * lv->H.p *
                                                   (4.0 * kFineThreads) * 8.0 : 0.0);
  size_t mem_free = 0, mem_total = 0;
  LTS_HIP(c, hipMemGetInfo(&mem_free, &mem_total));
  const double avail = 0.6 * ((double)mem_free + (double)c->adj.bytes + (double)c->adjscr.bytes);
  const int fit = std::max(1, std::min(n, (int)(avail / per_sample)));
  const int n_sub = (n + fit - 1) / fit;
  const int chunk = (n + n_sub - 1) / n_sub;
  const int p1 = lv->H.p + 1;
  for (int s0 = 0; s0 < n; s0 += chunk) {
    const int m = std::min(chunk, n - s0);
    std::vector<int> ns(st.nsteps.begin() + s0, st.nsteps.begin() + s0 + m);
    r = adjoint_device(c, *lv, m, d.kappa + (size_t)s0 * nb, d.coef + (size_t)s0 * p1, d.nsteps + s0,
                       d.x0 + 2 * (size_t)s0, S->width, ns, K, c->dldq.as<double>() + s0, c->Qd.as<double>() + s0,
                       c->gout.as<double>(), s0);
    if (r != LTS_OK) return r;
  }
  bool finite = true;
  if (st.ptr_kind == LTS_PTR_DEVICE) {
    k_zero_flag<<<1, 1, 0, c->stream>>>(d.flag);
    k_scatter_rows<<<grid_for((long long)n * nb), 256, 0, c->stream>>>(c->gout.as<double>(), d.perm, n, nb, dQ_dg_out,
                                                                     d.flag);
    LTS_HIP(c, hipGetLastError());
    int bad = 0;
    LTS_HIP(c, hipMemcpyAsync(&bad, d.flag, 4, hipMemcpyDeviceToHost, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));
    finite = bad == 0;
  } else {
    std::vector<double> gs((size_t)n * nb);
    LTS_HIP(c, hipMemcpyAsync(gs.data(), c->gout.p, gs.size() * 8, hipMemcpyDeviceToHost, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));
    for (int t = 0; t < n; ++t)
      for (int b = 0; b < nb; ++b) {
        const double v = gs[(size_t)t * nb + b];
        dQ_dg_out[(size_t)st.perm[t] * nb + b] = v;
        finite = finite && std::isfinite(v);
      }
  }
  // a large workspace is not kept between calls (it would starve other users
  // of the device); small ones are reused
  if (c->adj.bytes + c->adjscr.bytes > (size_t)48 << 30) {
    c->adj.release();
    c->adjscr.release();
  }
  if (!finite) {
    c->err = "non-finite gradient (unstable sample)";
    return LTS_ERR_UNSTABLE;
  }
  if (Q_out) return finish_Q(c, st, c->Qd.as<double>(), d, Q_out);
  return LTS_OK;
}

lts_status lts_moments(lts_ctx c, const double* x, int32_t n, int32_t ptr_kind, double* out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!out || (n > 0 && !x) || n < 0) return arg_fail(c, "bad moments arguments");
  if (ptr_kind != LTS_PTR_HOST && ptr_kind != LTS_PTR_DEVICE) return arg_fail(c, "bad ptr_kind");
  LTS_HIP(c, hipSetDevice(c->device));
  const bool dev = ptr_kind == LTS_PTR_DEVICE;
  LTS_HIP(c, c->red.ensure(std::max<size_t>(dev ? 64 : (size_t)n * 8 + 64, 64)));
  const double* dx = dev ? x : c->red.as<double>() + 8;   // device input is read in place
  if (n > 0 && !dev)
    LTS_HIP(c, hipMemcpyAsync(c->red.as<double>() + 8, x, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
  lts_status r = moments_device(c, dx, n, c->red.as<double>());
  if (r != LTS_OK) return r;
  LTS_HIP(c, hipMemcpyAsync(out, c->red.p, 24, hipMemcpyDeviceToHost, c->stream));
  LTS_HIP(c, hipStreamSynchronize(c->stream));
  return LTS_OK;
}

lts_status lts_set_timing(lts_ctx c, int32_t enable) {
  if (!c) return LTS_ERR_ARG;
  c->timing = enable != 0;
  return LTS_OK;
}

lts_status lts_get_timing(lts_ctx c, lts_timing* out) {
  if (!c || !out) return LTS_ERR_ARG;
  *out = c->last;
  return LTS_OK;
}

lts_status lts_set_barrier_timeout(lts_ctx c, double ms) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!(ms > 0.0) || !std::isfinite(ms) || ms > 3.6e6) return arg_fail(c, "barrier timeout must be in (0, 3.6e6] ms");
  c->barrier_ms = ms;
  return LTS_OK;
}

}  // extern "C"
