// Stabilized LF-LTS time stepping on the device (Algorithm 2, u-form).
//
// In the variables u = M^-1/2 z the scheme reads, with A_u = M^-1 K and the
// recurrence carried on the increments d_m = q_m/p - u_n:
//   w       = A_u (I - P) u_n
//   d_1     = -c1 (w + A_u P u_n)
//   d_m+1   = (1 + beta_m) d_m - beta_m d_m-1 - c2_m (w + A_u P (u_n + d_m))
//   u_n+1   = 2 u_n - u_n-1 + 2 d_p          (start-up: u_1 = u_0 + d_p)
// with c1 = 1/2 (dt/p)^2 2p^2/(omega delta), c2_m = (dt/p)^2 2p^2/omega beta_m+1/2.
// (Term by term the printed q-recurrence minus u_n; every coefficient that
// multiplies the state is exact, so binary64 rounding does not perturb the
// slow modes.)  A_u P q vanishes outside F+ (P and its neighbours), where
// d_m = a_m w and the whole step is u_n+1 = 2 u_n - u_n-1 + 2 a_p w: that part
// is a single stencil sweep.  Only F+ runs the p substeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ctx.h"

namespace lts {

namespace {

constexpr int TBX = 64, TBY = 4;

// ---------------------------------------------------------------------------
// Initial state: u_0 = exp(-|x - x0|^2 / width^2) on DOFs, 0 elsewhere.
template <class T>
__global__ __launch_bounds__(256) void k_init(LevelView L, const double* __restrict__ x0, double width,
                                              T* __restrict__ U, T* __restrict__ U1, size_t sstride) {
  const int s = blockIdx.z;
  const int i = blockIdx.x * TBX + threadIdx.x, j = blockIdx.y * TBY + threadIdx.y;
  if (i >= L.ld || j >= L.nyn) return;
  const size_t k = (size_t)j * L.ld + i;
  double v = 0.0;
  if (i < L.nxn && (L.flags[k] & F_DOF)) {
    const double dx = L.x[i] - x0[2 * s], dy = L.y[j] - x0[2 * s + 1];
    v = exp(-(dx * dx + dy * dy) / (width * width));
  }
  U[s * sstride + k] = (T)v;
  U1[s * sstride + k] = (T)0;   // the other time level: boundary nodes must read 0
}

// ---------------------------------------------------------------------------
// Q[s] = sum_k qoiw[k] u_k, one workgroup per sample, fixed summation order
// (per-lane strided sums, wavefront shuffles, then the four wavefronts in
// order), accumulated in binary64 also for binary32 states.
template <class T>
__global__ __launch_bounds__(256) void k_qoi(LevelView L, const int* __restrict__ nsteps,
                                             const T* __restrict__ B0, const T* __restrict__ B1,
                                             size_t sstride, size_t nodes, double* __restrict__ Q) {
  const int s = blockIdx.x;
  const T* __restrict__ u = ((nsteps[s] & 1) ? B1 : B0) + s * sstride;
  double acc = 0.0;
  for (size_t k = threadIdx.x; k < nodes; k += blockDim.x) {
    const double w = L.qoiw[k];
    if (w != 0.0) acc += w * (double)u[k];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) Q[s] = (part[0] + part[1]) + (part[2] + part[3]);
}

// ---------------------------------------------------------------------------
// (n, mean, M2) of x[0..n-1]: per-lane Welford, then pairwise Chan merges
// (wavefront shuffles, then across the workgroup's wavefronts).
struct Mom {
  double n, mean, m2;
};

__device__ __forceinline__ Mom chan_merge(Mom a, Mom b) {
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  const double nn = a.n + b.n;
  const double d = b.mean - a.mean;
  Mom r;
  r.n = nn;
  r.mean = a.mean + d * (b.n / nn);
  r.m2 = a.m2 + b.m2 + d * d * (a.n * b.n / nn);
  return r;
}

__global__ __launch_bounds__(1024) void k_moments(const double* __restrict__ x, int n,
                                                  double* __restrict__ out) {
  Mom m{0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double v = x[k];
    m.n += 1.0;
    const double d = v - m.mean;
    m.mean += d / m.n;
    m.m2 += d * (v - m.mean);
  }
  for (int o = 32; o > 0; o >>= 1) {
    Mom t;
    t.n = __shfl_down(m.n, o, 64);
    t.mean = __shfl_down(m.mean, o, 64);
    t.m2 = __shfl_down(m.m2, o, 64);
    m = chan_merge(m, t);
  }
  __shared__ Mom part[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    Mom r = part[0];
    const int nw = (blockDim.x + 63) / 64;
    for (int w = 1; w < nw; ++w) r = chan_merge(r, part[w]);
    out[0] = r.n;
    out[1] = r.mean;
    out[2] = r.m2;
  }
}

// (n, mean, M2) of every column of a row-major [n][nb] array: one workgroup
// per column, the same per-lane Welford updates and Chan merges as k_moments.
__global__ __launch_bounds__(256) void k_moments_cols(const double* __restrict__ x, int n, int nb,
                                                      double* __restrict__ out) {
  const int b = blockIdx.x;
  Mom m{0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double v = x[(size_t)k * nb + b];
    m.n += 1.0;
    const double d = v - m.mean;
    m.mean += d / m.n;
    m.m2 += d * (v - m.mean);
  }
  for (int o = 32; o > 0; o >>= 1) {
    Mom t;
    t.n = __shfl_down(m.n, o, 64);
    t.mean = __shfl_down(m.mean, o, 64);
    t.m2 = __shfl_down(m.m2, o, 64);
    m = chan_merge(m, t);
  }
  __shared__ Mom part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    Mom r = part[0];
    for (int w = 1; w < 4; ++w) r = chan_merge(r, part[w]);
    out[3 * b] = r.n;
    out[3 * b + 1] = r.mean;
    out[3 * b + 2] = r.m2;
  }
}

}  // namespace

lts_status moments_cols_device(lts_ctx c, const double* d_x, int n, int nb, double* d_out) {
  if (nb <= 0) return LTS_OK;
  k_moments_cols<<<nb, 256, 0, c->stream>>>(d_x, n, nb, d_out);
  LTS_HIP(c, hipGetLastError());
  return LTS_OK;
}

// ---------------------------------------------------------------------------

lts_status forward_device(lts_ctx c, const DevLevel& lv, int n, const double* d_kappa,
                          const double* d_coef, const int* d_nsteps, const double* d_x0, double width,
                          const std::vector<int>& h_nsteps, int precision, bool per_sample,
                          double* d_Q) {
  // Samples arrive sorted by decreasing step count, so the samples still
  // running at step `step` are a prefix of the batch.  FP32 stepping keeps
  // binary32 states (sstride elements of 4 bytes per sample) in the same buffers.
  const size_t bytes = (size_t)n * lv.nodes * (precision == LTS_FP32_STEP ? sizeof(float) : sizeof(double));
  LTS_HIP(c, c->st0.ensure(bytes));
  LTS_HIP(c, c->st1.ensure(bytes));
  return forward_device_states(c, lv, n, d_kappa, d_coef, d_nsteps, d_x0, width, h_nsteps, precision, per_sample,
                               d_Q, c->st0.as<double>(), c->st1.as<double>(), c->timing);
}

lts_status forward_device_states(lts_ctx c, const DevLevel& lv, int n, const double* d_kappa,
                                 const double* d_coef, const int* d_nsteps, const double* d_x0, double width,
                                 const std::vector<int>& h_nsteps, int precision, bool per_sample, double* d_Q,
                                 double* B0, double* B1, bool timing) {
  const bool fp32 = precision == LTS_FP32_STEP;
  const size_t sstride = lv.nodes;
  double* B[2] = {B0, B1};
  const int maxn = h_nsteps[0];

  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
  if (timing) {
    while (c->ev_pool.size() < 4) {
      hipEvent_t e;
      LTS_HIP(c, hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
    e0 = c->ev_pool[0]; e1 = c->ev_pool[1]; e2 = c->ev_pool[2]; e3 = c->ev_pool[3];
    LTS_HIP(c, hipEventRecord(e0, c->stream));
  }
  lts_status r = init_states(c, lv, n, d_x0, width, B[0], B[1], fp32);
  if (r != LTS_OK) return r;
  if (timing) LTS_HIP(c, hipEventRecord(e1, c->stream));
  int64_t launches = 0;
  if (per_sample) {
    for (int s = 0; s < n; ++s)
      for (int step = 0; step < h_nsteps[s]; ++step) {
        r = launch_step(c, lv, lv.tiling, d_kappa, d_coef, B[step & 1], B[(step + 1) & 1], sstride, s, 1,
                        step == 0, c->stream, fp32);
        if (r != LTS_OK) return r;
        ++launches;
      }
  } else {
    int active = n;
    for (int step = 0; step < maxn; ++step) {
      while (active > 0 && h_nsteps[active - 1] <= step) --active;
      r = launch_step(c, lv, lv.tiling, d_kappa, d_coef, B[step & 1], B[(step + 1) & 1], sstride, 0,
                      active, step == 0, c->stream, fp32);
      if (r != LTS_OK) return r;
      ++launches;
    }
  }
  LTS_HIP(c, hipGetLastError());
  if (timing) LTS_HIP(c, hipEventRecord(e2, c->stream));
  if ((r = qoi_device(c, lv, n, d_nsteps, B[0], B[1], d_Q, fp32)) != LTS_OK) return r;
  double dofu = 0.0, algb = 0.0;
  const double per_step = (double)(lv.H.n_dof - lv.H.n_P) + (double)lv.H.p * lv.H.n_P;
  for (int s = 0; s < n; ++s) {
    dofu += (double)h_nsteps[s] * per_step;
    algb += (double)h_nsteps[s] * (fp32 ? 12.0 : 24.0) * lv.H.n_dof;
  }
  c->last = lts_timing{};
  c->last.dof_updates = dofu;
  c->last.alg_bytes = algb;
  c->last.step_launches = launches;
  if (timing) {
    LTS_HIP(c, hipEventRecord(e3, c->stream));
    LTS_HIP(c, hipEventSynchronize(e3));
    float ta = 0, tb = 0;
    LTS_HIP(c, hipEventElapsedTime(&ta, e1, e2));
    LTS_HIP(c, hipEventElapsedTime(&tb, e0, e3));
    c->last.step_kernel_ms = ta;
    c->last.total_ms = tb;
  }
  return LTS_OK;
}

lts_status init_states(lts_ctx c, const DevLevel& lv, int n, const double* d_x0, double width, double* B0,
                       double* B1, bool fp32) {
  const LevelView L = lv.view();
  const size_t sstride = lv.nodes;
  const dim3 blk(TBX, TBY);
  const int gx = (L.ld + TBX - 1) / TBX, gy = (L.nyn + TBY - 1) / TBY;
  constexpr int kMaxZ = 32768;
  for (int z0 = 0; z0 < n; z0 += kMaxZ) {
    const int nz = std::min(kMaxZ, n - z0);
    if (fp32)
      k_init<float><<<dim3(gx, gy, nz), blk, 0, c->stream>>>(L, d_x0 + 2 * z0, width,
                                                              reinterpret_cast<float*>(B0) + z0 * sstride,
                                                              reinterpret_cast<float*>(B1) + z0 * sstride, sstride);
    else
      k_init<double><<<dim3(gx, gy, nz), blk, 0, c->stream>>>(L, d_x0 + 2 * z0, width, B0 + z0 * sstride,
                                                               B1 + z0 * sstride, sstride);
  }
  LTS_HIP(c, hipGetLastError());
  return LTS_OK;
}

lts_status qoi_device(lts_ctx c, const DevLevel& lv, int n, const int* d_nsteps, const double* B0,
                      const double* B1, double* d_Q, bool fp32) {
  if (n <= 0) return LTS_OK;
  if (fp32)
    k_qoi<float><<<n, 256, 0, c->stream>>>(lv.view(), d_nsteps, reinterpret_cast<const float*>(B0),
                                           reinterpret_cast<const float*>(B1), lv.nodes, lv.nodes, d_Q);
  else
    k_qoi<double><<<n, 256, 0, c->stream>>>(lv.view(), d_nsteps, B0, B1, lv.nodes, lv.nodes, d_Q);
  LTS_HIP(c, hipGetLastError());
  return LTS_OK;
}

lts_status moments_device(lts_ctx c, const double* d_x, int n, double* d_out3) {
  k_moments<<<1, 1024, 0, c->stream>>>(d_x, n, d_out3);
  LTS_HIP(c, hipGetLastError());
  return LTS_OK;
}

}  // namespace lts


