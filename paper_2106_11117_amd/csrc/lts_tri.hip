// Algorithm 2 (stabilized LF-LTS, in increment form) on a level given as a
// triangulation (Sec. 3.1: mass-lumped P1 elements on triangles; Sec. 3.3:
// the p local substeps act on the DOFs of P through A_u P).
//
// The operator is matrix-free in edge form: (K v)_i = sum over the couplings
// (i, j) of c_ij (v_i - v_j), c_ij = kappa_A w_A + kappa_B w_B summed over the
// (at most two) triangles of the edge, w = -|T| grad(l_i).grad(l_j) (host
// build).  A Dirichlet neighbour is the zero slot at index n of the state.
//
// One coarse step of all active samples is two launches:
//  * k_tri_coarse: the DOFs outside F+ (no P neighbour, so w = A_u u and
//    u_n+1 = 2 u_n - u_n-1 + 2 a_p w); a thread owns one DOF for kTriS
//    samples, so each coupling's mesh data is read once for all of them.
//  * k_tri_fine: one workgroup per (fine tile, sample) runs the p substeps on
//    the tile's region, the F+ DOFs within graph distance p of the tile,
//    compacted in LDS by increasing distance (two q buffers, one barrier per
//    substep).  A DOF at distance D influences the tile only after D more
//    substeps, so substep m updates the DOFs within p - 1 - m and only the
//    tile's own DOFs are written back; errors from the missing neighbours at
//    the region border never reach them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ctx.h"

namespace lts {

namespace {

constexpr int kTriS = 4;                              // samples per coarse thread
constexpr int kTriNT = 1024;                          // threads of a fine workgroup
constexpr int kTriNPT = kTriRegionCap / kTriNT;       // region DOFs per thread
static_assert(kTriNT * kTriNPT == kTriRegionCap, "region cap = threads x DOFs per thread");

struct TriView {
  int n, nb, p, n_coarse, n_tiles;
  const double* __restrict__ dx;
  const double* __restrict__ dy;
  const double* __restrict__ invm;
  const double* __restrict__ qoiw;
  const uint8_t* __restrict__ dflag;      // [n + 1] bit 0: P (the zero slot: 0)
  const int* __restrict__ rp;
  const int* __restrict__ col;
  const int* __restrict__ eblk;
  const double* __restrict__ ewa;
  const double* __restrict__ ewb;
  const int* __restrict__ coarse;
  const int* __restrict__ tiles;
  const int4* __restrict__ ent;
  const uint16_t* __restrict__ tslot;
  const double* __restrict__ beta;        // [p] beta_k, k = 1..p-1
};

struct TriStep {
  const double* __restrict__ kappa;       // [S][nb] (sorted sample order)
  const double* __restrict__ coef;        // [S][p+1]: a_p, c1, c2_1 .. c2_p-1
  const double* __restrict__ Ucur;        // u_n of sample s at Ucur + s*ld
  double* __restrict__ Uold;              // u_n-1 in, u_n+1 out
  size_t ld;
  int active, startup, per_xcd;
};

// u_0 = exp(-|x - x0|^2 / w^2) at the DOFs, the zero slots and u_-1 zero.
__global__ __launch_bounds__(256) void k_tri_init(TriView v, int S, const double* __restrict__ x0, double width,
                                                  double* __restrict__ B0, double* __restrict__ B1, size_t ld) {
  const long long tot = (long long)S * (long long)ld;
  const double iw2 = 1.0 / (width * width);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(e / (long long)ld), k = (int)(e - (long long)s * (long long)ld);
    double u = 0.0;
    if (k < v.n) {
      const double rx = v.dx[k] - x0[2 * s], ry = v.dy[k] - x0[2 * s + 1];
      u = exp(-(rx * rx + ry * ry) * iw2);
    }
    B0[e] = u;
    B1[e] = 0.0;
  }
}

template <int S>
__device__ __forceinline__ void load_kappa_groups(const TriStep& a, int nb, int s0, int ns,
                                                  double (*lk)[256]) {
  for (int t = threadIdx.x; t < S * 256; t += blockDim.x) {
    const int g = t >> 8, b = t & 255;
    lk[g][b] = (g < ns && b < nb) ? a.kappa[(size_t)(s0 + g) * nb + b] : 0.0;   // 255: no second triangle
  }
}

// Coarse DOFs: blockIdx.x = kTriS consecutive active samples (fastest, so
// that the blocks of one group of DOFs run together and share its coupling
// data in L2), blockIdx.y = 256 DOFs of the coarse list.
__global__ __launch_bounds__(256) void k_tri_coarse(TriView v, TriStep a) {
  __shared__ double lk[kTriS][256];
  const int s0 = blockIdx.x * kTriS;
  const int ns = min(kTriS, a.active - s0);
  load_kappa_groups<kTriS>(a, v.nb, s0, ns, lk);
  __syncthreads();
  const int c = blockIdx.y * 256 + threadIdx.x;
  if (c >= v.n_coarse) return;
  const int i = v.coarse[c];
  const int e0 = v.rp[i], e1 = v.rp[i + 1];
  double ui[kTriS], acc[kTriS];
#pragma unroll
  for (int g = 0; g < kTriS; ++g) {
    ui[g] = g < ns ? a.Ucur[(size_t)(s0 + g) * a.ld + i] : 0.0;
    acc[g] = 0.0;
  }
  for (int e = e0; e < e1; ++e) {
    const int j = v.col[e];
    const int bb = v.eblk[e];
    const double wa = v.ewa[e], wb = v.ewb[e];
#pragma unroll
    for (int g = 0; g < kTriS; ++g) {
      if (g >= ns) continue;
      const double cf = lk[g][bb & 255] * wa + lk[g][bb >> 8] * wb;
      acc[g] += cf * (ui[g] - a.Ucur[(size_t)(s0 + g) * a.ld + j]);
    }
  }
  const double im = v.invm[i];
#pragma unroll
  for (int g = 0; g < kTriS; ++g) {
    if (g >= ns) continue;
    const size_t o = (size_t)(s0 + g) * a.ld + i;
    const double d = a.coef[(size_t)(s0 + g) * (v.p + 1)] * (im * acc[g]);
    a.Uold[o] = a.startup ? ui[g] + d : 2.0 * ui[g] - a.Uold[o] + 2.0 * d;
  }
}

// One fine tile of one sample.  Region DOF e (lane e mod kTriNT, slot
// e / kTriNT) keeps u_n, P flag, the increments d_m, d_m-1, w = A_u (I - P) u_n
// and, per coupling, the scaled coefficient and the LDS byte offset of the
// neighbour's q (the zero slot for a neighbour that is not in P or not in the
// region).
// DEG: the level's largest F+ degree rounded up to 6, 8, 10 or 12 (the
// coupling arrays and loops are that long).
template <int DEG>
__global__ __launch_bounds__(kTriNT) void k_tri_fine(TriView v, TriStep a) {
  __shared__ double lk[256];
  __shared__ double qb[2 * (kTriRegionCap + 1)];
  const int G = v.n_tiles * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G) return;
  // sample-major: the tiles of one sample run back to back on one XCD, whose
  // L2 then holds the halo values a tile shares with its neighbours (measured
  // faster than tile-major, which would share the coupling data instead)
  const int s = Lid / v.n_tiles, tile = Lid - s * v.n_tiles;
  for (int t = threadIdx.x; t < 256; t += kTriNT) lk[t] = t < v.nb ? a.kappa[(size_t)s * v.nb + t] : 0.0;
  __syncthreads();
  const int off = v.tiles[tile], len = v.tiles[tile + 1] - off;
  const int p = v.p;
  const double* __restrict__ u_g = a.Ucur + (size_t)s * a.ld;
  double* __restrict__ uo_g = a.Uold + (size_t)s * a.ld;
  const double* __restrict__ cf = a.coef + (size_t)s * (p + 1);
  double* const q0 = qb;
  double* const q1 = qb + (kTriRegionCap + 1);
  const int tid = threadIdx.x;

  double u[kTriNPT], pm[kTriNPT], d0[kTriNPT], d1[kTriNPT], w[kTriNPT];
  double ac[kTriNPT][DEG];
  uint32_t ad[kTriNPT][DEG];
  int kk[kTriNPT], dd[kTriNPT];
#pragma unroll
  for (int r = 0; r < kTriNPT; ++r) {
    const int e = tid + r * kTriNT;
    u[r] = pm[r] = d0[r] = d1[r] = w[r] = 0.0;
    kk[r] = 0;
    dd[r] = p;                                          // never updated, never written
#pragma unroll
    for (int k = 0; k < DEG; ++k) {
      ac[r][k] = 0.0;
      ad[r][k] = (uint32_t)len * 8u;
    }
    if (e >= len) continue;
    const int4 en = v.ent[off + e];
    const int k0 = en.x & 0x7FFFFFFF;
    const bool isP = en.x < 0;
    const int deg = en.z & 0xFFFF;
    dd[r] = en.z >> 16;
    kk[r] = k0;
    const double uc = u_g[k0];
    u[r] = uc;
    pm[r] = isP ? 1.0 : 0.0;
    q0[e] = isP ? uc : 0.0;
    const double imu = dd[r] < p ? v.invm[k0] : 0.0;   // coefficients vanish where no substep updates
    const double vi = isP ? 0.0 : uc;
    double wr = 0.0;
#pragma unroll
    for (int k = 0; k < DEG; ++k) {
      if (k >= deg) continue;
      const int o = en.y + k;
      const int j = v.col[o];
      const int bb = v.eblk[o];
      const double c = (lk[bb & 255] * v.ewa[o] + lk[bb >> 8] * v.ewb[o]) * imu;
      ac[r][k] = c;
      ad[r][k] = (uint32_t)v.tslot[en.w + k] * 8u;
      const double uj = u_g[j];
      const double vj = (v.dflag[j] & 1) ? 0.0 : uj;
      wr += c * (vi - vj);
    }
    w[r] = wr;
  }
  if (tid == 0) q0[len] = q1[len] = 0.0;                // slot read for absent / non-P neighbours
  __syncthreads();

  // Substep m: d_m+1 = (1 + beta_m) d_m - beta_m d_m-1 - c_m (w + A_u q_m)
  // with d_0 = d_-1 = 0, beta_0 = 0, and q_m+1 = P (u_n + d_m+1).
  // At even m, d0 holds d_m and d1 d_m-1 (overwritten by d_m+1), q is read
  // from q0 and written to q1; at odd m the roles swap (fixed per call, so the
  // increments stay in registers).
  auto substep = [&](int m, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    double* dc = B == 0 ? d0 : d1;
    double* dq = B == 0 ? d1 : d0;
    const char* rq = reinterpret_cast<const char*>(B == 0 ? q0 : q1);
    double* wq = B == 0 ? q1 : q0;
    const double c = cf[1 + m];
    const double b = m > 0 ? v.beta[m] : 0.0;
    const int reach = p - 1 - m;
#pragma unroll
    for (int r = 0; r < kTriNPT; ++r) {
      if (dd[r] > reach) continue;
      const double qi = pm[r] * (u[r] + dc[r]);
      double apq = 0.0;
#pragma unroll
      for (int k = 0; k < DEG; ++k)
        apq += ac[r][k] * (qi - *reinterpret_cast<const double*>(rq + ad[r][k]));
      const double dn = (1.0 + b) * dc[r] - b * dq[r] - c * (w[r] + apq);
      dq[r] = dn;
      if (m + 1 < p) wq[tid + r * kTriNT] = pm[r] * (u[r] + dn);
    }
    if (m + 1 < p) __syncthreads();
  };
  int m = 0;
  for (; m + 1 < p; m += 2) {
    substep(m, std::integral_constant<int, 0>{});
    substep(m + 1, std::integral_constant<int, 1>{});
  }
  if (m < p) substep(m, std::integral_constant<int, 0>{});
  const bool podd = p & 1;
#pragma unroll
  for (int r = 0; r < kTriNPT; ++r) {
    if (dd[r] != 0) continue;                            // written back by the tile that owns it
    const double dfin = podd ? d1[r] : d0[r];            // d_p
    const size_t k = (size_t)kk[r];
    uo_g[k] = a.startup ? u[r] + dfin : 2.0 * u[r] - uo_g[k] + 2.0 * dfin;
  }
}

// Q_s = sum over the DOFs of qoi_w u(T); the state after n_steps[s] steps is
// in B[n_steps[s] & 1].
__global__ __launch_bounds__(256) void k_tri_qoi(TriView v, const int* __restrict__ nsteps,
                                                 const double* __restrict__ B0, const double* __restrict__ B1,
                                                 size_t ld, double* __restrict__ Q) {
  __shared__ double part[4];
  const int s = blockIdx.x;
  const double* u = ((nsteps[s] & 1) ? B1 : B0) + (size_t)s * ld;
  double acc = 0.0;
  for (int k = threadIdx.x; k < v.n; k += 256) acc += v.qoiw[k] * u[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) Q[s] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ __launch_bounds__(256) void k_tri_diff(const double* __restrict__ a, const double* __restrict__ b, int n,
                                                  double* __restrict__ d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) d[t] = a[t] - b[t];
}

TriView tri_view(const TriDev& M) {
  TriView v;
  v.n = M.H.n_dof;
  v.nb = M.H.shell.n_blocks;
  v.p = M.H.shell.p;
  v.n_coarse = (int)M.H.coarse.size();
  v.n_tiles = (int)M.H.tiles.size() - 1;
  v.dx = M.dx.as<double>();
  v.dy = M.dy.as<double>();
  v.invm = M.invm.as<double>();
  v.qoiw = M.qoiw.as<double>();
  v.dflag = M.dflag.as<uint8_t>();
  v.rp = M.rp.as<int>();
  v.col = M.col.as<int>();
  v.eblk = M.eblk.as<int>();
  v.ewa = M.ewa.as<double>();
  v.ewb = M.ewb.as<double>();
  v.coarse = M.coarse.as<int>();
  v.tiles = M.tiles.as<int>();
  v.ent = M.ent.as<int4>();
  v.tslot = M.tslot.as<uint16_t>();
  v.beta = M.beta.as<double>();
  return v;
}

template <class V>
lts_status upload_vec(lts_ctx c, DevBuf& b, const std::vector<V>& h) {
  LTS_HIP(c, b.ensure(std::max<size_t>(h.size() * sizeof(V), 16)));
  if (!h.empty()) LTS_HIP(c, hipMemcpy(b.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  return LTS_OK;
}

lts_status tri_upload(lts_ctx c, TriDev& M) {
  const TriHost& H = M.H;
  M.shell.H = H.shell;
  M.ld = ((size_t)H.n_dof + 1 + 63) / 64 * 64;
  std::vector<int4> ent(H.ent.size());
  static_assert(sizeof(TriEnt) == sizeof(int4), "region entry layout");
  std::memcpy(ent.data(), H.ent.data(), H.ent.size() * sizeof(int4));
  std::vector<double> beta(std::max(H.shell.p, 1), 0.0);
  for (int k = 1; k < H.shell.p; ++k) beta[k] = H.shell.beta[k];
  lts_status r;
  if ((r = upload_vec(c, M.dx, H.dx)) != LTS_OK || (r = upload_vec(c, M.dy, H.dy)) != LTS_OK ||
      (r = upload_vec(c, M.invm, H.invm)) != LTS_OK || (r = upload_vec(c, M.qoiw, H.qoiw)) != LTS_OK ||
      (r = upload_vec(c, M.dflag, H.dflag)) != LTS_OK || (r = upload_vec(c, M.rp, H.rp)) != LTS_OK ||
      (r = upload_vec(c, M.col, H.col)) != LTS_OK || (r = upload_vec(c, M.eblk, H.eblk)) != LTS_OK ||
      (r = upload_vec(c, M.ewa, H.ewa)) != LTS_OK || (r = upload_vec(c, M.ewb, H.ewb)) != LTS_OK ||
      (r = upload_vec(c, M.coarse, H.coarse)) != LTS_OK || (r = upload_vec(c, M.tiles, H.tiles)) != LTS_OK ||
      (r = upload_vec(c, M.ent, ent)) != LTS_OK || (r = upload_vec(c, M.tslot, H.tslot)) != LTS_OK ||
      (r = upload_vec(c, M.beta, beta)) != LTS_OK)
    return r;
  return LTS_OK;
}

// Forward solve of a staged batch; Q (sorted order) in c->Qd.
lts_status tri_solve(lts_ctx c, TriDev& M, const Staged& st, const StagedDev& d, double width) {
  const int n = st.n;
  const TriView v = tri_view(M);
  const size_t ld = M.ld;
  LTS_HIP(c, c->st0.ensure((size_t)n * ld * 8));
  LTS_HIP(c, c->st1.ensure((size_t)n * ld * 8));
  double* B[2] = {c->st0.as<double>(), c->st1.as<double>()};
  hipStream_t q = c->stream;
  const long long tot = (long long)n * (long long)ld;
  k_tri_init<<<(int)std::max(1LL, std::min((tot + 255) / 256, 8192LL)), 256, 0, q>>>(v, n, d.x0, width, B[0], B[1],
                                                                                     ld);
  LTS_HIP(c, hipGetLastError());
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
  int act = n;
  const int maxT = st.nsteps[0];
  for (int t = 0; t < maxT; ++t) {
    while (act > 0 && st.nsteps[act - 1] <= t) --act;
    TriStep a;
    a.kappa = d.kappa;
    a.coef = d.coef;
    a.Ucur = B[t & 1];
    a.Uold = B[(t + 1) & 1];
    a.ld = ld;
    a.active = act;
    a.startup = t == 0;
    a.per_xcd = 0;
    if (v.n_coarse > 0)
      k_tri_coarse<<<dim3((unsigned)((act + kTriS - 1) / kTriS), (unsigned)((v.n_coarse + 255) / 256)), 256, 0, q>>>(v,
                                                                                                                  a);
    if (v.n_tiles > 0) {
      const long long G = (long long)v.n_tiles * act;
      a.per_xcd = (int)((G + 7) / 8);
      const int md = M.H.max_deg;
      const dim3 g((unsigned)(8LL * a.per_xcd));
      if (md <= 6) k_tri_fine<6><<<g, kTriNT, 0, q>>>(v, a);
      else if (md <= 8) k_tri_fine<8><<<g, kTriNT, 0, q>>>(v, a);
      else if (md <= 10) k_tri_fine<10><<<g, kTriNT, 0, q>>>(v, a);
      else k_tri_fine<12><<<g, kTriNT, 0, q>>>(v, a);
    }
  }
  LTS_HIP(c, hipGetLastError());
  k_tri_qoi<<<n, 256, 0, q>>>(v, d.nsteps, B[0], B[1], ld, c->Qd.as<double>());
  LTS_HIP(c, hipGetLastError());
  c->last = lts_timing{};
  if (c->timing) {
    LTS_HIP(c, hipEventRecord(e1, q));
    LTS_HIP(c, hipEventSynchronize(e1));
    float ms = 0;
    LTS_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    c->last.total_ms = ms;
    c->last.step_kernel_ms = ms;
    c->last.step_launches = maxT;
  }
  const double per_step = (double)(M.H.n_dof - M.H.n_P) + (double)M.H.shell.p * M.H.n_P;
  for (int s = 0; s < n; ++s) {
    c->last.dof_updates += (double)st.nsteps[s] * per_step;
    c->last.alg_bytes += (double)st.nsteps[s] * 24.0 * M.H.n_dof;
  }
  return LTS_OK;
}

lts_status tri_forward(lts_ctx c, TriDev& M, const lts_samples* S, double* Q_out) {
  Staged st;
  lts_status r;
  if ((r = stage_samples(c, M.shell, S, st)) != LTS_OK) return r;
  if (st.n == 0) return LTS_OK;
  if (!Q_out) return arg_fail(c, "Q_out is NULL");
  StagedDev d;
  if ((r = ctx_staging(c, M.shell, st.n, d)) != LTS_OK) return r;
  if ((r = upload_staged(c, M.shell, st, S, d)) != LTS_OK) return r;
  if ((r = tri_solve(c, M, st, d, S->width)) != LTS_OK) return r;
  return finish_Q(c, st, c->Qd.as<double>(), d, Q_out);
}

TriDev* mesh_of(lts_ctx c, int32_t id) {
  if (!c || id < 0 || id >= (int32_t)c->meshes.size()) return nullptr;
  return c->meshes[id].get();
}

void fill_info(const TriHost& H, lts_mesh_info* out) {
  std::memset(out, 0, sizeof(*out));
  out->n_nodes = H.n_nodes;
  out->n_tris = H.n_tris;
  out->n_dof = H.n_dof;
  out->n_P = H.n_P;
  out->n_Fplus = H.n_F;
  out->n_edges = H.rp.empty() ? 0 : H.rp.back();
  out->max_degree = H.max_deg;
  out->n_tiles = (int)H.tiles.size() - 1;
  out->max_region = H.max_region;
  out->p = H.shell.p;
  out->n_blocks = H.shell.n_blocks;
  out->h = H.shell.h;
  out->nu = H.shell.nu;
  out->delta = H.shell.delta;
  out->omega = H.shell.omega;
  out->halo_ratio = H.halo_ratio;
}

}  // namespace

}  // namespace lts

using namespace lts;

extern "C" {

lts_status lts_add_mesh(lts_ctx c, const lts_mesh_desc* desc, int32_t* mesh_id_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!desc || !mesh_id_out) return arg_fail(c, "desc and mesh_id_out are required");
  auto M = std::make_unique<TriDev>();
  const std::string e = build_tri(*desc, M->H);
  if (!e.empty()) return arg_fail(c, e);
  LTS_HIP(c, hipSetDevice(c->device));
  lts_status r = tri_upload(c, *M);
  if (r != LTS_OK) return r;
  c->meshes.push_back(std::move(M));
  *mesh_id_out = (int32_t)c->meshes.size() - 1;
  return LTS_OK;
}

lts_status lts_mesh_info_get(lts_ctx c, int32_t mesh, lts_mesh_info* out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  TriDev* M = mesh_of(c, mesh);
  if (!M) return arg_fail(c, "no such mesh");
  if (!out) return arg_fail(c, "out is NULL");
  fill_info(M->H, out);
  return LTS_OK;
}

lts_status lts_mesh_host(const lts_mesh_desc* desc, lts_mesh_info* info, uint8_t* node_flags, double* mass) {
  if (!desc || !info) return LTS_ERR_ARG;
  TriHost H;
  if (!build_tri(*desc, H).empty()) return LTS_ERR_ARG;
  fill_info(H, info);
  if (node_flags) std::memcpy(node_flags, H.node_flags.data(), H.node_flags.size());
  if (mass) std::memcpy(mass, H.mass_node.data(), H.mass_node.size() * sizeof(double));
  return LTS_OK;
}

lts_status lts_mesh_forward(lts_ctx c, int32_t mesh, const lts_samples* samples, int32_t precision,
                            double* Q_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  TriDev* M = mesh_of(c, mesh);
  if (!M) return arg_fail(c, "no such mesh");
  if (precision != LTS_FP64) return arg_fail(c, "triangle-mesh levels step in FP64 only");
  LTS_HIP(c, hipSetDevice(c->device));
  return tri_forward(c, *M, samples, Q_out);
}

lts_status lts_mesh_forward_coupled(lts_ctx c, int32_t mesh_fine, int32_t mesh_coarse, const lts_samples* fine,
                                    const lts_samples* coarse, int32_t precision, double* Qf_out, double* Qc_out,
                                    double* dQ_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  TriDev* Mf = mesh_of(c, mesh_fine);
  TriDev* Mc = mesh_of(c, mesh_coarse);
  if (!Mf || !Mc) return arg_fail(c, "no such mesh");
  if (precision != LTS_FP64) return arg_fail(c, "triangle-mesh levels step in FP64 only");
  if (!fine || !coarse) return arg_fail(c, "samples are NULL");
  if (fine->n != coarse->n) return arg_fail(c, "fine and coarse batches differ in size");
  if (fine->ptr_kind != coarse->ptr_kind) return arg_fail(c, "fine and coarse batches differ in ptr_kind");
  const int n = fine->n;
  if (n <= 0) return n < 0 ? arg_fail(c, "samples.n must be >= 0") : LTS_OK;
  LTS_HIP(c, hipSetDevice(c->device));
  lts_status r;
  if (fine->ptr_kind == LTS_PTR_DEVICE) {
    LTS_HIP(c, c->qa.ensure((size_t)n * 8));
    LTS_HIP(c, c->qb.ensure((size_t)n * 8));
    double* qf = Qf_out ? Qf_out : c->qa.as<double>();
    double* qc = Qc_out ? Qc_out : c->qb.as<double>();
    if ((r = tri_forward(c, *Mf, fine, qf)) != LTS_OK) return r;
    if ((r = tri_forward(c, *Mc, coarse, qc)) != LTS_OK) return r;
    if (dQ_out) {
      k_tri_diff<<<(n + 255) / 256, 256, 0, c->stream>>>(qf, qc, n, dQ_out);
      LTS_HIP(c, hipGetLastError());
      LTS_HIP(c, hipStreamSynchronize(c->stream));
    }
    return LTS_OK;
  }
  std::vector<double> qf(n), qc(n);
  if ((r = tri_forward(c, *Mf, fine, qf.data())) != LTS_OK) return r;
  if ((r = tri_forward(c, *Mc, coarse, qc.data())) != LTS_OK) return r;
  for (int s = 0; s < n; ++s) {
    if (Qf_out) Qf_out[s] = qf[s];
    if (Qc_out) Qc_out[s] = qc[s];
    if (dQ_out) dQ_out[s] = qf[s] - qc[s];
  }
  return LTS_OK;
}

}  // extern "C"
