// Discrete adjoint of stabilized LF-LTS: dQ/d(block log wave speed) per sample.
//
// With R y = q_1(y) = y + d_p(y) (Algorithm 2 on increments, u-form, A_u =
// M^-1 K), the forward recurrence is u_1 = R u_0, u_n+1 = 2 R u_n - u_n-1 and
// Q = w^T u_N.  R is self-adjoint in the M inner product, so the adjoint runs
// the same recurrence backward:
//   mu_N = M^-1 w, mu_N+1 = 0, mu_n = 2 R mu_n+1 - mu_n+2   (n = N-1 .. 1),
//   dQ/dkappa = sum_{n>=1} 2 <mu_n+1, d(R u_n)>_M + <mu_1, d(R u_0)>_M.
// Each <mu, d(R y)/dkappa>_M is a reverse sweep over the p substeps for fixed
// y: with Lambda_p = f M mu (f = 2 or 1), Lambda_p+1 = 0,
//   Lambda_m = (1 + beta_m) Lambda_m+1 - c2_m P K (Lambda_m+1 / m) - beta_m+1 Lambda_m+2,
//   lw = -c1 Lambda_1 - sum_{m=1}^{p-1} c2_m Lambda_m+1,
// and the derivative pairs (a, b) = (-c2_m Lambda_m+1, P q_m), (-c1 Lambda_1, P q_0),
// (lw, (I - P) y) contract with dK/dkappa_cell: for every side (i, j) of a cell
// with leg weight g (hy/(2 hx) or hx/(2 hy)), g (a_i/m_i - a_j/m_j)(b_i - b_j),
// with a = b = 0 on Dirichlet nodes.  One thread owns one cell, so the
// accumulation is deterministic.  dQ/dg_b = 2 kappa_b sum_{cells of b} dQ/dkappa_cell.
// Forward states are checkpointed every K steps (pairs (u_k, u_k+1)); on
// levels with fine tiles the backward step also runs the forward step
// backward in time (u_n-1 = 2 R u_n - u_n+1, from R u_n's substeps, which it
// forms anyway), starting each segment from exact states, else each segment
// is recomputed forward with the step kernels; mu is
// advanced by the forward step kernels too (the recurrence is the same),
// except at the F+ DOFs of levels with fine tiles: there the reverse sweep
// already holds R^T Lambda_p = Lambda_p + K (lw / m), which gives mu_n
// (k_adj_fine on rect tilings, k_adj_mu_fplus on compact ones; the coarse
// items give the other DOFs).
// Per backward step: on rect tilings the fused k_adj_fine (below) and
// k_adj_cells; on compact tilings the two substep sweeps run per compact
// tile (launch_adj_compact in lts_fused.hip) and k_adj_contract contracts;
// the per-substep kernels over the list of P nodes remain for levels
// without fine tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"

namespace lts {

namespace {

constexpr int BX = 64, BY = 4;

struct AdjArgs {
  LevelView L;
  const double* __restrict__ kappa;  // [S][nb]
  const double* __restrict__ coef;   // [S][p+1]
  size_t sstride;
  int s_active;                      // samples 0..s_active-1 take part
  const int* __restrict__ plist;     // grid index j * ld + i of every node of P
  int np;
  const int* __restrict__ clist;     // cell index jb * ld + ia of every active cell with a corner in P
  int nc;
  const double* __restrict__ rho;    // rho[m], m = 1..p: Lambda_m = rho_m Lambda_p off P
  double* gam;                       // [S]: lw = gamma Lambda_p off P
  // k_adj_cells sums its cells per workgroup and block: slot of each cell's
  // block in its workgroup (255: cell not handled there), slots per workgroup,
  // block of each slot, and the sums over the steps [S][n_wg][max_slots]
  const uint8_t* __restrict__ cslot;
  const int* __restrict__ wslots;
  const int* __restrict__ wblock;
  double* gpart;
  int n_wg, max_slots;
};

// The P node of this thread (1D grid over the P list, z = sample); false past the end.
__device__ __forceinline__ bool p_node(const AdjArgs& a, int& i, int& j, size_t& k) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.np || (int)blockIdx.z >= a.s_active) return false;
  k = (size_t)a.plist[t];
  j = (int)(k / (size_t)a.L.ld);
  i = (int)(k - (size_t)j * a.L.ld);
  return true;
}

// w = A_u (I - P) y at the nodes of P (the only nodes whose increments the
// backward step reads: the pairs contract P q_m, and A_u P q_m reads P nodes).
__global__ __launch_bounds__(256) void k_adj_w(AdjArgs a, const double* __restrict__ Y,
                                               double* __restrict__ W) {
  const int s = blockIdx.z;
  const LevelView& L = a.L;
  int i, j;
  size_t k;
  if (!p_node(a, i, j, k)) return;
  const size_t so = (size_t)s * a.sstride;
  const double* __restrict__ y = Y + so;
  double cE, cW, cN, cS;
  edge_coefs(L, a.kappa + (size_t)s * L.nb, i, j, cE, cW, cN, cS);
  auto v = [&](size_t kk) { return (L.flags[kk] & F_P) ? 0.0 : y[kk]; };
  const double vi = v(k);
  W[so + k] = L.invm[k] * (cE * (vi - v(k + 1)) + cW * (vi - v(k - 1)) + cN * (vi - v(k + L.ld)) +
                           cS * (vi - v(k - L.ld)));
}

// d_m+1 from d_m (Dc, NULL: 0), d_m-1 (Dp, NULL: 0), w, at the nodes of P (m = 0 .. p-1).
__global__ __launch_bounds__(256) void k_adj_sub(AdjArgs a, int m, const double* __restrict__ Y,
                                                 const double* __restrict__ Dc,
                                                 const double* __restrict__ Dp,
                                                 const double* __restrict__ W, double* __restrict__ Dn) {
  const int s = blockIdx.z;
  const LevelView& L = a.L;
  int i, j;
  size_t k;
  if (!p_node(a, i, j, k)) return;
  const size_t so = (size_t)s * a.sstride;
  const double* __restrict__ y = Y + so;
  const double* __restrict__ dc = Dc ? Dc + so : nullptr;
  double cE, cW, cN, cS;
  edge_coefs(L, a.kappa + (size_t)s * L.nb, i, j, cE, cW, cN, cS);
  auto pq = [&](size_t kk) { return (L.flags[kk] & F_P) ? (dc ? y[kk] + dc[kk] : y[kk]) : 0.0; };
  const double pi = pq(k);
  const double apq = L.invm[k] * (cE * (pi - pq(k + 1)) + cW * (pi - pq(k - 1)) +
                                  cN * (pi - pq(k + L.ld)) + cS * (pi - pq(k - L.ld)));
  const double* cf = a.coef + (size_t)s * (L.p + 1);
  const double r = W[so + k] + apq;
  double dn;
  if (m == 0) {
    dn = -cf[1] * r;
  } else {
    const double b = L.beta[m];
    dn = (1.0 + b) * dc[k] - b * (Dp ? Dp[so + k] : 0.0) - cf[1 + m] * r;
  }
  Dn[so + k] = dn;
}

// Lambda_p = f m mu (and lw = 0).
__global__ __launch_bounds__(256) void k_adj_lam_init(AdjArgs a, double f, const double* __restrict__ MU,
                                                      double* __restrict__ Lp, double* __restrict__ LW) {
  const int s = blockIdx.z;
  if (s >= a.s_active) return;
  const LevelView& L = a.L;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
  if (i >= L.ld || j >= L.nyn) return;
  const size_t k = (size_t)j * L.ld + i, so = (size_t)s * a.sstride;
  const double im = L.invm[k];
  Lp[so + k] = im != 0.0 ? f * MU[so + k] / im : 0.0;
  LW[so + k] = 0.0;
}

// Lambda_m from Lambda_m+1 (L1) and Lambda_m+2 (L2, NULL: 0), m = p-1 .. 1,
// and lw -= c2_m Lambda_m+1, at the nodes of P; for m = 0 only lw -= c1
// Lambda_1 (Lout unused).  Off P no stencil acts, so Lambda_m = rho_m Lambda_p
// there (rho from the beta recursion alone) and the stencil reads it from Lp.
__global__ __launch_bounds__(256) void k_adj_rev(AdjArgs a, int m, const double* __restrict__ L1,
                                                 const double* __restrict__ L2, double* __restrict__ Lout,
                                                 double* __restrict__ LW, const double* __restrict__ Lp) {
  const int s = blockIdx.z;
  const LevelView& L = a.L;
  int i, j;
  size_t k;
  if (!p_node(a, i, j, k)) return;
  const size_t so = (size_t)s * a.sstride;
  const double* cf = a.coef + (size_t)s * (L.p + 1);
  const double* __restrict__ l1 = L1 + so;
  const double lam = l1[k];
  if (m == 0) {
    LW[so + k] -= cf[1] * lam;
    return;
  }
  const double c2 = cf[1 + m];
  LW[so + k] -= c2 * lam;
  double kt;   // (K (Lambda / m))_k
  {
    double cE, cW, cN, cS;
    edge_coefs(L, a.kappa + (size_t)s * L.nb, i, j, cE, cW, cN, cS);
    const double r1 = a.rho[m + 1];
    const double* __restrict__ lp = Lp + so;
    auto t = [&](size_t kk) {   // invm = 0 on Dirichlet nodes
      return ((L.flags[kk] & F_P) ? l1[kk] : r1 * lp[kk]) * L.invm[kk];
    };
    const double ti = t(k);
    kt = cE * (ti - t(k + 1)) + cW * (ti - t(k - 1)) + cN * (ti - t(k + L.ld)) + cS * (ti - t(k - L.ld));
  }
  const double bm = L.beta[m];
  const double bm1 = (m + 1 < L.p) ? L.beta[m + 1] : 0.0;
  const double l2 = L2 ? L2[so + k] : 0.0;
  Lout[so + k] = (1.0 + bm) * lam - c2 * kt - bm1 * l2;
}

// Per-cell accumulation of dQ/dkappa_cell over the derivative pairs of one step.
struct ContractArgs {
  const double* D1;                  // d_m at D1 + (m-1)*astride, m = 1..p (d_0 = 0)
  const double* L1;                  // Lambda_m at L1 + (m-1)*astride, m = 1..p
  size_t astride;
  const double* MU;                  // mu_n+1 (list form: Lambda_p / m = f mu, no Lambda_p array)
  double f;
};

// LIST: the cells of a.clist (those with a corner in P), grid (entries /
// (256 / kContractLanes), samples); each cell's pairs are split over
// kContractLanes adjacent lanes (pair m on lane m mod kContractLanes: that many
// times the loads in flight per cell) whose sums are added by lane shuffles.
// Otherwise one thread per cell of the grid.
constexpr int kContractLanes = 16;
template <bool LIST>
__global__ __launch_bounds__(256) void k_adj_contract(AdjArgs a, ContractArgs c,
                                                      const double* __restrict__ Y,
                                                      const double* __restrict__ LW,
                                                      double* __restrict__ G) {
  constexpr int NG = LIST ? kContractLanes : 1;      // lanes per cell
  const LevelView& L = a.L;
  int s, ia, jb, g = 0;
  bool on = true;
  if (LIST) {
    s = blockIdx.y;
    const int t = blockIdx.x * (256 / NG) + (int)(threadIdx.x / NG);
    g = (int)(threadIdx.x % NG);
    on = s < a.s_active && t < a.nc;
    const int kc0 = a.clist[on ? t : 0];
    jb = kc0 / L.ld;
    ia = kc0 - jb * L.ld;
  } else {
    s = blockIdx.z;
    if (s >= a.s_active) return;
    ia = blockIdx.x * BX + threadIdx.x;
    jb = blockIdx.y * BY + threadIdx.y;
    if (ia >= L.nxn - 1 || jb >= L.nyn - 1) return;
    const size_t kc = (size_t)jb * L.ld + ia;
    if (L.cblk[kc] == 255) return;
  }
  if (LIST && s >= a.s_active) s = 0;                // whole block off: read in bounds, write nothing
  // LIST: the workgroup's sample is uniform; its pair factors c_m and rho_m+1 go to LDS
  __shared__ double lcr[LIST ? 2 * kMaxAdjP : 1];
  if (LIST) {
    const double* cs = a.coef + (size_t)s * (L.p + 1);
    for (int m = (int)threadIdx.x; m < L.p; m += (int)blockDim.x) {
      lcr[2 * m] = cs[1 + m];                        // c1 for m = 0, c2_m otherwise
      lcr[2 * m + 1] = a.rho[m + 1];
    }
    __syncthreads();
  }
  const size_t kc = (size_t)jb * L.ld + ia;          // cell (ia, jb)
  const size_t so = (size_t)s * a.sstride;
  const size_t n00 = kc, n10 = kc + 1, n01 = kc + L.ld, n11 = kc + L.ld + 1;
  const double gx = L.hy[jb] * L.inv2hx[ia];   // bottom and top legs
  const double gy = L.hx[ia] * L.inv2hy[jb];   // left and right legs
  const double im00 = L.invm[n00], im10 = L.invm[n10], im01 = L.invm[n01], im11 = L.invm[n11];
  const bool p00 = L.flags[n00] & F_P, p10 = L.flags[n10] & F_P, p01 = L.flags[n01] & F_P,
             p11 = L.flags[n11] & F_P;
  const double* __restrict__ y = Y + so;
  const double y00 = y[n00], y10 = y[n10], y01 = y[n01], y11 = y[n11];
  const double* cf = a.coef + (size_t)s * (L.p + 1);
  auto side = [&](double a0, double a1, double a2, double a3, double b0, double b1, double b2,
                  double b3) {
    // corners 0 = (ia,jb), 1 = (ia+1,jb), 2 = (ia,jb+1), 3 = (ia+1,jb+1); a already divided by m
    return gx * ((a0 - a1) * (b0 - b1) + (a2 - a3) * (b2 - b3)) +
           gy * ((a0 - a2) * (b0 - b2) + (a1 - a3) * (b1 - b3));
  };
  // Lambda_m and lw are kept at the nodes of P only; off P, Lambda_m = rho_m
  // Lambda_p and lw = gamma Lambda_p with gamma = -(c1 rho_1 + sum_m c2_m rho_m+1)
  const double* __restrict__ lp = c.L1 + (size_t)(L.p - 1) * c.astride + so;
  const double* __restrict__ mu = LIST ? c.MU + so : nullptr;
  // Lambda_p / m at a corner: f mu in the list form, else from the Lambda_p array
  auto tp = [&](size_t n, double im) { return LIST ? c.f * mu[n] : lp[n] * im; };
  double acc = 0.0;
  // (lw, (I - P) y), on the first lane of the cell
  // Lambda_p / m at the corners off P, read once (the pairs take rho_m+1 times it there)
  const double t00 = p00 ? 0.0 : tp(n00, im00), t10 = p10 ? 0.0 : tp(n10, im10),
               t01 = p01 ? 0.0 : tp(n01, im01), t11 = p11 ? 0.0 : tp(n11, im11);
  if (g == 0) {
    const double gam = a.gam[s];
    const double* lw = LW + so;
    auto lwv = [&](size_t n, bool pn, double im, double tn) { return pn ? lw[n] * im : gam * tn; };
    acc += side(lwv(n00, p00, im00, t00), lwv(n10, p10, im10, t10), lwv(n01, p01, im01, t01),
                lwv(n11, p11, im11, t11), p00 ? 0.0 : y00, p10 ? 0.0 : y10, p01 ? 0.0 : y01, p11 ? 0.0 : y11);
  }
  // (-c1 Lambda_1, P y) and (-c2_m Lambda_m+1, P (y + d_m)), m = 1..p-1: zero
  // unless a corner is in P
  if (p00 || p10 || p01 || p11) {
    for (int m = g; m < L.p; m += NG) {
      const double cm = LIST ? lcr[2 * m] : cf[1 + m];
      const double rm = LIST ? lcr[2 * m + 1] : a.rho[m + 1];
      const double* la = c.L1 + (size_t)m * c.astride + so;
      const bool last = LIST && m + 1 == L.p;            // Lambda_p: f mu at the corners in P too
      auto lav = [&](size_t n, bool pn, double im, double tn) {
        return pn ? (last ? c.f * mu[n] : la[n] * im) : rm * tn;
      };
      const double* dm = m == 0 ? nullptr : c.D1 + (size_t)(m - 1) * c.astride + so;
      const double q00 = p00 ? y00 + (dm ? dm[n00] : 0.0) : 0.0;
      const double q10 = p10 ? y10 + (dm ? dm[n10] : 0.0) : 0.0;
      const double q01 = p01 ? y01 + (dm ? dm[n01] : 0.0) : 0.0;
      const double q11 = p11 ? y11 + (dm ? dm[n11] : 0.0) : 0.0;
      acc -= cm * side(lav(n00, p00, im00, t00), lav(n10, p10, im10, t10), lav(n01, p01, im01, t01),
                       lav(n11, p11, im11, t11), q00, q10, q01, q11);
    }
  }
  if (LIST) {
#pragma unroll
    for (int o = 1; o < NG; o <<= 1) acc += __shfl_xor(acc, o);
    if (g == 0 && on) G[so + kc] += acc;
  } else {
    G[so + kc] += acc;
  }
}

// mu_N = M^-1 w into buffer N_s % 2, 0 into the other.
__global__ __launch_bounds__(256) void k_adj_mu_init(AdjArgs a, const int* __restrict__ nsteps,
                                                     double* __restrict__ B0, double* __restrict__ B1) {
  const int s = blockIdx.z;
  const LevelView& L = a.L;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
  if (i >= L.ld || j >= L.nyn) return;
  const size_t k = (size_t)j * L.ld + i, so = (size_t)s * a.sstride;
  const double v = L.qoiw[k] * L.invm[k];
  double* a0 = (nsteps[s] & 1) ? B1 : B0;
  double* a1 = (nsteps[s] & 1) ? B0 : B1;
  a0[so + k] = v;
  a1[so + k] = 0.0;
}

// dQ/dg_b = 2 kappa_b sum over the cells of block b, times dLdQ[s]; one workgroup per sample.
__global__ __launch_bounds__(256) void k_adj_blocks(AdjArgs a, const double* __restrict__ G,
                                                    const double* __restrict__ dldq, int s_base,
                                                    double* __restrict__ out) {
  const int s = blockIdx.x;
  const LevelView& L = a.L;
  __shared__ double part[256];
  const double* g = G + (size_t)s * a.sstride;
  const double* gp = a.gpart + (size_t)s * a.n_wg * a.max_slots;
  for (int b = 0; b < L.nb; ++b) {
    double acc = 0.0;
    for (int c = threadIdx.x; c < (L.nyn - 1) * L.ld; c += blockDim.x)
      if (L.cblk[c] == b) acc += g[c];
    for (int w = threadIdx.x; w < a.n_wg; w += blockDim.x)
      for (int t = 0; t < a.wslots[w]; ++t)
        if (a.wblock[(size_t)w * a.max_slots + t] == b) acc += gp[(size_t)w * a.max_slots + t];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      out[(size_t)(s_base + s) * L.nb + b] = 2.0 * a.kappa[(size_t)s * L.nb + b] * part[0] * dldq[s];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fused form of one backward step on rect fine tiles.  One workgroup per
// (sample, fine tile), lane x of wavefront v = column x, rows 4v .. 4v+3 of the
// tile's region (the layout of the forward fine kernel).  For y = u_n and
// mu = mu_n+1 it recomputes the masked substep vectors q_0 .. q_p-1 of R y
// (stored in a per-tile global scratch, only at the nodes the contraction
// reads), runs the reverse sweep over the p substeps with Lambda in registers,
// and contracts every derivative pair on the cells it owns: the cells whose
// first corner in P (order: lower-left, lower-right, upper-left, upper-right)
// is inside the tile interior.  The other cells see Lambda_m = rho_m Lambda_p
// (no stencil acts there), so lw / m = gamma f mu and only the pair
// (lw, (I - P) y) contributes; k_adj_cells handles them.  Every value the
// contraction uses is exact at distance >= p - 1 from the region border (the
// forward q_m at >= m, Lambda_m+1 at >= p - m - 1), which covers the corners of
// all owned cells.
//
// With y_n+1 given, one more substep gives d_p on the interior and y_n-1 =
// (2 y - y_n+1) + 2 d_p at its F+ nodes (the step run backward in time).
//
// With mu_n+2 given, it also writes mu_n = 2 R mu_n+1 - mu_n+2 at the F+ nodes
// of the tile interior.  R is M-self-adjoint, so R mu = M^-1 R^T M mu, and the
// sweep started from Lambda_p = f M mu_n+1 yields R^T Lambda_p = Lambda_p +
// K (lw / m) (the last term from the derivative of every substep in y; off P,
// lw = gamma Lambda_p is the coarse update's weight):
//   mu_n = 2 mu_n+1 - mu_n+2 + (2/f) M^-1 K (lw / m),
// with lw / m exact at distance >= p - 1 from the region border, i.e. on the
// interior and its ring.  This replaces the forward substeps of a fine step
// on mu.
//
// The contraction of a pair (a, b) on cell (x, y) is
//   hy/(2 hx) [(a00 - a10)(b00 - b10) + (a01 - a11)(b01 - b11)]
// + hx/(2 hy) [(a00 - a01)(b00 - b01) + (a10 - a11)(b10 - b11)]
// (corners a_ij at (x + i, y + j)): a sum of products of differences along the
// cell's four edges with weights that do not depend on the pair.  So each
// lane accumulates, over all pairs, the products along its node's east edge
// (SH) and north edge (SV) with the pair's scalar factor, and the cell sums
// are formed once at the end; the differences are the ones the Lambda stencil
// uses anyway.
struct AdjTileArgs {
  LevelView L;
  const int4* __restrict__ rtiles;
  int n_fine, per_xcd, active;
  const double* __restrict__ kappa;  // [S][nb]
  const double* __restrict__ coef;   // [S][p+1]
  const double* __restrict__ Y;      // y = u_n of sample s at Y + s*sstride
  const double* __restrict__ MU;     // mu_n+1
  double* MU2;                       // mu_n+2 in, mu_n out at the F+ nodes of the tile interiors (NULL: no mu step)
  const double* Y1;                  // y_n+1 (read at the F+ nodes of the tile interiors), with
  double* Y0;                        // y_n-1 = 2 R y - y_n+1 out there (NULL: not formed)
  double* __restrict__ G;            // per-cell accumulators
  double* __restrict__ scr;          // q_0 .. q_p-1 per (sample, tile)
  size_t sstride;
  double f;                          // 2 (n >= 1) or 1 (n = 0)
};

__device__ __forceinline__ uint32_t lane_next_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, true);
}

__global__ __launch_bounds__(kFineThreads) void k_adj_fine(AdjTileArgs a) {
  constexpr int R = 4, W = 64;
  __shared__ double lk[256];
  __shared__ double lb[4 * kBndSlots];                 // boundary rows: 2 buffers x 2 quantities
  __shared__ double lL[4 * kFineThreads];              // Lambda_p of this lane's rows
  const int G_ = a.n_fine * a.active;
  const int Lid = (int)(blockIdx.x & 7) * a.per_xcd + (int)(blockIdx.x >> 3);
  if (Lid >= G_) return;
  const int s = Lid / a.n_fine, tile = Lid % a.n_fine;
  const LevelView& L = a.L;
  const int4 td = a.rtiles[tile];
  const int x0 = td.x & 0xFFFF, y0 = td.x >> 16;
  const int RX = td.y & 0xFFFF, RY = td.y >> 16;
  const int ix0 = td.z & 0xFFFF, ix1 = td.z >> 16, iy0 = td.w & 0xFFFF, iy1 = td.w >> 16;
  const int tid = threadIdx.x;
  const int x = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int yb = 4 * wv;
  const bool wave_on = yb < RY;
  const int gx = x0 + x, gyb = y0 + yb;
  const bool col_on = x < RX && gx < L.nxn;
  const double* __restrict__ y_g = a.Y + (size_t)s * a.sstride;
  const double* __restrict__ mu_g = a.MU + (size_t)s * a.sstride;
  const double* __restrict__ cf = a.coef + (size_t)s * (L.p + 1);
  const int ld = L.ld, p = L.p;
  double* __restrict__ scr = a.scr + ((size_t)s * a.n_fine + tile) * (size_t)p * (R * kFineThreads);
  // nodes whose q_m the contraction reads: corners of owned cells
  const bool col_b = gx >= ix0 - 1 && gx <= ix1;
  auto need_b = [&](int r) { return col_b && gyb + r >= iy0 - 1 && gyb + r <= iy1; };

  // ---- one batch of global reads
  const double kv = tid < L.nb ? a.kappa[(size_t)s * L.nb + tid] : 0.0;
  const int gxc = min(gx, L.nxn - 1);                  // column, in bounds off the grid
  const int gxw = max(gxc - 1, 0);
  const double hxE = L.hx[gxc], hxW = L.hx[gxw], ihE = L.inv2hx[gxc];
  double hyv[R + 1], ihy[R + 1];
  uint32_t ni[R + 2];                                  // node words of rows gy-1 .. gy+4
#pragma unroll
  for (int q = 0; q <= R + 1; ++q) {
    const int g = min(max(gyb - 1 + q, 0), L.nyn - 1);
    if (q <= R) {
      hyv[q] = L.hy[g];
      ihy[q] = L.inv2hy[g];
    }
    ni[q] = L.ninfo[g * ld + gxc];
  }
  double y[R], im[R];
  uint32_t f[R + 1];                                   // f[R]: row yb + 4
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    const bool ok = wave_on && col_on && yb + r < RY && gyb + r < L.nyn;
    f[r] = ok ? ni[r + 1] & 0xFFu : 0u;
    if (r < R) {
      const int k = ok ? (gyb + r) * ld + gx : ld + 1;
      y[r] = ok ? y_g[k] : 0.0;
      const double mu = ok ? mu_g[k] : 0.0;
      im[r] = ok ? L.invm[k] : 0.0;
      lL[r * kFineThreads + tid] = im[r] != 0.0 ? a.f * mu / im[r] : 0.0;   // Lambda_p = f M mu
    }
  }
  // Cell (gx, gyb + r), computed by the lane of its lower-left node, belongs to
  // this tile if its first corner in P is inside the tile: that node is in F+,
  // so its tile exists, and the cell's lower-left node, one node away at most,
  // lies in the region (the F+ bounding box grown by one).  Corner flags of the
  // next lane and row come by DPP and from the row above.
  uint32_t own = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t fn = lane_next_u(f[r]), fu = f[r + 1], fun = lane_next_u(f[r + 1]);
    const int gy = gyb + r;
    int cx = -1, cy = -1;
    if (f[r] & F_P) { cx = gx; cy = gy; }
    else if (fn & F_P) { cx = gx + 1; cy = gy; }
    else if (fu & F_P) { cx = gx; cy = gy + 1; }
    else if (fun & F_P) { cx = gx + 1; cy = gy + 1; }
    const bool in = cx >= ix0 && cx < ix1 && cy >= iy0 && cy < iy1;
    const bool cell = ((ni[r + 1] >> 8) & 0xFFu) != 255u;
    if (wave_on && col_on && yb + r < RY && in && cell) own |= 1u << r;
  }
  // ---- LDS: kappa (zero past the last block), boundary rows of q_0 = P y
  //      (buffer 0) and v = (I - P) y (buffer 1), zero rows of all four buffers
  double* const q0b = lb;
  double* const q1b = lb + kBndSlots;
  const int top = (2 * wv + 1) * W + x, bot = (2 * wv + 2) * W + x;
  const int below = 2 * wv * W + x, above = (2 * wv + 3) * W + x;
  if (tid < 256) lk[tid] = kv;
  double up[R], pm[R], v[R + 2];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool pi = f[r] & F_P;
    up[r] = pi ? y[r] : 0.0;
    pm[r] = pi ? 1.0 : 0.0;
    v[r + 1] = y[r] - up[r];
  }
  q0b[top] = up[0];
  q0b[bot] = up[R - 1];
  q1b[top] = v[1];
  q1b[bot] = v[R];
  for (int t = tid; t < 8 * W; t += kFineThreads) {
    const int buf = t / (2 * W), z = (t % (2 * W)) < W ? (t % W) : (kBndRows - 1) * W + (t % W);
    lb[buf * kBndSlots + z] = 0.0;
  }
  __syncthreads();

  // ---- edge coefficients: kappa of the cells east / west of the node, the
  //      vertical edges shared by consecutive rows, the west edge of a node the
  //      east edge of its west neighbour
  double cE[R], cV[R + 1];
  {
    double kE[R + 1], kW[R + 1];
#pragma unroll
    for (int c = 0; c <= R; ++c) {
      kE[c] = lk[(ni[c] >> 8) & 0xFFu];
      kW[c] = lk[(ni[c] >> 16) & 0xFFu];
    }
#pragma unroll
    for (int c = 0; c <= R; ++c) cV[c] = (kE[c] * hxE + kW[c] * hxW) * ihy[c];
#pragma unroll
    for (int r = 0; r < R; ++r) cE[r] = (kE[r + 1] * hyv[r + 1] + kE[r] * hyv[r]) * ihE;
  }
  // forward: coefficients scaled by 1/m on F+, w = A_u (I - P) y
  double aE[R], aW[R], aN[R], aS[R], w[R], q[R];
  {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double imf = (f[r] & F_FPLUS) ? im[r] : 0.0;
      aE[r] = imf * cE[r];
      aW[r] = imf * lane_prev(cE[r]);
      aN[r] = imf * cV[r + 1];
      aS[r] = imf * cV[r];
      q[r] = up[r];
      if (need_b(r)) scr[(size_t)r * kFineThreads + tid] = up[r];   // q_0
    }
    v[0] = q1b[below];
    v[R + 1] = q1b[above];
    double dN[R + 1];
#pragma unroll
    for (int c = 0; c <= R; ++c) dN[c] = v[c] - v[c + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double dE = v[r + 1] - lane_next(v[r + 1]);
      const double dWn = lane_prev(dE);
      w[r] = aS[r] * -dN[r] + (aN[r] * dN[r + 1] + (aW[r] * -dWn + aE[r] * dE));
    }
  }
  __syncthreads();   // buffer 1 is overwritten by the first substep

  // ---- forward substeps: q_1 .. q_p-1 into the scratch (q_m = P (y + d_m))
  double d0[R], d1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) d0[r] = d1[r] = 0.0;
  auto fsub = [&](int m, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    double* dc = B == 0 ? d0 : d1;
    double* dq = B == 0 ? d1 : d0;
    const double c = cf[1 + m];
    const double b = m > 0 ? L.beta[m] : 0.0;
    const double* rb = B == 0 ? q0b : q1b;
    double* wb = B == 0 ? q1b : q0b;
    // q_m+1 is needed within p-1-m rows of the tile interior (the contraction
    // reads q at the interior's rows and one beyond); wavefronts whose rows all
    // lie farther out skip the substep (rows left stale are read only by rows
    // outside the next band)
    const int reach = p - 1 - m;
    if (wave_on && gyb + R > iy0 - reach && gyb < iy1 + reach) {
      double dN[R + 1];
      dN[0] = rb[below] - q[0];
#pragma unroll
      for (int r = 0; r < R; ++r) dN[r + 1] = q[r] - (r + 1 < R ? q[r + 1] : rb[above]);
      double qn[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double dE = q[r] - lane_next(q[r]);
        const double dWn = lane_prev(dE);
        const double rr = aS[r] * -dN[r] + (aN[r] * dN[r + 1] + (aW[r] * -dWn + (aE[r] * dE + w[r])));
        const double dn = (dc[r] + b * (dc[r] - dq[r])) - c * rr;
        dq[r] = dn;
        qn[r] = pm[r] * dn + up[r];
        if (need_b(r) && m + 1 < p) scr[((size_t)(m + 1) * R + r) * kFineThreads + tid] = qn[r];   // q_m+1
      }
#pragma unroll
      for (int r = 0; r < R; ++r) q[r] = qn[r];
      wb[top] = q[0];
      wb[bot] = q[R - 1];
    }
    __syncthreads();
  };
  for (int m = 0; m < p - 1; m += 2) {
    fsub(m, std::integral_constant<int, 0>{});
    if (m + 1 < p - 1) fsub(m + 1, std::integral_constant<int, 1>{});
  }
  // the step run backward in time (the recurrence is symmetric): the last
  // substep gives d_p on the interior, and y_n-1 = (2 y - y_n+1) + 2 d_p at its F+ nodes
  if (a.Y0) {
    if ((p - 1) & 1) fsub(p - 1, std::integral_constant<int, 1>{});
    else fsub(p - 1, std::integral_constant<int, 0>{});
    const double* dp = ((p - 1) & 1) ? d0 : d1;        // d_p: the register set substep p-1 wrote
    const bool col_in = gx >= ix0 && gx < ix1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = wave_on && col_on && yb + r < RY && gyb + r < L.nyn;
      if (ok && col_in && gyb + r >= iy0 && gyb + r < iy1 && (f[r] & F_FPLUS)) {
        const size_t k = (size_t)s * a.sstride + (size_t)(gyb + r) * ld + gx;
        a.Y0[k] = (2.0 * a.Y[k] - a.Y1[k]) + 2.0 * dp[r];
      }
    }
  }

  // ---- reverse sweep: Lambda_p = f M mu, Lambda_p+1 = 0; m = p-1 .. 0
  double l1[R], l2[R], lw[R], SH[R], SV[R], imr[R];
  bool pr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    l1[r] = lL[r * kFineThreads + tid];
    l2[r] = lw[r] = SH[r] = SV[r] = 0.0;
    const bool ok = wave_on && col_on && yb + r < RY && gyb + r < L.nyn;
    imr[r] = ok ? L.invm[(gyb + r) * ld + gx] : 0.0;
    pr[r] = f[r] & F_P;
  }
  for (int m = p - 1; m >= 0; --m) {
    const int B = m & 1;
    const double nc = -cf[1 + m];                        // the pair's factor -c_m
    double t[R], bq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      t[r] = l1[r] * imr[r];                             // Lambda_m+1 / m
      bq[r] = need_b(r) ? scr[((size_t)m * R + r) * kFineThreads + tid] : 0.0;   // q_m
    }
    double* const tb = lb + B * kBndSlots;               // t boundary rows
    double* const bb = lb + (2 + B) * kBndSlots;         // q_m top rows
    if (wave_on) {
      tb[top] = t[0];
      tb[bot] = t[R - 1];
      bb[top] = bq[0];
    }
    __syncthreads();
    // Lambda_m is needed within m rows of the tile interior (at least one:
    // the contraction reads the interior's rows and one beyond)
    const int reach = m > 1 ? m : 1;
    if (wave_on && gyb + R > iy0 - reach && gyb < iy1 + reach) {
      double dNt[R + 1];                                 // dNt[r + 1] = t_r - t_r+1, dNt[0] = t_-1 - t_0
      dNt[0] = tb[below] - t[0];
      const double tN3 = tb[above], bN3 = bb[above];
#pragma unroll
      for (int r = 0; r < R; ++r) dNt[r + 1] = t[r] - (r + 1 < R ? t[r + 1] : tN3);
      double ln[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double dEt = t[r] - lane_next(t[r]);
        const double dEb = bq[r] - lane_next(bq[r]);
        const double dNb = bq[r] - (r + 1 < R ? bq[r + 1] : bN3);
        SH[r] += (nc * dEt) * dEb;
        SV[r] += (nc * dNt[r + 1]) * dNb;
        lw[r] += nc * l1[r];
        const double dWn = lane_prev(dEt);             // every lane takes part in the DPP
        const double cW = lane_prev(cE[r]);
        const double st = cV[r] * -dNt[r] + (cV[r + 1] * dNt[r + 1] + (cW * -dWn + cE[r] * dEt));
        ln[r] = pr[r] ? st : 0.0;                      // (P K) (Lambda_m+1 / m)
      }
      if (m > 0) {
        const double bm = L.beta[m];
        const double bm1 = m + 1 < p ? L.beta[m + 1] : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double lm = (1.0 + bm) * l1[r] + nc * ln[r] - bm1 * l2[r];   // Lambda_m
          l2[r] = l1[r];
          l1[r] = lm;
        }
      }
    }
  }
  // ---- pair (lw, (I - P) y), then the cell sums; the mu step at the F+ nodes
  //      of the tile interior
  {
    double aw[R], vv[R], m1[R], m2[R];
    const bool col_in = gx >= ix0 && gx < ix1;
    uint32_t wmask = 0;                                // bit r: mu_n is written at row r
#pragma unroll
    for (int r = 0; r < R; ++r) {
      aw[r] = lw[r] * imr[r];
      const bool ok = wave_on && col_on && yb + r < RY && gyb + r < L.nyn;
      const int k = (gyb + r) * ld + gx;
      vv[r] = (ok && !pr[r]) ? y_g[k] : 0.0;
      const bool wr = a.MU2 && ok && col_in && gyb + r >= iy0 && gyb + r < iy1 && (f[r] & F_FPLUS);
      if (wr) wmask |= 1u << r;
      m1[r] = wr ? mu_g[k] : 0.0;
      m2[r] = wr ? a.MU2[(size_t)s * a.sstride + k] : 0.0;
    }
    // buffers of the parity not read in the last reverse step (m = 0 used parity 0)
    double* const tb = lb + kBndSlots;
    double* const bb = lb + 3 * kBndSlots;
    if (wave_on) {
      tb[top] = aw[0];
      tb[bot] = aw[R - 1];
      bb[top] = vv[0];
    }
    __syncthreads();
    if (wave_on) {
      const double aN3 = tb[above], vN3 = bb[above];
      double dNs = tb[below] - aw[0];                  // lw / m of the row below minus this row's
      const double g2 = 2.0 / a.f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double dEa = aw[r] - lane_next(aw[r]), dEv = vv[r] - lane_next(vv[r]);
        const double dNa = aw[r] - (r + 1 < R ? aw[r + 1] : aN3), dNv = vv[r] - (r + 1 < R ? vv[r + 1] : vN3);
        SH[r] += dEa * dEv;
        SV[r] += dNa * dNv;
        if (a.MU2) {
          // the one-step map is M-self-adjoint, so R mu_n+1 = M^-1 R^T M mu_n+1;
          // with Lambda_p = f M mu_n+1 the sweep gives R^T Lambda_p = Lambda_p + K (lw / m)
          const double dWa = lane_prev(dEa);             // every lane takes part in the DPP
          const double cW = lane_prev(cE[r]);
          const double ka = cV[r] * -dNs + (cV[r + 1] * dNa + (cW * -dWa + cE[r] * dEa));
          if (wmask & (1u << r))
            a.MU2[(size_t)s * a.sstride + (size_t)(gyb + r) * ld + gx] = 2.0 * m1[r] - m2[r] + g2 * imr[r] * ka;
        }
        dNs = dNa;
      }
    }
  }
  // cell (x, r): its bottom edge is this node's east edge, its top edge the east
  // edge of the node above (the next wavefront's row 0 for r = 3), its left and
  // right edges the north edges of this node and of the east neighbour
  double* const sb = lb;   // buffer 0 (last read before the previous barrier): SH of each row 0
  if (wave_on) sb[top] = SH[0];
  __syncthreads();
  double* __restrict__ Gs = a.G + (size_t)s * a.sstride;
  if (wave_on) {
    // the cell geometry is read again here rather than kept in registers
    // through both sweeps (the opaque copy of the level view stops the
    // compiler from reusing the first reads)
    using gptr = const __attribute__((address_space(1))) double*;   // keeps global accesses
    gptr hxp = (gptr)L.hx, hyp = (gptr)L.hy, ihxp = (gptr)L.inv2hx, ihyp = (gptr)L.inv2hy;
    asm volatile("" : "+s"(hxp), "+s"(hyp), "+s"(ihxp), "+s"(ihyp));
    const double gxE = hxp[gxc], gihE = ihxp[gxc];
    const double shN = sb[above];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int g = min(gyb + r, L.nyn - 1);
      const double svE = lane_next(SV[r]);
      const double acc = hyp[g] * gihE * (SH[r] + (r + 1 < R ? SH[r + 1] : shN)) +
                         gxE * ihyp[g] * (SV[r] + svE);
      if (own & (1u << r)) Gs[(size_t)(gyb + r) * ld + gx] += acc;
    }
  }
}

// lw = gamma Lambda_p off P (no stencil acts there):
// gamma = -(c1 rho_1 + sum_{m=1}^{p-1} c2_m rho_m+1), rho_p = 1, rho_p+1 = 0,
// rho_m = (1 + beta_m) rho_m+1 - beta_m+1 rho_m+2.
__device__ double adj_gamma(const LevelView& L, const double* __restrict__ cf) {
  const int p = L.p;
  double r1 = 1.0, r2 = 0.0, gam = 0.0;            // rho_m+1, rho_m+2
  for (int m = p - 1; m >= 1; --m) {
    gam -= cf[1 + m] * r1;
    const double bm1 = m + 1 < p ? L.beta[m + 1] : 0.0;
    const double rm = (1.0 + L.beta[m]) * r1 - bm1 * r2;
    r2 = r1;
    r1 = rm;
  }
  return gam - cf[1] * r1;
}

__global__ __launch_bounds__(256) void k_adj_gamma(AdjArgs a, int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) a.gam[s] = adj_gamma(a.L, a.coef + (size_t)s * (a.L.p + 1));
}

// The F+ part of the mu step on compact tilings, from the reverse sweep's lw
// (as in k_adj_fine: R mu = M^-1 R^T M mu and R^T Lambda_p = Lambda_p + K (lw / m)):
//   mu_n = 2 mu_n+1 - mu_n+2 + (2/f) M^-1 K (lw / m)
// at the F+ DOFs (list), with lw / m from the sweep on P and gamma f mu_n+1
// elsewhere.  mu_n overwrites mu_n+2; the coarse items give the other DOFs.
__global__ __launch_bounds__(256) void k_adj_mu_fplus(AdjArgs a, const int* __restrict__ flist, int nf, double f,
                                                      const double* __restrict__ MU1,
                                                      const double* __restrict__ LW, double* __restrict__ MU2) {
  const int s = blockIdx.z;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf || s >= a.s_active) return;
  const LevelView& L = a.L;
  const size_t k = (size_t)flist[t];
  const int j = (int)(k / (size_t)L.ld), i = (int)(k - (size_t)j * L.ld);
  const size_t so = (size_t)s * a.sstride;
  const double gf = a.gam[s] * f;
  const double* __restrict__ mu = MU1 + so;
  const double* __restrict__ lw = LW + so;
  auto lwm = [&](size_t kk) { return (L.flags[kk] & F_P) ? lw[kk] * L.invm[kk] : gf * mu[kk]; };
  double cE, cW, cN, cS;
  edge_coefs(L, a.kappa + (size_t)s * L.nb, i, j, cE, cW, cN, cS);
  const double c = lwm(k);
  const double ka = cE * (c - lwm(k + 1)) + cW * (c - lwm(k - 1)) + cN * (c - lwm(k + L.ld)) +
                    cS * (c - lwm(k - L.ld));
  MU2[so + k] = 2.0 * mu[k] - MU2[so + k] + (2.0 / f) * L.invm[k] * ka;
}

// Cells without a node of P: with lw / m = gamma f mu (gamma from the substep
// scalars), only the pair (lw, (I - P) y) = (lw, y) contributes.  The cells of
// a workgroup are summed per block (a few blocks per workgroup) and the sums
// accumulate over the steps in gpart, so no per-cell accumulator is read and
// written every step.
__global__ __launch_bounds__(256) void k_adj_cells(AdjArgs a, const double* __restrict__ Y,
                                                   const double* __restrict__ MU, double f) {
  const int s = blockIdx.z;
  if (s >= a.s_active) return;
  const LevelView& L = a.L;
  const int ia = blockIdx.x * BX + threadIdx.x, jb = blockIdx.y * BY + threadIdx.y;
  double v = 0.0;
  int q = 255;
  if (ia < L.nxn - 1 && jb < L.nyn - 1) {
    const size_t kc = (size_t)jb * L.ld + ia;
    q = a.cslot[kc];
    if (q != 255) {
      const size_t n00 = kc, n10 = kc + 1, n01 = kc + L.ld, n11 = kc + L.ld + 1;
      const size_t so = (size_t)s * a.sstride;
      const double* __restrict__ y = Y + so;
      const double* __restrict__ mu = MU + so;
      const double gx = L.hy[jb] * L.inv2hx[ia], gy = L.hx[ia] * L.inv2hy[jb];
      const double a0 = mu[n00], a1 = mu[n10], a2 = mu[n01], a3 = mu[n11];
      const double b0 = y[n00], b1 = y[n10], b2 = y[n01], b3 = y[n11];
      const double sd = gx * ((a0 - a1) * (b0 - b1) + (a2 - a3) * (b2 - b3)) +
                        gy * ((a0 - a2) * (b0 - b2) + (a1 - a3) * (b1 - b3));
      v = a.gam[s] * f * sd;
    }
  }
  // per-slot workgroup sums: wavefront shuffles, then the four wavefronts in a fixed order
  __shared__ double part[BY];
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  const int ns = a.wslots[wg];
  double* gp = a.gpart + ((size_t)s * a.n_wg + wg) * a.max_slots;
  for (int t = 0; t < ns; ++t) {
    double x = q == t ? v : 0.0;
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (threadIdx.x == 0) part[threadIdx.y] = x;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) gp[t] += (part[0] + part[1]) + (part[2] + part[3]);
    __syncthreads();
  }
}

// p[0 .. n-1] = v with a grid-stride loop: the workspace can hold more than
// 2^32 doubles, beyond what one grid dimension can count in work-items.
__global__ __launch_bounds__(256) void k_fill(double* __restrict__ p, size_t n, double v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

}  // namespace

// Backward solve of one sub-batch (samples already sorted by decreasing n_steps,
// device tables staged).  Writes Q (sorted order) and dQ/dg * dLdQ rows
// s_base .. s_base+n-1 of out (sorted order).
lts_status adjoint_device(lts_ctx c, const DevLevel& lv, int n, const double* d_kappa,
                          const double* d_coef, const int* d_nsteps, const double* d_x0, double width,
                          const std::vector<int>& h_nsteps, int K, const double* d_dldq, double* d_Q,
                          double* d_out, int s_base) {
  const LevelView Lv = lv.view();
  const int p = lv.H.p;
  const size_t ss = lv.nodes;
  const size_t one = (size_t)n * ss;            // doubles in one batch-wide state array
  const int maxn = h_nsteps[0];
  const int n_ck = (maxn + K - 1) / K;
  // workspace layout (doubles): checkpoints 2*n_ck, segment K+1, d 1..p, Lambda 1..p+1 (+1 spare),
  // w, lw, mu 2, G, state 2
  const size_t n_arrays = 2 * (size_t)n_ck + (K + 1) + p + (p + 2) + 2 + 2 + 1;
  LTS_HIP(c, c->adj.ensure(n_arrays * one * sizeof(double)));
  double* base = c->adj.as<double>();
  auto arr = [&](size_t idx) { return base + idx * one; };
  size_t at = 0;
  const size_t ck0 = at; at += 2 * (size_t)n_ck;
  const size_t seg0 = at; at += K + 1;
  const size_t d0 = at; at += p;          // d_m at d0 + m - 1
  const size_t l0 = at; at += p + 2;      // Lambda_m at l0 + m - 1, m = 1..p+1
  const size_t iw = at++, ilw = at++, imu0 = at++, imu1 = at++, iG = at++;
  (void)ilw;

  AdjArgs a;
  a.L = Lv;
  a.kappa = d_kappa;
  a.coef = d_coef;
  a.sstride = ss;
  int* d_fl = nullptr;                          // F+ DOFs (list), for the mu step on compact tilings
  int nfl = 0;
  // the general backward step works on the nodes of P (list) and uses
  // Lambda_m = rho_m Lambda_p elsewhere: rho_p = 1, rho_p+1 = 0,
  // rho_m = (1 + beta_m) rho_m+1 - beta_m+1 rho_m+2 (beta_p := 0)
  {
    std::vector<int> pl, cl, fl;
    for (int j = 0; j < lv.H.nyn; ++j)
      for (int i = 0; i < lv.H.nxn; ++i) {
        const uint8_t fg = lv.H.flags[(size_t)j * lv.H.nxn + i];
        if (fg & LTS_NODE_P) pl.push_back(j * lv.ld + i);
        if ((fg & LTS_NODE_DOF) && (fg & LTS_NODE_FPLUS)) fl.push_back(j * lv.ld + i);
      }
    auto isP = [&](int i, int j) { return (lv.H.flags[(size_t)j * lv.H.nxn + i] & LTS_NODE_P) != 0; };
    for (int b = 0; b + 1 < lv.H.nyn; ++b)
      for (int i = 0; i + 1 < lv.H.nxn; ++i)
        if (lv.H.active[(size_t)b * lv.H.nxc + i] && (isP(i, b) || isP(i + 1, b) || isP(i, b + 1) || isP(i + 1, b + 1)))
          cl.push_back(b * lv.ld + i);
    std::vector<double> rho((size_t)p + 2, 0.0);
    rho[p] = 1.0;
    for (int m = p - 1; m >= 1; --m)
      rho[m] = (1.0 + lv.H.beta[m]) * rho[m + 1] - (m + 1 < p ? lv.H.beta[m + 1] : 0.0) * rho[m + 2];
    // k_adj_cells: per workgroup of its grid (BX x BY cells), the blocks of
    // the cells it handles (active, no corner in P) get slots 0, 1, ...
    const int gxw = (lv.H.nxn + BX - 1) / BX, gyw = (lv.H.nyn + BY - 1) / BY;
    const int n_wg = gxw * gyw;
    std::vector<uint8_t> cslot((size_t)(lv.H.nyn - 1) * lv.ld, 255);
    std::vector<std::vector<int>> wbl(n_wg);
    for (int wy = 0; wy < gyw; ++wy)
      for (int wx = 0; wx < gxw; ++wx) {
        std::vector<int>& bl = wbl[(size_t)wy * gxw + wx];
        for (int jb = wy * BY; jb < std::min((wy + 1) * BY, lv.H.nyn - 1); ++jb)
          for (int ia = wx * BX; ia < std::min((wx + 1) * BX, lv.H.nxn - 1); ++ia) {
            const size_t ci = (size_t)jb * lv.H.nxc + ia;
            if (!lv.H.active[ci] || isP(ia, jb) || isP(ia + 1, jb) || isP(ia, jb + 1) || isP(ia + 1, jb + 1)) continue;
            const int b = lv.H.block[ci];
            const size_t t = (size_t)(std::find(bl.begin(), bl.end(), b) - bl.begin());
            if (t == bl.size()) bl.push_back(b);
            cslot[(size_t)jb * lv.ld + ia] = (uint8_t)t;
          }
      }
    int max_slots = 1;
    for (const auto& bl : wbl) max_slots = std::max(max_slots, (int)bl.size());
    std::vector<int> wslots(n_wg), wblock((size_t)n_wg * max_slots, -1);
    for (int w = 0; w < n_wg; ++w) {
      wslots[w] = (int)wbl[w].size();
      for (size_t t = 0; t < wbl[w].size(); ++t) wblock[(size_t)w * max_slots + t] = wbl[w][t];
    }
    const size_t n_gp = (size_t)n * n_wg * max_slots;
    LTS_HIP(c, c->adjlist.ensure(
                   (rho.size() + n + n_gp) * sizeof(double) +
                   (pl.size() + cl.size() + fl.size() + wslots.size() + wblock.size()) * sizeof(int) + cslot.size() + 16));
    double* d_rho = c->adjlist.as<double>();
    a.gam = d_rho + rho.size();
    a.gpart = a.gam + n;
    int* d_pl = reinterpret_cast<int*>(a.gpart + n_gp);
    int* d_cl = d_pl + pl.size();
    d_fl = d_cl + cl.size();
    nfl = (int)fl.size();
    int* d_ws = d_fl + fl.size();
    int* d_wb = d_ws + wslots.size();
    uint8_t* d_cs = reinterpret_cast<uint8_t*>(d_wb + wblock.size());
    a.cslot = d_cs;
    a.wslots = d_ws;
    a.wblock = d_wb;
    a.n_wg = n_wg;
    a.max_slots = max_slots;
    LTS_HIP(c, hipMemcpyAsync(d_ws, wslots.data(), wslots.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    LTS_HIP(c, hipMemcpyAsync(d_wb, wblock.data(), wblock.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    LTS_HIP(c, hipMemcpyAsync(d_cs, cslot.data(), cslot.size(), hipMemcpyHostToDevice, c->stream));
    k_fill<<<(unsigned)std::min<size_t>((n_gp + 255) / 256, 65536), 256, 0, c->stream>>>(a.gpart, n_gp, 0.0);
    LTS_HIP(c, hipMemcpyAsync(d_rho, rho.data(), rho.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (!pl.empty())
      LTS_HIP(c, hipMemcpyAsync(d_pl, pl.data(), pl.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    if (!cl.empty())
      LTS_HIP(c, hipMemcpyAsync(d_cl, cl.data(), cl.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    if (!fl.empty())
      LTS_HIP(c, hipMemcpyAsync(d_fl, fl.data(), fl.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));   // host vectors end with this scope
    a.rho = d_rho;
    a.plist = d_pl;
    a.np = (int)pl.size();
    a.clist = d_cl;
    a.nc = (int)cl.size();
  }
  const dim3 blk(BX, BY);
  auto grid = [&](int cols, int nz) { return dim3((cols + BX - 1) / BX, (Lv.nyn + BY - 1) / BY, nz); };
  // zero the whole workspace region used (cells of G, Lambda spare, ...)
  {
    const size_t tot = at * one;
    const size_t blocks = std::min<size_t>((tot + 255) / 256, 65536);
    k_fill<<<(unsigned)blocks, 256, 0, c->stream>>>(base, tot, 0.0);
  }
  // ---- forward with checkpoints: states in the two state buffers
  LTS_HIP(c, c->st0.ensure(one * sizeof(double)));
  LTS_HIP(c, c->st1.ensure(one * sizeof(double)));
  double* B[2] = {c->st0.as<double>(), c->st1.as<double>()};
  lts_status r = init_states(c, lv, n, d_x0, width, B[0], B[1]);
  if (r != LTS_OK) return r;
  const size_t bytes1 = one * sizeof(double);
  int active = n;
  for (int step = 0; step < maxn; ++step) {
    if (step % K == 0) {
      // pair (u_step, u_step+1): copy u_step now, u_step+1 after the step
      LTS_HIP(c, hipMemcpyAsync(arr(ck0 + 2 * (step / K)), B[step & 1], bytes1, hipMemcpyDeviceToDevice, c->stream));
    }
    while (active > 0 && h_nsteps[active - 1] <= step) --active;
    r = launch_step(c, lv, lv.tiling, d_kappa, d_coef, B[step & 1], B[(step + 1) & 1], ss, 0, active,
                    step == 0, c->stream);
    if (r != LTS_OK) return r;
    if (step % K == 0)
      LTS_HIP(c, hipMemcpyAsync(arr(ck0 + 2 * (step / K) + 1), B[(step + 1) & 1], bytes1,
                                hipMemcpyDeviceToDevice, c->stream));
  }
  r = qoi_device(c, lv, n, d_nsteps, B[0], B[1], d_Q);
  if (r != LTS_OK) return r;

  // ---- backward
  // fused form on rect fine tiles: per-(sample, tile) scratch for q_0 .. q_p-1
  const TilingDev& T = lv.tiling;
  const bool fused = T.rect && T.n_fine > 0;
  if (fused)
    LTS_HIP(c, c->adjscr.ensure(std::max<size_t>((size_t)T.n_fine * n * (size_t)p *
                                                 (4 * kFineThreads) * sizeof(double), 8)));
  double* MU[2] = {arr(imu0), arr(imu1)};
  k_adj_mu_init<<<grid(Lv.ld, n), blk, 0, c->stream>>>(a, d_nsteps, MU[0], MU[1]);
  k_adj_gamma<<<(n + 255) / 256, 256, 0, c->stream>>>(a, n);
  ContractArgs ca;
  ca.D1 = arr(d0);
  ca.L1 = arr(l0);
  ca.astride = one;
  ca.MU = nullptr;
  ca.f = 0.0;
  // Levels with fine tiles run the step backward in time instead of
  // recomputing each segment forward: u_n-1 = 2 R u_n - u_n+1 is the same
  // recurrence, and the backward step forms R u_n's substeps anyway, so it
  // writes u_n-1 at the F+ nodes and the coarse items the rest.  Each segment
  // starts from exact states: the checkpoint pair above it for the samples
  // that continue from the segment above, a sample's last two states (still
  // in the forward buffers) when it joins at its last step.  Levels without
  // fine tiles recompute each segment forward from its checkpoint pair.
  const bool recon = T.n_fine > 0;
  auto count = [&](int last) {                  // samples with n_s - 1 >= last
    int k = 0;
    while (k < n && h_nsteps[k] - 1 >= last) ++k;
    return k;
  };
  for (int k0 = (n_ck - 1) * K; k0 >= 0; k0 -= K) {
    const int k1 = std::min(k0 + K - 1, maxn - 1);
    int seg_active = 0;
    while (seg_active < n && h_nsteps[seg_active] > k0) ++seg_active;
    if (seg_active == 0) continue;
    if (recon) {
      // samples that continue from the segment above: u_k1+1 and u_k1+2 from
      // the checkpoint pair at k1 + 1, then u_k1 by one step backward
      const int cont = count(k1 + 1);
      if (cont > 0) {
        const size_t cb = (size_t)cont * ss * sizeof(double);
        LTS_HIP(c, hipMemcpyAsync(arr(seg0 + (k1 + 1 - k0)), arr(ck0 + 2 * ((k1 + 1) / K)), cb,
                                  hipMemcpyDeviceToDevice, c->stream));
        r = launch_step(c, lv, lv.tiling, d_kappa, d_coef, arr(seg0 + (k1 + 1 - k0)), arr(ck0 + 2 * ((k1 + 1) / K) + 1),
                        ss, 0, cont, 0, c->stream, false, arr(seg0 + (k1 - k0)));
        if (r != LTS_OK) return r;
      }
    } else {
      // recompute the segment u_k0 .. u_k1 for every sample that reaches k0
      const size_t sb = (size_t)seg_active * ss * sizeof(double);
      LTS_HIP(c, hipMemcpyAsync(arr(seg0), arr(ck0 + 2 * (k0 / K)), sb, hipMemcpyDeviceToDevice, c->stream));
      LTS_HIP(c, hipMemcpyAsync(arr(seg0 + 1), arr(ck0 + 2 * (k0 / K) + 1), sb, hipMemcpyDeviceToDevice, c->stream));
      for (int jn = k0 + 1; jn < k1; ++jn) {
        int act = 0;
        while (act < n && h_nsteps[act] > jn) ++act;
        if (act == 0) break;
        // u_jn+1 out of place from u_jn and u_jn-1 (the segment keeps every state)
        r = launch_step(c, lv, lv.tiling, d_kappa, d_coef, arr(seg0 + (jn - k0)), arr(seg0 + (jn - k0) - 1), ss, 0,
                        act, 0, c->stream, false, arr(seg0 + (jn - k0) + 1));
        if (r != LTS_OK) return r;
      }
    }
    for (int nn = k1; nn >= k0; --nn) {
      const int act = count(nn);
      if (act == 0) continue;
      if (recon) {
        // samples whose last step is nn join with u_nn+1 = u_n_s and u_nn
        const int prev = count(nn + 1);
        if (act > prev) {
          const size_t off = (size_t)prev * ss, jb = (size_t)(act - prev) * ss * sizeof(double);
          LTS_HIP(c, hipMemcpyAsync(arr(seg0 + (nn + 1 - k0)) + off, B[(nn + 1) & 1] + off, jb,
                                    hipMemcpyDeviceToDevice, c->stream));
          LTS_HIP(c, hipMemcpyAsync(arr(seg0 + (nn - k0)) + off, B[nn & 1] + off, jb, hipMemcpyDeviceToDevice,
                                    c->stream));
        }
      }
      // u_nn-1 is formed (recon) while the segment has steps left below nn
      const double* y1 = recon ? arr(seg0 + (nn + 1 - k0)) : nullptr;
      double* y0 = recon && nn > k0 ? arr(seg0 + (nn - 1 - k0)) : nullptr;
      a.s_active = act;
      const double* y = arr(seg0 + (nn - k0));
      const double f = nn >= 1 ? 2.0 : 1.0;
      double* mu1 = MU[(nn + 1) & 1];   // mu_{n+1}
      double* mu2 = MU[nn & 1];         // mu_{n+2} (overwritten by mu_n)
      if (fused) {
        // fine tiles (cells with a node of P) and the remaining cells
        AdjTileArgs ta;
        ta.L = Lv;
        ta.rtiles = T.rtiles.as<int4>();
        ta.n_fine = T.n_fine;
        ta.active = act;
        ta.kappa = d_kappa;
        ta.coef = d_coef;
        ta.Y = y;
        ta.MU = mu1;
        ta.G = arr(iG);
        ta.scr = c->adjscr.as<double>();
        ta.sstride = ss;
        ta.f = f;
        // mu_n = 2 R mu_n+1 - mu_n+2: its F+ part by the tile kernel (from the
        // sweep it runs anyway), the other DOFs by the coarse items
        ta.MU2 = nn >= 1 ? mu2 : nullptr;
        ta.Y1 = y1;
        ta.Y0 = y0;
        const long long Gw = (long long)T.n_fine * act;
        ta.per_xcd = (int)((Gw + 7) / 8);
        if (Gw > 0) k_adj_fine<<<dim3((unsigned)(8LL * ta.per_xcd)), dim3(kFineThreads), 0, c->stream>>>(ta);
        k_adj_cells<<<grid(Lv.nxn, act), blk, 0, c->stream>>>(a, y, mu1, f);
        if (nn >= 1) {
          r = launch_coarse(c, lv, lv.tiling, d_kappa, d_coef, mu1, mu2, ss, act, 0, c->stream);
          if (r != LTS_OK) return r;
        }
        if (y0) {
          r = launch_coarse(c, lv, lv.tiling, d_kappa, d_coef, y, const_cast<double*>(y1), ss, act, 0, c->stream,
                            false, y0);
          if (r != LTS_OK) return r;
        }
        continue;
      }
      if (!T.rect && T.n_fine > 0) {
        // compact tiles: one launch per sweep (d_1 .. d_p, then Lambda_1 ..
        // Lambda_p-1 and lw, at the nodes of P); no Lambda_p array: the sweep
        // and the contraction take Lambda_p / m = f mu, and the reverse sweep
        // sets lw at every node of P
        ca.MU = mu1;
        ca.f = f;
        r = launch_adj_compact(c, lv, T, d_kappa, d_coef, y, nullptr, arr(d0), nullptr, nullptr, nullptr, one, ss,
                               act, f, false, c->stream, y1, y0);
        if (r != LTS_OK) return r;
        r = launch_adj_compact(c, lv, T, d_kappa, d_coef, y, mu1, nullptr, arr(l0), arr(ilw), a.rho, one, ss, act,
                               f, true, c->stream);
        if (r != LTS_OK) return r;
        // the cells with a corner in P from their list; the others by the closed form
        if (a.nc > 0)
          k_adj_contract<true><<<dim3((unsigned)((a.nc + 256 / kContractLanes - 1) / (256 / kContractLanes)),
                                      (unsigned)act), 256, 0, c->stream>>>(
              a, ca, y, arr(ilw), arr(iG));
        k_adj_cells<<<grid(Lv.nxn, act), blk, 0, c->stream>>>(a, y, mu1, f);
        if (nn >= 1) {
          // mu_n: the F+ DOFs from the sweep's lw, the others by the coarse items
          if (nfl > 0)
            k_adj_mu_fplus<<<dim3((unsigned)((nfl + 255) / 256), 1, (unsigned)act), 256, 0, c->stream>>>(
                a, d_fl, nfl, f, mu1, arr(ilw), mu2);
          r = launch_coarse(c, lv, lv.tiling, d_kappa, d_coef, mu1, mu2, ss, act, 0, c->stream);
          if (r != LTS_OK) return r;
        }
        if (y0) {
          r = launch_coarse(c, lv, lv.tiling, d_kappa, d_coef, y, const_cast<double*>(y1), ss, act, 0, c->stream,
                            false, y0);
          if (r != LTS_OK) return r;
        }
        continue;
      }
      // forward substeps of y, at the nodes of P
      const dim3 pgrid((unsigned)((a.np + 255) / 256), 1, (unsigned)act);
      if (a.np > 0) {
        k_adj_w<<<pgrid, 256, 0, c->stream>>>(a, y, arr(iw));
        for (int m = 0; m < p; ++m)
          k_adj_sub<<<pgrid, 256, 0, c->stream>>>(a, m, y, m == 0 ? nullptr : arr(d0 + m - 1),
                                                   m <= 1 ? nullptr : arr(d0 + m - 2), arr(iw), arr(d0 + m));
      }
      // reverse sweep
      k_adj_lam_init<<<grid(Lv.ld, act), blk, 0, c->stream>>>(a, f, mu1, arr(l0 + p - 1), arr(ilw));
      if (a.np > 0)
        for (int m = p - 1; m >= 0; --m)
          k_adj_rev<<<pgrid, 256, 0, c->stream>>>(a, m, arr(l0 + m), m + 1 < p ? arr(l0 + m + 1) : nullptr,
                                                  m > 0 ? arr(l0 + m - 1) : nullptr, arr(ilw), arr(l0 + p - 1));
      k_adj_contract<false><<<grid(Lv.nxn, act), blk, 0, c->stream>>>(a, ca, y, arr(ilw), arr(iG));
      // mu_n = 2 R mu_{n+1} - mu_{n+2}
      if (nn >= 1) {
        r = launch_step(c, lv, lv.tiling, d_kappa, d_coef, mu1, mu2, ss, 0, act, 0, c->stream);
        if (r != LTS_OK) return r;
      }
    }
  }
  LTS_HIP(c, hipGetLastError());
  k_adj_blocks<<<n, 256, 0, c->stream>>>(a, arr(iG), d_dldq, s_base, d_out);
  LTS_HIP(c, hipGetLastError());
  return LTS_OK;
}

}  // namespace lts
