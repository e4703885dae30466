// Level construction on the host: rectilinear grids split into P1 triangles,
// lumped mass, projector P, F+ and QoI weights (Sec. 3.1-3.4).
//
// Built with -ffp-contract=off: every coordinate, area, mass and weight here
// is exact dyadic arithmetic plus one final division by 6, so the arrays are
// reproducible bit for bit by any implementation of the same rules.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace lts {

static std::string check_axis(const double* v, int n, const char* name) {
  for (int k = 0; k + 1 < n; ++k)
    if (!(v[k + 1] > v[k]) || !std::isfinite(v[k]) || !std::isfinite(v[k + 1]))
      return std::string(name) + " must be finite and strictly increasing";
  return "";
}

std::string build_level_from_desc(const lts_grid_desc& d, HostLevel& L) {
  if (d.nx_cells < 2 || d.ny_cells < 2) return "nx_cells and ny_cells must be >= 2";
  if (d.nx_cells > (1 << 15) || d.ny_cells > (1 << 15)) return "grid too large";
  if (!d.x || !d.y || !d.cell_block || !d.cell_fine || !d.cell_qoi) return "NULL array in lts_grid_desc";
  if (d.n_blocks < 1 || d.n_blocks > 255) return "n_blocks must be in 1..255";
  if (d.p < 1 || d.p > 256) return "p must be in 1..256";
  if (!(d.nu >= 0.0 && d.nu <= 1.0)) return "nu must be in [0,1]";
  if (!(d.h > 0.0) || !std::isfinite(d.h)) return "h must be > 0";
  const int nxc = d.nx_cells, nyc = d.ny_cells, nxn = nxc + 1, nyn = nyc + 1;
  std::string e = check_axis(d.x, nxn, "x");
  if (!e.empty()) return e;
  e = check_axis(d.y, nyn, "y");
  if (!e.empty()) return e;

  L = HostLevel();
  L.nxc = nxc; L.nyc = nyc; L.nxn = nxn; L.nyn = nyn;
  L.x.assign(d.x, d.x + nxn);
  L.y.assign(d.y, d.y + nyn);
  const size_t nc = (size_t)nxc * nyc, nn = (size_t)nxn * nyn;
  L.active.assign(nc, 1);
  if (d.cell_active)
    for (size_t c = 0; c < nc; ++c) L.active[c] = d.cell_active[c] ? 1 : 0;
  L.block.assign(nc, -1);
  L.fine.assign(nc, 0);
  L.qoi.assign(nc, 0);
  for (size_t c = 0; c < nc; ++c) {
    if (!L.active[c]) continue;
    if (d.cell_block[c] < 0 || d.cell_block[c] >= d.n_blocks) return "cell_block out of range";
    L.block[c] = d.cell_block[c];
    L.fine[c] = d.cell_fine[c] ? 1 : 0;
    L.qoi[c] = d.cell_qoi[c] ? 1 : 0;
  }
  L.n_blocks = d.n_blocks;
  L.h = d.h;
  L.p = d.p;
  L.nu = d.nu;

  auto act = [&](int a, int b) -> bool {
    return a >= 0 && b >= 0 && a < nxc && b < nyc && L.active[(size_t)b * nxc + a];
  };
  // DOFs: all four incident cells active
  L.flags.assign(nn, 0);
  for (int j = 0; j < nyn; ++j)
    for (int i = 0; i < nxn; ++i)
      if (act(i, j) && act(i - 1, j) && act(i - 1, j - 1) && act(i, j - 1))
        L.flags[(size_t)j * nxn + i] |= LTS_NODE_DOF;

  // lumped mass and QoI weights: per node, (sum of 2|T| over incident triangles)/6.
  // Cell (a,b) = T1 {(a,b),(a+1,b),(a+1,b+1)} + T2 {(a,b),(a+1,b+1),(a,b+1)}, 2|T| = hx*hy.
  std::vector<double> s2(nn, 0.0), q2(nn, 0.0);
  for (int b = 0; b < nyc; ++b)
    for (int a = 0; a < nxc; ++a) {
      const size_t c = (size_t)b * nxc + a;
      if (!L.active[c]) continue;
      const double A2 = (L.x[a + 1] - L.x[a]) * (L.y[b + 1] - L.y[b]);
      const size_t n00 = (size_t)b * nxn + a, n10 = n00 + 1, n01 = n00 + nxn, n11 = n01 + 1;
      // T1 and T2 both contain (a,b) and (a+1,b+1); T1 has (a+1,b); T2 has (a,b+1)
      s2[n00] += A2; s2[n11] += A2; s2[n00] += A2; s2[n11] += A2;
      s2[n10] += A2; s2[n01] += A2;
      if (L.qoi[c]) {
        q2[n00] += A2; q2[n11] += A2; q2[n00] += A2; q2[n11] += A2;
        q2[n10] += A2; q2[n01] += A2;
      }
    }
  L.mass.resize(nn);
  L.qoiw.resize(nn);
  for (size_t k = 0; k < nn; ++k) {
    L.mass[k] = s2[k] / 6.0;
    L.qoiw[k] = (L.flags[k] & LTS_NODE_DOF) ? q2[k] / 6.0 : 0.0;
  }

  // P: DOFs that are vertices of a fine cell
  for (int b = 0; b < nyc; ++b)
    for (int a = 0; a < nxc; ++a) {
      const size_t c = (size_t)b * nxc + a;
      if (!L.active[c] || !L.fine[c]) continue;
      const size_t n00 = (size_t)b * nxn + a;
      const size_t v[4] = {n00, n00 + 1, n00 + nxn, n00 + nxn + 1};
      for (size_t k : v)
        if (L.flags[k] & LTS_NODE_DOF) L.flags[k] |= LTS_NODE_P;
    }
  // F+: P and every DOF with a stiffness neighbour (edge neighbour) in P.
  // Diagonal (hypotenuse) couplings of right triangles vanish.
  for (int j = 1; j + 1 < nyn; ++j)
    for (int i = 1; i + 1 < nxn; ++i) {
      const size_t k = (size_t)j * nxn + i;
      if (!(L.flags[k] & LTS_NODE_DOF)) continue;
      const bool f = (L.flags[k] & LTS_NODE_P) || (L.flags[k - 1] & LTS_NODE_P) ||
                     (L.flags[k + 1] & LTS_NODE_P) || (L.flags[k - nxn] & LTS_NODE_P) ||
                     (L.flags[k + nxn] & LTS_NODE_P);
      if (f) L.flags[k] |= LTS_NODE_FPLUS;
    }
  for (size_t k = 0; k < nn; ++k) {
    L.n_dof += (L.flags[k] & LTS_NODE_DOF) ? 1 : 0;
    L.n_P += (L.flags[k] & LTS_NODE_P) ? 1 : 0;
    L.n_F += (L.flags[k] & LTS_NODE_FPLUS) ? 1 : 0;
  }
  if (L.n_dof == 0) return "level has no DOFs";
  cheb_constants(L.p, L.nu, L.delta, L.omega, L.beta, L.beta_half);
  return "";
}

// ---------------------------------------------------------------------------

static std::vector<double> axis_box(double lo, double hi, int n, double blo, double bhi, int ref) {
  const double h = (hi - lo) / n;
  const double hf = (hi - lo) / ((double)n * ref);
  std::vector<double> v;
  for (int k = 0; k < n; ++k) {
    const double a = lo + k * h;
    const double b = lo + (k + 1) * h;
    if (b > blo && a < bhi) {
      for (int t = 0; t < ref; ++t) v.push_back(lo + (double)(k * ref + t) * hf);
    } else {
      v.push_back(lo + (double)(k * ref) * hf);
    }
  }
  v.push_back(hi);
  return v;
}

static bool axis_graded(double lo, double hi, int n, int layers, std::vector<double>& v) {
  const double h = (hi - lo) / n;
  int k0 = -1;
  for (int k = 0; k <= n; ++k)
    if (lo + k * h == 0.0) k0 = k;
  if (k0 <= 0 || k0 >= n) return false;
  v.clear();
  for (int k = 0; k < k0; ++k) v.push_back(lo + k * h);
  for (int j = 1; j <= layers; ++j) v.push_back(-std::ldexp(h, -j));
  v.push_back(0.0);
  for (int j = layers; j >= 1; --j) v.push_back(std::ldexp(h, -j));
  for (int k = k0 + 1; k <= n; ++k) v.push_back(lo + k * h);
  return true;
}

// DOFs (nodes whose four cells are active) and the DOFs that are a vertex of
// a fine cell, for per-cell flags on an nxc x nyc grid.
static void count_dof_p(int nxc, int nyc, const std::vector<uint8_t>& active, const std::vector<uint8_t>& fine,
                        long long& n_dof, long long& n_p) {
  n_dof = n_p = 0;
  auto cell = [&](const std::vector<uint8_t>& f, int a, int b) { return f[(size_t)b * nxc + a] != 0; };
  for (int j = 1; j < nyc; ++j)
    for (int i = 1; i < nxc; ++i) {
      if (!(cell(active, i, j) && cell(active, i - 1, j) && cell(active, i, j - 1) && cell(active, i - 1, j - 1)))
        continue;
      ++n_dof;
      if (cell(fine, i, j) || cell(fine, i - 1, j) || cell(fine, i, j - 1) || cell(fine, i - 1, j - 1)) ++n_p;
    }
}

// Fine set of the q smallest tiers of a graded level (Sec. 3.5): tier k holds
// the cells whose shorter leg is h 2^(k-1-layers), so the q smallest tiers are
// the cells with shorter leg < h 2^(q-layers).  The coarse step uses the
// spacing H = 2 x (shortest coarse leg) and p = ceil(H / h_min) (q = layers-1
// gives the rule "a leg < h/2" with H = h); with no fine cell, p = 1.
static void tier_fine_set(const std::vector<double>& x, const std::vector<double>& y,
                          const std::vector<uint8_t>& active, double h, int layers, int q,
                          std::vector<uint8_t>& fine, double& H, int& p) {
  const int nxc = (int)x.size() - 1, nyc = (int)y.size() - 1;
  const double thr = std::ldexp(h, q - layers);
  double cmin = INFINITY, hmin = INFINITY;
  bool any = false;
  fine.assign((size_t)nxc * nyc, 0);
  for (int b = 0; b < nyc; ++b)
    for (int a = 0; a < nxc; ++a) {
      const size_t c = (size_t)b * nxc + a;
      const double sh = std::min(x[a + 1] - x[a], y[b + 1] - y[b]);
      fine[c] = sh < thr;
      if (!active[c]) continue;
      hmin = std::min(hmin, sh);
      if (fine[c]) any = true;
      else cmin = std::min(cmin, sh);
    }
  H = 2.0 * cmin;
  p = any ? (int)std::ceil(H / hmin) : 1;
}

std::string build_rect_desc(const lts_rect_rule& r, std::vector<double>& x, std::vector<double>& y,
                            std::vector<uint8_t>& active, std::vector<int32_t>& block,
                            std::vector<uint8_t>& fine, std::vector<uint8_t>& qoi, double& h, int& p,
                            int& n_blocks) {
  if (!(r.hi > r.lo)) return "rule: hi must exceed lo";
  if (r.n_base < 2 || r.n_base > 8192) return "rule: n_base must be in 2..8192";
  if (r.nbx < 1 || r.nby < 1 || r.nbx * r.nby > 255) return "rule: block grid must have 1..255 blocks";
  const int kind = r.kind & ~LTS_RULE_LF;
  const bool lf = (r.kind & LTS_RULE_LF) != 0;
  if (kind == LTS_RULE_BOX) {
    if (r.ref < 1 || r.ref > 64) return "rule: ref must be in 1..64";
    x = axis_box(r.lo, r.hi, r.n_base, r.box_lo, r.box_hi, r.ref);
  } else if (kind == LTS_RULE_GRADED_L) {
    if (r.layers < 1 || r.layers > 20) return "rule: layers must be in 1..20";
    if (!axis_graded(r.lo, r.hi, r.n_base, r.layers, x)) return "rule: graded axis needs 0 as an interior node";
  } else {
    return "rule: unknown kind";
  }
  y = x;
  h = (r.hi - r.lo) / r.n_base;
  const int nxc = (int)x.size() - 1, nyc = (int)y.size() - 1;
  active.assign((size_t)nxc * nyc, 1);
  block.assign((size_t)nxc * nyc, 0);
  fine.assign((size_t)nxc * nyc, 0);
  qoi.assign((size_t)nxc * nyc, 0);
  double hmin = INFINITY;
  for (int a = 0; a < nxc; ++a) hmin = std::min(hmin, x[a + 1] - x[a]);
  for (int b = 0; b < nyc; ++b) hmin = std::min(hmin, y[b + 1] - y[b]);
  for (int b = 0; b < nyc; ++b)
    for (int a = 0; a < nxc; ++a) {
      const size_t c = (size_t)b * nxc + a;
      const double hx = x[a + 1] - x[a], hy = y[b + 1] - y[b];
      const double mx = 0.5 * (x[a] + x[a + 1]);
      const double my = 0.5 * (y[b] + y[b + 1]);
      if (kind == LTS_RULE_GRADED_L) active[c] = !(mx > 0.0 && my < 0.0);
      int bx = (int)std::floor((mx - r.lo) / (r.hi - r.lo) * r.nbx);
      int by = (int)std::floor((my - r.lo) / (r.hi - r.lo) * r.nby);
      bx = std::min(bx, r.nbx - 1);
      by = std::min(by, r.nby - 1);
      block[c] = by * r.nbx + bx;
      fine[c] = std::min(hx, hy) < 0.5 * h;
      qoi[c] = (r.qx_lo <= mx && mx <= r.qx_hi && r.qy_lo <= my && my <= r.qy_hi);
    }
  p = r.p > 0 ? r.p : (int)std::ceil(h / hmin);
  if (r.fine_rule != LTS_FINE_HALF_H) {
    if (kind != LTS_RULE_GRADED_L) return "rule: tier fine sets need a graded level";
    int q = r.fine_tiers;
    if (r.fine_rule == LTS_FINE_QOPT) {
      // q minimising the DOF-update rate ((N - |P_q|) + p_q |P_q|) / H_q, the
      // cost of Sec. 3.4 per unit time; the smallest q on a tie
      double best = INFINITY;
      for (int k = 0; k <= r.layers; ++k) {
        std::vector<uint8_t> f;
        double Hk;
        int pk;
        tier_fine_set(x, y, active, h, r.layers, k, f, Hk, pk);
        if (r.p_max > 0 && pk > r.p_max) continue;
        long long n, np;
        count_dof_p(nxc, nyc, active, f, n, np);
        const double rate = (double)((n - np) + (long long)pk * np) / Hk;
        if (rate < best) {
          best = rate;
          q = k;
        }
      }
    } else if (r.fine_rule != LTS_FINE_TIERS) {
      return "rule: unknown fine_rule";
    }
    if (q < 0 || q > r.layers) return "rule: fine_tiers must be in 0..layers";
    tier_fine_set(x, y, active, h, r.layers, q, fine, h, p);
    if (r.p > 0) p = r.p;
  }
  if (lf) {                                  // standard leapfrog twin: no fine cells, step dt/p
    std::fill(fine.begin(), fine.end(), (uint8_t)0);
    h /= p;
    p = 1;
  }
  n_blocks = r.nbx * r.nby;
  return "";
}

double solve_cost_model(const HostLevel& L, const lts_sample_rule& rule) {
  const double steps = std::ceil(rule.T / (rule.cfl * L.h));
  return steps * ((double)(L.n_dof - L.n_P) + (double)L.p * L.n_P);
}

}  // namespace lts
