// One-dimensional levels and samples on the host (Sec. 4.1, 4.2), exact
// arithmetic for the nodes and masses, -ffp-contract=off for the wave-speed
// fields (every operation rounds once, in a fixed order).
#include <algorithm>
#include <cmath>

#include "host.h"

namespace lts {

std::string build_line_level(const lts_line_rule& r, LineHost& L) {
  if (!(r.hi > r.lo) || !(r.H > 0.0) || !(r.h_fine > 0.0)) return "line rule: need lo < hi, H > 0, h_fine > 0";
  if (!(r.nu >= 0.0 && r.nu <= 1.0)) return "line rule: nu must be in [0, 1]";
  const double nc_d = std::round((r.hi - r.lo) / r.H);
  if (nc_d < 2 || nc_d > 1e6 || r.lo + nc_d * r.H != r.hi) return "line rule: (hi - lo) / H must be an integer >= 2";
  const int nc = (int)nc_d;
  const bool refine = r.H > r.h_fine;
  const double ref_d = std::round(r.H / r.h_fine);
  if (refine && ref_d * r.h_fine != r.H) return "line rule: H / h_fine must be an integer";
  L = LineHost();
  for (int k = 0; k < nc; ++k) {
    const double a = r.lo + (double)k * r.H, b = r.lo + (double)(k + 1) * r.H;
    if (refine && a >= r.fine_lo && b <= r.fine_hi) {
      for (int t = 0; t < (int)ref_d; ++t) L.x.push_back(a + (double)t * r.h_fine);
    } else {
      L.x.push_back(a);
    }
  }
  L.x.push_back(r.hi);
  const int n = (int)L.x.size();
  if (n > 65536) return "line rule: more than 65536 nodes";
  L.fine.assign(n - 1, 0);
  L.mass.assign(n, 0.0);
  L.P.assign(n, 0);
  bool any = false;
  for (int c = 0; c + 1 < n; ++c) {
    const double hc = L.x[c + 1] - L.x[c];
    L.fine[c] = hc < r.H;
    L.mass[c] += 0.5 * hc;
    L.mass[c + 1] += 0.5 * hc;
    if (L.fine[c]) {
      any = true;
      L.P[c] = L.P[c + 1] = 1;
    }
  }
  L.H = r.H;
  L.nu = r.nu;
  L.p = any ? (int)std::ceil(r.H / r.h_fine) : 1;
  if (r.lf && any) {                       // leapfrog twin: no local steps, dt from h_fine
    std::fill(L.P.begin(), L.P.end(), (uint8_t)0);
    L.H = r.H / L.p;
    L.p = 1;
    any = false;
  }
  if (L.p > 256) return "line rule: p above 256";
  if (any) {
    int lo = n, hi = -1;
    for (int i = 0; i < n; ++i)
      if (L.P[i]) {
        lo = std::min(lo, i);
        hi = std::max(hi, i);
      }
    for (int i = lo; i <= hi; ++i)
      if (!L.P[i]) return "line rule: the fine cells must form one interval";
    L.f0 = std::max(lo - 1, 0);
    L.nf = std::min(hi + 1, n - 1) - L.f0 + 1;
    if (L.nf > 64) return "line rule: more than 64 nodes in P and its neighbours";
  }
  cheb_constants(L.p, L.nu, L.delta, L.omega, L.beta, L.beta_half);
  return "";
}

std::string gen_line_samples(uint64_t seed, int32_t sample_level, int64_t first, int32_t n,
                             const lts_line_sample_rule& rule, const LineHost& L, double* kappa,
                             int32_t* n_steps, double* dt) {
  if (n < 0 || first < 0 || sample_level < 0) return "n, first and sample_level must be >= 0";
  if (!(rule.T > 0.0) || !(rule.cfl > 0.0)) return "T and cfl must be > 0";
  if (rule.kind != LTS_LINE_KL && rule.kind != LTS_LINE_JUMP) return "unknown line sample kind";
  const int nc = (int)L.x.size() - 1;
  std::vector<double> mid(nc), u(2 * kLineKlTerms), xi1(kLineKlTerms), xi2(kLineKlTerms), kap(nc);
  for (int c = 0; c < nc; ++c) mid[c] = 0.5 * (L.x[c] + L.x[c + 1]);
  for (int s = 0; s < n; ++s) {
    const int64_t i = first + s;
    if (rule.kind == LTS_LINE_KL) {
      // c^2(x) = 1 + sum_k (1/(4 pi^2 k^2)) (cos(k pi x/6) xi1_k + sin(k pi x/6) xi2_k), xi ~ U(-1, 1)
      philox_uniforms(seed, i, sample_level, 0, 2 * kLineKlTerms, u.data());
      for (int k = 0; k < kLineKlTerms; ++k) {
        xi1[k] = 2.0 * u[2 * k] - 1.0;
        xi2[k] = 2.0 * u[2 * k + 1] - 1.0;
      }
      for (int c = 0; c < nc; ++c) {
        double c2 = 1.0;
        for (int k = 1; k <= kLineKlTerms; ++k) {
          const double a = ((double)k * M_PI) * mid[c] / 6.0;
          const double coef = 1.0 / (4.0 * M_PI * M_PI * (double)k * (double)k);
          c2 += coef * (std::cos(a) * xi1[k - 1] + std::sin(a) * xi2[k - 1]);
        }
        kap[c] = c2;
      }
    } else {
      // c = c_left left of xi and c_right from xi on, xi ~ U(jump_lo, jump_hi)
      double u0;
      philox_uniforms(seed, i, sample_level, 0, 1, &u0);
      const double xi = rule.jump_lo + (rule.jump_hi - rule.jump_lo) * u0;
      for (int c = 0; c < nc; ++c)
        kap[c] = mid[c] >= xi ? rule.c_right * rule.c_right : rule.c_left * rule.c_left;
    }
    double kmax = 0.0;
    for (int c = 0; c < nc; ++c) {
      if (!(kap[c] > 0.0) || !std::isfinite(kap[c])) return "wave speed must be positive";
      kmax = std::max(kmax, kap[c]);
    }
    const double ns = std::ceil((rule.T * std::sqrt(kmax)) / (rule.cfl * L.H));
    if (!(ns >= 1.0) || ns > 2.0e9) return "step count out of range";
    if (kappa) std::copy(kap.begin(), kap.end(), kappa + (size_t)s * nc);
    if (n_steps) n_steps[s] = (int32_t)ns;
    if (dt) dt[s] = rule.T / ns;
  }
  return "";
}

}  // namespace lts
