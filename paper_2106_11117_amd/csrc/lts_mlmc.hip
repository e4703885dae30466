// Multilevel Monte Carlo driver (Algorithm 1, Sec. 2.2) on top of the forward
// solves: per-level coupled differences Delta Q_l on common samples, device
// moment reduction, optimal sample sizes, bias test, adaptive L.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "ctx.h"

using namespace lts;

namespace {

// Solve `n` new samples (indices first..first+n-1 of MLMC level l) and append
// Delta Q_l = Q_l - Q_{l-1} to dq (Q_{-1} = 0).
lts_status level_samples(lts_ctx c, const lts_mlmc_opts& o, int l, int64_t first, int n,
                         std::vector<double>& dq) {
  if (n <= 0) return LTS_OK;
  const DevLevel& fine = *c->levels[o.level_ids[l]];
  const int nb = o.rule.n_blocks;
  if (fine.H.n_blocks != nb) {
    c->err = "rule.n_blocks differs from the level's block count";
    return LTS_ERR_ARG;
  }
  std::vector<double> kappa((size_t)n * nb), x0((size_t)n * 2), dtf(n), dtc(n), qf(n), qc(n, 0.0);
  std::vector<int32_t> nsf(n), nsc(n);
  std::string e = gen_samples(o.seed, l, first, n, o.rule, fine.H.h, nullptr, kappa.data(), x0.data(),
                              nsf.data(), dtf.data());
  if (!e.empty()) {
    c->err = e;
    return LTS_ERR_ARG;
  }
  lts_samples sf{n, LTS_PTR_HOST, kappa.data(), x0.data(), nsf.data(), dtf.data(), o.rule.width};
  auto solve = [&](int32_t lid, const lts_samples* S, double* q) -> lts_status {
    return o.mode == LTS_MLMC_PLAIN ? lts_forward_plain(c, lid, S, LTS_FP64, q)
                                    : lts_forward(c, lid, S, LTS_FP64, q);
  };
  lts_status r = solve(o.level_ids[l], &sf, qf.data());
  if (r != LTS_OK) return r;
  if (l > 0) {
    const DevLevel& coarse = *c->levels[o.level_ids[l - 1]];
    e = gen_samples(o.seed, l, first, n, o.rule, coarse.H.h, nullptr, nullptr, nullptr, nsc.data(), dtc.data());
    if (!e.empty()) {
      c->err = e;
      return LTS_ERR_ARG;
    }
    lts_samples sc{n, LTS_PTR_HOST, kappa.data(), x0.data(), nsc.data(), dtc.data(), o.rule.width};
    if ((r = solve(o.level_ids[l - 1], &sc, qc.data())) != LTS_OK) return r;
  }
  for (int s = 0; s < n; ++s) dq.push_back(qf[s] - qc[s]);
  return LTS_OK;
}

}  // namespace

extern "C" lts_status lts_mlmc(lts_ctx c, const lts_mlmc_opts* op, lts_mlmc_result* out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!op || !out) return arg_fail(c, "NULL argument");
  const lts_mlmc_opts& o = *op;
  if (o.n_levels < 1 || o.n_levels > LTS_MAX_LEVELS) return arg_fail(c, "n_levels out of range");
  for (int l = 0; l < o.n_levels; ++l) {
    if (o.level_ids[l] < 0 || o.level_ids[l] >= (int)c->levels.size()) return arg_fail(c, "bad level id");
    if (o.N_init[l] < 2) return arg_fail(c, "N_init must be >= 2 (variance estimates)");
  }
  if (!(o.eps > 0.0) || !(o.alpha > 0.0)) return arg_fail(c, "eps and alpha must be > 0");
  const int Lmax = o.n_levels - 1;
  int L = std::min(std::max(o.L_start, 0), Lmax);
  // cost model C_l in DOF updates per Delta Q_l sample
  std::vector<double> cs(o.n_levels), C(o.n_levels);
  for (int l = 0; l < o.n_levels; ++l) cs[l] = solve_cost_model(c->levels[o.level_ids[l]]->H, o.rule);
  for (int l = 0; l < o.n_levels; ++l) C[l] = l == 0 ? cs[0] : cs[l] + cs[l - 1];
  std::vector<int64_t> N(o.n_levels, 0);
  for (int l = 0; l <= L; ++l) N[l] = o.N_init[l];
  std::vector<std::vector<double>> dq(o.n_levels);
  std::vector<double> mean(o.n_levels, 0.0), var(o.n_levels, 0.0);
  auto t0 = std::chrono::steady_clock::now();
  bool grew = true;
  lts_status r;
  while (grew) {
    int64_t total = 0;
    for (int l = 0; l <= L; ++l) total += N[l];
    if (o.max_total_samples > 0 && total > o.max_total_samples) {
      c->err = "sample budget exceeded before convergence";
      return LTS_ERR_STATE;
    }
    for (int l = 0; l <= L; ++l) {
      const int64_t have = (int64_t)dq[l].size();
      if ((r = level_samples(c, o, l, have, (int)(N[l] - have), dq[l])) != LTS_OK) return r;
    }
    for (int l = 0; l <= L; ++l) {
      double m3[3];
      if ((r = lts_moments(c, dq[l].data(), (int32_t)N[l], LTS_PTR_HOST, m3)) != LTS_OK) return r;
      mean[l] = m3[1];
      var[l] = N[l] > 1 ? m3[2] / (double)(N[l] - 1) : 0.0;
    }
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
    const double bias = std::fabs(mean[L]) / (std::pow(2.0, o.alpha) - 1.0);
    if (bias * bias >= 0.5 * o.eps * o.eps && L < Lmax) {
      ++L;
      N[L] = o.N_init[L];
      grew = true;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = lts_mlmc_result{};
  double est = 0.0, vsum = 0.0;
  for (int l = 0; l <= L; ++l) {
    est += mean[l];
    vsum += var[l] / (double)N[l];
    out->N[l] = (int32_t)N[l];
    out->mean[l] = mean[l];
    out->var[l] = var[l];
    out->cost[l] = C[l];
  }
  const double bias = std::fabs(mean[L]) / (std::pow(2.0, o.alpha) - 1.0);
  out->estimate = est;
  out->L = L;
  out->bias = bias;
  out->rmse = std::sqrt(vsum + bias * bias);
  out->converged = bias * bias < 0.5 * o.eps * o.eps;
  out->seconds = secs;
  return LTS_OK;
}
