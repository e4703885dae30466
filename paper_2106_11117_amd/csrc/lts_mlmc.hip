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

// New samples of one level: indices first..first+n-1 of MLMC level l, drawn
// once and solved on mesh l (fine) and mesh l-1 (coarse).
struct LevelBatch {
  int l = 0, n = 0;
  std::vector<double> kappa, x0, dtf, dtc, qf, qc;
  std::vector<int32_t> nsf, nsc;
};

// The host header of level l of the hierarchy (grid level or triangle mesh):
// block count, spacing h, p and the sizes the cost model reads.
const HostLevel& level_header(lts_ctx c, const lts_mlmc_opts& o, int l) {
  if (o.level_kind == LTS_LEVELS_MESH) return c->meshes[o.level_ids[l]]->H.shell;
  return c->levels[o.level_ids[l]]->H;
}

lts_status draw_level(lts_ctx c, const lts_mlmc_opts& o, int l, int64_t first, int n, LevelBatch& b) {
  b.l = l;
  b.n = n;
  const HostLevel& fine = level_header(c, o, l);
  const int nb = o.rule.n_blocks;
  if (fine.n_blocks != nb) {
    c->err = "rule.n_blocks differs from the level's block count";
    return LTS_ERR_ARG;
  }
  b.kappa.resize((size_t)n * nb);
  b.x0.resize((size_t)n * 2);
  b.dtf.resize(n);
  b.dtc.resize(n);
  b.nsf.resize(n);
  b.nsc.resize(n);
  b.qf.assign(n, 0.0);
  b.qc.assign(n, 0.0);
  std::string e = gen_samples(o.seed, l, first, n, o.rule, fine.h, nullptr, b.kappa.data(), b.x0.data(),
                              b.nsf.data(), b.dtf.data());
  if (e.empty() && l > 0)
    e = gen_samples(o.seed, l, first, n, o.rule, level_header(c, o, l - 1).h, nullptr, nullptr, nullptr,
                    b.nsc.data(), b.dtc.data());
  if (!e.empty()) {
    c->err = e;
    return LTS_ERR_ARG;
  }
  return LTS_OK;
}

// Solve the batches: plain form = one solve call per level and mesh with one
// launch per sample and step (multi-level LTS: one solve per level and mesh);
// batched form = every fine and coarse job of every level in one
// graph-captured lts_batch_run.
lts_status solve_batches(lts_ctx c, const lts_mlmc_opts& o, std::vector<LevelBatch>& bs) {
  lts_status r;
  const bool tiers = o.level_kind == LTS_LEVELS_MLTS;
  if (o.level_kind == LTS_LEVELS_MESH || (tiers && o.mode == LTS_MLMC_PLAIN)) {
    // triangle meshes, and the plain form of multi-level LTS: one solve per
    // level and mesh
    const bool mesh = o.level_kind == LTS_LEVELS_MESH;
    auto solve = [&](int32_t id, const lts_samples* S, double* q) {
      return mesh ? lts_mesh_forward(c, id, S, LTS_FP64, q) : lts_mlts_forward(c, id, S, LTS_FP64, q);
    };
    for (auto& b : bs) {
      if (b.n == 0) continue;
      lts_samples sf{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsf.data(), b.dtf.data(), o.rule.width};
      if ((r = solve(o.level_ids[b.l], &sf, b.qf.data())) != LTS_OK) return r;
      if (b.l > 0) {
        lts_samples sc{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsc.data(), b.dtc.data(), o.rule.width};
        if ((r = solve(o.level_ids[b.l - 1], &sc, b.qc.data())) != LTS_OK) return r;
      }
    }
    return LTS_OK;
  }
  if (o.mode == LTS_MLMC_PLAIN) {
    for (auto& b : bs) {
      if (b.n == 0) continue;
      lts_samples sf{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsf.data(), b.dtf.data(), o.rule.width};
      if ((r = lts_forward_plain(c, o.level_ids[b.l], &sf, LTS_FP64, b.qf.data())) != LTS_OK) return r;
      if (b.l > 0) {
        lts_samples sc{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsc.data(), b.dtc.data(), o.rule.width};
        if ((r = lts_forward_plain(c, o.level_ids[b.l - 1], &sc, LTS_FP64, b.qc.data())) != LTS_OK) return r;
      }
    }
    return LTS_OK;
  }
  std::vector<lts_job> jobs;
  int off = 0;
  for (auto& b : bs) {
    if (b.n == 0) continue;
    jobs.push_back(lts_job{o.level_ids[b.l],
                           lts_samples{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsf.data(), b.dtf.data(),
                                       o.rule.width},
                           off});
    off += b.n;
    if (b.l > 0) {
      jobs.push_back(lts_job{o.level_ids[b.l - 1],
                             lts_samples{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsc.data(),
                                         b.dtc.data(), o.rule.width},
                             off});
      off += b.n;
    }
  }
  if (jobs.empty()) return LTS_OK;
  std::vector<double> q(off);
  const int32_t flags = LTS_BATCH_GRAPH | (tiers ? LTS_BATCH_MLTS : 0);
  if ((r = lts_batch_run(c, jobs.data(), (int32_t)jobs.size(), flags, q.data())) != LTS_OK) return r;
  off = 0;
  for (auto& b : bs) {
    if (b.n == 0) continue;
    std::copy(q.begin() + off, q.begin() + off + b.n, b.qf.begin());
    off += b.n;
    if (b.l > 0) {
      std::copy(q.begin() + off, q.begin() + off + b.n, b.qc.begin());
      off += b.n;
    }
  }
  return LTS_OK;
}

// Gradient form: the new samples of each level solved by the backward LF-LTS
// on the fine and the coarse mesh (dL/dQ = 1), which returns each QoI (equal
// bit for bit to the forward solve's) and dQ/dg; the rows of dG_l = dQ_l/dg -
// dQ_l-1/dg are appended to dg[l].
lts_status solve_batches_grad(lts_ctx c, const lts_mlmc_opts& o, std::vector<LevelBatch>& bs, int K,
                              std::vector<std::vector<double>>& dg) {
  lts_status r;
  const int nb = o.rule.n_blocks;
  for (auto& b : bs) {
    if (b.n == 0) continue;
    std::vector<double> ones(b.n, 1.0), gf((size_t)b.n * nb), gc((size_t)b.n * nb, 0.0);
    lts_samples sf{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsf.data(), b.dtf.data(), o.rule.width};
    if ((r = lts_backward(c, o.level_ids[b.l], &sf, ones.data(), K, b.qf.data(), gf.data())) != LTS_OK) return r;
    if (b.l > 0) {
      lts_samples sc{b.n, LTS_PTR_HOST, b.kappa.data(), b.x0.data(), b.nsc.data(), b.dtc.data(), o.rule.width};
      if ((r = lts_backward(c, o.level_ids[b.l - 1], &sc, ones.data(), K, b.qc.data(), gc.data())) != LTS_OK)
        return r;
    }
    for (size_t k = 0; k < gf.size(); ++k) dg[b.l].push_back(gf[k] - gc[k]);
  }
  return LTS_OK;
}

// Algorithm 1 (see lts_mlmc); with dg != nullptr every sample is solved by the
// backward form and the gradient differences are collected per level.
lts_status mlmc_run(lts_ctx c, const lts_mlmc_opts* op, lts_mlmc_result* out, int K,
                    std::vector<std::vector<double>>* dg) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!op || !out) return arg_fail(c, "NULL argument");
  lts_mlmc_opts o = *op;                    // level_ids grows with generated levels
  const int n_total = std::max(o.n_levels, o.n_levels_max);
  if (o.n_levels < 0 || n_total < 1 || n_total > LTS_MAX_LEVELS) return arg_fail(c, "n_levels out of range");
  if (o.level_kind != LTS_LEVELS_GRID && o.level_kind != LTS_LEVELS_MESH && o.level_kind != LTS_LEVELS_MLTS)
    return arg_fail(c, "bad level_kind");
  const bool meshes = o.level_kind == LTS_LEVELS_MESH, tiers = o.level_kind == LTS_LEVELS_MLTS;
  if (meshes && (n_total > o.n_levels || dg))
    return arg_fail(c, "triangle-mesh hierarchies are given in full and have no gradient form");
  if (tiers && dg) return arg_fail(c, "multi-level LTS has no gradient form");
  if (tiers && n_total > o.n_levels && o.gen_mlts.cell_tier)
    return arg_fail(c, "gen_mlts of generated levels must use the halving rule (cell_tier NULL)");
  for (int l = 0; l < o.n_levels; ++l) {
    if (o.level_ids[l] < 0 || o.level_ids[l] >= (int)(meshes ? c->meshes.size() : c->levels.size()))
      return arg_fail(c, "bad level id");
    if (tiers && !c->levels[o.level_ids[l]]->mlts) return arg_fail(c, "a level has no tiers attached (lts_set_mlts)");
  }
  for (int l = 0; l < n_total; ++l)
    if (o.N_init[l] < 2) return arg_fail(c, "N_init must be >= 2 (variance estimates)");
  if (!(o.eps > 0.0) || !(o.alpha > 0.0)) return arg_fail(c, "eps and alpha must be > 0");
  if (n_total > o.n_levels) {
    // the generated levels must be valid rules (checked on the host, no device work)
    for (int l = o.n_levels; l < n_total; ++l) {
      lts_rect_rule g = o.gen_rule;
      g.n_base = o.gen_rule.n_base << l;
      lts_level_info info;
      if (lts_rect_level_host(&g, &info, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != LTS_OK)
        return arg_fail(c, "gen_rule does not build level " + std::to_string(l));
      lts_mlts_info mi;
      if (tiers && lts_mlts_host(&g, &o.gen_mlts, &mi, nullptr) != LTS_OK)
        return arg_fail(c, "gen_mlts does not fit generated level " + std::to_string(l));
    }
  }
  const int Lmax = n_total - 1;
  auto t0 = std::chrono::steady_clock::now();
  // level l exists in the context (built from gen_rule on first use)
  auto ensure_level = [&](int l) -> lts_status {
    if (l < o.n_levels) return LTS_OK;
    lts_rect_rule g = o.gen_rule;
    g.n_base = o.gen_rule.n_base << l;
    int32_t id = -1;
    lts_status rr = lts_build_rect_level(c, &g, &id);
    if (rr != LTS_OK) return rr;
    if (tiers && (rr = lts_set_mlts(c, id, &o.gen_mlts)) != LTS_OK) return rr;
    o.level_ids[l] = id;
    o.n_levels = l + 1;
    return LTS_OK;
  };
  int L = std::min(std::max(o.L_start, 0), Lmax);
  lts_status r;
  for (int l = 0; l <= L; ++l)
    if ((r = ensure_level(l)) != LTS_OK) return r;
  // cost model C_l in DOF updates per Delta Q_l sample, formed as levels are added
  std::vector<double> cs(n_total, 0.0), C(n_total, 0.0);
  auto add_cost = [&](int l) {
    const HostLevel& H = level_header(c, o, l);
    cs[l] = tiers ? std::ceil(o.rule.T / (o.rule.cfl * H.h)) * c->levels[o.level_ids[l]]->mlts->updates
                  : solve_cost_model(H, o.rule);
    C[l] = l == 0 ? cs[0] : cs[l] + cs[l - 1];
  };
  for (int l = 0; l <= L; ++l) add_cost(l);
  std::vector<int64_t> N(n_total, 0);
  for (int l = 0; l <= L; ++l) N[l] = o.N_init[l];
  std::vector<std::vector<double>> dq(n_total);
  std::vector<double> mean(n_total, 0.0), var(n_total, 0.0);
  bool grew = true;
  while (grew) {
    int64_t total = 0;
    for (int l = 0; l <= L; ++l) total += N[l];
    if (o.max_total_samples > 0 && total > o.max_total_samples) {
      c->err = "sample budget exceeded before convergence";
      return LTS_ERR_STATE;
    }
    std::vector<LevelBatch> bs(L + 1);
    for (int l = 0; l <= L; ++l) {
      const int64_t have = (int64_t)dq[l].size();
      if ((r = draw_level(c, o, l, have, (int)(N[l] - have), bs[l])) != LTS_OK) return r;
    }
    if (dg) {
      if ((r = solve_batches_grad(c, o, bs, K, *dg)) != LTS_OK) return r;
    } else if ((r = solve_batches(c, o, bs)) != LTS_OK) {
      return r;
    }
    for (int l = 0; l <= L; ++l)
      for (int s = 0; s < bs[l].n; ++s) dq[l].push_back(bs[l].qf[s] - bs[l].qc[s]);
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
      if ((r = ensure_level(L)) != LTS_OK) return r;
      add_cost(L);
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
    out->level_ids[l] = o.level_ids[l];
  }
  const double bias = std::fabs(mean[L]) / (std::pow(2.0, o.alpha) - 1.0);
  out->estimate = est;
  out->L = L;
  out->bias = bias;
  out->rmse = std::sqrt(vsum + bias * bias);
  out->converged = bias * bias < 0.5 * o.eps * o.eps;
  out->seconds = secs;
  if (dg) dg->resize(L + 1);
  return LTS_OK;
}

}  // namespace

extern "C" lts_status lts_mlmc(lts_ctx c, const lts_mlmc_opts* op, lts_mlmc_result* out) {
  return mlmc_run(c, op, out, 0, nullptr);
}

extern "C" lts_status lts_mlmc_grad(lts_ctx c, const lts_mlmc_opts* op, int32_t K_ckpt, lts_mlmc_result* out,
                                    double* grad_estimate, double* grad_mean, double* grad_var) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!op || !out || !grad_estimate || !grad_mean || !grad_var) return arg_fail(c, "NULL argument");
  if (K_ckpt < 1 || K_ckpt > 4096) return arg_fail(c, "K_ckpt must be in 1..4096");
  const int nb = op->rule.n_blocks;
  if (nb < 2 || nb > 255) return arg_fail(c, "rule.n_blocks out of range");
  std::vector<std::vector<double>> dg(LTS_MAX_LEVELS);
  lts_status r = mlmc_run(c, op, out, K_ckpt, &dg);
  if (r != LTS_OK) return r;
  const int L = out->L;
  // per level and block: mean and unbiased variance of dG on the device
  size_t rows = 0;
  for (int l = 0; l <= L; ++l) rows = std::max(rows, dg[l].size() / nb);
  LTS_HIP(c, hipSetDevice(c->device));
  LTS_HIP(c, c->red.ensure(std::max<size_t>((rows * nb + 3 * (size_t)nb) * 8, 64)));
  double* dx = c->red.as<double>() + 3 * (size_t)nb;
  std::vector<double> m3(3 * (size_t)nb);
  for (int b = 0; b < nb; ++b) grad_estimate[b] = 0.0;
  for (int l = 0; l < LTS_MAX_LEVELS; ++l)
    for (int b = 0; b < nb; ++b) grad_mean[(size_t)l * nb + b] = grad_var[(size_t)l * nb + b] = 0.0;
  for (int l = 0; l <= L; ++l) {
    const int n = out->N[l];
    if ((size_t)n * nb > dg[l].size()) {
      c->err = "gradient rows missing";
      return LTS_ERR_STATE;
    }
    LTS_HIP(c, hipMemcpyAsync(dx, dg[l].data(), (size_t)n * nb * 8, hipMemcpyHostToDevice, c->stream));
    if ((r = moments_cols_device(c, dx, n, nb, c->red.as<double>())) != LTS_OK) return r;
    LTS_HIP(c, hipMemcpyAsync(m3.data(), c->red.p, m3.size() * 8, hipMemcpyDeviceToHost, c->stream));
    LTS_HIP(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nb; ++b) {
      grad_mean[(size_t)l * nb + b] = m3[3 * b + 1];
      grad_var[(size_t)l * nb + b] = n > 1 ? m3[3 * b + 2] / (double)(n - 1) : 0.0;
      grad_estimate[b] += m3[3 * b + 1];
    }
  }
  return LTS_OK;
}
