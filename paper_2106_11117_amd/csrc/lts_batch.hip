// Batched form: many (level, samples) jobs advanced by shared launches, with
// optional capture of the whole launch sequence into a HIP graph, and the
// autotuner that picks each level's fine-tile shape by measurement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "ctx.h"

namespace lts {

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ULL + (h << 6) + (h >> 2);
  return h;
}

uint64_t shape_key(const HostLevel& H) {
  uint64_t h = mix(mix(mix(0, (uint64_t)H.nxn), (uint64_t)H.nyn), (uint64_t)H.p);
  for (uint8_t f : H.flags) h = mix(h, f);
  return h;
}

struct TuneChoice {
  int TX, TY, ox, oy;
  bool rect, mix;
  double ms;
};

std::map<uint64_t, TuneChoice>& tune_cache() {
  static std::map<uint64_t, TuneChoice> m;
  return m;
}

}  // namespace

// Time candidate tilings of `lv` on synthetic samples (unit coefficient,
// centred pulse, CFL step) and keep the fastest.  Candidates: every tile size
// of level_tile_candidates() with the grid origin at 0 and aligned to F+, in
// rect mode where it fits and in compact mode; the six best-ranked of each mode
// by region overhead (12 in all).
lts_status autotune_level(lts_ctx c, DevLevel& lv) {
  if (lv.H.n_F == 0) {                       // no fine tiles (e.g. a leapfrog twin): nothing to tune
    lts_status r = default_tiling(c, lv);
    if (r != LTS_OK) return r;
    lv.tuned = true;
    lv.tuned_ms = 0.0;
    return LTS_OK;
  }
  const uint64_t key = shape_key(lv.H);
  auto hit = tune_cache().find(key);
  std::vector<TilingHost> cands;
  if (hit != tune_cache().end()) {
    TilingHost T;
    const TuneChoice& t = hit->second;
    if (build_tiling(lv.H, lv.ld, t.TX, t.TY, t.ox, t.oy, t.rect, T).empty()) {
      lts_status r = upload_tiling(c, T, lv.tiling);
      if (r != LTS_OK) return r;
      lv.tiling.mix = t.mix;
      lv.tuned = true;
      lv.tuned_ms = t.ms;
      return LTS_OK;
    }
  }
  std::vector<TilingHost> by_mode[2];
  for (int mode = 1; mode >= 0; --mode)
    for (auto& tc : level_tile_candidates(lv.H))
      for (auto& org : tile_origins(lv.H, tc.first, tc.second)) {
        TilingHost T;
        if (build_tiling(lv.H, lv.ld, tc.first, tc.second, org.first, org.second, mode == 1, T).empty())
          by_mode[mode].push_back(std::move(T));
      }
  // the best-ranked candidates of each mode, 12 in all
  for (int mode = 1; mode >= 0; --mode) {
    auto& v = by_mode[mode];
    std::sort(v.begin(), v.end(), [](const TilingHost& a, const TilingHost& b) {
      return a.halo_ratio * (1.0 + 0.01 * a.wg_per_sample) < b.halo_ratio * (1.0 + 0.01 * b.wg_per_sample);
    });
  }
  for (int k = 0; k < 12; ++k) {
    const int mode = k % 2 ? 0 : 1, idx = k / 2;
    if (idx < (int)by_mode[mode].size()) cands.push_back(std::move(by_mode[mode][idx]));
  }
  for (int mode = 1; mode >= 0 && cands.size() < 12; --mode)
    for (size_t idx = 6; idx < by_mode[mode].size() && cands.size() < 12; ++idx)
      cands.push_back(std::move(by_mode[mode][idx]));
  if (cands.empty()) {
    c->err = "no fine-tile size fits the workgroup capacity for this level";
    return LTS_ERR_ARG;
  }
  // synthetic batch that fills the device with every candidate (at least 1024
  // fine workgroups), within 1 GiB of states
  int min_wg = 1 << 30;
  for (const auto& T : cands) min_wg = std::min(min_wg, std::max(1, T.n_fine));
  const int s_mem = (int)std::max<size_t>(4, (size_t(1) << 30) / (16 * std::max<size_t>(lv.nodes, 1)));
  const int S = std::max(4, std::min({(1024 + min_wg - 1) / min_wg, s_mem, 4096}));
  const int nb = lv.H.n_blocks, p = lv.H.p;
  std::vector<double> kappa((size_t)S * nb, 1.0), x0((size_t)2 * S), coef((size_t)S * (p + 1));
  const double dt = 0.2 * lv.H.h;
  for (int s = 0; s < S; ++s) {
    x0[2 * s] = 0.5 * (lv.H.x.front() + lv.H.x.back());
    x0[2 * s + 1] = 0.5 * (lv.H.y.front() + lv.H.y.back());
    step_coefficients(lv.H, dt, &coef[(size_t)s * (p + 1)]);
  }
  LTS_HIP(c, hipSetDevice(c->device));
  LTS_HIP(c, c->kappa.ensure(kappa.size() * 8));
  LTS_HIP(c, c->coef.ensure(coef.size() * 8));
  LTS_HIP(c, c->x0.ensure(x0.size() * 8));
  LTS_HIP(c, hipMemcpyAsync(c->kappa.p, kappa.data(), kappa.size() * 8, hipMemcpyHostToDevice, c->stream));
  LTS_HIP(c, hipMemcpyAsync(c->coef.p, coef.data(), coef.size() * 8, hipMemcpyHostToDevice, c->stream));
  LTS_HIP(c, hipMemcpyAsync(c->x0.p, x0.data(), x0.size() * 8, hipMemcpyHostToDevice, c->stream));
  const size_t bytes = (size_t)S * lv.nodes * 8;
  LTS_HIP(c, c->st0.ensure(bytes));
  LTS_HIP(c, c->st1.ensure(bytes));
  double* B[2] = {c->st0.as<double>(), c->st1.as<double>()};
  hipEvent_t e0, e1;
  LTS_HIP(c, hipEventCreate(&e0));
  LTS_HIP(c, hipEventCreate(&e1));
  double best = 1e300;
  int bi = 0;
  bool best_mix = false;
  TilingDev Td;
  // each candidate with separate coarse and fine launches; the winner, if in
  // rect mode, also with both in one launch (k_step_mix)
  for (size_t ci = 0; ci <= cands.size(); ++ci) {
    const bool mix = ci == cands.size();
    if (mix && !cands[bi].rect) break;
    lts_status r = upload_tiling(c, cands[mix ? bi : ci], Td);
    if (r != LTS_OK) return r;
    Td.mix = mix;
    if ((r = init_states(c, lv, S, c->x0.as<double>(), 0.05, B[0], B[1])) != LTS_OK) return r;
    constexpr int kWarm = 2, kTimed = 6;
    for (int t = 0; t < kWarm + kTimed; ++t) {
      if (t == kWarm) LTS_HIP(c, hipEventRecord(e0, c->stream));
      r = launch_step(c, lv, Td, c->kappa.as<double>(), c->coef.as<double>(), B[t & 1], B[(t + 1) & 1],
                      lv.nodes, 0, S, t == 0, c->stream);
      if (r != LTS_OK) return r;
    }
    LTS_HIP(c, hipEventRecord(e1, c->stream));
    LTS_HIP(c, hipEventSynchronize(e1));
    float ms = 0;
    LTS_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      if (mix) best_mix = true;
      else bi = (int)ci;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LTS_HIP(c, hipStreamSynchronize(c->stream));
  const TilingHost& W = cands[bi];
  lts_status r = upload_tiling(c, W, lv.tiling);
  if (r != LTS_OK) return r;
  lv.tiling.mix = best_mix;
  lv.tuned = true;
  lv.tuned_ms = best / 6.0 / S;
  tune_cache()[key] = TuneChoice{W.TX, W.TY, W.ox, W.oy, W.rect, best_mix, lv.tuned_ms};
  return LTS_OK;
}

}  // namespace lts

using namespace lts;

extern "C" lts_status lts_autotune(lts_ctx c, int32_t level) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (level < 0 || level >= (int32_t)c->levels.size()) return arg_fail(c, "no such level");
  c->levels[level]->pinned = false;
  return autotune_level(c, *c->levels[level]);
}

extern "C" lts_status lts_set_tiling(lts_ctx c, int32_t level, int32_t tile_x, int32_t tile_y, int32_t rect) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (level < 0 || level >= (int32_t)c->levels.size()) return arg_fail(c, "no such level");
  const bool adaptive = tile_x == 0 && tile_y == 0 && rect == 0;
  if (!adaptive && (tile_x < 1 || tile_y < 1 || tile_x > 4096 || tile_y > 4096))
    return arg_fail(c, "tile size out of range");
  if (rect < 0 || rect > 2) return arg_fail(c, "rect must be 0, 1 or 2");
  DevLevel& lv = *c->levels[level];
  TilingHost best;
  bool have = false;
  std::string why;
  for (auto& org : tile_origins(lv.H, tile_x, tile_y)) {
    TilingHost T;
    std::string e = build_tiling(lv.H, lv.ld, tile_x, tile_y, org.first, org.second, rect >= 1, T);
    if (!e.empty()) {
      why = e;
      continue;
    }
    if (!have || T.halo_ratio * T.n_fine < best.halo_ratio * best.n_fine) {
      best = std::move(T);
      have = true;
    }
  }
  if (!have) return arg_fail(c, "tiling does not fit: " + why);
  LTS_HIP(c, hipSetDevice(c->device));
  lts_status r = upload_tiling(c, best, lv.tiling);
  if (r != LTS_OK) return r;
  lv.tiling.mix = rect == 2;
  lv.tuned = false;
  lv.pinned = true;
  lv.tuned_ms = 0.0;
  return LTS_OK;
}

extern "C" lts_status lts_batch_run(lts_ctx c, const lts_job* jobs, int32_t n_jobs, int32_t flags,
                                    double* Q_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (!jobs || n_jobs < 1 || n_jobs > kMaxJobs) return arg_fail(c, "n_jobs must be in 1..32");
  if (flags &
      ~(LTS_BATCH_GRAPH | LTS_BATCH_FP32 | LTS_BATCH_PERSIST | LTS_BATCH_SB_MASK | LTS_BATCH_AUTO | LTS_BATCH_MLTS))
    return arg_fail(c, "unknown flags");
  const bool mlts = (flags & LTS_BATCH_MLTS) != 0;
  if (mlts && (flags & (LTS_BATCH_PERSIST | LTS_BATCH_SB_MASK | LTS_BATCH_AUTO)))
    return arg_fail(c, "LTS_BATCH_MLTS excludes the persistent and automatic forms");
  const bool autof = (flags & LTS_BATCH_AUTO) != 0;
  if (autof && (flags & (LTS_BATCH_GRAPH | LTS_BATCH_PERSIST | LTS_BATCH_SB_MASK)))
    return arg_fail(c, "LTS_BATCH_AUTO excludes the other form flags");
  bool persist = (flags & LTS_BATCH_PERSIST) != 0;
  bool graph = (flags & LTS_BATCH_GRAPH) != 0;
  if (persist && graph) return arg_fail(c, "LTS_BATCH_PERSIST and LTS_BATCH_GRAPH exclude each other");
  const int sb_code = (flags & LTS_BATCH_SB_MASK) / LTS_BATCH_SB1;   // 0: largest S_b that fits
  if (sb_code == 3 || (sb_code && !persist)) return arg_fail(c, "bad S_b cap");
  int sb_cap = sb_code == 0 ? 4 : sb_code == 1 ? 1 : 2;
  const bool fp32 = (flags & LTS_BATCH_FP32) != 0;
  const size_t es = fp32 ? sizeof(float) : sizeof(double);   // bytes per state value
  const int kind = jobs[0].samples.ptr_kind;
  int total = 0;
  for (int j = 0; j < n_jobs; ++j) {
    if (jobs[j].level < 0 || jobs[j].level >= (int32_t)c->levels.size()) return arg_fail(c, "bad level id");
    if (jobs[j].samples.ptr_kind != kind) return arg_fail(c, "all jobs must use the same ptr_kind");
    if (jobs[j].q_offset < 0) return arg_fail(c, "q_offset must be >= 0");
    if (mlts && !c->levels[jobs[j].level]->mlts) {
      c->err = "a job's level has no tiers attached (lts_set_mlts)";
      return LTS_ERR_STATE;
    }
    total = std::max(total, jobs[j].q_offset + std::max(jobs[j].samples.n, 0));
  }
  if (total > 0 && !Q_out) return arg_fail(c, "Q_out is NULL");
  std::vector<Staged> st(n_jobs);
  lts_status r;
  for (int j = 0; j < n_jobs; ++j)
    if ((r = stage_samples(c, *c->levels[jobs[j].level], &jobs[j].samples, st[j])) != LTS_OK) return r;
  LTS_HIP(c, hipSetDevice(c->device));
  for (int j = 0; j < n_jobs; ++j) {
    DevLevel& lv = *c->levels[jobs[j].level];
    if (!mlts && !lv.tuned && !lv.pinned && (r = autotune_level(c, lv)) != LTS_OK) return r;
  }
  // device layout: per-job tables, states, Q
  std::vector<size_t> o_k(n_jobs), o_c(n_jobs), o_n(n_jobs), o_x(n_jobs), o_p(n_jobs), o_s(n_jobs), o_q(n_jobs),
      o_c0(n_jobs);
  size_t tab = 256, sts = 0, qb = 0;                   // the first 256 bytes: the staging flag
  for (int j = 0; j < n_jobs; ++j) {
    const DevLevel& lv = *c->levels[jobs[j].level];
    const size_t n = (size_t)st[j].n;
    o_k[j] = tab; tab += align256(n * lv.H.n_blocks * 8);
    o_c[j] = tab; tab += align256(n * (lv.H.p + 1) * 8);
    o_n[j] = tab; tab += align256(n * 4);
    o_x[j] = tab; tab += align256(n * 16);
    o_p[j] = tab; tab += align256(n * 4);
    o_c0[j] = tab; tab += mlts ? align256(n * 8) : 0;
    o_s[j] = sts; sts += align256(n * lv.nodes * es) * 2;
    o_q[j] = qb; qb += align256(n * 8);
  }
  LTS_HIP(c, c->b_tab.ensure(std::max<size_t>(tab, 256)));
  LTS_HIP(c, c->b_states.ensure(std::max<size_t>(sts, 256)));
  LTS_HIP(c, c->b_Q.ensure(std::max<size_t>(qb, 256)));
  LTS_HIP(c, c->b_jobs.ensure(step_args_size() * n_jobs));
  if (mlts) LTS_HIP(c, c->b_mjobs.ensure(mlts_record_size() * n_jobs));
  char* tb = c->b_tab.as<char>();
  char* sb = c->b_states.as<char>();
  char* qbp = c->b_Q.as<char>();
  auto staged_dev = [&](int j) {
    return StagedDev{(double*)(tb + o_k[j]), (double*)(tb + o_x[j]), (double*)(tb + o_c[j]), (int*)(tb + o_n[j]),
                     (int*)(tb + o_p[j]), (int*)tb};
  };
  std::vector<char> recs(step_args_size() * n_jobs), mrecs(mlts ? mlts_record_size() * n_jobs : 0);
  std::vector<std::vector<double>> c0h(n_jobs);
  std::vector<const TilingDev*> T(n_jobs);
  std::vector<const MltsDev*> Mv(mlts ? n_jobs : 0);
  int maxT = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const DevLevel& lv = *c->levels[jobs[j].level];
    const Staged& S = st[j];
    if (S.n > 0) {
      if ((r = upload_staged(c, lv, S, &jobs[j].samples, staged_dev(j))) != LTS_OK) return r;
      maxT = std::max(maxT, S.nsteps[0]);
    }
    double* B0 = (double*)(sb + o_s[j]);
    double* B1 = (double*)(sb + o_s[j] + align256((size_t)S.n * lv.nodes * es));
    job_record(lv, lv.tiling, (const double*)(tb + o_k[j]), (const double*)(tb + o_c[j]), B0, B1, lv.nodes,
               recs.data() + j * step_args_size());
    T[j] = &lv.tiling;
    if (mlts) {
      Mv[j] = lv.mlts.get();
      c0h[j].resize(S.n);
      mlts_c0(*lv.mlts, S.dt.data(), S.n, c0h[j].data());
      if (S.n > 0)
        LTS_HIP(c, hipMemcpyAsync(tb + o_c0[j], c0h[j].data(), (size_t)S.n * 8, hipMemcpyHostToDevice, c->stream));
      mlts_record(lv, (const double*)(tb + o_k[j]), (const double*)(tb + o_c0[j]), B0, B1,
                  mrecs.data() + j * mlts_record_size());
    }
  }
  LTS_HIP(c, hipMemcpyAsync(c->b_jobs.p, recs.data(), recs.size(), hipMemcpyHostToDevice, c->stream));
  if (mlts) LTS_HIP(c, hipMemcpyAsync(c->b_mjobs.p, mrecs.data(), mrecs.size(), hipMemcpyHostToDevice, c->stream));
  LTS_HIP(c, hipStreamSynchronize(c->stream));   // host staging buffers may be released after this

  // active samples of every job at every step (samples sorted by decreasing n_steps)
  std::vector<int> act_tab((size_t)maxT * n_jobs);
  {
    std::vector<int> act(n_jobs);
    for (int j = 0; j < n_jobs; ++j) act[j] = st[j].n;
    for (int t = 0; t < maxT; ++t)
      for (int j = 0; j < n_jobs; ++j) {
        while (act[j] > 0 && st[j].nsteps[act[j] - 1] <= t) --act[j];
        act_tab[(size_t)t * n_jobs + j] = act[j];
      }
  }
  // S_b of every job under a cap (0 for rect mode)
  auto sb_for = [&](int cap) {
    std::vector<int> v(n_jobs, 0);
    for (int j = 0; j < n_jobs; ++j)
      if (!T[j]->rect) v[j] = std::max(1, std::min(persist_sb_max(*T[j]), cap));
    return v;
  };
  if (persist || autof) {
    LTS_HIP(c, c->b_act.ensure(std::max<size_t>(act_tab.size() * sizeof(int), 256)));
    if (!act_tab.empty())
      LTS_HIP(c, hipMemcpyAsync(c->b_act.p, act_tab.data(), act_tab.size() * sizeof(int), hipMemcpyHostToDevice,
                                c->stream));
  }

  // steps 0 .. n_t-1 of every job (from the initial states), then the QoIs
  auto record_n = [&](int n_t, bool with_qoi, bool use_persist, const std::vector<int>& sbv) -> lts_status {
    lts_status rr;
    for (int j = 0; j < n_jobs; ++j) {
      const DevLevel& lv = *c->levels[jobs[j].level];
      if (st[j].n == 0) continue;
      double* B0 = (double*)(sb + o_s[j]);
      double* B1 = (double*)(sb + o_s[j] + align256((size_t)st[j].n * lv.nodes * es));
      if ((rr = init_states(c, lv, st[j].n, (const double*)(tb + o_x[j]), jobs[j].samples.width, B0, B1, fp32)) !=
          LTS_OK)
        return rr;
    }
    if (use_persist) {
      if ((rr = launch_persist(c, (const StepArgs*)c->b_jobs.p, T, act_tab, c->b_act.as<int>(), n_t, sbv, c->stream,
                               fp32)) != LTS_OK)
        return rr;
    } else {
      std::vector<int> act(n_jobs);
      for (int t = 0; t < n_t; ++t) {
        for (int j = 0; j < n_jobs; ++j) act[j] = act_tab[(size_t)t * n_jobs + j];
        if ((rr = launch_multi_step(c, (const StepArgs*)c->b_jobs.p, T, act, t, c->stream, fp32, mlts ? 1 : 5)) !=
            LTS_OK)
          return rr;
        if (mlts && (rr = launch_mlts(c, c->b_mjobs.p, Mv, act, t, c->stream, fp32)) != LTS_OK) return rr;
      }
    }
    for (int j = 0; j < n_jobs && with_qoi; ++j) {
      const DevLevel& lv = *c->levels[jobs[j].level];
      if (st[j].n == 0) continue;
      double* B0 = (double*)(sb + o_s[j]);
      double* B1 = (double*)(sb + o_s[j] + align256((size_t)st[j].n * lv.nodes * es));
      if ((rr = qoi_device(c, lv, st[j].n, (const int*)(tb + o_n[j]), B0, B1, (double*)(qbp + o_q[j]), fp32)) !=
          LTS_OK)
        return rr;
    }
    return LTS_OK;
  };

  if (autof && maxT > 0) {
    // the form of this job-list shape: cached, or timed on its first steps
    std::vector<uint64_t> key = {(uint64_t)n_jobs, (uint64_t)fp32};
    for (int j = 0; j < n_jobs; ++j) {
      key.push_back(c->levels[jobs[j].level]->tiling.gen);
      key.push_back((uint64_t)st[j].n);
    }
    auto hit = c->batch_forms.find(key);
    if (hit != c->batch_forms.end()) {
      graph = hit->second.first == 1;
      persist = hit->second.first == 2;
      sb_cap = hit->second.second;
    } else {
      int sbm = 0;
      for (int j = 0; j < n_jobs; ++j)
        if (!T[j]->rect && T[j]->n_fine > 0) sbm = std::max(sbm, persist_sb_max(*T[j]));
      std::vector<std::pair<int, int>> cand = {{1, 0}, {2, 4}};
      if (sbm >= 4) cand.push_back({2, 2});
      if (sbm >= 2) cand.push_back({2, 1});
      const int K = std::min(maxT, 48);
      hipEvent_t a0, a1;
      LTS_HIP(c, hipEventCreate(&a0));
      LTS_HIP(c, hipEventCreate(&a1));
      double best = 1e300;
      std::pair<int, int> win = cand[0];
      lts_status rr = LTS_OK;
      for (const auto& f : cand) {
        hipGraphExec_t ge = nullptr;
        if (f.first == 1) {
          hipGraph_t g;
          LTS_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
          rr = record_n(K, false, false, {});
          hipError_t ec = hipStreamEndCapture(c->stream, &g);
          if (rr != LTS_OK) break;
          if (ec != hipSuccess) return hip_fail(c, ec, "hipStreamEndCapture");
          ec = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          if (ec != hipSuccess) return hip_fail(c, ec, "hipGraphInstantiate");
        }
        float ms = 0.f;
        for (int rep = 0; rep < 2 && rr == LTS_OK; ++rep) {   // the second run is timed
          LTS_HIP(c, hipEventRecord(a0, c->stream));
          if (ge) {
            hipError_t ec = hipGraphLaunch(ge, c->stream);
            if (ec != hipSuccess) {
              (void)hipGraphExecDestroy(ge);
              return hip_fail(c, ec, "hipGraphLaunch");
            }
          } else {
            rr = record_n(K, false, true, sb_for(f.second));
          }
          LTS_HIP(c, hipEventRecord(a1, c->stream));
          LTS_HIP(c, hipEventSynchronize(a1));
          LTS_HIP(c, hipEventElapsedTime(&ms, a0, a1));
        }
        if (ge) (void)hipGraphExecDestroy(ge);
        if (rr != LTS_OK) break;
        if (ms < best) {
          best = ms;
          win = f;
        }
      }
      (void)hipEventDestroy(a0);
      (void)hipEventDestroy(a1);
      if (rr != LTS_OK) return rr;
      c->batch_forms[key] = win;
      graph = win.first == 1;
      persist = win.first == 2;
      sb_cap = win.second;
    }
  }
  auto record = [&]() { return record_n(maxT, true, persist, sb_for(sb_cap)); };

  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    while (c->ev_pool.size() < 4) {
      hipEvent_t e;
      LTS_HIP(c, hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
    e0 = c->ev_pool[0];
    e1 = c->ev_pool[1];
    LTS_HIP(c, hipEventRecord(e0, c->stream));
  }
  if (graph) {
    // key: job shapes, step counts and every device address baked into the graph
    std::vector<uint64_t> key = {(uint64_t)n_jobs, (uint64_t)fp32, (uint64_t)(uintptr_t)tb, (uint64_t)(uintptr_t)sb,
                                 (uint64_t)(uintptr_t)qbp, (uint64_t)(uintptr_t)c->b_jobs.p, (uint64_t)mlts,
                                 (uint64_t)(uintptr_t)(mlts ? c->b_mjobs.p : nullptr)};
    for (int j = 0; j < n_jobs; ++j) {
      key.push_back((uint64_t)jobs[j].level);
      key.push_back(c->levels[jobs[j].level]->tiling.gen);
      key.push_back(mlts ? c->levels[jobs[j].level]->mlts->tiling.gen : 0);
      key.push_back((uint64_t)st[j].n);
      key.push_back((uint64_t)(std::llround(jobs[j].samples.width * 1e15)));
      for (int v : st[j].nsteps) key.push_back((uint64_t)v);
    }
    if (!c->graph || key != c->graph_key) {
      if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
      }
      hipGraph_t g;
      LTS_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      r = record();
      hipError_t ec = hipStreamEndCapture(c->stream, &g);
      if (r != LTS_OK) return r;
      if (ec != hipSuccess) return hip_fail(c, ec, "hipStreamEndCapture");
      ec = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ec != hipSuccess) return hip_fail(c, ec, "hipGraphInstantiate");
      c->graph_key = key;
    }
    LTS_HIP(c, hipGraphLaunch(c->graph, c->stream));
  } else {
    if ((r = record()) != LTS_OK) return r;
  }
  LTS_HIP(c, hipGetLastError());
  c->last = lts_timing{};
  if (c->timing) {
    LTS_HIP(c, hipEventRecord(e1, c->stream));
    LTS_HIP(c, hipEventSynchronize(e1));
    float ms = 0;
    LTS_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    c->last.total_ms = ms;
    c->last.step_kernel_ms = ms;
    c->last.step_launches = maxT;
  }
  c->last.batch_form = persist ? 2 : graph ? 1 : 0;
  c->last.batch_sb_cap = persist ? sb_cap : 0;
  for (int j = 0; j < n_jobs; ++j) {
    const DevLevel& lv = *c->levels[jobs[j].level];
    const double per_step =
        mlts ? lv.mlts->updates : (double)(lv.H.n_dof - lv.H.n_P) + (double)lv.H.p * lv.H.n_P;
    for (int v : st[j].nsteps) {
      c->last.dof_updates += (double)v * per_step;
      c->last.alg_bytes += (double)v * 24.0 * lv.H.n_dof;
    }
  }
  // results: per job in sorted order -> caller order at q_offset (only the
  // ranges the jobs own are written)
  bool bad = false;
  for (int j = 0; j < n_jobs; ++j) {
    if (st[j].n == 0) continue;
    r = finish_Q(c, st[j], (const double*)(qbp + o_q[j]), staged_dev(j), Q_out + jobs[j].q_offset);
    if (r == LTS_ERR_UNSTABLE) bad = true;
    else if (r != LTS_OK) return r;
  }
  if (bad) {
    c->err = "non-finite QoI (unstable sample)";
    return LTS_ERR_UNSTABLE;
  }
  return LTS_OK;
}
