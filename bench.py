"""Benchmark: batched LF-LTS throughput on one MI355X.

Workload (the single-level batched throughput configuration): unit square,
512 base cells per axis, refined 8x in the coarse cells meeting (0.48, 0.52)
(442,225 DOFs, |P| = 204,081, p = 8, nu = 0.01), 256 samples of a 4x4 block
log-normal wave speed (sigma 0.25), Gaussian pulse (width 0.05, centre in
[0.2,0.4]^2), T = 1, dt = 0.2 h / max c per sample, FP64, QoI = lumped
integral over [0.6,0.8]^2.  Synthetic inputs from Philox seed 0.

One step = one pass of the whole hot path over the batch: the initial state,
every LF-LTS time step of every sample (coarse sweep + p local substeps), the
QoI and the per-level moment reduction.  Inputs (per-sample coefficients,
pulse centres, step counts) are resident in HBM before the timed region.

Prints one JSON line (see the repository's benchmark contract).  After the
timed throughput run the same line also carries, measured outside the timed
region, the rest of the metric on the graded L-shape hierarchy (5 levels,
p = 64, T = 2): Algorithm 1 at eps = 1e-4, batched + graph against the plain
one-launch-per-sample form at identical N_l ("mlmc_graded_L"), the batched
multi-level throughput with N_l = 4096, 1024, 256, 64, 16 ("batch_graded_L"),
and Algorithm 1 at eps = 1e-4 with multi-level LTS against single-tier LTS,
both batched + graph ("mlts_mlmc_graded_L").  --no-extra leaves them out.

Other modes (one JSON line each): --mlmc (Algorithm 1, batched + graph against
the plain form and the CPU oracle), --batch [--plain] (all five graded L-shape
levels in shared launches), --lf (LF-LTS against the standard leapfrog
baseline), --line (the one-dimensional workloads, LF-LTS against leapfrog),
--adjoint (discrete adjoint against the forward solve),
--stream-check and --copy-check (HBM reference rates and counter calibration).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_BASE, BOX, REF = 512, (0.48, 0.52), 8
N_SAMPLES = 256
HBM_PEAK_GBS = 8000.0
# HBM bytes per step launch (one k_coarse + one k_fine) from the FETCH_SIZE /
# WRITE_SIZE counter runs, scaled by a plain copy kernel
# (profiles/lts_step_kernels_C1_256samples_counters.md): counter bytes are 1.354x
# the algorithmic bytes on the profiled launches (all samples active), applied
# to the average launch's 1.7105e9 algorithmic bytes.  Valid only for the
# step-kernel sources the counters were taken with.
TRAFFIC = {"bytes_per_launch": 1.3540 * 1.7105e9,
           "sources_sha256": "12a494a876a68def51ec0258378ad6a3f88ded3a1d654705c27f852604a6bf0e"}
STEP_SOURCES = ("lts_fused.hip", "fused.h", "device.h", "lts_step.hip")
WORKLOAD = ("unit square 512x512 base refined 8x in (0.48,0.52): 442225 DOFs, |P|=204081, p=8, "
            "nu=0.01, 256 samples, 4x4 blocks sigma=0.25, T=1, FP64")


def step_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_11117_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _cpu_worker(args):
    """Oracle (test infrastructure) timing of `steps` coarse steps of one sample."""
    i, steps = args
    import numpy as np
    from oracle import fem, lts, mesh, rng
    lv = mesh.box_refined_level(N_BASE, box=BOX, ref=REF)
    ops = fem.operators(lv)
    rule = rng.SampleRule()
    smp = rng.draw(0, 0, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    s = lts.Solver(ops, smp.kappa)
    z0 = lts.pulse(ops, smp.x0)
    t0 = time.perf_counter()
    zm, zc = z0, s.q1(z0, dt)
    for _ in range(1, steps):
        zm, zc = zc, 2.0 * zc - zm + 2.0 * s.d1(zc, dt)
    el = time.perf_counter() - t0
    n_dof, n_p = ops.Pd.size, int(ops.Pd.sum())
    return steps * ((n_dof - n_p) + lv.p * n_p), el, bool(np.isfinite(zc).all())


def cpu_baseline(steps_per_sample: int = 150):
    import multiprocessing as mp
    procs = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_cpu_worker, [(i, steps_per_sample) for i in range(procs)])
    wall = time.perf_counter() - t0
    upd = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": upd / busy, "unit": "DOF-updates/s", "cores": procs, "kind": "oracle",
            "host_cpu": model, "host_cpu_count": os.cpu_count(),
            "sample": f"samples 0..{procs - 1} of the same workload, first {steps_per_sample} coarse "
                      f"steps each (one process per core, scipy CSR, FP64); wall {wall:.1f} s incl. setup"}


# MLMC workload: graded L-shape hierarchy, 5 levels, Algorithm 1 at fixed RMSE
MLMC_BASES = (32, 64, 128, 256, 512)      # cells across [-1, 1]: h = 1/16 .. 1/256
MLMC_EPS = (1e-3, 1e-4)                   # the workload's eps, and a tighter extra point
MLMC_N_INIT = (256, 64, 16, 8, 4)


def _mlmc_rule_oracle():
    from oracle import rng
    return rng.SampleRule(n_blocks=64, sigma=0.3, pulse_box=(-0.8, -0.4, 0.4, 0.8), T=2.0)


def _mlmc_cpu_worker(args):
    """Oracle (test infrastructure) seconds per coarse step of one sample on level `lvl`."""
    lvl, i, steps = args
    from oracle import fem, lts, mesh, rng
    lv = mesh.graded_L_level(MLMC_BASES[lvl])
    ops = fem.operators(lv)
    rule = _mlmc_rule_oracle()
    smp = rng.draw(0, lvl, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    s = lts.Solver(ops, smp.kappa)
    z0 = lts.pulse(ops, smp.x0)
    t0 = time.perf_counter()
    zm, zc = z0, s.q1(z0, dt)
    for _ in range(1, steps):
        zm, zc = zc, 2.0 * zc - zm + 2.0 * s.d1(zc, dt)
    return lvl, (time.perf_counter() - t0) / steps


def mlmc_bench(no_cpu: bool, eps_list=MLMC_EPS, emit: bool = True, plain: bool = True, fine_tiers=None):
    """Algorithm 1 on the graded L-shape hierarchy (h = 1/16 .. 1/256, p = 64, 8x8
    blocks sigma 0.3, T = 2) at the workload's eps = 1e-3 and a tighter 1e-4: wall
    time of the batched + graph form and of the plain form (one launch per sample
    and step) at identical N_l, and an extrapolated CPU-oracle time for the same N_l.
    The CPU timing runs first, before this process touches the GPU."""
    import multiprocessing as mp

    import numpy as np

    procs = max(1, min(os.cpu_count() or 1, 16))
    per_step = None
    if not no_cpu:
        # oracle seconds per coarse step on every level (4 samples each, 10 steps,
        # one process per core)
        work = [(l, i, 10) for l in range(len(MLMC_BASES)) for i in range(4)]
        with mp.get_context("spawn").Pool(procs) as pool:
            res = pool.map(_mlmc_cpu_worker, work)
        per_step = {l: float(np.mean([t for (ll, t) in res if ll == l])) for l in range(len(MLMC_BASES))}

    import paper_2106_11117_amd as P

    ctx = P.Context(0)
    # the cost-optimal tiers with p <= 64: a larger p on the finest level leaves
    # fine-tile regions (the F+ band within p of a tile) beyond one workgroup
    ids = [ctx.add_rect_level(P.graded_L_rule(nb, fine_tiers=fine_tiers, p_max=64 if fine_tiers else 0))
           for nb in MLMC_BASES]
    rule = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), width=0.05, T=2.0)
    t0 = time.perf_counter()
    for lid in ids:
        ctx.autotune(lid)
    setup = time.perf_counter() - t0
    info = [ctx.level_info(l) for l in ids]
    print("levels (h, p, |P|): " + ", ".join(f"({i['h']}, {i['p']}, {i['n_P']})" for i in info), file=sys.stderr,
          flush=True)
    runs = []
    for eps in eps_list:
        t0 = time.perf_counter()
        rb = ctx.mlmc(ids, rule, eps=eps, N_init=MLMC_N_INIT, L_start=2)
        wall_b = time.perf_counter() - t0
        wall_p = None
        if plain:
            t0 = time.perf_counter()
            rp = ctx.mlmc(ids, rule, eps=eps, N_init=MLMC_N_INIT, L_start=2, mode=P.LTS_MLMC_PLAIN)
            wall_p = time.perf_counter() - t0
            assert rb["N"] == rp["N"] and rb["estimate"] == rp["estimate"]
        run = {"eps": eps, "batched_graph_s": wall_b, "plain_s": wall_p,
               "speedup_vs_plain": None if wall_p is None else wall_p / wall_b,
               "L": rb["L"], "N": rb["N"], "estimate": rb["estimate"], "rmse": rb["rmse"],
               "bias": rb["bias"], "mean": rb["mean"], "var": rb["var"], "converged": rb["converged"]}
        print(f"eps {eps}: L {rb['L']} N {rb['N']} batched {wall_b:.3f} s", file=sys.stderr, flush=True)
        if per_step is not None:
            # the run's own step counts for the same N_l, spread over the cores
            total = 0.0
            for l in range(rb["L"] + 1):
                n = rb["N"][l]
                total += float(P.gen_samples(0, l, 0, n, rule, info[l]["h"])["n_steps"].sum()) * per_step[l]
                if l > 0:
                    total += float(P.gen_samples(0, l, 0, n, rule, info[l - 1]["h"])["n_steps"].sum()) \
                        * per_step[l - 1]
            run["cpu_oracle_s_extrapolated"] = total / procs
            run["speedup_vs_cpu"] = total / procs / wall_b
        runs.append(run)
    out = {"metric": "MLMC wall time at fixed RMSE (Algorithm 1), batched + graph vs plain",
           "unit": "s", "higher_is_better": False, "data": "synthetic (Philox seed 0)",
           "config": {"workload": "graded L-shape, 5 levels h = 1/16..1/256, 6 graded layers "
                                  "(h_min = h/64, p = 64), 8x8 blocks sigma 0.3, T = 2, "
                                  "QoI [0.5,0.9]x[0.2,0.6]; eps absolute",
                      "N_init": list(MLMC_N_INIT), "L_start": 2,
                      "fine_set": "leg < h/2" if fine_tiers is None else f"tiers {fine_tiers}, p <= 64",
                      "dofs": [i["n_dof"] for i in info], "P": [i["n_P"] for i in info],
                      "p": [i["p"] for i in info], "h_step": [i["h"] for i in info]},
           "setup_autotune_s": setup, "runs": runs,
           "cpu_oracle": None if per_step is None else {
               "seconds_per_step_by_level": [per_step[l] for l in range(len(ids))], "cores": procs,
               "kind": "oracle",
               "sample": "oracle seconds per coarse step timed on every level (4 samples x 10 steps, one "
                         "process per core), times each run's step counts for the same N_l, divided by "
                         "the cores (an extrapolation, not a full oracle run)"}}
    if emit:
        print(json.dumps(out), flush=True)
    ctx.close()
    return out


def lf_bench():
    """Standard leapfrog baseline (the cost comparison of Sec. 3.4 and the MLMC
    comparisons of Sec. 4) on the graded L-shape hierarchy: every level against
    its leapfrog twin (the same grid with P empty, stepping at dt/p everywhere).
    Per level, one batched forward of N_l = 4096, 1024, 256, 64, 16 samples on each, whose wall
    time ratio is the measured C_l^LF / C_l^LTS, beside the ratio of DOF updates;
    then Algorithm 1 on both hierarchies (batched + graph) at the MLMC eps."""
    import numpy as np

    import paper_2106_11117_amd as P

    ctx = P.Context(0)
    lts_ids = [ctx.add_rect_level(P.graded_L_rule(nb)) for nb in MLMC_BASES]
    lf_ids = [ctx.add_rect_level(P.lf_rule(P.graded_L_rule(nb))) for nb in MLMC_BASES]
    rule = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), width=0.05, T=2.0)
    for lid in lts_ids + lf_ids:
        ctx.autotune(lid)
    levels = []
    for lev, n in enumerate(BATCH_N):
        row = {"level": lev, "samples": n}
        for kind, lid in (("lts", lts_ids[lev]), ("lf", lf_ids[lev])):
            info = ctx.level_info(lid)
            s = P.gen_samples(0, lev, 0, n, rule, info["h"])
            args = (s["kappa"], s["x0"], s["n_steps"], s["dt"])
            ctx.forward(lid, *(a[:2] for a in args))                  # warm-up (2 samples)
            t0 = time.perf_counter()
            q = np.asarray(ctx.forward(lid, *args))
            t = time.perf_counter() - t0
            steps = float(s["n_steps"].sum())
            upd = steps * ((info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"])
            row[kind] = {"s": t, "sum_n_steps": int(steps), "dof_updates": upd,
                         "dof_updates_per_s": upd / t, "mean_Q": float(q.mean())}
            print(f"level {lev} {kind}: {t:.3f} s", file=sys.stderr, flush=True)
        row["measured_cost_ratio_lf_over_lts"] = row["lf"]["s"] / row["lts"]["s"]
        row["dof_update_ratio_lf_over_lts"] = row["lf"]["dof_updates"] / row["lts"]["dof_updates"]
        levels.append(row)
    runs = []
    for eps in MLMC_EPS:
        res = {}
        for kind, ids in (("lts", lts_ids), ("lf", lf_ids)):
            t0 = time.perf_counter()
            r = ctx.mlmc(ids, rule, eps=eps, N_init=MLMC_N_INIT, L_start=2)
            res[kind] = {"s": time.perf_counter() - t0, "L": r["L"], "N": r["N"], "var": r["var"],
                         "estimate": r["estimate"], "rmse": r["rmse"], "converged": r["converged"]}
        res["eps"] = eps
        res["speedup_lts_over_lf"] = res["lf"]["s"] / res["lts"]["s"]
        runs.append(res)
    out = {"metric": "LF-LTS against the standard leapfrog baseline (dt/p on every element): per-level cost "
                     "and MLMC wall time at fixed RMSE", "unit": "s", "higher_is_better": False,
           "data": "synthetic (Philox seed 0)",
           "config": {"workload": "graded L-shape, 5 levels h = 1/16..1/256, 6 graded layers (h_min = h/64, "
                                  "p = 64), 8x8 blocks sigma 0.3, T = 2; leapfrog twins with P empty, p = 1, "
                                  "spacing h/64", "N_init": list(MLMC_N_INIT), "L_start": 2},
           "levels": levels, "mlmc": runs}
    print(json.dumps(out), flush=True)
    ctx.close()


def adjoint_bench(samples: int, K: int):
    """Discrete adjoint (backward LF-LTS) on the throughput workload: time of one
    lts_backward over the batch (checkpoints every K steps, forward states
    recomputed per segment) against one forward solve of the same batch."""
    import numpy as np
    import torch

    import paper_2106_11117_amd as P

    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    lid = ctx.add_rect_level(P.box_rule(N_BASE, box=BOX, ref=REF))
    info = ctx.level_info(lid)
    s = P.gen_samples(0, 0, 0, samples, P.sample_rule(), info["h"])
    kap = torch.tensor(s["kappa"], device=dev)
    x0 = torch.tensor(s["x0"], device=dev)
    ns = torch.tensor(s["n_steps"], device=dev)
    dt = torch.tensor(s["dt"], device=dev)
    dl = torch.ones(samples, dtype=torch.float64, device=dev)
    ctx.forward(lid, kap[:8], x0[:8], ns[:8], dt[:8])      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qf = ctx.forward(lid, kap, x0, ns, dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    q, g = ctx.backward(lid, kap, x0, ns, dt, dl, K=K)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    per_step = (info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"]
    out = {"metric": "discrete adjoint (backward LF-LTS) time, relative to the forward solve",
           "unit": "s", "higher_is_better": False, "data": "synthetic (Philox seed 0)",
           "config": {"workload": WORKLOAD, "samples": samples, "K_ckpt": K, "dtype": "f64"},
           "forward_s": t_fwd, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
           "forward_dof_updates_per_s": float(s["n_steps"].sum()) * per_step / t_fwd,
           "qoi_equal_to_forward": bool(torch.equal(q, qf)),
           "grad_abs_max": float(g.abs().max())}
    print(json.dumps(out), flush=True)
    ctx.close()


def adjoint_graded_bench(K: int = 64):
    """Discrete adjoint on the graded L-shape levels (compact tilings, p = 64,
    T = 2): lts_backward against lts_forward on the same samples, level 2 with
    64 samples and level 3 with 16 (K = 64)."""
    import numpy as np

    import paper_2106_11117_amd as P

    ctx = P.Context(0)
    rule = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), width=0.05, T=2.0)
    out = {"metric": "discrete adjoint time relative to the forward solve, graded L-shape (compact tiles, p = 64)",
           "unit": "s", "higher_is_better": False, "data": "synthetic (Philox seed 0)", "K_ckpt": K, "runs": []}
    for lev, nb, S in ((2, 128, 64), (3, 256, 16)):
        lid = ctx.add_rect_level(P.graded_L_rule(nb))
        ctx.autotune(lid)
        info = ctx.level_info(lid)
        s = P.gen_samples(0, lev, 0, S, rule, info["h"])
        args = (s["kappa"], s["x0"], s["n_steps"], s["dt"])
        ctx.forward(lid, *(a[:2] for a in args))
        ctx.backward(lid, *(a[:1] for a in args), np.ones(1), K=K)      # warm-up
        t0 = time.perf_counter()
        qf = np.asarray(ctx.forward(lid, *args))
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        q, g = ctx.backward(lid, *args, np.ones(S), K=K)
        tb = time.perf_counter() - t0
        out["runs"].append({"level": lev, "dofs": info["n_dof"], "P": info["n_P"], "samples": S,
                            "tile_rect": info["tile_rect"], "forward_s": tf, "backward_s": tb,
                            "backward_over_forward": tb / tf, "qoi_equal_to_forward": bool(np.array_equal(q, qf))})
    print(json.dumps(out), flush=True)
    ctx.close()


def mlts_bench(T: float = 2.0, per_level: bool = True, eps_list=MLMC_EPS, emit: bool = True):
    """Multi-level LTS (lts_mlts_forward: five tiers by halving legs, p_j = 2)
    against the single-tier LTS solve (lts_forward, p = 64, autotuned tiling)
    on the graded L-shape levels 2-4 at the workload's horizon T = 2, the same
    samples for both (level 2: 64, level 3: 64, level 4: 16).  Wall time with
    the inputs staged, the step kernels' event time, DOF updates per step
    (each scheme's own count), and the largest QoI difference (time
    discretisation) relative to max |Q|.  Then Algorithm 1 on the five-level
    hierarchy at the MLMC benchmark's eps with either scheme: wall time, L,
    N_l and the cost model sum_l N_l C_l."""
    import numpy as np

    import paper_2106_11117_amd as P

    ctx = P.Context(0)
    ctx.set_timing(True)
    rule = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), width=0.05, T=T)
    out = {"metric": "multi-level LTS vs single-tier LTS wall time, graded L-shape (T = 2)",
           "unit": "s", "higher_is_better": False, "data": "synthetic (Philox seed 0)", "dtype": "f64",
           "tiers": [2, 2, 2, 2, 2], "runs": []}
    for lev, nb, S in ((2, 128, 64), (3, 256, 64), (4, 512, 16)) if per_level else ():
        lid = ctx.add_rect_level(P.graded_L_rule(nb))
        ctx.autotune(lid)
        info = ctx.level_info(lid)
        mi = ctx.set_mlts(lid, [2, 2, 2, 2, 2])
        s = P.gen_samples(0, lev, 0, S, rule, info["h"])
        args = (s["kappa"], s["x0"], s["n_steps"], s["dt"])
        ctx.forward(lid, *(a[:2] for a in args))                 # warm-up
        ctx.mlts_forward(lid, *(a[:2] for a in args))
        t0 = time.perf_counter()
        ql = np.asarray(ctx.forward(lid, *args))
        tl = time.perf_counter() - t0
        kl = ctx.timing()["step_kernel_ms"]
        t0 = time.perf_counter()
        qm = np.asarray(ctx.mlts_forward(lid, *args))
        tm = time.perf_counter() - t0
        km = ctx.timing()["step_kernel_ms"]
        ctx.mlts_forward(lid, *(a[:2] for a in args), precision=P.LTS_FP32_STEP)
        t0 = time.perf_counter()
        q32 = np.asarray(ctx.mlts_forward(lid, *args, precision=P.LTS_FP32_STEP))
        t32 = time.perf_counter() - t0
        k32 = ctx.timing()["step_kernel_ms"]
        steps = float(s["n_steps"].sum())
        upd_l = (info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"]
        print(f"level {lev}: lts {tl:.3f} s, mlts {tm:.3f} s, mlts fp32 {t32:.3f} s", flush=True)
        out["runs"].append({
            "level": lev, "dofs": info["n_dof"], "samples": S, "sum_n_steps": int(steps),
            "n_P_tiers": mi["n_P"], "mlts_tiles": mi["n_tiles"], "mlts_halo_ratio": mi["halo_ratio"],
            "mlts_max_region": mi["max_region"], "lts_halo_ratio": info["halo_ratio"],
            "lts": {"s": tl, "step_kernel_ms": kl, "updates_per_step": upd_l,
                    "dof_updates_per_s": steps * upd_l / tl},
            "mlts": {"s": tm, "step_kernel_ms": km, "updates_per_step": mi["updates_per_step"],
                     "dof_updates_per_s": steps * mi["updates_per_step"] / tm},
            "mlts_fp32": {"s": t32, "step_kernel_ms": k32,
                          "dof_updates_per_s": steps * mi["updates_per_step"] / t32,
                          "max_dq_vs_fp64_over_max_q": float(np.max(np.abs(q32 - qm)) / np.max(np.abs(qm)))},
            "speedup": tl / tm,
            "max_dq_over_max_q": float(np.max(np.abs(qm - ql)) / np.max(np.abs(ql)))})
    # Algorithm 1 on the five-level graded hierarchy: single-tier LTS (batched +
    # graph) against multi-level LTS (one solve per level and mesh), same eps
    ids = []
    for nb in MLMC_BASES:
        lid = ctx.add_rect_level(P.graded_L_rule(nb))
        ctx.autotune(lid)
        ctx.set_mlts(lid, [2, 2, 2, 2, 2])
        ids.append(lid)
    out["mlmc"] = []
    for eps in eps_list:
        t0 = time.perf_counter()
        rl = ctx.mlmc(ids, rule, eps=eps, N_init=MLMC_N_INIT, L_start=2)
        wl = time.perf_counter() - t0
        t0 = time.perf_counter()
        rm = ctx.mlmc(ids, rule, eps=eps, N_init=MLMC_N_INIT, L_start=2, mlts=True)
        wm = time.perf_counter() - t0
        print(f"mlmc eps {eps}: lts {wl:.3f} s, mlts {wm:.3f} s", flush=True)
        out["mlmc"].append({
            "eps": eps,
            "lts": {"s": wl, "L": rl["L"], "N": rl["N"], "estimate": rl["estimate"], "rmse": rl["rmse"],
                    "cost_model": float(sum(n * c for n, c in zip(rl["N"], rl["cost"])))},
            "mlts": {"s": wm, "L": rm["L"], "N": rm["N"], "estimate": rm["estimate"], "rmse": rm["rmse"],
                     "cost_model": float(sum(n * c for n, c in zip(rm["N"], rm["cost"])))}})
    if emit:
        print(json.dumps(out), flush=True)
    ctx.close()
    return out


BATCH_N = (4096, 1024, 256, 64, 16)       # samples per level of the multi-level throughput run


def batch_bench(plain: bool, fp32: bool = True, emit: bool = True):
    """Form 2 throughput on the graded L-shape hierarchy (5 levels, h = 1/16 ..
    1/256, p = 64, 8x8 blocks sigma 0.3, T = 2): the samples of all levels
    (N_l = 4096, 1024, 256, 64, 16) advanced together by lts_batch_run, with and
    without graph capture, against one lts_forward call per level and, with
    --plain, the one-launch-per-sample form.  Autotuning is setup, outside the
    timed region; every form must return the same QoIs."""
    import numpy as np

    import paper_2106_11117_amd as P

    ctx = P.Context(0)
    ids = [ctx.add_rect_level(P.graded_L_rule(nb)) for nb in MLMC_BASES]
    rule = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), width=0.05, T=2.0)
    t0 = time.perf_counter()
    for lid in ids:
        ctx.autotune(lid)
    setup = time.perf_counter() - t0
    jobs, levels = [], []
    dof_upd = alg_bytes = 0.0
    for lev, (lid, n) in enumerate(zip(ids, BATCH_N)):
        info = ctx.level_info(lid)
        smp = P.gen_samples(0, lev, 0, n, rule, info["h"])
        jobs.append((lid, smp["kappa"], smp["x0"], smp["n_steps"], smp["dt"], 0.05))
        steps = float(smp["n_steps"].sum())
        per_step = (info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"]
        dof_upd += steps * per_step
        alg_bytes += steps * 24.0 * info["n_dof"]
        levels.append({"dofs": info["n_dof"], "P": info["n_P"], "p": info["p"], "samples": n,
                       "sum_n_steps": int(steps)})

    def median_time(fn, reps):
        ts, out = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), out

    ctx.batch_run(jobs, graph=True)                      # warm-up; captures the graph
    t_graph, q_graph = median_time(lambda: ctx.batch_run(jobs, graph=True), 3)
    t_batch, q_batch = median_time(lambda: ctx.batch_run(jobs, graph=False), 3)
    persist = {}
    for cap in (4, 1):                                   # the persistent form, S_b capped at 4 and at 1
        ctx.batch_run(jobs, persist=True, sb_cap=cap)                   # warm-up
        t_p, q_p = median_time(lambda: ctx.batch_run(jobs, persist=True, sb_cap=cap), 1)
        persist[f"sb_cap_{cap}"] = {"s": t_p, "dof_updates_per_s": dof_upd / t_p,
                                    "q_equal": bool(np.array_equal(np.asarray(q_p), np.asarray(q_graph)))}
    ctx.batch_run(jobs, auto=True)                       # measures the forms on the first steps, caches the choice
    t_auto, q_auto = median_time(lambda: ctx.batch_run(jobs, auto=True), 3)
    tm = ctx.timing()
    per_level = lambda **kw: np.concatenate([np.asarray(ctx.forward(j[0], *j[1:5], width=j[5], **kw))
                                             for j in jobs])
    t_level, q_level = median_time(per_level, 3)
    q64 = np.asarray(q_graph)
    if fp32:
        ctx.batch_run(jobs, graph=True, precision=P.LTS_FP32_STEP)       # warm-up; captures the graph
        t_f32, q_f32 = median_time(lambda: ctx.batch_run(jobs, graph=True, precision=P.LTS_FP32_STEP), 3)
        rel32 = np.abs(np.asarray(q_f32) - q64) / np.max(np.abs(q64))
    out = {"metric": "batched multi-level LF-LTS throughput (form 2), graded L-shape hierarchy",
           "unit": "DOF-updates/s", "higher_is_better": True, "data": "synthetic (Philox seed 0)", "dtype": "f64",
           "config": {"workload": "graded L-shape, 5 levels h = 1/16..1/256, 6 graded layers (h_min = h/64, "
                                  "p = 64), 8x8 blocks sigma 0.3, T = 2", "levels": levels},
           "setup_autotune_s": setup,
           "batched_graph": {"s": t_graph, "dof_updates_per_s": dof_upd / t_graph,
                             "hbm_frac_algorithmic": alg_bytes / t_graph / (HBM_PEAK_GBS * 1e9)},
           "batched_no_graph": {"s": t_batch, "dof_updates_per_s": dof_upd / t_batch},
           "batched_persistent": persist,
           "batched_auto": {"s": t_auto, "dof_updates_per_s": dof_upd / t_auto,
                            "form": {0: "step launches", 1: "graph", 2: "persistent"}[tm["batch_form"]],
                            "sb_cap": tm["batch_sb_cap"],
                            "q_equal": bool(np.array_equal(np.asarray(q_auto), np.asarray(q_graph)))},
           "one_forward_per_level": {"s": t_level, "dof_updates_per_s": dof_upd / t_level},
           "batched_graph_fp32_step": None if not fp32 else {
               "s": t_f32, "dof_updates_per_s": dof_upd / t_f32,
               "qoi_max_err_rel_to_max_abs_q": float(rel32.max()),
               "qoi_median_err_rel_to_max_abs_q": float(np.median(rel32))},
           "q_equal": bool(np.array_equal(np.asarray(q_graph), np.asarray(q_batch)) and
                           np.array_equal(np.asarray(q_graph), q_level))}
    if plain:
        t_plain, q_plain = median_time(lambda: per_level(plain=True), 1)
        out["plain"] = {"s": t_plain, "dof_updates_per_s": dof_upd / t_plain,
                        "speedup_batched_graph_vs_plain": t_plain / t_graph}
        out["q_equal"] = out["q_equal"] and bool(np.array_equal(np.asarray(q_graph), q_plain))
    if emit:
        print(json.dumps(out), flush=True)
    ctx.close()
    return out


LINE_EPS = {"kl": (5e-3, 2e-3, 1e-3), "jump": (5e-3, 2e-3, 1e-3)}


def mesh_bench(samples: int = 64, T: float = 0.25):
    """Levels given as triangulations (lts_add_mesh): the unit square with 512
    cells across refined 8x in the cells meeting (0.48, 0.52), every interior
    node jittered by up to 0.1 of its spacing and the cells split along
    alternating diagonals (442,225 DOFs, |P| = 204,081, p = 8: the C1 sizes
    on an unstructured mesh), `samples` samples to T; the same samples on the
    C1 grid level by the grid path.  Wall time with the samples' inputs
    staged; build and first-call costs outside the timed region."""
    import numpy as np

    import paper_2106_11117_amd as P
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import meshgen

    ctx = P.Context(0)
    m = meshgen.criss_cross(n=N_BASE, ref=REF, box=BOX, jitter=0.1)
    t0 = time.perf_counter()
    mid = ctx.add_mesh(m)
    build = time.perf_counter() - t0
    info = ctx.mesh_info(mid)
    lid = ctx.add_rect_level(P.box_rule(N_BASE, box=BOX, ref=REF, nu=0.01))
    ctx.autotune(lid)
    s = P.gen_samples(0, 0, 0, samples, P.sample_rule(T=T), 1.0 / N_BASE)
    args = (s["kappa"], s["x0"], s["n_steps"], s["dt"])
    ctx.mesh_forward(mid, *(a[:2] for a in args))                   # warm-up
    ctx.forward(lid, *(a[:2] for a in args))
    t0 = time.perf_counter()
    qm = np.asarray(ctx.mesh_forward(mid, *args))
    tm = time.perf_counter() - t0
    t0 = time.perf_counter()
    qg = np.asarray(ctx.forward(lid, *args))
    tg = time.perf_counter() - t0
    per_step = (info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"]
    upd = float(s["n_steps"].sum()) * per_step
    out = {"metric": "LF-LTS DOF-updates/s on a triangle mesh (lts_mesh_forward) vs the tensor-grid path",
           "unit": "DOF-updates/s", "higher_is_better": True, "data": "synthetic (Philox seed 0)", "dtype": "f64",
           "config": {"workload": "unit square 512 base refined 8x in (0.48,0.52), nodes jittered 0.1, "
                                  "alternating diagonals", "samples": samples, "T": T,
                      "sum_n_steps": int(s["n_steps"].sum())},
           "mesh": {k: info[k] for k in ("n_dof", "n_P", "n_Fplus", "n_edges", "max_degree", "n_tiles",
                                         "max_region", "halo_ratio")},
           "build_s": build,
           "mesh_path": {"s": tm, "dof_updates_per_s": upd / tm,
                         "q_finite": bool(np.all(np.isfinite(qm)))},
           "grid_path_c1": {"s": tg, "dof_updates_per_s": upd / tg}}
    print(json.dumps(out), flush=True)
    ctx.close()


def line_bench():
    """The one-dimensional workloads of Sec. 4.1 (continuous random wave speed,
    T = 11) and Sec. 4.2 (random jump, T = 6), Neumann data, Q = u(T) in
    L^2(D): Algorithm 1 with LF-LTS against the standard leapfrog twins (the
    same meshes, P empty, the step of the refined cells everywhere) at the
    same RMSE targets, five levels H = 2^-4 .. 2^-8.  Wall time of each run,
    L, N_l and the cost model sum N_l C_l of both (the paper's own measure)."""
    import paper_2106_11117_amd as P

    ctx = P.Context(0)
    out = {"metric": "1D MLMC wall time at fixed RMSE, LF-LTS vs standard leapfrog (L^2(D)-valued QoI)",
           "unit": "s", "higher_is_better": False, "data": "synthetic (Philox seed 0)", "runs": []}
    for kind in ("kl", "jump"):
        rule = P.line_sample_rule(kind)
        lts_ids = [ctx.add_line_level(P.line_rule(kind, l)) for l in range(5)]
        lf_ids = [ctx.add_line_level(P.line_rule(kind, l, lf=True)) for l in range(5)]
        ctx.line_mlmc(lts_ids[:2], rule, eps=0.1, N_init=(4, 4), L_start=1)        # warm-up
        for eps in LINE_EPS[kind]:
            row = {"kind": kind, "eps": eps}
            for name, ids in (("lts", lts_ids), ("lf", lf_ids)):
                t0 = time.perf_counter()
                r = ctx.line_mlmc(ids, rule, eps=eps, N_init=(32, 16, 8, 4, 4), L_start=2)
                row[name] = {"s": time.perf_counter() - t0, "L": r["L"], "N": r["N"],
                             "model_cost": float(sum(n * c for n, c in zip(r["N"], r["cost"]))),
                             "rmse": r["rmse"], "converged": r["converged"]}
                print(f"{kind} eps {eps} {name}: L {r['L']} N {r['N']} {row[name]['s']:.3f} s", file=sys.stderr,
                      flush=True)
            row["speedup_wall"] = row["lf"]["s"] / row["lts"]["s"]
            row["speedup_model"] = row["lf"]["model_cost"] / row["lts"]["model_cost"]
            out["runs"].append(row)
    print(json.dumps(out), flush=True)
    ctx.close()


def copy_check(mib: int):
    """Four device-to-device copies of `mib` MiB (read mib, write mib each): the
    reference point that turns the FETCH_SIZE / WRITE_SIZE counters of a profiled
    run into bytes."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_check_mib": mib, "copies": 4, "bytes_read_per_copy": n * 8,
                      "bytes_written_per_copy": n * 8}), flush=True)


def stream_check(mib: int = 2048, reps: int = 10):
    """Achieved HBM rates of plain torch streaming kernels over `mib` MiB fp64
    arrays: a copy (1 read, 1 write), c = a + 2b (2 reads, 1 write, the coarse
    sweep's mix) and a sum (1 read).  The practical ceiling beside the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    out = {"stream_check_mib": mib}
    for name, f, nbytes in (("copy_1r1w", lambda: c.copy_(a), 16 * n),
                            ("axpy_2r1w", lambda: torch.add(a, b, alpha=2.0, out=c), 24 * n),
                            ("sum_1r", lambda: torch.sum(a), 8 * n)):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_GBps"] = round(nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--plain", action="store_true", help="time the one-launch-per-sample form")
    ap.add_argument("--samples", type=int, default=N_SAMPLES)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-stepping run")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the MLMC and multi-level batched runs that follow the throughput line")
    ap.add_argument("--copy-check", type=int, default=0, metavar="MIB",
                    help="only run 4 plain device copies of MIB MiB (calibrates HBM byte counters)")
    ap.add_argument("--lf", action="store_true",
                    help="only compare LF-LTS with the standard leapfrog baseline (graded L-shape hierarchy)")
    ap.add_argument("--mesh", action="store_true",
                    help="the triangle-mesh path on a C1-sized unstructured mesh against the grid path")
    ap.add_argument("--line", action="store_true",
                    help="only run the one-dimensional workloads' MLMC, LF-LTS against leapfrog")
    ap.add_argument("--stream-check", action="store_true",
                    help="only time plain torch copy / axpy / sum kernels (practical HBM rates)")
    ap.add_argument("--mlts", action="store_true",
                    help="multi-level LTS against single-tier LTS on the graded L-shape levels 2-4")
    ap.add_argument("--adjoint-graded", action="store_true",
                    help="the discrete adjoint on graded L-shape levels 2 and 3 (compact tiles) against the forward")
    ap.add_argument("--adjoint", action="store_true",
                    help="only time the discrete adjoint against the forward solve (K = 64)")
    ap.add_argument("--mlmc", action="store_true",
                    help="only run the MLMC wall-time comparison (graded L-shape, Algorithm 1)")
    ap.add_argument("--eps", type=float, nargs="+", help="with --mlmc: the RMSE targets (default 1e-3 1e-4)")
    ap.add_argument("--no-plain", action="store_true", help="with --mlmc: skip the plain form")
    ap.add_argument("--qopt", action="store_true",
                    help="with --mlmc: fine sets of the q cost-optimal tiers (Sec. 3.5) instead of legs < h/2")
    ap.add_argument("--batch", action="store_true",
                    help="only time the batched multi-level form on the graded L-shape hierarchy "
                         "(with --plain: also the one-launch-per-sample form)")
    args = ap.parse_args()
    if args.batch:
        batch_bench(args.plain)
        return
    if args.mlts:
        mlts_bench()
        return
    if args.adjoint_graded:
        adjoint_graded_bench()
        return
    if args.adjoint:
        adjoint_bench(args.samples, 64)
        return
    if args.mlmc:
        mlmc_bench(args.no_cpu, tuple(args.eps) if args.eps else MLMC_EPS, plain=not args.no_plain,
                   fine_tiers="opt" if args.qopt else None)
        return
    if args.copy_check:
        copy_check(args.copy_check)
        return
    if args.stream_check:
        stream_check()
        return
    if args.lf:
        lf_bench()
        return
    if args.mesh:
        mesh_bench()
        return
    if args.line:
        line_bench()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the workload is one GPU's "
                                   "share (samples shard across GPUs with one moment all-reduce)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    cpu = None if args.no_cpu else cpu_baseline()

    import numpy as np
    import torch

    import paper_2106_11117_amd as P

    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    lid = ctx.add_rect_level(P.box_rule(N_BASE, box=BOX, ref=REF))
    info = ctx.level_info(lid)
    rule = P.sample_rule()
    s = P.gen_samples(0, 0, 0, args.samples, rule, info["h"])
    kap = torch.tensor(s["kappa"], device=dev)
    x0 = torch.tensor(s["x0"], device=dev)
    ns = torch.tensor(s["n_steps"], device=dev)
    dt = torch.tensor(s["dt"], device=dev)
    torch.cuda.synchronize()

    def step():
        q = ctx.forward(lid, kap, x0, ns, dt, plain=args.plain)
        m = ctx.moments(q)
        return q, m

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    kern_ms, launches = 0.0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, m = step()
        t = ctx.timing()
        kern_ms += t["step_kernel_ms"]
        launches += t["step_launches"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.set_timing(False)

    fp32 = None
    if not args.no_fp32:
        # FP32 stepping beside FP64: one timed solve of the same batch (after one
        # untimed solve), QoI error against the FP64 results of the same samples
        ctx.forward(lid, kap, x0, ns, dt, precision=P.LTS_FP32_STEP)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        q32 = ctx.forward(lid, kap, x0, ns, dt, precision=P.LTS_FP32_STEP)
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t1
        q64 = q.cpu().numpy()
        d = np.abs(q32.cpu().numpy() - q64)
        fp32 = {"ms_per_solve": el32 * 1e3,
                "dof_updates_per_s": float(s["n_steps"].sum()) * ((info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"]) / el32,
                "qoi_max_abs_err_vs_fp64": float(d.max()),
                "qoi_max_err_rel_to_max_abs_q": float(d.max() / np.abs(q64).max()),
                "qoi_median_rel_err": float(np.median(d / np.maximum(np.abs(q64), 1e-300)))}

    per_step = (info["n_dof"] - info["n_P"]) + info["p"] * info["n_P"]
    sum_ns = int(s["n_steps"].sum())
    dof_upd = float(sum_ns) * per_step * args.steps
    alg_bytes = 24.0 * info["n_dof"] * sum_ns * args.steps
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = TRAFFIC["bytes_per_launch"] if step_sources_sha256() == TRAFFIC["sources_sha256"] else None
    out = {
        "metric": "LF-LTS DOF-updates/s & % HBM peak; MLMC time at fixed RMSE, batched vs plain",
        "value": dof_upd / el,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Philox seed 0)",
        "config": {"workload": WORKLOAD, "samples": args.samples, "sum_n_steps": sum_ns,
                   "dofs": info["n_dof"], "P": info["n_P"], "p": info["p"],
                   "form": "plain" if args.plain else "batched",
                   "fine_tile": [info["tile_x"], info["tile_y"]], "tile_rect": info["tile_rect"],
                   "halo_ratio": info["halo_ratio"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "LF-LTS step (k_coarse + k_fine launches)",
                     "algorithmic_bytes_per_launch": alg_bytes / max(launches, 1),
                     "launches": launches, "kernel_ms": kern_ms},
        "cpu_baseline": cpu,
        "fp32_step": fp32,
        "mean_Q": float(m[1]), "var_Q": float(m[2] / max(m[0] - 1, 1)),
    }
    ctx.close()
    if not args.no_extra:
        # the rest of the metric, outside the timed region above: MLMC wall time at
        # fixed RMSE (batched + graph against the plain form, identical N_l), the
        # batched multi-level throughput and MLMC with multi-level LTS, all on the
        # graded L-shape hierarchy
        t0 = time.perf_counter()
        mb = mlmc_bench(True, (1e-4,), emit=False)
        bb = batch_bench(False, fp32=False, emit=False)
        ml = mlts_bench(per_level=False, eps_list=(1e-4,), emit=False)["mlmc"][0]
        r = mb["runs"][0]
        out["mlmc_graded_L"] = {k: r[k] for k in ("eps", "batched_graph_s", "plain_s", "speedup_vs_plain", "L",
                                                  "N", "estimate", "rmse", "converged")}
        out["mlmc_graded_L"]["workload"] = mb["config"]["workload"]
        out["batch_graded_L"] = {"workload": bb["config"]["workload"],
                                 "samples_per_level": [lv["samples"] for lv in bb["config"]["levels"]],
                                 "batched_graph_s": bb["batched_graph"]["s"],
                                 "dof_updates_per_s": bb["batched_graph"]["dof_updates_per_s"],
                                 "hbm_frac_algorithmic": bb["batched_graph"]["hbm_frac_algorithmic"],
                                 "one_forward_per_level_s": bb["one_forward_per_level"]["s"],
                                 "q_equal": bb["q_equal"]}
        out["mlts_mlmc_graded_L"] = {"eps": ml["eps"], "tiers": [2, 2, 2, 2, 2],
                                     "single_tier_s": ml["lts"]["s"], "multi_level_s": ml["mlts"]["s"],
                                     "speedup": ml["lts"]["s"] / ml["mlts"]["s"],
                                     "N_single_tier": ml["lts"]["N"], "N_multi_level": ml["mlts"]["N"],
                                     "cost_model_ratio": ml["lts"]["cost_model"] / ml["mlts"]["cost_model"]}
        out["extra_wall_s"] = time.perf_counter() - t0
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
