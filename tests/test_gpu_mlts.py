"""GPU parity of multi-level LTS (lts_set_mlts, lts_mlts_forward) against the
oracle's multi-level LTS (oracle/mlts.py; Sec. 3.5, closing remark).

Graded L-shape levels 0-2 (32, 64, 128 cells across) with five tiers by the
halving rule and p_j = 2 (every tier at the coarse cells' ratio of step to
leg) at the workload's horizon T = 2, batches of 16 samples, oracle solves in
worker processes; caller-given tiers with a three-stage tier on the
box-refined level; one tier against the single-tier LTS solve; device
pointers, the g input and the error paths.  Metric as in the other parity
tests: |Q_gpu - Q_oracle| <= 1e-11 sum_i w_i |u_i| (FP64)."""
import numpy as np
import pytest

import oracle_jobs
import paper_2106_11117_amd as P
from oracle import fem, lts, mesh, mlts, rng

pytestmark = pytest.mark.gpu
T_END = 2.0
TOL = 1e-11
PS = [2, 2, 2, 2, 2]
BASES = (32, 64, 128)
LIVE = {0: (0, 1, 2, 15), 1: (0, 7), 2: (0,)}
BATCH = 16


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rule(T=T_END):
    return P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=T)


@pytest.fixture(scope="module")
def ctx():
    _torch()
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def oracle():
    jobs = [("mlts", BASES[l], l, i, T_END, PS) for l, ii in LIVE.items() for i in ii]
    print(f"oracle: {len(jobs)} multi-level LTS solves in worker processes", flush=True)
    res = oracle_jobs.run_all(jobs)
    return {(j[1], j[2], j[3]): r for j, r in zip(jobs, res)}


def _fp32_bound(n_steps, stages):
    """FP32 stepping: every coarse step applies `stages` binary32 recurrence and
    stencil updates to O(|u|) values (relative rounding 2^-24 each), which add up
    at most linearly in the stable, non-dissipative recurrence: |dQ| <= 4 n_s
    stages 2^-24 sum_i w_i |u_i| (the bound of the single-tier FP32 tests with p
    replaced by the innermost stage count)."""
    return 4.0 * n_steps * stages * 2.0 ** -24


def _check(q, ref):
    e = abs(q - ref["Q"]) / ref["abs_wu"]
    assert e <= TOL, (q, ref["Q"], e)
    return e


def test_graded_levels_0_2_at_T2(ctx, oracle):
    for l, ii in LIVE.items():
        lid = ctx.add_rect_level(P.graded_L_rule(BASES[l]))
        info = ctx.set_mlts(lid, PS)
        assert info["phases"] == 31 and info["n_tiles"] >= 1 and info["max_region"] <= 2048
        s = P.gen_samples(0, l, 0, BATCH, _rule(), ctx.level_info(lid)["h"])
        print(f"level {l}: {info['n_tiles']} tiles, {BATCH} samples", flush=True)
        q = ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        for i in ii:
            ref = oracle[(BASES[l], l, i)]
            assert ref["n_steps"] == int(s["n_steps"][i])
            _check(q[i], ref)
        # the multi-level step differs from the single-tier one by time discretisation only
        # (about 1e-5 of Q in the oracle on level 0)
        ql = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        assert np.max(np.abs(q - ql)) < 1e-3 * np.max(np.abs(ql))
        # FP32 stepping against the FP64 oracle within the derived bound: every
        # coarse step applies prod p_j innermost stages of binary32 updates
        q32 = ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP)
        for i in ii:
            ref = oracle[(BASES[l], l, i)]
            e = abs(q32[i] - ref["Q"]) / ref["abs_wu"]
            assert 1e-12 < e <= _fp32_bound(ref["n_steps"], int(np.prod(PS))), (l, i, e)


def test_one_tier_is_the_single_tier_solve(ctx):
    """T = 1 with p_1 = p: Algorithm 2 itself, up to the rounding of A u + A P e
    against w + A P (u + d) (box-refined level, p = 4; graded level with four layers, p = 16,
    T = 0.5)."""
    for rule, p, T in [(P.box_rule(32, box=(0.4375, 0.5625)), 4, 1.0), (P.graded_L_rule(32, layers=4), 16, 0.5)]:
        lid = ctx.add_rect_level(rule)
        ctx.set_mlts(lid, [p])
        s = P.gen_samples(0, 0, 0, 8, P.sample_rule(n_blocks=ctx.level_info(lid)["n_blocks"], T=T),
                          ctx.level_info(lid)["h"])
        q = ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        ql = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        assert np.max(np.abs(q - ql)) <= 1e-12 * np.max(np.abs(ql))


def test_given_tiers_with_three_stages(ctx):
    """Caller-given cell tiers on the box-refined level (tier 2: the fine cells
    near the box centre), p = (3, 2), against the oracle."""
    lv = mesh.box_refined_level(32, box=(0.4375, 0.5625))
    mx = 0.5 * (lv.xs[:-1] + lv.xs[1:])
    MX, MY = np.meshgrid(mx, mx)
    inner = (abs(MX - 0.5) < 0.03) & (abs(MY - 0.5) < 0.03)
    ct = np.where(lv.cell_active & lv.cell_fine, np.where(inner, 2, 1), 0).astype(np.uint8)
    ps = [3, 2]
    lid = ctx.add_rect_level(P.box_rule(32, box=(0.4375, 0.5625)))
    info = ctx.set_mlts(lid, ps, ct)
    assert info["phases"] == 2 + 3 * 1
    T = 1.0
    s = P.gen_samples(0, 0, 0, 5, P.sample_rule(T=T), lv.h)
    q = ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    # smaller tiles on 256-thread workgroups: a tiling only decides which workgroup updates a node
    assert ctx.set_mlts(lid, ps, ct, max_region=512)["threads"] == 256
    assert np.array_equal(ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"]), q)
    ops = fem.operators(lv)
    Ps = mlts.tier_projectors(lv, ct, 2)
    rule = rng.SampleRule(T=T)
    for i in (0, 4):
        smp = rng.draw(0, 0, i, rule)
        n, dt = rng.steps_for(smp, rule, lv.h)
        assert n == int(s["n_steps"][i])
        u = mlts.MltsSolver(ops, smp.kappa, Ps, ps).run(lts.pulse(ops, smp.x0), dt, n)
        _check(q[i], {"Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u))})


def test_device_pointers_g_and_errors(ctx):
    torch = _torch()
    lid = ctx.add_rect_level(P.graded_L_rule(32))
    s = P.gen_samples(0, 0, 0, 6, _rule(0.5), ctx.level_info(lid)["h"])
    with pytest.raises(P.LtsError):                    # no tiers attached yet
        ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    ctx.set_mlts(lid, [2, 2])
    ctx.set_mlts(lid, PS)                              # replaces the tiers
    assert ctx.mlts_info(lid)["n_tiers"] == 5
    q = ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    d = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, device=d)
    qd = ctx.mlts_forward(lid, T(s["kappa"]), T(s["x0"]), T(s["n_steps"]), T(s["dt"]))
    assert np.array_equal(qd.cpu().numpy(), q)
    qg = ctx.mlts_forward(lid, None, T(s["x0"]), T(s["n_steps"]), T(s["dt"]), g=T(0.5 * np.log(s["kappa"])))
    assert np.max(np.abs(qg.cpu().numpy() - q)) <= 1e-13 * np.max(np.abs(q))
    assert len(ctx.mlts_forward(lid, s["kappa"][:0], s["x0"][:0], s["n_steps"][:0], s["dt"][:0])) == 0
    with pytest.raises(P.LtsError):                    # FP64 only
        P._check(ctx.lib.lts_mlts_forward(ctx.h, lid, None, P.LTS_FP32_STEP, None), ctx.h)
    with pytest.raises(P.LtsError):
        ctx.mlts_info(99)
    # a level without fine cells (the leapfrog twin): no fine tiles, the coarse sweep alone
    tw = ctx.add_rect_level(P.lf_rule(P.graded_L_rule(32)))
    info = ctx.set_mlts(tw, [1])
    assert info["n_tiles"] == 0 and info["n_P"] == [0]
    st = P.gen_samples(0, 0, 0, 3, _rule(0.5), ctx.level_info(tw)["h"])
    assert np.array_equal(ctx.mlts_forward(tw, st["kappa"], st["x0"], st["n_steps"], st["dt"]),
                          ctx.forward(tw, st["kappa"], st["x0"], st["n_steps"], st["dt"]))


def test_mlmc_with_multi_level_lts(ctx):
    """Algorithm 1 over graded levels with 16, 32 and 64 cells across, each
    with the five tiers (LTS_LEVELS_MLTS), T = 0.5 and the QoI over
    [-0.35,0.05]x[0.05,0.45] next to the graded corner: the same L, N_l,
    estimate, moments and cost model as the oracle's Algorithm 1 with the
    oracle's multi-level LTS solves and the multi-level update count as cost;
    the same results with levels 1-2 generated on demand."""
    import math

    from oracle import mlmc
    bases, qb = (16, 32, 64), (-0.35, 0.05, 0.05, 0.45)
    ids = []
    for b in bases:
        lid = ctx.add_rect_level(P.graded_L_rule(b, qoi=qb))
        ctx.set_mlts(lid, PS)
        ids.append(lid)
    eps, N_init = 2e-4, (24, 12, 6)
    res = ctx.mlmc(ids, _rule(0.5), eps=eps, N_init=N_init, L_start=1, mlts=True)
    ops = [fem.operators(mesh.graded_L_level(b, qoi_box=qb)) for b in bases]
    Ps = [mlts.tier_projectors(o.lv, mlts.tiers_by_leg(o.lv, 5), 5) for o in ops]
    orule = rng.SampleRule(T=0.5, n_blocks=64, sigma=0.3, pulse_box=(-0.8, -0.4, 0.4, 0.8))

    def q(l, smp):
        n, dt = rng.steps_for(smp, orule, ops[l].lv.h)
        u = mlts.MltsSolver(ops[l], smp.kappa, Ps[l], PS).run(lts.pulse(ops[l], smp.x0), dt, n)
        return float(lts.qoi(ops[l], u))

    def eval_dq(l, i):
        smp = rng.draw(0, l, i, orule)
        return q(l, smp) - (q(l - 1, smp) if l > 0 else 0.0)

    cs = []
    for o, Pl in zip(ops, Ps):
        nP = [int(v.sum()) for v in Pl]
        upd, rate = o.lv.n_dof - nP[0], 1
        for j in range(5):
            rate *= PS[j]
            upd += rate * (nP[j] - (nP[j + 1] if j + 1 < 5 else 0))
        cs.append(math.ceil(orule.T / (orule.cfl * o.lv.h)) * upd)
    costs = [cs[0]] + [cs[l] + cs[l - 1] for l in (1, 2)]
    print("oracle Algorithm 1 with multi-level LTS", flush=True)
    ores = mlmc.mlmc(ops, orule, eps=eps, N_init=N_init, L_start=1, eval_dq=eval_dq, costs=costs)
    assert ores.L == 2
    assert res["L"] == ores.L and res["N"] == ores.N
    assert res["cost"] == [float(c) for c in ores.cost[:ores.L + 1]]
    scale = max(abs(v) for v in ores.mean)
    assert abs(res["estimate"] - ores.estimate) <= 1e-11 * scale
    for l in range(res["L"] + 1):
        assert abs(res["mean"][l] - ores.mean[l]) <= 1e-11 * scale
        assert abs(res["var"][l] - ores.var[l]) <= 1e-9 * ores.var[l]
    # the same hierarchy with levels 1 and 2 built (and given their tiers) when Algorithm 1 first needs them
    rg = ctx.mlmc(ids[:1], _rule(0.5), eps=eps, N_init=N_init, L_start=1, mlts=True,
                  gen_rule=P.graded_L_rule(16, qoi=qb), n_levels_max=3, gen_mlts=PS)
    for k in ("L", "N", "estimate", "mean", "var", "cost"):
        assert rg[k] == res[k], k
    with pytest.raises(P.LtsError):                    # a level without tiers
        lid = ctx.add_rect_level(P.graded_L_rule(16, qoi=qb))
        ctx.mlmc([lid] + ids[1:], _rule(0.5), eps=eps, N_init=N_init, L_start=1, mlts=True)


def test_batched_form_is_bit_identical(ctx):
    """LTS_BATCH_MLTS: jobs of graded levels 0-2 (with the tiers) and of the
    box-refined level with given three-stage tiers in shared launches, with and
    without the graph, give the QoIs of lts_mlts_forward bit for bit; a level
    without tiers is refused."""
    jobs, singles = [], []
    for l, b in enumerate(BASES):
        lid = ctx.add_rect_level(P.graded_L_rule(b))
        ctx.set_mlts(lid, PS)
        s = P.gen_samples(0, l, 0, (24, 9, 5)[l], _rule(0.5), ctx.level_info(lid)["h"])
        jobs.append((lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], 0.05))
        singles.append(ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"]))
    lv = mesh.box_refined_level(32, box=(0.4375, 0.5625))
    mx = 0.5 * (lv.xs[:-1] + lv.xs[1:])
    MX, MY = np.meshgrid(mx, mx)
    ct = np.where(lv.cell_active & lv.cell_fine, np.where((abs(MX - 0.5) < 0.03) & (abs(MY - 0.5) < 0.03), 2, 1),
                  0).astype(np.uint8)
    lid = ctx.add_rect_level(P.box_rule(32, box=(0.4375, 0.5625)))
    ctx.set_mlts(lid, [3, 2], ct)
    s = P.gen_samples(0, 0, 0, 7, P.sample_rule(T=0.5), lv.h)
    jobs.append((lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], 0.05))
    singles.append(ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"]))
    want = np.concatenate(singles)
    for graph in (False, True, True):                 # the second graph run replays the cached graph
        q = ctx.batch_run(jobs, graph=graph, mlts=True)
        assert np.array_equal(q, want)
    # FP32 stepping: batched (with and without the graph) equals the plain form bit for bit
    want32 = np.concatenate([np.asarray(ctx.mlts_forward(j[0], *j[1:5], precision=P.LTS_FP32_STEP)) for j in jobs])
    for graph in (False, True, True):
        assert np.array_equal(ctx.batch_run(jobs, graph=graph, mlts=True, precision=P.LTS_FP32_STEP), want32)
    assert not np.array_equal(want32, want)
    plain = ctx.add_rect_level(P.graded_L_rule(32))
    with pytest.raises(P.LtsError):
        ctx.batch_run([(plain,) + jobs[0][1:]], mlts=True)
    with pytest.raises(P.LtsError):
        ctx.batch_run(jobs[:1], mlts=True, auto=True)


def test_graded_levels_3_4_at_T2_in_the_bench_configuration(ctx):
    """The two finest graded levels (53,333 and 204,885 DOFs, 7 and 12 fine
    tiles of up to 2,048 region nodes) in the launch configuration bench.py
    --mlts times (64 and 16 samples in one call), first and last sample
    against stored oracle values (tests/golden/mlts_gradedL_qoi.json, written
    by tests/golden/make_mlts_golden.py, which calls only the oracle)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mlts_gradedL_qoi.json")))
    assert gold["tiers"] == PS
    bases, batch = {3: 256, 4: 512}, {3: 64, 4: 16}
    for l in (3, 4):
        lid = ctx.add_rect_level(P.graded_L_rule(bases[l]))
        info = ctx.set_mlts(lid, PS)
        assert info["n_tiles"] == (7 if l == 3 else 12)
        s = P.gen_samples(0, l, 0, batch[l], _rule(), ctx.level_info(lid)["h"])
        print(f"level {l}: {batch[l]} samples", flush=True)
        q = ctx.mlts_forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        refs = [r for r in gold["samples"] if r["level"] == l]
        assert len(refs) == 2
        for ref in refs:
            i = ref["i"]
            assert ref["n_steps"] == int(s["n_steps"][i])
            _check(q[i], ref)
