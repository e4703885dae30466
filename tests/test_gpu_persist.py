"""GPU tests of the persistent batched form (LTS_BATCH_PERSIST): one cooperative
launch advances every job of every level through all its steps, with a
device-wide barrier after each step; compact tiles of small regions run S_b
samples side by side in one workgroup.  Results must equal the per-level
solves bit for bit (the same arithmetic per node) and the oracle within the
FP64 bound; the bounded barrier wait must end the launch with an error, not
a hang, when it runs out."""
import numpy as np
import pytest

import paper_2106_11117_amd as P
from oracle import fem, lts, mesh

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    c = P.Context(0)
    yield c
    c.close()


def _mixed_jobs(ctx):
    """One rect-mode level (box, 16 x 16 tiles), compact levels whose regions fit
    256-, 512- and 1024-thread tiles (S_b = 4, 2, 1), ragged step counts, and a
    job with fewer samples than S_b."""
    lr = ctx.add_rect_level(P.box_rule(32))
    lg = ctx.add_rect_level(P.graded_L_rule(32))
    l0 = ctx.add_rect_level(P.box_rule(32))
    l1 = ctx.add_rect_level(P.box_rule(64))
    assert ctx.set_tiling(lr, 16, 16, True)["tile_rect"] == 1
    for lid in (lg, l0, l1):
        ctx.set_tiling(lid, 0, 0, False)
    rg = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    r = P.sample_rule(T=0.3)
    sr = P.gen_samples(3, 0, 0, 7, r, 1 / 32)
    sg = P.gen_samples(3, 1, 0, 61, rg, 1 / 16)
    s0 = P.gen_samples(3, 2, 0, 13, r, 1 / 32)
    s1 = P.gen_samples(3, 3, 0, 3, r, 1 / 64)
    jobs = [(lr, sr, 0.05), (lg, sg, 0.05), (l0, s0, 0.05), (l1, s1, 0.05)]
    return [(l, s["kappa"], s["x0"], s["n_steps"], s["dt"], w) for l, s, w in jobs]


def _per_level(ctx, jobs, **kw):
    return np.concatenate([np.asarray(ctx.forward(j[0], *j[1:5], width=j[5], **kw)) for j in jobs])


def test_persistent_equals_per_level_and_oracle(ctx):
    jobs = _mixed_jobs(ctx)
    # the compact tilings' workgroup sizes: S_b = 4, 2 and 1 fit
    assert [P.tiling_host(r, 0, 0, False)["threads"] for r in
            (P.graded_L_rule(32), P.box_rule(32), P.box_rule(64))] == [256, 512, 1024]
    ql = _per_level(ctx, jobs)
    for cap in (4, 2, 1):
        qp = ctx.batch_run(jobs, persist=True, sb_cap=cap)
        assert np.array_equal(qp, ql), cap
        t = ctx.timing()
        assert t["batch_form"] == 2 and t["batch_sb_cap"] == cap
    off = 0
    for (lid, kap, x0, ns, dt, w), lv in zip(jobs, (mesh.box_refined_level(32), mesh.graded_L_level(32),
                                                    mesh.box_refined_level(32), mesh.box_refined_level(64))):
        ops = fem.operators(lv)
        for k in sorted({0, len(ns) - 1}):
            u = lts.Solver(ops, kap[k]).run(lts.pulse(ops, x0[k], w), dt[k], int(ns[k]))
            sc = float(ops.qoi_w @ np.abs(u))
            assert abs(qp[off + k] - float(lts.qoi(ops, u))) <= 1e-11 * sc, (lid, k)
        off += len(ns)


def test_persistent_fp32_equals_per_level_fp32(ctx):
    jobs = _mixed_jobs(ctx)
    q32 = ctx.batch_run(jobs, persist=True, precision=P.LTS_FP32_STEP)
    assert np.array_equal(q32, _per_level(ctx, jobs, precision=P.LTS_FP32_STEP))


def test_persistent_repeats_and_device_pointers(ctx):
    """Two persistent runs in a row with unrelated eager work between them give
    the same bits; device-resident sample arrays give the same bits as host ones."""
    torch = _torch()
    jobs = _mixed_jobs(ctx)
    a = ctx.batch_run(jobs, persist=True)
    x = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
    (x * 2.0).sum().item()
    torch.cuda.synchronize()
    b = ctx.batch_run(jobs, persist=True)
    d = torch.device("cuda:0")
    tj = [(l, torch.tensor(k, device=d), torch.tensor(x0, device=d), torch.tensor(n, device=d),
           torch.tensor(t, device=d), w) for (l, k, x0, n, t, w) in jobs]
    c = ctx.batch_run(tj, persist=True)
    assert np.array_equal(a, b) and np.array_equal(c.cpu().numpy(), a)


def test_barrier_wait_bound_ends_the_launch(ctx):
    """A barrier wait bound far below one step's time (forced from the host):
    the workgroups that wait give up, every workgroup leaves at its next
    barrier, the call reports LTS_ERR_STATE, and the next run with the default
    bound is exact again."""
    jobs = _mixed_jobs(ctx)
    ref = ctx.batch_run(jobs, persist=True)
    ctx.set_barrier_timeout(1e-6)
    try:
        with pytest.raises(P.LtsError) as e:
            ctx.batch_run(jobs, persist=True)
        assert e.value.code == -5
    finally:
        ctx.set_barrier_timeout(2000.0)
    assert np.array_equal(ctx.batch_run(jobs, persist=True), ref)
    with pytest.raises(P.LtsError):
        ctx.set_barrier_timeout(0.0)


def test_auto_form_is_cached_and_exact(ctx):
    """LTS_BATCH_AUTO times the graph form and the persistent form with each
    S_b cap on the first steps, runs the fastest, and reuses the choice for the
    same job list; every choice gives the per-level bits."""
    jobs = _mixed_jobs(ctx)
    ql = _per_level(ctx, jobs)
    qa = ctx.batch_run(jobs, auto=True)
    t1 = ctx.timing()
    assert t1["batch_form"] in (1, 2)
    assert np.array_equal(qa, ql)
    qb = ctx.batch_run(jobs, auto=True)
    t2 = ctx.timing()
    assert (t2["batch_form"], t2["batch_sb_cap"]) == (t1["batch_form"], t1["batch_sb_cap"])
    assert np.array_equal(qb, ql)
    with pytest.raises(P.LtsError):
        ctx.batch_run(jobs, auto=True, graph=True)


def test_persistent_graded_hierarchy_at_T2(ctx):
    """Three graded L-shape levels (h = 1/16, 1/32, 1/64; p = 64) to the
    workload's horizon T = 2, 48 / 12 / 3 samples: persistent == per-step graph
    launches, bit for bit."""
    rule = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    jobs = []
    for lev, (nb, n) in enumerate(zip((32, 64, 128), (48, 12, 3))):
        lid = ctx.add_rect_level(P.graded_L_rule(nb))
        ctx.autotune(lid)
        s = P.gen_samples(0, lev, 0, n, rule, ctx.level_info(lid)["h"])
        jobs.append((lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], 0.05))
    qg = ctx.batch_run(jobs, graph=True)
    for cap in (4, 1):
        assert np.array_equal(ctx.batch_run(jobs, persist=True, sb_cap=cap), qg), cap
