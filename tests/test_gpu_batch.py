"""GPU tests of the batched form: jobs of several levels (uneven mesh sizes and
step counts) advanced by shared launches, HIP-graph capture and replay, and the
autotuner."""
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


def _jobs(ctx):
    """Two unit-square levels and one reentrant-corner level, ragged step counts."""
    l0 = ctx.add_rect_level(P.box_rule(32))
    l1 = ctx.add_rect_level(P.box_rule(64))
    lg = ctx.add_rect_level(P.graded_L_rule(32))
    r = P.sample_rule(T=0.4)
    rg = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    s0 = P.gen_samples(0, 0, 0, 9, r, 1 / 32)
    s1 = P.gen_samples(0, 1, 0, 5, r, 1 / 64)
    sg = P.gen_samples(0, 2, 0, 3, rg, 1 / 16)
    jobs = [(l0, s0["kappa"], s0["x0"], s0["n_steps"], s0["dt"], 0.05),
            (l1, s1["kappa"], s1["x0"], s1["n_steps"], s1["dt"], 0.05),
            (lg, sg["kappa"], sg["x0"], sg["n_steps"], sg["dt"], 0.05)]
    return jobs


def test_batch_matches_per_level_solves_and_oracle(ctx):
    jobs = _jobs(ctx)
    q = ctx.batch_run(jobs)
    off = 0
    makers = [lambda: mesh.box_refined_level(32), lambda: mesh.box_refined_level(64),
              lambda: mesh.graded_L_level(32)]
    for (lid, kap, x0, ns, dt, w), mk in zip(jobs, makers):
        qf = ctx.forward(lid, kap, x0, ns, dt, w)
        n = len(ns)
        scale = np.max(np.abs(qf)) + 1e-300
        assert np.max(np.abs(q[off:off + n] - qf)) <= 1e-14 * scale
        lv = mk()
        ops = fem.operators(lv)
        for k in range(min(n, 3)):
            u = lts.Solver(ops, kap[k]).run(lts.pulse(ops, x0[k], w), dt[k], int(ns[k]))
            sc = float(ops.qoi_w @ np.abs(u))
            assert abs(q[off + k] - float(lts.qoi(ops, u))) <= 1e-11 * sc
        off += n
    for lid in (jobs[0][0], jobs[1][0], jobs[2][0]):
        info = ctx.level_info(lid)
        assert info["tuned"] == 1 and info["halo_ratio"] >= 1.0
        assert info["tile_x"] > 0 or (info["tile_y"] == 0 and info["tile_rect"] == 0)   # 0 x 0: adaptive


def test_batch_compact_workgroup_sizes(ctx):
    """Compact tilings whose regions fit 256-, 512- and 1024-thread workgroups,
    with enough samples that the launches switch workgroup size as samples
    finish (the small sizes while the launch has workgroups to spare): the
    batched QoIs equal one solve per level bit for bit, and the oracle's."""
    lg = ctx.add_rect_level(P.graded_L_rule(32))    # adaptive: 777-node region, 256 threads
    l0 = ctx.add_rect_level(P.box_rule(32))          # adaptive: 1,273 nodes, 512 threads
    l1 = ctx.add_rect_level(P.box_rule(64))          # adaptive: up to 4,060 nodes, 1024 threads
    for lid in (lg, l0, l1):
        ctx.set_tiling(lid, 0, 0, False)
    rg = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    r = P.sample_rule(T=0.2)
    sg = P.gen_samples(1, 0, 0, 700, rg, 1 / 16)
    s0 = P.gen_samples(1, 1, 0, 300, r, 1 / 32)
    s1 = P.gen_samples(1, 2, 0, 40, r, 1 / 64)
    jobs = [(lg, sg["kappa"], sg["x0"], sg["n_steps"], sg["dt"], 0.05),
            (l0, s0["kappa"], s0["x0"], s0["n_steps"], s0["dt"], 0.05),
            (l1, s1["kappa"], s1["x0"], s1["n_steps"], s1["dt"], 0.05)]
    q = ctx.batch_run(jobs)
    qg = ctx.batch_run(jobs, graph=True)
    ql = np.concatenate([np.asarray(ctx.forward(j[0], *j[1:5], width=j[5])) for j in jobs])
    assert np.array_equal(q, ql) and np.array_equal(qg, ql)
    off = 0
    for (lid, kap, x0, ns, dt, w), lv in zip(jobs, (mesh.graded_L_level(32), mesh.box_refined_level(32),
                                                    mesh.box_refined_level(64))):
        ops = fem.operators(lv)
        for k in (0, len(ns) - 1):
            u = lts.Solver(ops, kap[k]).run(lts.pulse(ops, x0[k], w), dt[k], int(ns[k]))
            sc = float(ops.qoi_w @ np.abs(u))
            assert abs(q[off + k] - float(lts.qoi(ops, u))) <= 1e-11 * sc
        off += len(ns)


def test_graph_replays_match_eager(ctx):
    torch = _torch()
    jobs = _jobs(ctx)
    eager = ctx.batch_run(jobs)
    for rep in range(3):
        g = ctx.batch_run(jobs, graph=True)      # capture on the first call, replay after
        assert np.array_equal(g, eager), rep
        # unrelated eager device work and a synchronisation between replays
        x = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
        (x * 2.0).sum().item()
        torch.cuda.synchronize()
        e2 = ctx.batch_run(jobs)
        assert np.array_equal(e2, eager)


def test_graph_recaptures_on_new_samples(ctx):
    jobs = _jobs(ctx)
    a = ctx.batch_run(jobs, graph=True)
    lid, kap, x0, ns, dt, w = jobs[0]
    jobs[0] = (lid, kap[::-1].copy(), x0[::-1].copy(), ns[::-1].copy(), dt[::-1].copy(), w)
    b = ctx.batch_run(jobs, graph=True)
    n0 = len(ns)
    assert np.array_equal(b[:n0], a[:n0][::-1]) and np.array_equal(b[n0:], a[n0:])


def test_batch_device_pointers_and_offsets(ctx):
    torch = _torch()
    jobs = _jobs(ctx)
    host = ctx.batch_run(jobs)
    d = torch.device("cuda:0")
    tj = [(l, torch.tensor(k, device=d), torch.tensor(x, device=d), torch.tensor(n, device=d),
           torch.tensor(t, device=d), w) for (l, k, x, n, t, w) in jobs]
    dev = ctx.batch_run(tj, graph=True)
    assert np.array_equal(dev.cpu().numpy(), host)


def test_batch_argument_errors(ctx):
    jobs = _jobs(ctx)
    bad = list(jobs)
    bad[1] = (99,) + bad[1][1:]
    with pytest.raises(P.LtsError):
        ctx.batch_run(bad)


def test_batch_fp32_stepping(ctx):
    """FP32 stepping in the batched form (LTS_BATCH_FP32): the same QoIs, bit for
    bit, as FP32 stepping of one solve per level (with and without the graph),
    within the FP32 error bound of the FP64 QoIs, and measurably not FP64."""
    jobs = _jobs(ctx)
    q32 = ctx.batch_run(jobs, precision=P.LTS_FP32_STEP)
    q32g = ctx.batch_run(jobs, graph=True, precision=P.LTS_FP32_STEP)
    q64 = ctx.batch_run(jobs)
    ql = np.concatenate([np.asarray(ctx.forward(j[0], *j[1:5], width=j[5], precision=P.LTS_FP32_STEP))
                         for j in jobs])
    assert np.array_equal(q32, ql) and np.array_equal(q32g, ql)
    off = 0
    for (lid, kap, x0, ns, dt, w) in jobs:
        p = ctx.level_info(lid)["p"]
        n = len(ns)
        scale = np.max(np.abs(q64[off:off + n]))
        err = np.abs(q32[off:off + n] - q64[off:off + n])
        assert np.all(err <= 4 * ns * p * 2.0 ** -24 * scale)      # loose form of the derived bound
        assert np.max(err) > 1e-12 * scale                             # binary32 really ran
        off += n
