"""GPU parity of the forward LF-LTS path (through the C ABI) against the oracle.

Metric (R16 reading of "relative error 1e-11" when Q can be near 0): per
sample, |Q_gpu - Q_oracle| / sum_i w_i |u_i(T)| <= 1e-11, and also relative
to |Q_oracle| when |Q_oracle| >= 1e-3 sum_i w_i |u_i(T)|.
"""
import json
import math
import os

import numpy as np
import pytest

import paper_2106_11117_amd as P
from oracle import fem, lts, mesh, mlmc, rng

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(__file__)
TOL = 1e-11


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


def oracle_solve(ops, lv, kappa, x0, n, dt, width=0.05, nu=None):
    s = lts.Solver(ops, kappa)
    u = s.run(lts.pulse(ops, x0, width), dt, n)
    return float(lts.qoi(ops, u)), float(ops.qoi_w @ np.abs(u))


def check(qg, qo, scale, tol=TOL):
    e_abs = abs(qg - qo) / scale
    assert e_abs <= tol, (qg, qo, e_abs)
    if abs(qo) >= 1e-3 * scale:
        assert abs(qg - qo) / abs(qo) <= tol, (qg, qo)
    return e_abs


def _c0_rule():
    return P.sample_rule(n_blocks=16, sigma=0.25, pulse=(0.2, 0.4, 0.2, 0.4), width=0.05, T=1.0)


def test_c0_level0_batch(ctx):
    """Two-level unit-square workload, level 0: 64 samples in one batched call."""
    lid = ctx.add_rect_level(P.box_rule(32))
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    s = P.gen_samples(0, 0, 0, 64, _c0_rule(), lv.h)
    q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    assert len(set(s["n_steps"].tolist())) > 10        # ragged step counts in one batch
    worst = 0.0
    for k in range(64):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(s["n_steps"][k]), s["dt"][k])
        worst = max(worst, check(q[k], qo, sc))
    print(f"C0 level 0: worst |dQ| / sum w|u| = {worst:.3g}")


def test_c0_level1_coupled(ctx):
    """Level-1 differences: the same 16 samples on the 1/64 and the 1/32 mesh."""
    lf = ctx.add_rect_level(P.box_rule(64))
    lc = ctx.add_rect_level(P.box_rule(32))
    lvf, lvc = mesh.box_refined_level(64), mesh.box_refined_level(32)
    opf, opc = fem.operators(lvf), fem.operators(lvc)
    r = _c0_rule()
    sf = P.gen_samples(0, 1, 0, 16, r, lvf.h)
    sc_ = P.gen_samples(0, 1, 0, 16, r, lvc.h)
    qf, qc, dq = ctx.forward_coupled(lf, lc, sf["kappa"], sf["x0"], sf["n_steps"], sf["dt"],
                                     sc_["n_steps"], sc_["dt"])
    for k in range(16):
        of, af = oracle_solve(opf, lvf, sf["kappa"][k], sf["x0"][k], int(sf["n_steps"][k]), sf["dt"][k])
        oc, ac = oracle_solve(opc, lvc, sf["kappa"][k], sf["x0"][k], int(sc_["n_steps"][k]), sc_["dt"][k])
        check(qf[k], of, af)
        check(qc[k], oc, ac)
        assert abs(dq[k] - (of - oc)) <= TOL * (af + ac)
        assert dq[k] == qf[k] - qc[k]


def test_graded_L_p64(ctx):
    """Reentrant-corner mesh (p = 64 substeps) at the horizon T = 2."""
    lid = ctx.add_rect_level(P.graded_L_rule(32))
    lv = mesh.graded_L_level(32)
    ops = fem.operators(lv)
    r = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    s = P.gen_samples(0, 0, 0, 3, r, lv.h)
    q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    for k in range(3):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(s["n_steps"][k]), s["dt"][k])
        check(q[k], qo, sc)


@pytest.mark.parametrize("nu,p", [(0.0, 3), (1.0, 5), (0.01, 1)])
def test_other_p_and_nu(ctx, nu, p):
    """Explicit p (including p = 1: plain leapfrog) and the extreme nu values."""
    lid = ctx.add_rect_level(P.box_rule(16, ref=4, p=p, nu=nu))
    lv = mesh.box_refined_level(16, ref=4, p=p, nu=nu)
    ops = fem.operators(lv)
    kap = np.exp(2 * np.linspace(-0.3, 0.3, 16))[None, :]
    dt = 0.15 / 16 / math.exp(0.3) * (p if p > 1 else 0.5)
    x0 = np.array([[0.3, 0.35]])
    q = ctx.forward(lid, kap, x0, np.array([40], dtype=np.int32), np.array([dt]))
    qo, sc = oracle_solve(ops, lv, kap[0], x0[0], 40, dt)
    check(q[0], qo, sc)


def test_plain_form_is_bitwise_equal_to_batched(ctx):
    lid = ctx.add_rect_level(P.box_rule(32))
    s = P.gen_samples(0, 0, 100, 8, _c0_rule(), 1 / 32)
    a = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    b = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], plain=True)
    assert np.array_equal(a, b)
    # deterministic run to run
    c = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    assert np.array_equal(a, c)


def test_device_pointer_path(ctx):
    torch = _torch()
    lid = ctx.add_rect_level(P.box_rule(32))
    s = P.gen_samples(0, 0, 0, 5, _c0_rule(), 1 / 32)
    a = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    d = torch.device("cuda:0")
    b = ctx.forward(lid, torch.tensor(s["kappa"], device=d), torch.tensor(s["x0"], device=d),
                    torch.tensor(s["n_steps"], device=d), torch.tensor(s["dt"], device=d))
    assert np.array_equal(a, b.cpu().numpy())


def test_edge_cases(ctx):
    lid = ctx.add_rect_level(P.box_rule(32))
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    # empty batch
    q = ctx.forward(lid, np.zeros((0, 16)), np.zeros((0, 2)), np.zeros(0, dtype=np.int32), np.zeros(0))
    assert q.shape == (0,)
    # one step only (start-up), and a mix with a long one
    s = P.gen_samples(0, 0, 0, 3, _c0_rule(), 1 / 32)
    ns = np.array([1, 2, int(s["n_steps"][2])], dtype=np.int32)
    q = ctx.forward(lid, s["kappa"], s["x0"], ns, s["dt"])
    for k in range(3):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(ns[k]), s["dt"][k])
        check(q[k], qo, sc)


def test_argument_errors(ctx):
    lid = ctx.add_rect_level(P.box_rule(32))
    s = P.gen_samples(0, 0, 0, 2, _c0_rule(), 1 / 32)
    bad = s["kappa"].copy()
    bad[1, 3] = -1.0
    with pytest.raises(P.LtsError) as e:
        ctx.forward(lid, bad, s["x0"], s["n_steps"], s["dt"])
    assert e.value.code == -1
    with pytest.raises(P.LtsError):
        ctx.forward(lid, s["kappa"], s["x0"], np.array([0, 5], dtype=np.int32), s["dt"])
    with pytest.raises(P.LtsError):
        ctx.forward(99, s["kappa"], s["x0"], s["n_steps"], s["dt"])


def test_unstable_step_reported(ctx):
    """A step far beyond the stability limit (forced from the host) gives NaN/inf QoIs
    for that sample only and LTS_ERR_UNSTABLE."""
    lid = ctx.add_rect_level(P.box_rule(32))
    s = P.gen_samples(0, 0, 0, 2, _c0_rule(), 1 / 32)
    dt = s["dt"].copy()
    ns = np.array([3000, int(s["n_steps"][1])], dtype=np.int32)
    dt[0] = 3.0 / 32
    with pytest.raises(P.LtsError) as e:
        ctx.forward(lid, s["kappa"], s["x0"], ns, dt)
    assert e.value.code == -4


def test_moments_match_oracle(ctx):
    x = np.random.default_rng(5).standard_normal(1001) * 1e-4 + 0.3
    out = ctx.moments(x)
    m, v = mlmc.mean_var(x)
    assert out[0] == 1001
    assert abs(out[1] - m) <= 1e-15 * abs(m)
    assert abs(out[2] / 1000 - v) <= 1e-12 * v
    out = ctx.moments(np.array([]))
    assert out[0] == 0
    out = ctx.moments(np.array([2.5]))
    assert out[0] == 1 and out[1] == 2.5 and out[2] == 0


def test_c1_full_size_sampled(ctx):
    """Full single-level throughput workload (442,225 DOFs, p = 8, 256 samples in one
    batched call, as timed by the benchmark) against oracle QoIs of sampled outputs."""
    path = os.path.join(HERE, "golden", "c1_qoi.json")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    gold = json.load(open(path))
    lid = ctx.add_rect_level(P.box_rule(512, box=(0.48, 0.52), ref=8))
    s = P.gen_samples(0, 0, 0, gold["n_samples"], _c0_rule(), 1 / 512)
    assert int(s["n_steps"].sum()) == gold["sum_n_steps"]
    q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    worst = 0.0
    for g in gold["samples"]:
        assert int(s["n_steps"][g["i"]]) == g["n_steps"] and s["dt"][g["i"]] == g["dt"]
        worst = max(worst, check(q[g["i"]], g["Q"], g["abs_wu"]))
    print(f"C1 sampled: worst |dQ| / sum w|u| = {worst:.3g}")


def _fp32_bound(n_steps, p):
    """Derived bound for FP32 stepping: every coarse step applies n_s * p binary32
    stencil/recurrence updates to O(|u|) values (relative rounding 2^-24 each); in a
    stable, non-dissipative three-term recurrence these errors add up at most
    linearly, so |dQ| <= 4 * n_s * p * 2^-24 * sum_i w_i |u_i| (factor 4: the few
    roundings per update)."""
    return 4.0 * n_steps * p * 2.0 ** -24


def _fp32_case(ctx, graded):
    if not graded:
        lid = ctx.add_rect_level(P.box_rule(32))
        lv = mesh.box_refined_level(32)
        s = P.gen_samples(0, 0, 0, 12, _c0_rule(), lv.h)
    else:
        lid = ctx.add_rect_level(P.graded_L_rule(32))
        lv = mesh.graded_L_level(32)
        r = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
        s = P.gen_samples(0, 0, 0, 3, r, lv.h)
    return lid, lv, s


@pytest.mark.parametrize("graded,rect", [(False, True), (False, False), (True, True), (True, False)])
def test_fp32_stepping(ctx, graded, rect):
    """FP32 stepping (binary32 states, increments and stencil; binary64 QoI sum)
    against the FP64 oracle in both fine-tile modes: within the derived bound,
    and measurably not FP64."""
    lid, lv, s = _fp32_case(ctx, graded)
    info = ctx.set_tiling(lid, 48, 48, rect) if not graded else ctx.set_tiling(lid, 16, 16, rect)
    assert bool(info["tile_rect"]) == rect
    ops = fem.operators(lv)
    q32 = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP)
    q32b = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP,
                       plain=True)
    assert np.array_equal(q32, q32b)
    worst = 0.0
    for k in range(len(q32)):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(s["n_steps"][k]), s["dt"][k])
        e = abs(q32[k] - qo) / sc
        worst = max(worst, e / _fp32_bound(int(s["n_steps"][k]), lv.p))
        assert e <= _fp32_bound(int(s["n_steps"][k]), lv.p), (k, e)
        assert e > 1e-12          # binary32 really ran
    print(f"fp32 worst error / bound = {worst:.3g}")


@pytest.mark.parametrize("graded", [False, True])
def test_fine_tile_modes_and_shapes(ctx, graded):
    """FP64 parity in compact mode and in rect mode at several tile shapes: rect
    shapes agree bitwise (same per-node arithmetic), compact within rounding."""
    lid, lv, s = _fp32_case(ctx, graded)
    ops = fem.operators(lv)
    shapes = [(48, 48), (64, 16), (24, 40)] if not graded else [(16, 16), (32, 8), (8, 24)]
    ref = None
    for tx, ty in shapes:
        ctx.set_tiling(lid, tx, ty, True)
        q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        if ref is None:
            ref = q
        assert np.array_equal(q, ref), (tx, ty)
    # coarse items and fine tiles in one launch: the same per-node arithmetic
    ctx.set_tiling(lid, *shapes[0], True)
    q32 = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP)
    _, g = ctx.backward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], np.ones(len(ref)), K=7)
    assert ctx.set_tiling(lid, *shapes[0], True, mix=True)["tile_rect"] == 2
    assert np.array_equal(ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"]), ref)
    assert np.array_equal(ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], plain=True), ref)
    assert np.array_equal(ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP),
                          q32)
    _, gm = ctx.backward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], np.ones(len(ref)), K=7)
    assert np.array_equal(gm, g)
    ctx.set_tiling(lid, *shapes[0], False)
    qc = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    for k in range(len(qc)):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(s["n_steps"][k]), s["dt"][k])
        check(qc[k], qo, sc)
        check(ref[k], qo, sc)
    for bad in [(0, 8), (8, 5000)]:
        with pytest.raises(P.LtsError):
            ctx.set_tiling(lid, *bad, True)
    big = ctx.add_rect_level(P.box_rule(128))      # 200 x 200 tiles: region beyond one workgroup
    for rect in (True, False):
        with pytest.raises(P.LtsError):
            ctx.set_tiling(big, 200, 200, rect)


@pytest.mark.parametrize("graded", [False, True])
def test_adaptive_tiling(ctx, graded):
    """The adaptive compact tiling (recursive bisection of F+): same QoIs, bit
    for bit, as a uniform compact tiling (a tiling only decides which workgroup
    updates a node), oracle parity, and rect mode refused."""
    lid, lv, s = _fp32_case(ctx, graded)
    ops = fem.operators(lv)
    ctx.set_tiling(lid, *((16, 16) if graded else (48, 48)), False)
    qu = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    info = ctx.set_tiling(lid, 0, 0, False)
    assert (info["tile_x"], info["tile_y"], info["tile_rect"]) == (0, 0, 0)
    qa = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    assert np.array_equal(qa, qu)
    for k in range(len(qa)):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(s["n_steps"][k]), s["dt"][k])
        check(qa[k], qo, sc)
    with pytest.raises(P.LtsError):
        ctx.set_tiling(lid, 0, 0, True)


def test_adaptive_tiling_halo(ctx):
    """On a graded L-shape level (F+ a cross of thin bands, p = 64) the adaptive
    tiling needs far fewer region nodes than square tiles."""
    lid = ctx.add_rect_level(P.graded_L_rule(256))
    square = ctx.set_tiling(lid, 40, 40, False)["halo_ratio"]
    adaptive = ctx.set_tiling(lid, 0, 0, False)["halo_ratio"]
    print(f"halo ratio: 40 x 40 tiles {square:.3f}, adaptive {adaptive:.3f}")
    assert adaptive < 0.6 * square


@pytest.mark.parametrize("precision", [P.LTS_FP64, P.LTS_FP32_STEP])
def test_compact_workgroup_size_does_not_change_results(ctx, precision):
    """A sample's QoI does not depend on what it is batched with: the first
    samples solved alone (1024-thread compact workgroups) and at the head of a
    700-sample batch (256- and 512-thread workgroups while many are active)
    agree bit for bit, in FP64 and in FP32 stepping."""
    lid = ctx.add_rect_level(P.graded_L_rule(32))
    info = ctx.set_tiling(lid, 0, 0, False)          # one 777-node region: 256-thread workgroups fit
    assert info["tile_rect"] == 0
    r = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    s = P.gen_samples(2, 0, 0, 700, r, 1 / 16)
    big = np.asarray(ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=precision))
    k = 5
    small = np.asarray(ctx.forward(lid, s["kappa"][:k], s["x0"][:k], s["n_steps"][:k], s["dt"][:k],
                                   precision=precision))
    assert np.array_equal(big[:k], small)
    assert np.isfinite(big).all()


def test_compact_mode_beyond_rect_p128(ctx):
    """p = 128 (seven graded layers), beyond what rect mode allows: compact
    tiles against the oracle, the batched form bit for bit against one solve,
    and rect mode refused."""
    lid = ctx.add_rect_level(P.graded_L_rule(16, layers=7))
    info = ctx.level_info(lid)
    assert info["p"] == 128 and info["tile_rect"] == 0
    with pytest.raises(P.LtsError):
        ctx.set_tiling(lid, 16, 16, True)
    ctx.autotune(lid)
    lv = mesh.graded_L_level(16, layers=7)
    ops = fem.operators(lv)
    r = P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=2.0)
    s = P.gen_samples(3, 0, 0, 6, r, lv.h)
    q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
    qb = ctx.batch_run([(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], 0.05)], graph=True)
    assert np.array_equal(np.asarray(q), np.asarray(qb))
    for k in range(2):
        qo, sc = oracle_solve(ops, lv, s["kappa"][k], s["x0"][k], int(s["n_steps"][k]), s["dt"][k])
        check(q[k], qo, sc)
