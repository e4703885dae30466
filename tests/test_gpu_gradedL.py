"""GPU parity on the graded L-shape hierarchy at the workload's horizon T = 2.

The L-shape [-1,1]^2 minus (0,1]x[-1,0], spacing graded toward the reentrant
corner (6 layers of ratio 1/2, smallest cell h/64, so p = 64 on every level,
Sec. 3.5), levels with 32, 64, 128, 256, 512 cells across, 8x8 blocks of
g ~ N(0, 0.3^2), pulse centred in [-0.8,-0.4]x[0.4,0.8], QoI over
[0.5,0.9]x[0.2,0.6].  At T = 2 the pulse has crossed the graded corner and
reached the QoI box (|Q| of order 1e-3), so these cases compare the solution
itself, not a precursor tail.

Levels 0-2 are checked against the oracle run live (in worker processes),
levels 3-4 against stored oracle values (tests/golden/gradedL_qoi.json,
written by tests/golden/make_gradedL_golden.py, which calls only the oracle).
Each level is autotuned first, so the tiling the solves run on is the one the
batched and MLMC forms use (compact adaptive tiles on the finer levels).
Metric as in the other parity tests: |Q_gpu - Q_oracle| <= 1e-11 sum_i w_i |u_i|
(FP64), and the derived FP32-stepping bound.
"""
import json
import os

import numpy as np
import pytest

import paper_2106_11117_amd as P
import oracle_jobs

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(__file__)
BASES = (32, 64, 128, 256, 512)
T_END = 2.0
TOL = 1e-11
LIVE = {0: (0, 1, 2, 3), 1: (0, 1, 2, 3), 2: (0, 1, 2)}      # level -> sample indices
LF_LIVE = {0: (0, 1), 1: (0, 1), 2: (0,)}
BATCH = 16


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rule(T=T_END):
    return P.sample_rule(n_blocks=64, sigma=0.3, pulse=(-0.8, -0.4, 0.4, 0.8), T=T)


def _fp32_bound(n_steps, p):
    return 4.0 * n_steps * p * 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    _torch()
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def levels(ctx):
    ids = []
    for b in BASES:
        lid = ctx.add_rect_level(P.graded_L_rule(b))
        ctx.autotune(lid)
        ids.append(lid)
    return ids


@pytest.fixture(scope="module")
def oracle():
    """Every live oracle solve of this module, in one pool of worker processes."""
    jobs = [("fwd", BASES[l], l, i, T_END, False) for l, ii in LIVE.items() for i in ii]
    jobs += [("fwd", BASES[l], l, i, T_END, True) for l, ii in LF_LIVE.items() for i in ii]
    jobs += [("adj", 32, 0, i, T_END, 64) for i in (0, 1)]
    jobs += [("adj", 64, 1, 0, T_END, 64)]
    print(f"oracle: {len(jobs)} solves in worker processes", flush=True)
    res = oracle_jobs.run_all(jobs)
    return {j[:4] + (j[5],): r for j, r in zip(jobs, res)}


def _check(q, ref, tol=TOL):
    e = abs(q - ref["Q"]) / ref["abs_wu"]
    assert e <= tol, (q, ref["Q"], e)
    if abs(ref["Q"]) >= 1e-3 * ref["abs_wu"]:
        assert abs(q - ref["Q"]) / abs(ref["Q"]) <= tol
    return e


def test_levels_0_2_at_T2(ctx, levels, oracle):
    worst = 0.0
    for l, ii in LIVE.items():
        lid = levels[l]
        info = ctx.level_info(lid)
        s = P.gen_samples(0, l, 0, BATCH, _rule(), info["h"])
        q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        q32 = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP)
        for i in ii:
            ref = oracle[("fwd", BASES[l], l, i, False)]
            assert int(s["n_steps"][i]) == ref["n_steps"]
            assert abs(ref["Q"]) > 1e-2 * ref["abs_wu"]        # the wave has reached the QoI box
            worst = max(worst, _check(q[i], ref))
            assert abs(q32[i] - ref["Q"]) <= _fp32_bound(ref["n_steps"], info["p"]) * ref["abs_wu"]
        print(f"level {l}: tiling {info['tile_x']}x{info['tile_y']} rect={info['tile_rect']}, "
              f"worst FP64 error {worst:.2e}")


def test_levels_3_4_at_T2_golden(ctx, levels):
    path = os.path.join(HERE, "golden", "gradedL_qoi.json")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    gold = json.load(open(path))
    assert gold["batch"] == BATCH
    for l in (3, 4):
        lid = levels[l]
        info = ctx.level_info(lid)
        assert info["tile_rect"] == 0        # the autotuned compact tiling
        s = P.gen_samples(0, l, 0, BATCH, _rule(), info["h"])
        # a batch this small has fewer fine workgroups than CUs: 1024-thread workgroups
        q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        q32 = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], precision=P.LTS_FP32_STEP)
        rows = [r for r in gold["samples"] if r["level"] == l]
        assert rows
        for r in rows:
            i = r["i"]
            assert int(s["n_steps"][i]) == r["n_steps"] and s["dt"][i] == r["dt"]
            e = _check(q[i], r)
            assert abs(q32[i] - r["Q"]) <= _fp32_bound(r["n_steps"], info["p"]) * r["abs_wu"]
            print(f"level {l} sample {i}: Q {q[i]:.15e} oracle {r['Q']:.15e} rel {e:.2e}")


def test_batched_all_levels_at_T2(ctx, levels, oracle):
    """All five levels in shared launches, graph captured: the per-level solves'
    QoIs bit for bit, and the oracle's where it is known."""
    path = os.path.join(HERE, "golden", "gradedL_qoi.json")
    gold = json.load(open(path))["samples"] if os.path.exists(path) else []
    jobs, samples = [], []
    for l, lid in enumerate(levels):
        s = P.gen_samples(0, l, 0, BATCH, _rule(), ctx.level_info(lid)["h"])
        jobs.append((lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], 0.05))
        samples.append(s)
    qb = ctx.batch_run(jobs, graph=True)
    for l, lid in enumerate(levels):
        s = samples[l]
        ql = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        assert np.array_equal(qb[l * BATCH:(l + 1) * BATCH], ql)
        for i in LIVE.get(l, ()):
            _check(ql[i], oracle[("fwd", BASES[l], l, i, False)])
        for r in gold:
            if r["level"] == l:
                _check(ql[r["i"]], r)


def test_lf_twins_at_T2(ctx, oracle):
    """The standard leapfrog twins (P empty, p = 1, step dt/64) of levels 0-2."""
    for l, ii in LF_LIVE.items():
        lid = ctx.add_rect_level(P.lf_rule(P.graded_L_rule(BASES[l])))
        s = P.gen_samples(0, l, 0, 4, _rule(), ctx.level_info(lid)["h"])
        q = ctx.forward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"])
        for i in ii:
            ref = oracle[("fwd", BASES[l], l, i, True)]
            assert int(s["n_steps"][i]) == ref["n_steps"]
            _check(q[i], ref)


@pytest.mark.parametrize("l,K,mode", [(0, 7, "rect"), (0, 64, "rect"), (0, 7, "compact"),
                                      (0, 64, "adaptive"), (1, 64, "adaptive"), (1, 7, "compact")])
def test_adjoint_p64_at_T2(ctx, oracle, l, K, mode):
    """Backward LF-LTS at p = 64 on graded levels 0-1 (the fused rect-tile step,
    and the per-substep kernels of compact and adaptive tilings) against the
    oracle's discrete adjoint."""
    lid = ctx.add_rect_level(P.graded_L_rule(BASES[l]))
    info = ctx.level_info(lid)
    if mode == "rect":
        ctx.set_tiling(lid, info["nx_nodes"], info["ny_nodes"], True)
    elif mode == "compact":
        ctx.set_tiling(lid, 16, 16, False)
    else:
        ctx.set_tiling(lid, 0, 0, False)
    ii = (0, 1) if l == 0 else (0,)
    s = P.gen_samples(0, l, 0, 2, _rule(), info["h"])
    dl = np.array([1.0, -0.5])
    q, g = ctx.backward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], dl, K=K)
    for i in ii:
        ref = oracle[("adj", BASES[l], l, i, 64)]
        go = np.asarray(ref["g"])
        assert abs(q[i] - ref["Q"]) <= 1e-11 * abs(ref["Q"])
        err = np.max(np.abs(g[i] - dl[i] * go)) / np.max(np.abs(dl[i] * go))
        assert err <= 1e-10, (i, err)


def test_adjoint_p64_vs_finite_differences(ctx, levels):
    """Central differences (step 1e-6, dt and step counts fixed) of the GPU QoI on
    graded level 1 at T = 2 against the adjoint gradient, 2 samples x 64 blocks."""
    lid = levels[1]
    s = P.gen_samples(0, 1, 0, 2, _rule(), ctx.level_info(lid)["h"])
    _, g = ctx.backward(lid, s["kappa"], s["x0"], s["n_steps"], s["dt"], np.ones(2), K=64)
    eps = 1e-6
    gl = np.log(s["kappa"]) / 2
    kp, x0, ns, dt = [], [], [], []
    for k in range(2):
        for b in range(64):
            for sgn in (1.0, -1.0):
                gg = gl[k].copy()
                gg[b] += sgn * eps
                kp.append(np.exp(2 * gg))
                x0.append(s["x0"][k])
                ns.append(s["n_steps"][k])
                dt.append(s["dt"][k])
    qq = ctx.forward(lid, np.array(kp), np.array(x0), np.array(ns, dtype=np.int32), np.array(dt))
    fd = ((qq[0::2] - qq[1::2]) / (2 * eps)).reshape(2, 64)
    for k in range(2):
        e = np.max(np.abs(g[k] - fd[k])) / np.max(np.abs(fd[k]))
        assert e <= 1e-5, (k, e)
