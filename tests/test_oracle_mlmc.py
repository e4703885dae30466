"""Pins of the oracle's Algorithm 1 (Sec. 2.2) by closed forms.

The level differences here are synthetic sequences whose sample means and
unbiased variances are known exactly, so the sample sizes of eq. (optimal
N_l), the bias estimate of eq. (bias_est) and the level L where the bias test
passes follow by hand.  The cost model is pinned against eq.
(cost_waveeq_LTS) and eq. (C_l_LTS) on a mesh whose fine DOFs are counted by
hand.
"""
from __future__ import annotations

import math

import pytest

from oracle import fem, mesh, mlmc, rng


def _alternating(m: float, s: float):
    """Delta Q(i) = m + s (-1)^i: every even-length prefix has mean m exactly
    (m +- s dyadic) and unbiased variance s^2 N/(N-1)."""
    return lambda i: m + (s if i % 2 == 0 else -s)


def _unit_variance_sequence(n: int):
    """r_0 = 0, r_N = mean(r_0..r_{N-1}) +- sqrt((N+1)/N): each new term adds
    exactly 1 to the sum of squared deviations (Welford's update
    M2_{N+1} = M2_N + (x - mean_N)^2 N/(N+1)), so every prefix of length
    N >= 2 has unbiased sample variance 1."""
    r = [0.0]
    for N in range(1, n):
        mu = math.fsum(r) / N
        r.append(mu + (1.0 if N % 2 else -1.0) * math.sqrt((N + 1) / N))
    return r


def test_unit_variance_sequence_is_unit_variance():
    r = _unit_variance_sequence(600)
    for N in (2, 3, 7, 64, 599, 600):
        _, v = mlmc.mean_var(r[:N])
        assert abs(v - 1.0) < 1e-12


def test_alg1_bias_test_adds_exactly_the_needed_levels():
    """Means 4^-l: the bias estimate at L is 4^-L / (2^2 - 1).  With
    eps/sqrt(2) = 0.018 the test fails at L = 2 (1/48 = 0.0208) and passes at
    L = 3 (1/192 = 0.0052), so Algorithm 1 started at L = 2 ends at L = 3 of a
    five-level hierarchy, and level 4 is never sampled.  The variances are so
    small that eq. (optimal N_l) asks for fewer than N_init = (8, 8, 8, 6, 4)
    samples on every level (ceil(2/eps^2 * 2^-18 * 8/7 * sum sqrt(C) /
    sqrt(C_0)) = 1), so N stays at N_init; a level added by the bias test
    starts at its own N_init."""
    s = 2.0 ** -9
    m = [4.0 ** -l for l in range(5)]
    seqs = [_alternating(m[l], s) for l in range(5)]
    calls = []

    def eval_dq(l, i):
        calls.append(l)
        return seqs[l](i)

    eps = 0.018 * math.sqrt(2.0)
    C = [1.0, 5.0, 20.0, 80.0, 320.0]
    res = mlmc.mlmc([None] * 5, None, eps, N_init=(8, 8, 8, 6, 4), L_start=2, eval_dq=eval_dq, costs=C)
    assert res.L == 3
    assert res.N == [8, 8, 8, 6]
    assert 4 not in calls
    assert res.mean == m[:4]
    V = [s * s * n / (n - 1.0) for n in (8, 8, 8, 6)]
    for v, ve in zip(res.var, V):
        assert abs(v - ve) <= 1e-15 * ve
    assert res.estimate == 1.0 + 0.25 + 0.0625 + 0.015625
    assert res.bias == (1.0 / 64.0) / 3.0
    assert abs(res.rmse - math.sqrt(sum(v / n for v, n in zip(V, (8, 8, 8, 6))) + res.bias ** 2)) <= 1e-15
    # eq. (bias_est) with alpha = 1 and eps/sqrt(2) = 0.01: the bias 4^-L / 1
    # passes only at L = 4 (1/256 = 0.0039 < 0.01 < 1/64), the top level
    res1 = mlmc.mlmc([None] * 5, None, 0.01 * math.sqrt(2.0), N_init=(8, 8, 8, 6, 4), alpha=1.0, L_start=2,
                     eval_dq=eval_dq, costs=C)
    assert res1.L == 4 and res1.N == [8, 8, 8, 6, 4] and res1.bias == 1.0 / 256.0
    # a bias test that passes at once: L stays at L_start
    res2 = mlmc.mlmc([None] * 5, None, 0.1, N_init=(8,) * 5, L_start=2, eval_dq=eval_dq, costs=C)
    assert res2.L == 2 and res2.N == [8, 8, 8]


def test_alg1_level_cap():
    """The bias test still fails at the top level: L stops at the hierarchy's
    depth and the result reports the failing bias (1/16 / 3 >= eps/sqrt 2)."""
    seqs = [_alternating(4.0 ** -l, 2.0 ** -9) for l in range(3)]
    res = mlmc.mlmc([None] * 3, None, 0.02, N_init=(8, 8, 8), L_start=1,
                    eval_dq=lambda l, i: seqs[l](i), costs=[1.0, 1.0, 1.0])
    assert res.L == 2 and res.N == [8, 8, 8]
    assert res.bias == 0.0625 / 3.0
    assert res.bias ** 2 >= 0.5 * 0.02 ** 2


def test_alg1_sample_sizes_closed_form():
    """Unit-variance sequences scaled by s_l = (1, 1/2, 1/4) give V_l = s_l^2
    for every N, with costs C_l = (1, 4, 16): sqrt(V C) = 1 on every level, so
    eq. (optimal N_l) gives N_l = ceil(2/eps^2 * 3 * s_l / sqrt(C_l)) =
    ceil(600/(100 eps^2) * (1, 1/4, 1/16)).  eps = 0.11 gives
    (495.87.., 123.96.., 30.99..) -> (496, 124, 31) after one update, and the
    next pass leaves them unchanged.  The top level has mean 0, so the bias
    test passes at L = 2."""
    r = _unit_variance_sequence(600)
    sc = [1.0, 0.5, 0.25]
    mu = [3.0, -1.0, 0.0]
    res = mlmc.mlmc([None] * 3, None, 0.11, N_init=(16, 8, 4), L_start=2,
                    eval_dq=lambda l, i: mu[l] + sc[l] * r[i], costs=[1.0, 4.0, 16.0])
    assert res.L == 2
    assert res.N == [496, 124, 31]
    for l in range(3):
        assert abs(res.var[l] - sc[l] ** 2) <= 1e-12
    # the stochastic error then meets eps^2/2
    assert sum(v / n for v, n in zip(res.var, res.N)) <= 0.5 * 0.11 ** 2


def test_cost_model_counts_dof_updates():
    """eq. (cost_waveeq_LTS): per coarse step, one update of each coarse DOF
    and p updates of each fine DOF.  8 base cells, box (0.45, 0.55) refined
    4x: the intervals [0.375, 0.5] and [0.5, 0.625] split, 15 nodes per axis,
    13 x 13 = 169 DOFs.  Fine cells lie in columns or rows 3..10, so a DOF is
    in P iff its column or row index lies in 3..11: all but 4 x 4 = 16 DOFs.
    p = ceil(h / (h/4)) = 4, so a step is 16 + 4 * 153 = 628 updates; with
    T = 0.99 and dt = 0.2 h there are ceil(39.6) = 40 steps.  eq. (C_l_LTS):
    a level-l sample costs a solve on mesh l plus one on mesh l-1."""
    rule = rng.SampleRule(T=0.99)
    lv = mesh.box_refined_level(8, box=(0.45, 0.55), ref=4)
    assert lv.n_dof == 169 and int((lv.Pmask & lv.dof).sum()) == 153 and lv.p == 4
    ops = fem.operators(lv)
    assert mlmc.cost_per_solve(ops, rule) == 40 * 628
    lv2 = mesh.box_refined_level(16, box=(0.45, 0.55), ref=4)
    ops2 = fem.operators(lv2)
    C = mlmc.level_costs([ops, ops2], rule)
    assert C == [40 * 628, 40 * 628 + mlmc.cost_per_solve(ops2, rule)]


@pytest.mark.parametrize("graded", [False, True])
def test_cost_model_of_leapfrog_twin(graded):
    """Sec. 3.4: plain leapfrog at step dt/p updates every DOF once per step,
    p times as many steps: the twin's cost is p n_nominal N."""
    rule = rng.SampleRule(T=0.99) if not graded else rng.SampleRule(T=0.5, cfl=0.2)
    lv = mesh.graded_L_level(8, layers=3) if graded else mesh.box_refined_level(8, box=(0.45, 0.55), ref=4)
    tw = mesh.lf_twin(lv)
    ops = fem.operators(tw)
    steps = math.ceil(rule.T / (rule.cfl * lv.h / lv.p))
    assert mlmc.cost_per_solve(ops, rule) == steps * lv.n_dof


def test_mlmc_gradient_is_the_derivative_of_the_estimator():
    """The MLMC gradient estimate sum_l mean_i (dQ_l/dg_b - dQ_{l-1}/dg_b) is the
    derivative of the MLMC estimate itself when every sample's g_b is shifted
    by the same amount (N_l, L, step counts and dt held fixed): central
    differences of the estimator, computed from forward solves only, match it.
    A dropped coarse term, a wrong sign or a wrong per-level average fails."""
    import numpy as np
    from oracle import lts
    T = 0.25
    levels = [8, 16]
    ops = [fem.operators(mesh.box_refined_level(nb)) for nb in levels]
    rule = rng.SampleRule(T=T)
    res, est, means, _ = mlmc.mlmc_grad(ops, rule, eps=2e-3, seed=0, N_init=(6, 4), L_start=1, K=8)
    assert res.L == 1
    d = 1e-6

    def estimate(b, shift):
        tot = 0.0
        for l in range(res.L + 1):
            acc = []
            for i in range(res.N[l]):
                smp = rng.draw(0, l, i, rule)
                kap = list(smp.kappa)
                kap[b] *= math.exp(2.0 * shift)           # g_b -> g_b + shift
                q = []
                for o in ([ops[l], ops[l - 1]] if l > 0 else [ops[l]]):
                    n, dt = rng.steps_for(smp, rule, o.lv.h)
                    u = lts.Solver(o, kap).run(lts.pulse(o, smp.x0), dt, n)
                    q.append(float(lts.qoi(o, u)))
                acc.append(q[0] - (q[1] if l > 0 else 0.0))
            tot += math.fsum(acc) / len(acc)
        return tot
    scale = max(abs(v) for v in est)
    for b in (0, 5, 10, 15):
        fd = (estimate(b, d) - estimate(b, -d)) / (2 * d)
        assert abs(fd - est[b]) <= 1e-6 * scale, (b, fd, est[b])
    assert np.allclose(est, np.sum(np.array(means), axis=0), rtol=0, atol=1e-15 * scale)
