"""Pins of the oracle's multi-level LTS (oracle/mlts.py; Sec. 3.5, closing
remark: tiers of equally sized elements, each stepping with its own step).

The scheme is a reading (Algorithm 2 nested once per tier), so it is pinned to
what must hold whatever the nesting details: one tier is Algorithm 2; an
inner tier without stiffness or with one stage changes nothing; the stages of
Algorithm 2 share one half step (the Chebyshev identity the nesting rests
on); the effective operator is M-self-adjoint with its spectrum inside the
leapfrog stability interval at the coarse step, where plain leapfrog and
one-tier LTS with the outer ratio alone are unstable; the discrete energy is
conserved; and the error against the exact semi-discrete solution (from an
eigendecomposition) falls by four when the step is halved."""
import math

import numpy as np
import pytest

from oracle import cheby, fem, lts, mesh, mlts, rng


def _setup(lv, n_tiers, seed=3):
    ops = fem.operators(lv)
    kap = np.exp(2 * np.random.default_rng(seed).normal(0, 0.3, lv.n_blocks))
    ct = mlts.tiers_by_leg(lv, n_tiers)
    return ops, kap, mlts.tier_projectors(lv, ct, n_tiers)


def _G(s, dt, n):
    """The effective operator G y = -(2/dt^2) E_1(A y), column by column."""
    return np.stack([-2.0 * s.d1(np.eye(n)[k], dt) / (dt * dt) for k in range(n)], axis=1)


def test_tier_sets_by_brute_force():
    """tiers_by_leg and tier_projectors against loops over cells and
    triangles; the sets are nested and P_1 is the level's P."""
    lv = mesh.graded_L_level(8)
    T = 5
    ct = mlts.tiers_by_leg(lv, T)
    hx, hy = np.diff(lv.xs), np.diff(lv.ys)
    for b in range(len(hy)):
        for a in range(len(hx)):
            want = 0
            if lv.cell_active[b, a] and lv.cell_fine[b, a]:
                leg = min(hx[a], hy[b])
                want = 1 + sum(1 for j in range(2, T + 1) if leg < lv.h / 2 ** j)
            assert ct[b, a] == want
    Ps = mlts.tier_projectors(lv, ct, T)
    ids = list(lv.dof_ids)
    for j in range(1, T + 1):
        want = np.zeros(lv.n_dof)
        for t, c in zip(lv.tris, lv.tri_cell):
            if ct.ravel()[c] >= j:
                for v in t:
                    if v in ids:
                        want[ids.index(v)] = 1.0
        assert np.array_equal(Ps[j - 1], want)
        if j > 1:
            assert np.all(Ps[j - 1] <= Ps[j - 2]) and Ps[j - 1].sum() < Ps[j - 2].sum()
    assert np.array_equal(Ps[0], fem.operators(lv).Pd)
    # on the graded L-shape tier j holds exactly the cells of shorter leg h 2^-(j+1) and below
    legs = np.minimum.outer(hy, hx)
    for j in range(1, T):
        sel = (ct == j) & lv.cell_active
        assert np.all(np.isclose(legs[sel], lv.h * 2.0 ** -(j + 1)))


def test_one_tier_is_algorithm_2():
    """T = 1 with p_1 = p is the increment form of Algorithm 2 (``lts``),
    up to the rounding of A z + A P d against w + A P (z + d)."""
    for lv, T_end in [(mesh.box_refined_level(16), 0.6), (mesh.graded_L_level(16), 0.5)]:
        ops = fem.operators(lv)
        rule = rng.SampleRule(T=T_end, n_blocks=lv.n_blocks)
        smp = rng.draw(0, 0, 2, rule)
        n, dt = rng.steps_for(smp, rule, lv.h)
        u0 = lts.pulse(ops, smp.x0)
        a = lts.Solver(ops, smp.kappa).run(u0, dt, n)
        b = mlts.MltsSolver(ops, smp.kappa, [ops.Pd], [lv.p]).run(u0, dt, n)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_empty_or_one_stage_inner_tier_changes_nothing():
    """An inner tier whose set is empty (A P_2 = 0: the recurrence is exact
    for a constant force) or that has one stage gives the one-tier scheme."""
    lv = mesh.graded_L_level(16)
    ops, kap, Ps = _setup(lv, 2)
    rule = rng.SampleRule(T=0.3, n_blocks=lv.n_blocks)
    smp = rng.draw(0, 0, 5, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    u0 = lts.pulse(ops, smp.x0)
    one = mlts.MltsSolver(ops, smp.kappa, [ops.Pd], [64]).run(u0, dt, n)
    empty = mlts.MltsSolver(ops, smp.kappa, [ops.Pd, np.zeros(lv.n_dof)], [64, 3]).run(u0, dt, n)
    single = mlts.MltsSolver(ops, smp.kappa, Ps, [64, 1]).run(u0, dt, n)
    sc = np.max(np.abs(one))
    assert np.max(np.abs(empty - one)) <= 1e-12 * sc
    assert np.max(np.abs(single - one)) <= 1e-12 * sc
    # ... while a real inner tier does change the solution
    two = mlts.MltsSolver(ops, smp.kappa, Ps, [32, 2]).run(u0, dt, n)
    assert np.max(np.abs(two - one)) > 1e-9 * sc


@pytest.mark.parametrize("nu", [0.0, 0.01, 0.3, 1.0])
@pytest.mark.parametrize("p", [2, 3, 5, 8, 64])
def test_stages_share_one_half_step(p, nu):
    """c_m = (1 + beta_m) c_0 for m >= 1 (T_{m+1} + T_{m-1} = 2 delta T_m),
    so every stage of Algorithm 2 is built on the half step of time
    sqrt(2 c_0) that MLTS hands to the inner tier."""
    cc = cheby.cheb_consts(p, nu)
    c0 = 0.5 / (cc.omega * cc.delta)
    for m in range(1, p):
        cm = cc.beta_half[m] / cc.omega
        assert abs(cm - (1.0 + cc.beta[m]) * c0) <= 1e-14 * cm


@pytest.mark.parametrize("layers,ps", [(6, [2, 2, 2, 2, 2]), (4, [3, 2, 2]), (4, [2, 3, 2])])
def test_effective_operator_self_adjoint_and_stable(layers, ps):
    """M G symmetric; dt^2 G has its spectrum in (0, 4) at dt = 0.2 h / c_max,
    the coarse step, where plain leapfrog is unstable (and, with six layers
    of grading, so is the outer tier alone)."""
    lv = mesh.graded_L_level(8, layers=layers)
    ops, kap, Ps = _setup(lv, len(ps))
    n = lv.n_dof
    dt = 0.2 * lv.h / math.sqrt(kap.max())
    G = _G(mlts.MltsSolver(ops, kap, Ps, ps), dt, n)
    MG = ops.m[:, None] * G
    assert np.max(np.abs(MG - MG.T)) <= 1e-13 * np.max(np.abs(MG))
    sm = np.sqrt(ops.m)
    S = (sm[:, None] * G) / sm[None, :]
    ev = np.linalg.eigvalsh(0.5 * (S + S.T)) * dt * dt
    assert ev.min() > 0.0 and ev.max() < 4.0
    A = fem.sym_operator(ops, kap).toarray()
    assert np.linalg.eigvalsh(A).max() * dt * dt > 4.0
    if layers == 6:
        # cells down to h/64: tier 1 alone (p_1 = 2) is not enough
        G1 = _G(mlts.MltsSolver(ops, kap, Ps[:1], ps[:1]), dt, n)
        S1 = (sm[:, None] * G1) / sm[None, :]
        ev1 = np.linalg.eigvalsh(0.5 * (S1 + S1.T)) * dt * dt
        assert ev1.min() < 0.0 or ev1.max() >= 4.0


def test_energy_conserved():
    lv = mesh.graded_L_level(16)
    ops, _, Ps = _setup(lv, 5)
    rule = rng.SampleRule(T=1.0, n_blocks=lv.n_blocks)
    smp = rng.draw(0, 0, 1, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    s = mlts.MltsSolver(ops, smp.kappa, Ps, [2, 2, 2, 2, 2])
    _, zs = s.run(lts.pulse(ops, smp.x0), dt, n, keep=True)
    E = np.array([s.energy(zs[k + 1], zs[k], dt) for k in range(0, n, 3)])
    assert np.max(np.abs(E - E[0])) <= 1e-12 * E[0]


def test_second_order_against_exact_semi_discrete_solution():
    """u(t) = M^-1/2 cos(t S^1/2) M^1/2 u_0 with S = M^-1/2 K M^-1/2 (exact in
    time); the MLTS error at T falls by about 4 per halving of dt, and is as
    small as that of one-tier LTS with p = 64 at the same dt."""
    lv = mesh.graded_L_level(8)
    ops, kap, Ps = _setup(lv, 5)
    w, V = np.linalg.eigh(fem.sym_operator(ops, kap).toarray())
    sm = np.sqrt(ops.m)
    u0 = lts.pulse(ops, (-0.5, 0.5), 0.3)
    T_end = 0.5
    exact = (V @ (np.cos(T_end * np.sqrt(w)) * (V.T @ (sm * u0)))) / sm
    s = mlts.MltsSolver(ops, kap, Ps, [2, 2, 2, 2, 2])
    s1 = lts.Solver(ops, kap)
    n0 = int(math.ceil(T_end * math.sqrt(kap.max()) / (0.2 * lv.h)))
    err, err1 = [], []
    for k in (1, 2, 4):
        n = n0 * k
        e = s.run(u0, T_end / n, n) - exact
        e1 = s1.run(u0, T_end / n, n) - exact
        err.append(math.sqrt(e @ (ops.m * e)))
        err1.append(math.sqrt(e1 @ (ops.m * e1)))
    for a, b in zip(err, err[1:]):
        assert 3.4 < a / b < 4.6
    for a, b in zip(err, err1):
        assert a < 2.0 * b
