"""Pins of the oracle's choice of the fine set on graded meshes (Sec. 3.5) and
of Algorithm 1 on a hierarchy built level by level (Sec. 2.2).

The paper's cost model of one LTS solve on the radially graded mesh
T_{m,s} with q fine layers (eq. cost_waveeq_LTSgraded), the resulting speed-up
over leapfrog (eq. speedup_det_graded), the derivative condition for the
optimal q (eq. ddqS) and its asymptotics (eq. LTSgraded_qopt) are transcribed
separately in the oracle; these tests tie them to each other and to brute
force, so that a wrong sign or exponent in any one of them fails.  The tier
family on the rectilinear graded L-shape is pinned to the workload's level and
to a count by hand.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import mesh, mlmc, rng

CASES = [(10, 2.0, 2), (40, 2.0, 2), (100, 3.0, 2), (50, 2.0, 3), (200, 1.5, 2), (30, 2.0, 1), (500, 2.5, 3)]


@pytest.mark.parametrize("m,s,d", CASES)
def test_speedup_is_lf_cost_over_lts_cost(m, s, d):
    """eq. speedup_det_graded equals eq. cost_waveeq_LFgraded (m^(s+d)) over eq.
    cost_waveeq_LTSgraded, and q = m (everything fine) gives no speed-up."""
    for q in (1, 2, 3, m // 3, m - 1):
        c = mesh.cost_lts_graded_model(m, s, d, q)
        assert abs(mesh.speedup_graded_model(m, s, d, q) - m ** (s + d) / c) <= 1e-12 * (m ** (s + d) / c)
    # all m layers fine: the LTS cost is m^d elements at the smallest step h_1 ~ m^-s
    top = mesh.cost_lts_graded_model(m, s, d, m)
    g = (m + 1.0) ** s - m ** s
    assert abs(top - (m ** (s + d) + m ** (s + d) * (g - 1.0)) / g) <= 1e-12 * top
    assert abs(mesh.speedup_graded_model(m, s, d, m) - 1.0) <= 1e-12


@pytest.mark.parametrize("m,s,d", CASES)
def test_integer_optimum_sits_at_the_sign_change_of_ddqS(m, s, d):
    """Brute force over q = 1..m: the q with the largest speed-up is where the
    left-hand side of eq. ddqS (the q-derivative of the speed-up, up to a
    positive factor) changes sign, and it lies strictly inside (1, m)."""
    qs = np.arange(1, m + 1)
    S = np.array([mesh.speedup_graded_model(m, s, d, q) for q in qs])
    qstar = int(qs[np.argmax(S)])
    assert 1 < qstar < m
    assert mesh.ddq_speedup_graded_model(m, s, d, qstar - 1) > 0
    assert mesh.ddq_speedup_graded_model(m, s, d, qstar + 1) < 0
    # the real root by bisection lies within one of the integer optimum
    lo, hi = 1.0, float(m)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mesh.ddq_speedup_graded_model(m, s, d, mid) > 0:
            lo = mid
        else:
            hi = mid
    assert math.floor(lo) <= qstar <= math.ceil(lo)
    # the derivative matches a central difference of the speed-up in sign and
    # up to the positive factor m^d / denominator^2
    for q in (qstar - 0.5, qstar + 0.5, 1.5):
        g = (q + 1.0) ** s - q ** s
        den = m ** d + q ** d * (g - 1.0)
        h = 1e-6 * q
        fd = (mesh.speedup_graded_model(m, s, d, q + h) - mesh.speedup_graded_model(m, s, d, q - h)) / (2 * h)
        an = mesh.ddq_speedup_graded_model(m, s, d, q) * m ** d / den ** 2
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-12


@pytest.mark.parametrize("s,d", [(2.0, 2), (2.0, 3), (3.0, 2), (1.5, 2)])
def test_optimal_q_grows_like_m_to_d_over_d_plus_s_minus_1(s, d):
    """eq. LTSgraded_qopt: for large m the root of eq. ddqS behaves like
    ((s-1) m^d / (s d))^(1/(d+s-1)) (the balance of its two leading terms)."""
    def root(m):
        lo, hi = 1.0, float(m)
        for _ in range(300):
            mid = math.sqrt(lo * hi)
            if mesh.ddq_speedup_graded_model(m, s, d, mid) > 0:
                lo = mid
            else:
                hi = mid
        return lo
    expo = d / (d + s - 1.0)
    for m in (1e5, 1e6):
        pred = ((s - 1.0) * m ** d / (s * d)) ** (1.0 / (d + s - 1.0))
        assert abs(root(m) / pred - 1.0) < 0.05, (m, root(m), pred)
    slope = math.log(root(1e7) / root(1e5)) / math.log(100.0)
    assert abs(slope - expo) < 0.01, (slope, expo)


@pytest.mark.parametrize("n_base", [16, 32])
def test_tier_family_contains_the_workload_level(n_base):
    """q = layers - 1 fine tiers is the workload's graded level exactly: fine
    cells with a leg < h/2, step spacing h, p = ceil(h / h_min) = 64."""
    a = mesh.graded_L_level(n_base)
    t = mesh.graded_L_tiers(n_base, 5)
    assert (t.h, t.p) == (a.h, a.p) == (2.0 / n_base, 64)
    for f in ("cell_fine", "Pmask", "dof", "mass", "qoi_w", "cell_block", "cell_active"):
        assert np.array_equal(getattr(t, f), getattr(a, f)), f


def test_tiers_counted_by_hand():
    """Base 8 on [-1,1] (h = 1/4) with 2 graded layers: per axis the cells are
    three of 1/4, one of 1/8, four of 1/16, one of 1/8, three of 1/4.  Tier 1
    (legs 1/16) is the 4 middle columns and rows, tier 2 (1/8) one more on each
    side.  q = 0: no fine cell, step spacing 2 x 1/16, p = 1; q = 1: spacing
    2 x 1/8, p = 4; q = 2: spacing 2 x 1/4, p = 8.  P: the DOFs that are
    vertices of a fine cell, counted cell by cell."""
    want = {0: (0.125, 1), 1: (0.25, 4), 2: (0.5, 8)}
    for q, (H, p) in want.items():
        lv = mesh.graded_L_tiers(8, q, layers=2)
        assert (lv.h, lv.p) == (H, p)
        xs = lv.xs
        assert list(np.diff(xs)) == [0.25] * 3 + [0.125] + [0.0625] * 4 + [0.125] + [0.25] * 3
        thr = [0.0625, 0.125, 0.25][q]
        P = set()
        nodes = len(xs)
        for b in range(nodes - 1):
            for a in range(nodes - 1):
                mx, my = 0.5 * (xs[a] + xs[a + 1]), 0.5 * (xs[b] + xs[b + 1])
                if mx > 0 and my < 0:
                    continue                     # the removed quadrant
                if min(xs[a + 1] - xs[a], xs[b + 1] - xs[b]) < thr:
                    P.update({(a, b), (a + 1, b), (a, b + 1), (a + 1, b + 1)})
        P = {v for v in P if lv.dof[v[1], v[0]]}
        assert int(lv.Pmask.sum()) == len(P)
        assert bool(lv.cell_fine.any()) == (q > 0)


def test_qopt_minimises_the_cost_rate():
    """The oracle's choice is the argmin of ((N - |P_q|) + p_q |P_q|) / H_q over
    q = 0..layers, recomputed here from the tier levels; on the workload's
    graded hierarchy it grows with the level (coarse levels take fewer tiers)."""
    qs = []
    for n_base in (32, 64, 128):
        q, costs = mesh.qopt_tiers(n_base)
        lvs = [mesh.graded_L_tiers(n_base, k) for k in range(7)]
        rates = [((lv.n_dof - int(lv.Pmask.sum())) + lv.p * int(lv.Pmask.sum())) / lv.h for lv in lvs]
        assert rates == costs
        assert q == int(np.argmin(rates))
        qs.append(q)
    assert qs == sorted(qs) and qs[0] < qs[-1]


class _FakeOps:
    """Stands in for a level's operators in the cost model: N DOFs, |P|, p, h."""

    def __init__(self, n, nP, p, h):
        self.Pd = np.array([1.0] * nP + [0.0] * (n - nP))

        class _L:
            pass
        self.lv = _L()
        self.lv.p, self.lv.h = p, h


def test_algorithm1_builds_levels_only_when_the_bias_test_asks():
    """A lazily built hierarchy: Algorithm 1 started at L = 1 with level means
    4^-l (bias estimate 4^-L / 3 against eps/sqrt(2) = 0.018: fails at L = 2,
    passes at L = 3) builds levels 0..3 only, and returns what the same run on
    a fully built list returns."""
    built = []

    def make(l):
        built.append(l)
        return _FakeOps(100 * 4 ** l, 10 * 2 ** l, 8, 2.0 ** -l)

    s = 2.0 ** -9
    dq = lambda l, i: 4.0 ** -l + (s if i % 2 == 0 else -s)
    rule = rng.SampleRule(T=1.0)
    eps = 0.018 * math.sqrt(2.0)
    lazy = mlmc.LazyLevels(make, 8)
    r1 = mlmc.mlmc(lazy, rule, eps=eps, N_init=(8,) * 8, L_start=1, eval_dq=dq)
    assert r1.L == 3 and lazy.built == [0, 1, 2, 3] and sorted(built) == [0, 1, 2, 3]
    r2 = mlmc.mlmc([make(l) for l in range(8)], rule, eps=eps, N_init=(8,) * 8, L_start=1, eval_dq=dq)
    assert (r1.L, r1.N, r1.estimate, r1.cost) == (r2.L, r2.N, r2.estimate, r2.cost)


def test_qopt_with_a_cap_on_p():
    """With p capped the choice is the cheapest tier level whose p fits: on the
    finest workload level (512 cells across) the unconstrained optimum takes
    all six tiers (p = 128), with p <= 64 it takes five (the workload's rule)."""
    q, costs = mesh.qopt_tiers(512)
    assert q == 6 and mesh.graded_L_tiers(512, 6).p == 128
    qc, costs_c = mesh.qopt_tiers(512, p_max=64)
    assert qc == 5 and costs_c == costs
    ok = [k for k in range(7) if mesh.graded_L_tiers(512, k).p <= 64]
    assert qc == min(ok, key=lambda k: costs[k])
