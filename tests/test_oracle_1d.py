"""Pins of the oracle's one-dimensional workloads (Sec. 4.1, 4.2): the lumped
P1 operator with Neumann data, leapfrog and LF-LTS closed forms, energy
conservation, the two random wave-speed models, nested meshes, the
prolongation and the V = L^2(D) estimator pieces of Algorithm 1."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import cheby, mlmc, oned


def _uniform(n_cells, L=6.0, p=1, nu=0.0):
    lv = oned.line_level(L / n_cells, (0.0, 0.0), L / n_cells, hi=L, nu=nu)
    lv.p = p
    return lv


@pytest.mark.parametrize("k", [1, 3, 7])
def test_neumann_cosines_are_exact_eigenvectors(k):
    """cos(k pi x / 6) on a uniform mesh, boundary nodes with half masses:
    M^-1 K v = (4 c^2 / h^2) sin^2(k pi h / 12) v exactly (to rounding)."""
    lv = _uniform(96)
    h = 6.0 / 96
    c2 = 1.7
    v = np.cos(k * math.pi * lv.x / 6.0)
    Av = oned._Au(lv, np.full(96, c2)) @ v
    lam = 4.0 * c2 / h ** 2 * math.sin(k * math.pi * h / 12.0) ** 2
    assert np.max(np.abs(Av - lam * v)) <= 1e-11 * lam


@pytest.mark.parametrize("k", [1, 4])
def test_leapfrog_and_lts_standing_waves(k):
    """P = 0: plain leapfrog, u_n = cos(n theta) v, cos theta = 1 - dt^2 lam / 2.
    P = I with p substeps: cos Theta = T_p(delta - dt^2 lam / omega) / T_p(delta)."""
    lv = _uniform(64, nu=0.01)
    h = 6.0 / 64
    c2 = 1.0
    v = np.cos(k * math.pi * lv.x / 6.0)
    lam = 4.0 * c2 / h ** 2 * math.sin(k * math.pi * h / 12.0) ** 2
    dt, n = 0.4 * h, 150
    u = oned.solve(lv, np.full(64, c2), dt, n, Pd=np.zeros(lv.n), u0=v, p=1)
    th = 2.0 * math.asin(dt * math.sqrt(lam) / 2.0)          # 1 - cos th = dt^2 lam / 2
    assert np.max(np.abs(u - math.cos(n * th) * v)) <= 5e-12
    p = 4
    cc = cheby.cheb_consts(p, 0.01)
    Tp = lambda x: math.cos(p * math.acos(x)) if abs(x) <= 1 else math.cosh(p * math.acosh(x))
    ratio = Tp(cc.delta - dt * dt * lam / cc.omega) / Tp(cc.delta)
    u = oned.solve(lv, np.full(64, c2), dt, n, Pd=np.ones(lv.n), u0=v, p=p)
    assert np.max(np.abs(u - math.cos(n * math.acos(ratio)) * v)) <= 5e-12


def test_lts_energy_is_conserved_on_the_refined_level():
    """Level 0 of Sec. 4.1 (16 fine cells of 2^-8, p = 16) with a KL sample:
    the discrete energy E_{n+1/2} is constant."""
    lv = oned.kl_level(0)
    assert lv.p == 16 and int(lv.fine.sum()) == 16 and int(lv.Pd.sum()) == 17
    kap = oned.cell_kappa(lv, "kl", 0, 0, 3)
    n, dt = oned.steps(lv, kap, 3.0)
    _, hist = oned.solve(lv, kap, dt, n, keep=True)
    E = [oned.energy(lv, kap, hist[j + 1], hist[j], dt) for j in range(1, n)]
    assert max(abs(e - E[0]) for e in E) <= 1e-12 * abs(E[0])


def test_kl_field_statistics_and_bounds():
    """c^2 of Sec. 4.1: mean 1 and variance (1/3) sum_k 1/(16 pi^4 k^4) at every x
    (E xi = 0, Var xi = 1/3), and |c^2 - 1| <= sqrt(2) sum_k 1/(4 pi^2 k^2)."""
    xs = (0.3, 2.0, 4.7)
    vals = {x: [] for x in xs}
    for i in range(1500):
        xi1, xi2 = oned.kl_xi(7, 0, i)
        assert all(-1.0 < a < 1.0 for a in xi1 + xi2)
        for x in xs:
            vals[x].append(oned.kl_c2(x, xi1, xi2))
    var = sum(1.0 / (16.0 * math.pi ** 4 * k ** 4) for k in range(1, 101)) / 3.0
    bound = math.sqrt(2.0) * sum(1.0 / (4.0 * math.pi ** 2 * k * k) for k in range(1, 101))
    for x in xs:
        m, v = mlmc.mean_var(vals[x])
        assert abs(m - 1.0) <= 5.0 * math.sqrt(var / 1500)
        assert abs(v / var - 1.0) <= 0.12
        assert max(abs(c - 1.0) for c in vals[x]) <= bound


def test_jump_field():
    """Sec. 4.2: xi in [4 - 1/16, 4); c^2 = 1 on the cells left of xi and 4 from the
    first cell whose midpoint is >= xi; the jump cell sits in the refined part."""
    lv = oned.jump_level(1)
    assert lv.p == 16 and int(lv.fine.sum()) == 32
    for i in range(20):
        xi = oned.jump_xi(0, 1, i)
        assert 4.0 - 1.0 / 16 <= xi < 4.0
        kap = oned.cell_kappa(lv, "jump", 0, 1, i)
        mid = oned.midpoints(lv)
        j = int(np.argmax(kap > 1.0))
        assert np.all(kap[:j] == 1.0) and np.all(kap[j:] == 4.0)
        assert mid[j] >= xi and (j == 0 or mid[j - 1] < xi) and lv.fine[j]


@pytest.mark.parametrize("maker,nf,hf", [(oned.kl_level, 16, 2.0 ** -8), (oned.jump_level, 32, 2.0 ** -9)])
def test_nested_meshes_and_masses(maker, nf, hf):
    """Levels are nested (every coarse node is a fine node), the masses sum to
    |D| = 6, and the fine part always holds the same cells of size h_f until
    H reaches h_f."""
    prev = None
    for l in range(5):
        lv = maker(l)
        assert abs(lv.m.sum() - 6.0) <= 1e-14
        H = 2.0 ** -(l + 4)
        if H > hf:
            assert int(lv.fine.sum()) == nf and lv.p == int(H / hf)
            assert np.all(np.diff(lv.x)[lv.fine] == hf)
        else:
            assert not lv.fine.any() and lv.p == 1
        if prev is not None:
            assert set(prev.x.tolist()) <= set(lv.x.tolist())
        prev = lv


def test_prolongation_and_norm():
    """Interpolation onto the finer nested mesh reproduces linear functions
    exactly and keeps coarse nodal values; |1|_V^2 = |D|."""
    c, f = oned.kl_level(1), oned.kl_level(2)
    u = 0.5 - 0.25 * c.x
    assert np.max(np.abs(oned.prolong(c, u, f) - (0.5 - 0.25 * f.x))) <= 1e-15
    g = np.sin(c.x)
    pg = oned.prolong(c, g, f)
    idx = np.searchsorted(f.x, c.x)
    assert np.array_equal(pg[idx], g)
    assert abs(oned.norm2(f, np.ones(f.n)) - 6.0) <= 1e-14


def test_telescoping_with_common_samples():
    """With one sample on every level, sum_l I(u_l - I u_{l-1}) is u_L: the
    vector differences and the prolongation telescope."""
    rule = oned.Rule1D(kind="jump", T=1.0)
    levels = [oned.jump_level(l) for l in range(3)]
    us = [oned.solve_sample(lv, rule, 0, 0, 5) for lv in levels]
    total = us[0]
    for l in range(1, 3):
        total = oned.prolong(levels[l - 1], total, levels[l]) + (us[l] - oned.prolong(levels[l - 1], us[l - 1],
                                                                                       levels[l]))
    assert np.max(np.abs(total - us[2])) <= 1e-14 * np.max(np.abs(us[2]))


def test_vector_algorithm1_reduces_to_the_scalar_one_on_constants():
    """Delta Q_l(i) = (4^-l + s (-1)^i) * 1 on mesh l: |.|_V = sqrt(6) |.|, so the
    V-valued Algorithm 1 takes the path of the scalar one on sqrt(6) (4^-l +
    s (-1)^i): the same L and N_l, and bias and variances in proportion."""
    levels = [oned.kl_level(l) for l in range(4)]
    s = 2.0 ** -9
    dq_s = lambda l, i: math.sqrt(6.0) * (4.0 ** -l + (s if i % 2 == 0 else -s))
    dq_v = lambda l, i: np.full(levels[l].n, 4.0 ** -l + (s if i % 2 == 0 else -s))
    costs = [100.0 * 4 ** l for l in range(4)]
    eps = 0.05
    rv = oned.mlmc_vec(levels, oned.Rule1D(), eps, N_init=(8, 8, 8, 8), L_start=1, eval_dq=dq_v, costs=costs)
    rs = mlmc.mlmc(list(range(4)), None, eps, N_init=(8, 8, 8, 8), L_start=1, eval_dq=dq_s, costs=costs)
    assert (rv.L, rv.N) == (rs.L, rs.N)
    assert abs(rv.bias - rs.bias) <= 1e-12 * rs.bias
    for a, b in zip(rv.var, rs.var):
        assert abs(a - b) <= 1e-12 * b
    assert np.allclose(rv.estimate, sum(4.0 ** -l for l in range(rv.L + 1)), rtol=0, atol=1e-15)
