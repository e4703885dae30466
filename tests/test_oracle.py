"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: known-answer
vectors, closed forms (discrete standing waves, Chebyshev identities), exact
invariants (energy, symmetry, reduction of LF-LTS to leapfrog), special cases
and independent routines.
"""
import math
import os

import numpy as np
import pytest
import scipy.stats

from oracle import adjoint, cheby, fem, lts, mesh, mlmc, rng

HERE = os.path.dirname(__file__)


# ---------------------------------------------------------------------------
# Random inputs
# ---------------------------------------------------------------------------

def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split("|")
            a = [int(v, 16) for v in lhs.split()]
            b = [int(v, 16) for v in rhs.split()]
            rows.append((a[:4], a[4:], b))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert rng.philox_block_key(key, ctr) == out


def test_philox_stream_counter_layout():
    # block j of stream (i, l, purpose) is Philox at counter (j, i, l, purpose), key (seed, 0)
    a = rng.philox_block(7, (3, 11, 2, 1))
    b = rng.philox_block_key((7, 0), (3, 11, 2, 1))
    assert a == b
    assert rng.philox_block(7, (0, 11, 2, 1)) != a


def test_uniform_open_interval():
    assert rng.to_uniform(0) == 0.5 * 2.0 ** -52
    assert 0.0 < rng.to_uniform(0) < 1.0
    assert rng.to_uniform((1 << 64) - 1) < 1.0
    assert rng.to_uniform((1 << 64) - 1) == 1.0 - 0.5 * 2.0 ** -52


def test_field_statistics():
    rule = rng.SampleRule(n_blocks=16, sigma=0.25)
    g = np.array([rng.draw(0, 0, i, rule).g for i in range(400)]).ravel()
    # N(0, sigma^2): Kolmogorov-Smirnov against the exact normal law
    ks = scipy.stats.kstest(g / 0.25, "norm")
    assert ks.pvalue > 1e-3
    assert abs(np.mean(g)) < 4 * 0.25 / math.sqrt(g.size)
    assert abs(np.var(g) / 0.0625 - 1) < 0.05


def test_sample_fields_and_steps():
    rule = rng.SampleRule(n_blocks=16, sigma=0.25, pulse_box=(0.2, 0.4, 0.2, 0.4), T=1.0)
    s = rng.draw(0, 1, 5, rule)
    assert s.kappa == [math.exp(2.0 * g) for g in s.g]
    assert 0.2 <= s.x0[0] <= 0.4 and 0.2 <= s.x0[1] <= 0.4
    n, dt = rng.steps_for(s, rule, 1 / 32)
    assert n == math.ceil(s.c_max / (0.2 / 32))
    assert abs(dt * n - 1.0) < 1e-15
    assert dt <= 0.2 / 32 / s.c_max * (1 + 1e-15)
    # same omega on the fine and the coarse mesh of a difference
    assert rng.draw(0, 1, 5, rule).g == s.g
    assert rng.draw(0, 0, 5, rule).g != s.g


# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n_base,box,ref,N,nP,nF", [
    (32, (0.45, 0.55), 4, 1849, 1173, 1273),
    (64, (0.45, 0.55), 4, 7569, 4653, 4865),
])
def test_box_mesh_counts(n_base, box, ref, N, nP, nF):
    lv = mesh.box_refined_level(n_base, box=box, ref=ref)
    fem.operators(lv)
    assert lv.n_dof == N and lv.Pmask.sum() == nP and lv.Fplus.sum() == nF
    assert lv.p == ref
    # the refined box snaps outward to coarse grid lines
    assert 0.4375 in lv.xs and 0.5625 in lv.xs
    assert np.all(np.diff(lv.xs) > 0)


def test_box_mesh_c1_counts():
    lv = mesh.box_refined_level(512, box=(0.48, 0.52), ref=8)
    assert lv.n_dof == 442225 and lv.Pmask.sum() == 204081 and lv.p == 8
    assert lv.xs[245 + 0] == 245 / 512 and 267 / 512 in lv.xs


@pytest.mark.parametrize("n_base,N,nP", [(32, 1365, 690), (64, 4181, 1298), (128, 14421, 2514)])
def test_graded_L_counts(n_base, N, nP):
    lv = mesh.graded_L_level(n_base)
    assert lv.n_dof == N and lv.Pmask.sum() == nP and lv.p == 64
    h = 2.0 / n_base
    assert np.min(np.diff(lv.xs)) == h / 64


@pytest.mark.parametrize("maker", [lambda: mesh.box_refined_level(32),
                                   lambda: mesh.graded_L_level(32)])
def test_mass_and_qoi_weight_sums(maker):
    lv = maker()
    area = 3.0 if lv.xs[0] == -1.0 else 1.0
    assert lv.mass.sum() == area                    # exact: dyadic areas
    # QoI weights integrate 1 over the QoI cells (minus what sits on Dirichlet nodes)
    hx = np.diff(lv.xs)
    hy = np.diff(lv.ys)
    cell_area = np.outer(hy, hx)
    qa = cell_area[lv.cell_qoi & lv.cell_active].sum()
    assert abs(lv.qoi_w.sum() - qa) < 1e-15
    assert lv.qoi_w[~lv.dof].sum() == 0.0


def test_dirichlet_L_shape():
    lv = mesh.graded_L_level(32)
    X, Y = np.meshgrid(lv.xs, lv.ys)
    # nodes of the closed removed quadrant are never DOFs
    assert not np.any(lv.dof & (X >= 0) & (Y <= 0))
    assert np.all(lv.dof[1:-1, 1:-1][((X < 0) | (Y > 0))[1:-1, 1:-1]])


# ---------------------------------------------------------------------------
# Chebyshev constants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3, 4, 8, 19, 64])
def test_cheby_nu0_is_original_scheme(p):
    c = cheby.cheb_consts(p, 0.0)
    assert c.delta == 1.0 and c.omega == 2.0 * p * p
    assert all(b == 1.0 for b in c.beta[1:]) and all(b == 1.0 for b in c.beta_half[1:])


def test_cheby_worked_example():
    # worked example for p = 2: printed omega ~ 7.882, beta_{3/2} ~ 0.985, given delta = 1.005
    c = cheby.cheb_consts_from_delta(2, 1.005)
    assert round(c.omega, 3) == 7.882
    assert round(c.beta_half[1], 3) == 0.985
    assert abs(c.beta[1] - 1 / (2 * 1.005 ** 2 - 1)) < 1e-15
    # with the definition delta = 1 + nu/p^2
    d = cheby.cheb_consts(2, 0.01)
    assert d.delta == 1.0025


@pytest.mark.parametrize("p,nu", [(2, 0.01), (4, 0.01), (8, 0.1), (19, 1.0), (64, 0.01)])
def test_cheby_closed_forms(p, nu):
    c = cheby.cheb_consts(p, nu)
    x = c.delta
    a = math.acosh(x)
    Tp = math.cosh(p * a)
    dTp = p * math.sinh(p * a) / math.sqrt(x * x - 1)
    assert abs(c.omega - 2 * dTp / Tp) < 1e-9 * c.omega
    for k in range(1, p):
        assert abs(c.beta[k] - math.cosh((k - 1) * a) / math.cosh((k + 1) * a)) < 1e-12
        assert abs(c.beta_half[k] - math.cosh(k * a) / math.cosh((k + 1) * a)) < 1e-12
        # three-term identity 2 delta beta_{k+1/2} = 1 + beta_k
        assert abs(2 * x * c.beta_half[k] - 1 - c.beta[k]) < 1e-14


@pytest.mark.parametrize("p,nu", [(1, 0.0), (2, 0.01), (4, 0.01), (8, 0.01), (19, 0.1), (64, 1.0)])
def test_coarse_coefficient_is_leapfrog(p, nu):
    """Away from P the substeps act on a scalar multiple of w: q_m = z + a_m w and
    a_p = -dt^2/2, i.e. LF-LTS is plain leapfrog there regardless of p, nu."""
    c = cheby.cheb_consts(p, nu)
    dt = 0.37
    c1 = 0.5 * (dt / p) ** 2 * (2 * p * p / (c.omega * c.delta))
    a_prev, a = 0.0, -c1
    for m in range(1, p):
        c2 = (dt / p) ** 2 * (2 * p * p / c.omega) * c.beta_half[m]
        a_prev, a = a, (1 + c.beta[m]) * a - c.beta[m] * a_prev - c2
    assert abs(a + 0.5 * dt * dt) < 1e-14 * dt * dt


# ---------------------------------------------------------------------------
# Operators and time stepping: closed forms on uniform grids
# ---------------------------------------------------------------------------

def _uniform(n, p=1, all_fine=False, c=1.0):
    # a box that meets no cell -> uniform grid; n cells of size 1/n
    lv = mesh.box_refined_level(n, box=(2.0, 3.0), ref=1, p=p)
    if all_fine:
        lv.cell_fine[:] = True
        lv.Pmask = lv.dof.copy()
    ops = fem.operators(lv)
    return lv, ops


def _mode(lv, k, l):
    X, Y = np.meshgrid(lv.xs, lv.ys)
    ids = lv.dof_ids
    return (np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)).ravel()[ids]


@pytest.mark.parametrize("k,l", [(1, 1), (2, 3), (7, 5)])
def test_operator_eigenpair(k, l):
    n = 16
    lv, ops = _uniform(n)
    h = 1.0 / n
    c2 = 1.7
    K = fem.stiffness(ops.ed, np.full(16, c2))
    v = _mode(lv, k, l)
    lam = (4 * c2 / h ** 2) * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
    assert np.allclose(ops.m, h * h, rtol=0, atol=1e-18)
    Av = (K @ v) / ops.m
    assert np.max(np.abs(Av - lam * v)) < 1e-12 * lam


def test_stiffness_hypotenuse_entries_vanish():
    lv = mesh.box_refined_level(16)
    ops = fem.operators(lv)
    K = fem.stiffness(ops.ed, np.linspace(0.5, 2.0, 16)).tocoo()
    ids = lv.dof_ids
    ri, ci = ids[K.row] % lv.nxn, ids[K.col] % lv.nxn
    rj, cj = ids[K.row] // lv.nxn, ids[K.col] // lv.nxn
    diag_pair = (ri != ci) & (rj != cj)
    assert np.all(K.data[diag_pair] == 0.0)
    # symmetric, zero row sums away from the boundary (constants in the kernel)
    Kc = K.tocsr()
    assert abs(Kc - Kc.T).max() == 0.0


@pytest.mark.parametrize("k,l", [(1, 2), (3, 3)])
def test_leapfrog_discrete_standing_wave(k, l):
    n = 16
    lv, ops = _uniform(n)
    h = 1.0 / n
    v = _mode(lv, k, l)
    lam = (4 / h ** 2) * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
    dt = 0.2 * h
    theta = math.acos(1 - dt * dt * lam / 2)
    s = lts.Solver(ops, np.ones(16))
    for N in (1, 2, 37, 200):
        u = s.run_lf(v, dt, N)
        assert np.max(np.abs(u - math.cos(N * theta) * v)) < 1e-12


@pytest.mark.parametrize("p,nu,k,l", [(4, 0.0, 1, 2), (4, 0.01, 2, 5), (8, 0.1, 3, 1), (3, 1.0, 6, 6)])
def test_lts_all_fine_is_chebyshev_standing_wave(p, nu, k, l):
    """P = I: q_1 = T_p(delta - dt^2 lam/omega)/T_p(delta) z on an eigenvector."""
    n = 16
    lv, ops = _uniform(n, p=p, all_fine=True)
    lv.nu = nu
    h = 1.0 / n
    v = _mode(lv, k, l)
    lam = (4 / h ** 2) * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
    c = cheby.cheb_consts(p, nu)
    dt = 0.5 * h * p / 2
    x = c.delta - dt * dt * lam / c.omega

    def T(pp, xx):
        return math.cos(pp * math.acos(xx)) if abs(xx) <= 1 else math.cosh(pp * math.acosh(xx))

    rho = T(p, x) / T(p, c.delta)
    assert abs(rho) <= 1
    Theta = math.acos(rho)
    s = lts.Solver(ops, np.ones(16))
    assert np.all(s.Pd == 1.0)
    for N in (1, 5, 60):
        u = s.run(v, dt, N)
        assert np.max(np.abs(u - math.cos(N * Theta) * v)) < 1e-12


def test_lts_all_fine_nu0_equals_leapfrog_substeps():
    n, p = 16, 4
    lv, ops = _uniform(n, p=p, all_fine=True)
    lv.nu = 0.0
    v = _mode(lv, 2, 1) + 0.3 * _mode(lv, 5, 7)
    s = lts.Solver(ops, np.ones(16))
    dt = 0.3 / n
    u_lts = s.run(v, dt, 1)
    # p leapfrog steps of size dt/p from rest (start-up included) give the same q_1
    z0 = v
    zm, zc = z0, z0 - 0.5 * (dt / p) ** 2 * (s.A @ z0)
    for _ in range(1, p):
        zm, zc = zc, lts.lf_step(s.A, zc, zm, dt / p)
    assert np.max(np.abs(u_lts - zc)) < 1e-13


@pytest.mark.parametrize("which", ["P0", "p1"])
def test_lts_reduces_to_leapfrog(which):
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    rule = rng.SampleRule()
    smp = rng.draw(0, 0, 3, rule)
    u0 = lts.pulse(ops, smp.x0)
    if which == "P0":
        s = lts.Solver(ops, smp.kappa, Pd=np.zeros_like(ops.Pd))
    else:
        s = lts.Solver(ops, smp.kappa, p=1)
    dt = 0.1 / 32 / smp.c_max       # below the plain leapfrog CFL limit
    # one step: equal up to rounding of a_p = -dt^2/2
    u1 = s.run(u0, dt, 2)
    u2 = s.run_lf(u0, dt, 2)
    assert np.max(np.abs(u1 - u2)) < 1e-14 * np.max(np.abs(u2))
    # a long run: rounding differences accumulate, nothing else
    N = 400
    u1 = s.run(u0, dt, N)
    u2 = s.run_lf(u0, dt, N)
    assert np.max(np.abs(u1 - u2)) < 1e-10 * np.max(np.abs(u2))


def test_lts_is_leapfrog_outside_fplus():
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    s = lts.Solver(ops, np.exp(np.linspace(-0.5, 0.5, 16)))
    rs = np.random.default_rng(1)
    z = rs.standard_normal(ops.Pd.size)
    dt = 0.2 / 32
    q1 = s.q1(z, dt)
    out = ~lv.Fplus.ravel()[lv.dof_ids]
    ref = z - 0.5 * dt * dt * (s.A @ ((1 - s.Pd) * z))
    assert np.max(np.abs(q1[out] - ref[out])) < 1e-13 * np.max(np.abs(z))
    # and differs inside (the local steps do something)
    assert np.max(np.abs(q1[~out] - ref[~out])) > 1e-3


def test_energy_conserved_c0_mesh():
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    rule = rng.SampleRule()
    smp = rng.draw(0, 0, 0, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    s = lts.Solver(ops, smp.kappa)
    u, zs = s.run(lts.pulse(ops, smp.x0), dt, n, keep=True)
    E = np.array([s.energy(zs[k + 1], zs[k], dt) for k in range(0, n, 7)])
    assert np.max(np.abs(E - E[0])) < 1e-12 * E[0]


def test_effective_operator_symmetric_and_stable():
    lv = mesh.box_refined_level(8, box=(0.45, 0.55), ref=4)
    ops = fem.operators(lv)
    s = lts.Solver(ops, np.exp(2 * np.linspace(-0.3, 0.3, 16)))
    n = ops.Pd.size
    dt = 0.2 * lv.h / math.exp(0.3)
    I = np.eye(n)
    R = np.stack([s.q1(I[:, k], dt) for k in range(n)], axis=1)
    Ap = 2 * (I - R) / (dt * dt)
    # M A_p is symmetric (A_p self-adjoint in the M inner product)
    MAp = ops.m[:, None] * Ap
    assert np.max(np.abs(MAp - MAp.T)) < 1e-12 * np.max(np.abs(MAp))
    # spectrum of dt^2 A_p (similar to the symmetric M^1/2 A_p M^-1/2) inside (0, 4)
    sq = np.sqrt(ops.m)
    S = sq[:, None] * Ap / sq[None, :]
    ev = np.linalg.eigvalsh(0.5 * (S + S.T)) * dt * dt
    assert ev.min() > 0 and ev.max() < 4


def test_plain_leapfrog_unstable_at_lts_step():
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    s = lts.Solver(ops, np.ones(16))
    rs = np.random.default_rng(0)
    u0 = rs.standard_normal(ops.Pd.size)
    dt = 0.2 * lv.h                      # the LTS step; plain LF needs < 0.1776 h here
    u = s.run_lf(u0, dt, 300)
    assert np.max(np.abs(u)) > 1e6 * np.max(np.abs(u0))
    u = s.run(u0, dt, 300)               # LF-LTS (p = 4) stays bounded
    assert np.max(np.abs(u)) < 10 * np.max(np.abs(u0))


@pytest.mark.parametrize("graded", [False, True])
def test_lf_twin_is_plain_leapfrog_at_dt_over_p(graded):
    """The standard leapfrog twin of a level (Sec. 3.4): the same grid with P
    empty and p = 1. Its spacing h/p makes a sample take p times the steps of
    the LTS level (up to the ceiling), LF-LTS on it is the plain leapfrog
    scheme, and that step is stable: dt^2 lambda_max(M^-1 K(kappa)) < 4."""
    lv = mesh.graded_L_level(32) if graded else mesh.box_refined_level(32)
    tw = mesh.lf_twin(lv)
    assert tw.p == 1 and not tw.Pmask.any() and tw.h == lv.h / lv.p
    assert np.array_equal(tw.dof, lv.dof) and np.array_equal(tw.mass, lv.mass)
    assert np.array_equal(tw.qoi_w, lv.qoi_w)
    ops = fem.operators(tw)
    assert not tw.Fplus.any()
    rule = rng.SampleRule(n_blocks=64, sigma=0.3, pulse_box=(-0.8, -0.4, 0.4, 0.8), T=2.0) if graded \
        else rng.SampleRule()
    smp = rng.draw(0, 0, 1, rule)
    n, dt = rng.steps_for(smp, rule, tw.h)
    n0, _ = rng.steps_for(smp, rule, lv.h)
    assert lv.p * (n0 - 1) < n <= lv.p * n0
    s = lts.Solver(ops, smp.kappa)
    u0 = lts.pulse(ops, smp.x0)
    u1 = s.run(u0, dt, 300)
    u2 = s.run_lf(u0, dt, 300)
    assert np.max(np.abs(u1 - u2)) < 1e-11 * np.max(np.abs(u2))
    K = fem.stiffness(fem.element_data(tw), smp.kappa)
    sq = 1.0 / np.sqrt(ops.m)
    S = (K.multiply(sq[:, None])).multiply(sq[None, :]).toarray()
    lam = np.linalg.eigvalsh(0.5 * (S + S.T)).max()
    assert dt * dt * lam < 4.0


# ---------------------------------------------------------------------------
# MLMC pieces
# ---------------------------------------------------------------------------

def test_mean_var_matches_numpy():
    x = np.random.default_rng(3).standard_normal(1000) * 1e-3 + 5.0
    m, v = mlmc.mean_var(x)
    assert abs(m - np.mean(x)) < 1e-14 * 5
    assert abs(v - np.var(x, ddof=1)) < 1e-12 * v


def test_optimal_N_formula():
    V = [1e-2, 1e-3, 1e-4]
    C = [1.0, 4.0, 16.0]
    eps = 1e-2
    N = mlmc.optimal_N(eps, V, C)
    # by construction the total variance meets eps^2/2 ...
    assert sum(v / n for v, n in zip(V, N)) <= 0.5 * eps * eps * (1 + 1e-12)
    # ... and the Lagrange optimum N_l ~ sqrt(V_l/C_l)
    s = sum(math.sqrt(v * c) for v, c in zip(V, C))
    assert N == [math.ceil(2 / eps ** 2 * math.sqrt(v / c) * s) for v, c in zip(V, C)]


def test_telescoping_with_common_samples():
    rule = rng.SampleRule()
    lvs = [mesh.box_refined_level(8, box=(0.45, 0.55), ref=4),
           mesh.box_refined_level(16, box=(0.45, 0.55), ref=4),
           mesh.box_refined_level(32, box=(0.45, 0.55), ref=4)]
    ops = [fem.operators(lv) for lv in lvs]
    rule.T = 0.25
    i = 4
    Q = [mlmc.solve_Q(o, rng.draw(0, 2, i, rule), rule) for o in ops]
    d = [mlmc.delta_Q(ops, 0, l, i, rule) for l in range(3)]
    # same omega on both meshes of a difference
    assert d[2][0] == Q[2] and d[2][1] == Q[1]
    # telescoping: Q_L = Q_0 + sum (Q_l - Q_{l-1}) along one omega
    assert abs((Q[0] + (Q[1] - Q[0]) + (Q[2] - Q[1])) - Q[2]) < 1e-16


def test_mlmc_algorithm_meets_variance_target():
    rule = rng.SampleRule(T=0.25)
    lvs = [mesh.box_refined_level(8, box=(0.45, 0.55), ref=4),
           mesh.box_refined_level(16, box=(0.45, 0.55), ref=4),
           mesh.box_refined_level(32, box=(0.45, 0.55), ref=4)]
    ops = [fem.operators(lv) for lv in lvs]
    res = mlmc.mlmc(ops, rule, eps=2e-4, N_init=(16, 8, 4))
    assert sum(v / n for v, n in zip(res.var, res.N)) <= 0.5 * (2e-4) ** 2 * (1 + 1e-12)
    assert abs(res.estimate - sum(np.mean(res.samples[l]) for l in range(res.L + 1))) < 1e-15


# ---------------------------------------------------------------------------
# Discrete adjoint
# ---------------------------------------------------------------------------

def _tiny_case():
    lv = mesh.box_refined_level(8, box=(0.45, 0.55), ref=4)
    ops = fem.operators(lv)
    rule = rng.SampleRule()
    smp = rng.draw(0, 0, 1, rule)
    u0 = lts.pulse(ops, (0.5, 0.45), 0.2)
    return lv, ops, np.array(smp.g), u0


@pytest.mark.parametrize("K", [1, 8, 64])
def test_adjoint_matches_complex_step(K):
    lv, ops, g, u0 = _tiny_case()
    dt, N = 0.011, 41
    Q, gk, gg = adjoint.gradient(ops, np.exp(2 * g), u0, dt, N, K=K)
    cs = np.array([adjoint.q_complex_step(ops, g, b, u0, dt, N) for b in range(16)])
    assert np.max(np.abs(gg - cs)) < 1e-12 * np.max(np.abs(cs))


def test_adjoint_matches_central_differences():
    lv, ops, g, u0 = _tiny_case()
    dt, N = 0.011, 41
    Q, gk, gg = adjoint.gradient(ops, np.exp(2 * g), u0, dt, N)
    eps = 1e-6
    fd = []
    for b in range(16):
        e = np.zeros(16)
        e[b] = eps
        qp = lts.qoi(ops, lts.Solver(ops, np.exp(2 * (g + e))).run(u0, dt, N))
        qm = lts.qoi(ops, lts.Solver(ops, np.exp(2 * (g - e))).run(u0, dt, N))
        fd.append((qp - qm) / (2 * eps))
    fd = np.array(fd)
    assert np.max(np.abs(gg - fd)) < 1e-5 * np.max(np.abs(fd))


def test_adjoint_scaling_identity():
    """The scheme sees kappa only through dt^2 kappa: sum_b dQ/dg_b = dQ/dlog dt."""
    lv, ops, g, u0 = _tiny_case()
    dt, N = 0.011, 41
    Q, gk, gg = adjoint.gradient(ops, np.exp(2 * g), u0, dt, N)
    s = lts.Solver(ops, np.exp(2 * g))
    e = 1e-6
    qp = lts.qoi(ops, s.run(u0, dt * math.exp(e), N))
    qm = lts.qoi(ops, s.run(u0, dt * math.exp(-e), N))
    assert abs(gg.sum() - (qp - qm) / (2 * e)) < 1e-7 * np.max(np.abs(gg))


# ---------------------------------------------------------------------------
# Evaluation form: increments vs the printed recurrence
# ---------------------------------------------------------------------------

def test_increment_form_equals_printed_form_one_step():
    lv = mesh.box_refined_level(32)
    ops = fem.operators(lv)
    s = lts.Solver(ops, np.exp(np.linspace(-0.5, 0.5, 16)))
    z = np.random.default_rng(2).standard_normal(ops.Pd.size)
    dt = 0.2 / 32
    a = lts.lts_q1(s.A, s.Pd, z, dt, s.cc)
    b = z + s.d1(z, dt)
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(z))


def _printed_extended(ops, kappa, u0, dt, n):
    """The printed recurrence of Algorithm 2 evaluated in x87 extended precision
    (64-bit significand; coefficients, masses and stiffness entries promoted from
    their binary64 values) for z = M^1/2 u with A = M^-1/2 K M^-1/2, K in edge form."""
    LD = np.longdouble
    K = fem.EdgeStiffness(ops.ed, kappa)
    sqm = np.sqrt(ops.m.astype(LD))

    class A:
        def __matmul__(self, v):
            return (K @ (v / sqm)) / sqm

    A = A()
    Pd = ops.Pd.astype(LD)
    cc = cheby.cheb_consts(ops.lv.p, ops.lv.nu)
    p = cc.p

    def q1(z):
        w = A @ ((LD(1) - Pd) * z)
        c1 = LD(0.5) * (LD(dt) / p) ** 2 * (LD(2 * p * p) / (LD(cc.omega) * LD(cc.delta)))
        qp, q = z, z - c1 * (w + A @ (Pd * z))
        for m in range(1, p):
            c2 = (LD(dt) / p) ** 2 * (LD(2 * p * p) / LD(cc.omega)) * LD(cc.beta_half[m])
            b = LD(cc.beta[m])
            qp, q = q, (LD(1) + b) * q - b * qp - c2 * (w + A @ (Pd * q))
        return q

    z0 = sqm * u0.astype(LD)
    zm, zc = z0, q1(z0)
    for _ in range(1, n):
        zm, zc = zc, -zm + LD(2) * q1(zc)
    return zc / sqm


@pytest.mark.parametrize("n_base,i", [(32, 0), (32, 5), (64, 0)])
def test_increment_form_tracks_extended_precision(n_base, i):
    """The binary64 increment form stays within 1e-13 of the printed algorithm
    evaluated in extended precision over a whole solve; the binary64 printed form
    drifts by orders of magnitude more on the finer mesh."""
    lv = mesh.box_refined_level(n_base)
    ops = fem.operators(lv)
    rule = rng.SampleRule()
    smp = rng.draw(0, 0, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    u0 = lts.pulse(ops, smp.x0)
    uL = _printed_extended(ops, smp.kappa, u0, dt, n)
    qL = float(ops.qoi_w.astype(np.longdouble) @ uL)
    scale = float(ops.qoi_w @ np.abs(uL.astype(np.float64)))
    s = lts.Solver(ops, smp.kappa)
    qi = float(lts.qoi(ops, s.run(u0, dt, n)))
    assert abs(qi - qL) <= 1e-13 * scale
    if n_base == 64:
        qp = float(lts.qoi(ops, s.run(u0, dt, n, form="printed")))
        assert abs(qp - qL) > 100 * abs(qi - qL)


def test_edge_form_stiffness():
    """K v in edge form: the same matrix as the assembled one, constants exactly in
    its kernel away from the boundary, symmetric."""
    lv = mesh.box_refined_level(16)
    ops = fem.operators(lv)
    kap = np.exp(np.linspace(-0.7, 0.6, 16))
    Ke = fem.EdgeStiffness(ops.ed, kap)
    Km = Ke.matrix()
    v = np.random.default_rng(4).standard_normal(ops.Pd.size)
    assert np.max(np.abs(Ke @ v - Km @ v)) < 1e-12 * np.max(np.abs(Km @ v))
    assert abs(Km - Km.T).max() == 0.0
    # interior rows whose neighbours are all DOFs annihilate constants exactly
    ones = np.ones(ops.Pd.size)
    # rows with a nonzero coupling to a Dirichlet node (an incidence row with one entry)
    single = np.diff(Ke.E.indptr) == 1
    ge = np.flatnonzero(single & (Ke.w != 0.0))
    boundary_row = np.zeros(ops.Pd.size, dtype=bool)
    boundary_row[Ke.E.indices[Ke.E.indptr[ge]]] = True
    r = Ke @ ones
    assert np.all(r[~boundary_row] == 0.0)
    # and Dirichlet couplings act like u = 0 outside: K 1 = sum of couplings to the boundary
    assert np.all(r[boundary_row] > 0.0)


def test_edge_form_is_the_closer_binary64_evaluation_of_Kv():
    """K v on a graded L-shape level (smallest cell h/64) for a smooth v, in exact
    rational arithmetic from the binary64 edge weights c_ij (K_ii = sum_j c_ij,
    Dirichlet neighbours included), against two binary64 evaluations of the same
    matrix: the edge form sum_j c_ij (v_i - v_j) that the oracle and the kernels
    use, and the assembled form K_ii v_i - sum_j c_ij v_j with the diagonal
    summed in binary64, at the DOFs away from the Dirichlet boundary.  On a
    locally nearly constant v the exact K v is small next to K_ii v_i,
    and the assembled form's rounding of K_ii v_i swamps it; the edge form
    stays within a few roundings of the exact value.  A constant v gives
    exactly 0 in the edge form there."""
    from fractions import Fraction
    lv = mesh.graded_L_level(32)
    ops = fem.operators(lv)
    kap = np.exp(2.0 * np.linspace(-0.3, 0.3, lv.n_blocks))
    E = fem.EdgeStiffness(ops.ed, kap)
    ids = lv.dof_ids
    X, Y = np.meshgrid(lv.xs, lv.ys)
    px, py = X.ravel()[ids], Y.ravel()[ids]
    n = ids.size
    Ecoo = E.E.tocoo()
    # edges: (i, j or -1, c); rows of E hold +1 at i and -1 at j
    ends = {}
    for r, c, v in zip(Ecoo.row, Ecoo.col, Ecoo.data):
        ends.setdefault(int(r), [None, -1])[0 if v > 0 else 1] = int(c)
    edges = [(ends[e][0], ends[e][1], float(E.w[e])) for e in range(E.w.size)]
    # a smooth mode on top of a constant: locally nearly constant, as the
    # smooth modes are on the h/64 cells
    for v in (1.0 + 1e-3 * np.cos(px) * np.cos(py), np.full(n, 0.3)):
        exact = [Fraction(0)] * n
        diag = np.zeros(n)
        for i, j, c in edges:
            vj = Fraction(float(v[j])) if j >= 0 else Fraction(0)
            d = Fraction(c) * (Fraction(float(v[i])) - vj)
            exact[i] += d
            diag[i] += c
            if j >= 0:
                exact[j] -= d
                diag[j] += c
        edge = E @ v
        off = np.zeros(n)
        for i, j, c in edges:
            if j >= 0:
                off[i] += c * v[j]
                off[j] += c * v[i]
        assembled = diag * v - off
        ex = np.array([float(x) for x in exact])
        # away from the Dirichlet boundary (next to it both forms round c_i0 v_i alike)
        inner = np.ones(n, dtype=bool)
        inner[[i for i, j, _ in edges if j < 0]] = False
        scale = np.abs(diag * v)[inner].max()
        err_edge = np.abs(edge - ex)[inner].max()
        err_asm = np.abs(assembled - ex)[inner].max()
        if np.all(v == v[0]):
            assert np.all(edge[inner] == 0.0) and np.all(ex[inner] == 0.0)
            assert err_asm > 0.0                       # the assembled diagonal leaves a residue
        else:
            assert err_edge <= 1e-15 * scale
            assert err_edge * 10 <= err_asm, (err_edge, err_asm)
