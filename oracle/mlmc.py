"""MLMC estimator pieces, oracle side (test infrastructure only).

Sec. 2.2: Delta Q_0 = Q_0, Delta Q_l = Q_l - Q_{l-1} evaluated on the same
omega; the estimator is sum_l N_l^-1 sum_i Delta Q_l(omega^(i,l)) with
independent samples per level; V_l is estimated with the 1/(N_l - 1)
normalisation; the optimal sample sizes are
N_l >= 2/eps^2 sqrt(V_l / C_l) sum_l' sqrt(V_l' C_l'); the bias is estimated as
|E[Q_L - Q_{L-1}]| / (2^alpha - 1); Algorithm 1 repeats "compute the missing
samples, update V_l and N_l, test the bias, maybe add a level" until no N_l
grows.

Readings: variances are computed two-pass with math.fsum instead of the
single-pass sum-of-squares form (same value, no cancellation); C_l is the cost
model of Sec. 3.3 counted in DOF updates per Delta Q_l sample with the
nominal step dt = cfl*h (so that any two implementations choose the same
N_l); the number of levels is capped by the given hierarchy, which may build
its levels on first use (LazyLevels), so that L grows beyond the levels that
exist when Algorithm 1 starts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import rng
from .fem import Operators
from .lts import Solver, pulse, qoi


def mean_var(x):
    """Sample mean and unbiased variance (1/(n-1)), two-pass with fsum."""
    x = [float(v) for v in x]
    n = len(x)
    if n == 0:
        return float("nan"), float("nan")
    mu = math.fsum(x) / n
    if n == 1:
        return mu, float("nan")
    var = math.fsum((v - mu) ** 2 for v in x) / (n - 1)
    return mu, var


def optimal_N(eps: float, V, C):
    """Smallest integers satisfying N_l >= 2/eps^2 sqrt(V_l/C_l) sum sqrt(V C)."""
    s = math.fsum(math.sqrt(v * c) for v, c in zip(V, C))
    return [int(math.ceil(2.0 / (eps * eps) * math.sqrt(v / c) * s)) for v, c in zip(V, C)]


def bias_estimate(mean_dQ_L: float, alpha: float = 2.0) -> float:
    return abs(mean_dQ_L) / (2.0 ** alpha - 1.0)


def cost_per_solve(ops: Operators, rule: rng.SampleRule) -> float:
    """DOF updates of one solve: n_nominal ((N - |P|) + p |P|), n_nominal = ceil(T/(cfl h))."""
    n = ops.Pd.size
    nP = int(ops.Pd.sum())
    steps = math.ceil(rule.T / (rule.cfl * ops.lv.h))
    return float(steps * ((n - nP) + ops.lv.p * nP))


def level_costs(ops_list, rule):
    c = [cost_per_solve(o, rule) for o in ops_list]
    return [c[0]] + [c[l] + c[l - 1] for l in range(1, len(c))]


def solve_Q(ops: Operators, smp: rng.Sample, rule: rng.SampleRule, width: float = 0.05):
    n, dt = rng.steps_for(smp, rule, ops.lv.h)
    s = Solver(ops, smp.kappa)
    u = s.run(pulse(ops, smp.x0, width), dt, n)
    return float(qoi(ops, u))


def delta_Q(ops_list, seed: int, level: int, i: int, rule, width: float = 0.05):
    """(Q_l, Q_{l-1}, Delta Q_l) for sample i of level l (Q_{-1} := 0)."""
    smp = rng.draw(seed, level, i, rule)
    qf = solve_Q(ops_list[level], smp, rule, width)
    qc = solve_Q(ops_list[level - 1], smp, rule, width) if level > 0 else 0.0
    return qf, qc, qf - qc


class LazyLevels:
    """A level hierarchy whose level l is built by ``make(l)`` on first use,
    l < n_max: Algorithm 1 adds a level whenever the bias test asks for one,
    so the hierarchy need not exist in advance (Sec. 2.2)."""

    def __init__(self, make, n_max: int):
        self.make, self.n_max, self._lv = make, n_max, {}

    def __len__(self):
        return self.n_max

    def __getitem__(self, l):
        if not 0 <= l < self.n_max:
            raise IndexError(l)
        if l not in self._lv:
            self._lv[l] = self.make(l)
        return self._lv[l]

    @property
    def built(self):
        return sorted(self._lv)


@dataclass
class MLMCResult:
    estimate: float
    L: int
    N: list
    mean: list
    var: list
    cost: list
    bias: float
    rmse: float
    samples: dict = field(default_factory=dict)


def mlmc(ops_list, rule, eps: float, seed: int = 0, N_init=(256, 64, 16, 8, 4), alpha: float = 2.0,
         L_start: int = 2, eval_dq=None, costs=None):
    """Algorithm 1 with eq. (optimal N_l) and the bias test against eps^2/2.

    ``eval_dq(level, i) -> Delta Q`` may be supplied (defaults to the oracle
    solver), and so may the per-sample costs ``costs[l]`` = C_l (defaults to
    the cost model on ``ops_list``; then ``ops_list`` may be any sequence
    whose length is the number of levels)."""
    if eval_dq is None:
        def eval_dq(level, i):
            return delta_Q(ops_list, seed, level, i, rule)[2]
    Lmax = len(ops_list) - 1
    L = min(L_start, Lmax)
    solve_cost = {}

    def cost_of(l):
        """C_l, computed when level l is first used (ops_list may build levels lazily)."""
        if costs is not None:
            return costs[l]
        for k in (l, l - 1):
            if k >= 0 and k not in solve_cost:
                solve_cost[k] = cost_per_solve(ops_list[k], rule)
        return solve_cost[l] + (solve_cost[l - 1] if l > 0 else 0.0)

    C = [cost_of(l) for l in range(L + 1)]
    N = [N_init[l] for l in range(L + 1)]
    dq = {l: [] for l in range(Lmax + 1)}
    grew = True
    while grew:
        for l in range(L + 1):
            for i in range(len(dq[l]), N[l]):
                dq[l].append(eval_dq(l, i))
        mv = [mean_var(dq[l]) for l in range(L + 1)]
        V = [v for _, v in mv]
        newN = optimal_N(eps, V, C)
        grew = False
        for l in range(L + 1):
            if newN[l] > N[l]:
                N[l] = newN[l]
                grew = True
        bias = bias_estimate(mv[L][0], alpha)
        if bias * bias >= 0.5 * eps * eps and L < Lmax:
            L += 1
            N.append(N_init[L])
            C.append(cost_of(L))
            grew = True
    mv = [mean_var(dq[l][:N[l]]) for l in range(L + 1)]
    est = math.fsum(m for m, _ in mv)
    bias = bias_estimate(mv[L][0], alpha)
    var_est = math.fsum(v / n for (_, v), n in zip(mv, N))
    return MLMCResult(estimate=est, L=L, N=N, mean=[m for m, _ in mv], var=[v for _, v in mv],
                      cost=C, bias=bias, rmse=math.sqrt(var_est + bias * bias),
                      samples={l: dq[l][:N[l]] for l in range(L + 1)})


def delta_grad(ops_list, seed: int, level: int, i: int, rule, K: int = 64, width: float = 0.05):
    """dQ_l/dg - dQ_{l-1}/dg (dQ_{-1}/dg := 0) for sample i of level l: the
    discrete adjoint on both meshes of the coupled difference, each with its
    own step count and dt held fixed."""
    from .adjoint import gradient
    smp = rng.draw(seed, level, i, rule)

    def g_on(ops):
        n, dt = rng.steps_for(smp, rule, ops.lv.h)
        return np.asarray(gradient(ops, smp.kappa, pulse(ops, smp.x0, width), dt, n, K=K)[2])
    gf = g_on(ops_list[level])
    return gf - g_on(ops_list[level - 1]) if level > 0 else gf


def mlmc_grad(ops_list, rule, eps: float, seed: int = 0, N_init=(256, 64, 16, 8, 4), alpha: float = 2.0,
              L_start: int = 2, K: int = 64):
    """Algorithm 1 for the QoI (mlmc) and, on the same samples of every level,
    the mean and unbiased variance of each block's gradient difference
    dQ_l/dg_b - dQ_{l-1}/dg_b; their sum over the levels estimates dE[Q]/dg_b
    (the derivative of the MLMC estimator of E[Q], term by term).
    Returns (MLMCResult, estimate[nb], mean[L+1][nb], var[L+1][nb])."""
    res = mlmc(ops_list, rule, eps, seed=seed, N_init=N_init, alpha=alpha, L_start=L_start)
    means, vars_ = [], []
    for l in range(res.L + 1):
        rows = [delta_grad(ops_list, seed, l, i, rule, K) for i in range(res.N[l])]
        mv = [mean_var([r[b] for r in rows]) for b in range(len(rows[0]))]
        means.append([m for m, _ in mv])
        vars_.append([v for _, v in mv])
    est = [math.fsum(means[l][b] for l in range(res.L + 1)) for b in range(len(means[0]))]
    return res, est, means, vars_
