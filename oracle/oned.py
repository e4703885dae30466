"""One-dimensional workloads of Sec. 4.1 and Sec. 4.2, oracle side (test
infrastructure only; see the package header).

Model (Sec. 4.1): u_tt - (c^2 u_x)_x = 0 in D = (0, 6), homogeneous Neumann
data, u_0(x) = exp(-(x - 3)^2 / 0.09), u_t(0) = 0.  Space: continuous P1 with
mass lumping (Sec. 3.1); under Neumann data every node is a DOF.  The lumped
mass of node i is the sum of |cell|/2 over its cells, and K is applied in edge
form, (K v)_i = sum_j (kappa_cell / |cell|) (v_i - v_j) over the neighbours j
(kappa = c^2 on the cell joining i and j).  Time: Algorithm 2 (stabilized
LF-LTS) with P the nodes of the fine cells, in u-form as in ``lts``.

Readings (the paper leaves them open):
* kappa = c^2 per cell is the field at the cell midpoint (midpoint rule for
  the stiffness integral).
* Level meshes: uniform cells of size H on D; every coarse cell inside the
  closed fine interval D_fine is split into cells of size h_f (Sec. 4.1:
  D_fine = [5 - H_0, 5], h_f = 2^-8; Sec. 4.2: [4 - H_0, 4], h_f = 2^-9, with
  H_0 = 1/16 and H_l = 2^-(l+4)); P = the nodes of fine cells, p = H / h_f.
  A level with H <= h_f has no fine cells (plain leapfrog, p = 1).
* Continuous field (Sec. 4.1): c^2(x) = 1 + sum_{k=1}^{100} (1/(4 pi^2 k^2))
  (cos(k pi x / 6) xi1_k + sin(k pi x / 6) xi2_k), xi ~ U(-1, 1) from the
  sample's Philox stream (purpose 0): xi1_k = 2 u_{2k-2} - 1,
  xi2_k = 2 u_{2k-1} - 1, summed in the order k = 1..100.
* Jump (Sec. 4.2): c = 1 left of xi and 2 from xi on, xi = (4 - H_0) + H_0 u_0
  (purpose 0); a cell takes c^2 = 4 when its midpoint is >= xi.
* Steps: n = ceil(T c_max / (cfl H)) with c_max = sqrt(max_cell kappa) and
  cfl = 0.5 (plain leapfrog in 1D is stable up to c dt / h = 1), dt = T / n.
* Q = u(T) in V = L^2(D) as nodal values.  Delta Q_l = u_l - I u_{l-1}, with I
  the nodal interpolation onto the finer mesh (exact: the meshes are nested);
  |v|_V^2 = sum_i m_i v_i^2 with the lumped masses of v's mesh.  V_l =
  sum_i |Delta Q_l(i) - mean|_V^2 / (N_l - 1); bias = |mean Delta Q_L|_V /
  (2^alpha - 1); the estimate sum_l I mean Delta Q_l lives on the finest mesh
  used (Sec. 2.1: Q a Lipschitz map into the Hilbert space V).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import rng
from .cheby import cheb_consts
from .lts import lts_d1
from .mlmc import mean_var, optimal_N

KL_TERMS = 100


@dataclass
class Line:
    x: np.ndarray          # [n] node coordinates
    fine: np.ndarray       # [n-1] bool, fine cells
    H: float               # coarse spacing (the step rule uses it)
    p: int
    nu: float
    m: np.ndarray = None   # [n] lumped masses
    Pd: np.ndarray = None  # [n] 0/1 diagonal of P

    @property
    def n(self):
        return self.x.size


def line_level(H: float, fine_box, h_f: float, lo: float = 0.0, hi: float = 6.0, nu: float = 0.01,
               lf: bool = False) -> Line:
    """Uniform cells of size H on (lo, hi); those inside the closed fine_box split
    into cells of size h_f.  lf: the standard leapfrog twin (the comparison of
    Sec. 4): the same nodes with P empty, p = 1, and the step spacing H / p of
    the refined cells."""
    nc = int(round((hi - lo) / H))
    xs = []
    refine = H > h_f
    for k in range(nc):
        a, b = lo + k * H, lo + (k + 1) * H
        if refine and a >= fine_box[0] and b <= fine_box[1]:
            r = int(round(H / h_f))
            xs += [a + t * h_f for t in range(r)]
        else:
            xs.append(a)
    xs.append(hi)
    x = np.array(xs)
    hc = np.diff(x)
    fine = hc < H
    p = int(math.ceil(H / h_f)) if fine.any() else 1
    lv = Line(x=x, fine=fine, H=H, p=p, nu=nu)
    m = np.zeros(x.size)
    m[:-1] += 0.5 * hc
    m[1:] += 0.5 * hc
    lv.m = m
    Pd = np.zeros(x.size)
    Pd[:-1][fine] = 1.0
    Pd[1:][fine] = 1.0
    lv.Pd = Pd
    if lf and fine.any():
        lv.Pd = np.zeros(x.size)
        lv.H = H / p
        lv.p = 1
    return lv


def kl_level(l: int, nu: float = 0.01, lf: bool = False) -> Line:
    """Level l of the continuous-wave-speed workload (Sec. 4.1)."""
    return line_level(2.0 ** -(l + 4), (5.0 - 1.0 / 16, 5.0), 2.0 ** -8, nu=nu, lf=lf)


def jump_level(l: int, nu: float = 0.01, lf: bool = False) -> Line:
    """Level l of the random-jump workload (Sec. 4.2)."""
    return line_level(2.0 ** -(l + 4), (4.0 - 1.0 / 16, 4.0), 2.0 ** -9, nu=nu, lf=lf)


def midpoints(lv: Line) -> np.ndarray:
    return 0.5 * (lv.x[:-1] + lv.x[1:])


def kl_xi(seed: int, level: int, i: int):
    u = rng.uniforms(seed, i, level, 0, 2 * KL_TERMS)
    return [2.0 * u[2 * k] - 1.0 for k in range(KL_TERMS)], [2.0 * u[2 * k + 1] - 1.0 for k in range(KL_TERMS)]


def kl_c2(x: float, xi1, xi2) -> float:
    """c^2(x) of Sec. 4.1 for one realisation, terms summed in order k = 1..100."""
    c2 = 1.0
    for k in range(1, KL_TERMS + 1):
        a = (k * math.pi) * x / 6.0
        coef = 1.0 / (4.0 * math.pi * math.pi * k * k)
        c2 += coef * (math.cos(a) * xi1[k - 1] + math.sin(a) * xi2[k - 1])
    return c2


def jump_xi(seed: int, level: int, i: int, H0: float = 1.0 / 16) -> float:
    u = rng.uniforms(seed, i, level, 0, 1)[0]
    return (4.0 - H0) + H0 * u


def cell_kappa(lv: Line, kind: str, seed: int, level: int, i: int) -> np.ndarray:
    """kappa = c^2 on every cell of lv for sample i of MLMC level `level`."""
    mid = midpoints(lv)
    if kind == "kl":
        xi1, xi2 = kl_xi(seed, level, i)
        return np.array([kl_c2(float(xm), xi1, xi2) for xm in mid])
    xi = jump_xi(seed, level, i)
    return np.where(mid >= xi, 4.0, 1.0)


def steps(lv: Line, kappa, T: float, cfl: float = 0.5):
    c_max = math.sqrt(float(np.max(kappa)))
    n = int(math.ceil((T * c_max) / (cfl * lv.H)))
    return n, T / n


class _Au:
    """A_u = M^-1 K(kappa) on a line, K in edge form."""

    def __init__(self, lv: Line, kappa):
        self.c = np.asarray(kappa) / np.diff(lv.x)
        self.m = lv.m

    def __matmul__(self, v):
        d = v[:-1] - v[1:]                   # v_i - v_i+1 on every cell
        f = self.c * d
        kv = np.zeros_like(v)
        kv[:-1] += f
        kv[1:] -= f
        return kv / self.m


def pulse(lv: Line) -> np.ndarray:
    return np.exp(-(lv.x - 3.0) ** 2 / 0.09)


def solve(lv: Line, kappa, dt: float, n: int, Pd=None, keep=False, u0=None, p=None):
    """u(T) by Algorithm 2 (increment form, start-up u_1 = u_0 + d_p(u_0));
    u0 defaults to the pulse, Pd to the level's P, p to the level's p."""
    A = _Au(lv, kappa)
    P = lv.Pd if Pd is None else Pd
    cc = cheb_consts(lv.p if p is None else p, lv.nu)
    zm = pulse(lv) if u0 is None else u0
    zc = zm + lts_d1(A, P, zm, dt, cc)
    hist = [zm, zc] if keep else None
    for _ in range(1, n):
        zm, zc = zc, 2.0 * zc - zm + 2.0 * lts_d1(A, P, zc, dt, cc)
        if keep:
            hist.append(zc)
    return (zc, hist) if keep else zc


def energy(lv: Line, kappa, z_np1, z_n, dt):
    """E_{n+1/2} = 1/2 |u_{n+1} - u_n|_M^2 / dt^2 + 1/2 u_{n+1}^T M A_p u_n,
    A_p y = -2 d_p(y) / dt^2 (as lts.Solver.energy)."""
    A = _Au(lv, kappa)
    cc = cheb_consts(lv.p, lv.nu)
    d = z_np1 - z_n
    Ap = -2.0 * lts_d1(A, lv.Pd, z_n, dt, cc) / (dt * dt)
    return 0.5 * float(d @ (lv.m * d)) / (dt * dt) + 0.5 * float(z_np1 @ (lv.m * Ap))


def prolong(coarse: Line, u, fine: Line) -> np.ndarray:
    """Nodal interpolation of the P1 function u on `coarse` at the nodes of `fine`."""
    a = np.searchsorted(coarse.x, fine.x, side="right") - 1
    a = np.clip(a, 0, coarse.n - 2)
    xa, xb = coarse.x[a], coarse.x[a + 1]
    t = (fine.x - xa) / (xb - xa)
    return u[a] + t * (u[a + 1] - u[a])


def norm2(lv: Line, v) -> float:
    """|v|_V^2 = sum_i m_i v_i^2 (lumped L^2 norm), summed with fsum."""
    return math.fsum(float(w) for w in lv.m * v * v)


@dataclass
class Rule1D:
    kind: str = "kl"        # "kl" (Sec. 4.1) or "jump" (Sec. 4.2)
    T: float = 11.0
    cfl: float = 0.5


def solve_sample(lv: Line, rule: Rule1D, seed: int, level: int, i: int):
    kap = cell_kappa(lv, rule.kind, seed, level, i)
    n, dt = steps(lv, kap, rule.T, rule.cfl)
    return solve(lv, kap, dt, n)


def delta_Q(levels, rule: Rule1D, seed: int, l: int, i: int):
    """Delta Q_l(omega^(i,l)) on mesh l: u_l - I u_{l-1} (same sample on both)."""
    uf = solve_sample(levels[l], rule, seed, l, i)
    if l == 0:
        return uf
    uc = solve_sample(levels[l - 1], rule, seed, l, i)
    return uf - prolong(levels[l - 1], uc, levels[l])


def cost_per_solve(lv: Line, rule: Rule1D) -> float:
    """DOF updates of one solve at the nominal step cfl * H: ceil(T / (cfl H)) ((N - |P|) + p |P|)."""
    nP = int(lv.Pd.sum())
    return float(math.ceil(rule.T / (rule.cfl * lv.H)) * ((lv.n - nP) + lv.p * nP))


@dataclass
class VecResult:
    estimate: np.ndarray    # on the finest mesh used
    L: int
    N: list
    var: list
    mean_norm: list         # |mean Delta Q_l|_V
    cost: list
    bias: float
    rmse: float


def vec_moments(lv: Line, rows):
    """Mean vector and V_l = sum |row - mean|_V^2 / (N - 1) (two-pass)."""
    X = np.array(rows)
    n = X.shape[0]
    mean = np.array([math.fsum(X[:, j]) / n for j in range(X.shape[1])])
    var = math.fsum(norm2(lv, r - mean) for r in X) / (n - 1) if n > 1 else float("nan")
    return mean, var


def mlmc_vec(levels, rule: Rule1D, eps: float, seed: int = 0, N_init=(64, 32, 16, 8, 4), alpha: float = 2.0,
             L_start: int = 2, eval_dq=None, costs=None):
    """Algorithm 1 for the V-valued QoI: V_l and the bias in the norm of V."""
    if eval_dq is None:
        def eval_dq(l, i):
            return delta_Q(levels, rule, seed, l, i)
    Lmax = len(levels) - 1
    L = min(L_start, Lmax)

    def cost(l):
        if costs is not None:
            return costs[l]
        c = cost_per_solve(levels[l], rule)
        return c + (cost_per_solve(levels[l - 1], rule) if l > 0 else 0.0)
    C = [cost(l) for l in range(L + 1)]
    N = [N_init[l] for l in range(L + 1)]
    dq = {l: [] for l in range(Lmax + 1)}
    grew = True
    while grew:
        for l in range(L + 1):
            for i in range(len(dq[l]), N[l]):
                dq[l].append(eval_dq(l, i))
        mv = [vec_moments(levels[l], dq[l][:N[l]]) for l in range(L + 1)]
        V = [v for _, v in mv]
        newN = optimal_N(eps, V, C)
        grew = False
        for l in range(L + 1):
            if newN[l] > N[l]:
                N[l] = newN[l]
                grew = True
        bias = math.sqrt(norm2(levels[L], mv[L][0])) / (2.0 ** alpha - 1.0)
        if bias * bias >= 0.5 * eps * eps and L < Lmax:
            L += 1
            N.append(N_init[L])
            C.append(cost(L))
            grew = True
    mv = [vec_moments(levels[l], dq[l][:N[l]]) for l in range(L + 1)]
    est = mv[0][0]
    for l in range(1, L + 1):
        est = prolong(levels[l - 1], est, levels[l]) + mv[l][0]
    bias = math.sqrt(norm2(levels[L], mv[L][0])) / (2.0 ** alpha - 1.0)
    var_est = math.fsum(v / n for (_, v), n in zip(mv, N))
    return VecResult(estimate=est, L=L, N=N, var=[v for _, v in mv],
                     mean_norm=[math.sqrt(norm2(levels[l], mv[l][0])) for l in range(L + 1)], cost=C,
                     bias=bias, rmse=math.sqrt(var_est + bias * bias))
