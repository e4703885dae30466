"""Discrete adjoint of stabilized LF-LTS, oracle side (test infrastructure only).

In u = M^-1/2 z variables (see lts.py), write R y := q_1(y) = y + d_p(y)
(Algorithm 2, lines 1-4, applied to q_0 = y; linear in y and self-adjoint in
the M inner product, since every term is a polynomial (A_u P)^k A_u with
M A_u = K symmetric).  The forward recurrence is u_1 = R u_0,
u_{n+1} = 2 R u_n - u_{n-1} and Q = w^T u_N.  Its adjoint is the same
recurrence run backward in the M inner product:

  mu_N = M^-1 w,  mu_{N+1} = 0,  mu_n = 2 R mu_{n+1} - mu_{n+2},
  dQ/dkappa_b = sum_{n=1}^{N-1} 2 <mu_{n+1}, d_b(R u_n)>_M + <mu_1, d_b(R u_0)>_M,

where d_b(R y) is the derivative of the substep recurrence for fixed y with
respect to kappa_b (dA_u/dkappa_b = M^-1 K_b, K_b the stiffness of the cells
of block b with unit coefficient).  Each <mu, d_b(R y)>_M is obtained by a
reverse sweep over the p substeps.  dQ/dg_b = 2 kappa_b dQ/dkappa_b since
kappa = exp(2 g).  dt and the step count are held fixed (they are functions of
max_b c_b, which is not smooth).  States are checkpointed every K steps and
recomputed segment by segment.  As in the forward solver, the recurrences are
evaluated on increments: u_{n+1} = 2 u_n - u_{n-1} + 2 d_p(u_n),
mu_n = 2 mu_{n+1} - mu_{n+2} + 2 d_p(mu_{n+1}).
"""
from __future__ import annotations

import numpy as np

from .lts import Solver


def _block_contract(ops, a, b):
    """a^T (dA_u/dkappa_blk) b = (a/m)^T K_blk b for every block, over the element
    entries of the block, with K_blk's diagonal minus its off-diagonal row sums:
    (K_blk b)_r = sum_e geo_e (b_c - b_r), b_c = 0 on Dirichlet nodes."""
    ed = ops.ed
    am = a / ops.m
    bc = np.where(ed.cols >= 0, b[np.maximum(ed.cols, 0)], 0.0)
    wts = am[ed.rows] * ed.geo * (bc - b[ed.rows])
    return np.bincount(ed.block, weights=wts.real, minlength=ops.lv.n_blocks) + (
        1j * np.bincount(ed.block, weights=wts.imag, minlength=ops.lv.n_blocks)
        if np.iscomplexobj(wts) else 0.0)


def vjp_R_kappa(s: Solver, y, lam, dt):
    """<lam, d(R y)/dkappa_b>_M for all b, by a reverse sweep over the substeps."""
    A, Pd, cc, p = s.A, s.Pd, s.cc, s.p
    ops = s.ops
    c1 = 0.5 * (dt / p) * (dt / p) * (2.0 * p * p / (cc.omega * cc.delta))
    # forward substeps on the increments (kept): q_m = y + d_m
    w = A @ ((1.0 - Pd) * y)
    d = [np.zeros_like(y), -c1 * (w + A @ (Pd * y))]
    c2 = [None]
    for m in range(1, p):
        c2m = (dt / p) * (dt / p) * (2.0 * p * p / cc.omega) * cc.beta_half[m]
        c2.append(c2m)
        d.append((1.0 + cc.beta[m]) * d[m] - cc.beta[m] * d[m - 1] - c2m * (w + A @ (Pd * (y + d[m]))))
    q = [y + dm for dm in d]
    # reverse, with the Euclidean cotangent of q_p equal to M lam
    lq = [np.zeros_like(y) for _ in range(p + 1)]
    lq[p] = ops.m * lam
    lw = np.zeros_like(y)
    g = np.zeros(ops.lv.n_blocks, dtype=np.result_type(y, lam, A.dtype))
    for m in range(p - 1, 0, -1):
        L = lq[m + 1]
        lq[m] = lq[m] + (1.0 + cc.beta[m]) * L - c2[m] * (Pd * (A.T @ L))
        lq[m - 1] = lq[m - 1] - cc.beta[m] * L
        lw = lw - c2[m] * L
        g = g + _block_contract(ops, -c2[m] * L, Pd * q[m])
    L = lq[1]
    lw = lw - c1 * L
    g = g + _block_contract(ops, -c1 * L, Pd * q[0])
    g = g + _block_contract(ops, lw, (1.0 - Pd) * y)
    return g


def gradient(ops, kappa_blocks, u0, dt, n_steps, K: int = 64):
    """(Q, dQ/dkappa_b, dQ/dg_b) for one sample by the checkpointed discrete adjoint."""
    s = Solver(ops, kappa_blocks)
    kb = np.asarray(kappa_blocks, dtype=np.float64)
    N = n_steps
    z0 = u0
    z1 = s.q1(z0, dt)
    # forward, keeping the pairs (u_k, u_{k+1}) for k = 0, K, 2K, ...
    pairs = {0: (z0, z1)}
    zm, zc = z0, z1
    for n in range(1, N):
        zm, zc = zc, 2.0 * zc - zm + 2.0 * s.d1(zc, dt)      # (u_n, u_{n+1})
        if n % K == 0:
            pairs[n] = (zm, zc)
    Q = float(ops.qoi_w @ zc)

    grad_k = np.zeros(ops.lv.n_blocks)
    mu_np2 = np.zeros_like(u0)           # mu_{n+2}
    mu_np1 = ops.qoi_w / ops.m           # mu_{n+1}, starting at n = N-1
    for k0 in sorted(pairs, reverse=True):
        k1 = min(k0 + K - 1, N - 1)
        seg = list(pairs[k0])
        while len(seg) < k1 - k0 + 1:
            seg.append(2.0 * seg[-1] - seg[-2] + 2.0 * s.d1(seg[-1], dt))
        for n in range(k1, k0 - 1, -1):
            zn = seg[n - k0]
            if n >= 1:
                grad_k += 2.0 * vjp_R_kappa(s, zn, mu_np1, dt)
                mu_n = 2.0 * mu_np1 - mu_np2 + 2.0 * s.d1(mu_np1, dt)
                mu_np2, mu_np1 = mu_np1, mu_n
            else:
                grad_k += vjp_R_kappa(s, zn, mu_np1, dt)
    grad_g = 2.0 * kb * grad_k
    return Q, grad_k, grad_g


def q_complex_step(ops, g_blocks, b: int, u0, dt, n_steps, hstep: float = 1e-30):
    """dQ/dg_b by the complex step: Im Q(g + i h e_b) / h, dt and n held fixed."""
    g = np.asarray(g_blocks, dtype=np.complex128).copy()
    g[b] += 1j * hstep
    kappa = np.exp(2.0 * g)
    s = Solver(ops, kappa)
    z0 = u0.astype(np.complex128)
    zm, zc = z0, s.q1(z0, dt)
    for _ in range(1, n_steps):
        zm, zc = zc, 2.0 * zc - zm + 2.0 * s.d1(zc, dt)
    Q = ops.qoi_w @ zc
    return float(np.imag(Q) / hstep)
