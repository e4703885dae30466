"""Leapfrog and stabilized LF-LTS time stepping, oracle side (test infrastructure only).

Algorithm 2 (stabilized LF-LTS, Sec. 3.3) is stated for z = M^1/2 u and
A = M^-1/2 K M^-1/2; because M and P are diagonal they commute, and the same
algorithm written for u with A_u = M^-1 K produces the iterates
u_n = M^-1/2 z_n.  The oracle runs it in u (reading: in binary64 the rounded
entries of M^-1/2 K M^-1/2 no longer annihilate the discrete constants, which
shifts the frequencies of smooth modes by far more than the rounding of
(K v)/m does), on *all* DOFs, with P kept as a 0/1 diagonal:

  w_n      = A (I - P) q_0,                       q_0 = z_n
  q_{1/p}  = q_0 - 1/2 (dt/p)^2 (2p^2/(omega delta)) (w_n + A P q_0)
  q_{(m+1)/p} = (1 + beta_m) q_{m/p} - beta_m q_{(m-1)/p}
               - (dt/p)^2 (2p^2/omega) beta_{m+1/2} (w_n + A P q_{m/p}),  m = 1..p-1
  z_{n+1}  = -z_{n-1} + 2 q_1

Reading: the index k of beta_k, beta_{k+1/2} inside the substep loop is the
loop index m.  Start-up (the paper gives none for LTS): z_1 = q_1(z_0) +
dt M^1/2 v_0, the LTS analogue of the leapfrog start-up of Sec. 3.1 (for
P = 0 the two coincide).  The sign of the v_0 term follows the Taylor
expansion (+).

Evaluation (a reading of how to carry out the printed recurrence in binary64):
the solver runs the same recurrence on the increments d_m = q_{m/p} - z_n,

  d_0 = 0,  d_1 = -c1 (w_n + A P z_n),
  d_{m+1} = (1 + beta_m) d_m - beta_m d_{m-1} - c2_m (w_n + A P (z_n + d_m)),
  z_{n+1} = 2 z_n - z_{n-1} + 2 d_p,

which is the printed algorithm term by term (subtract z_n from every q and use
(1 + beta_m) - beta_m = 1).  In binary64 the printed form multiplies the full
state by the rounded (1 + beta_m) and beta_m, whose difference is 1 only up to
an ulp; that systematic O(1e-16) error on z is large next to the dt^2 A z
increment of smooth modes on fine meshes and drifts their phase (~1e-11 after
a few hundred steps, growing with the step count).  The increment form keeps
every coefficient of z exact.  ``lts_q1`` keeps the printed form; the tests
pin the increment form against the printed form evaluated in extended
precision.
"""
from __future__ import annotations

import numpy as np

from .cheby import ChebConsts, cheb_consts
from .fem import Operators, mass_scaled_operator


def lts_q1(A, Pd, z, dt, cc: ChebConsts):
    """q_1^n of Algorithm 2 for q_0 = z (lines 1-4).  Linear in z."""
    p = cc.p
    w = A @ ((1.0 - Pd) * z)
    c1 = 0.5 * (dt / p) * (dt / p) * (2.0 * p * p / (cc.omega * cc.delta))
    q_prev = z
    q = z - c1 * (w + A @ (Pd * z))
    for m in range(1, p):
        c2 = (dt / p) * (dt / p) * (2.0 * p * p / cc.omega) * cc.beta_half[m]
        q_next = (1.0 + cc.beta[m]) * q - cc.beta[m] * q_prev - c2 * (w + A @ (Pd * q))
        q_prev, q = q, q_next
    return q


def lts_d1(A, Pd, z, dt, cc: ChebConsts):
    """Increment d_p = q_1^n - z of Algorithm 2 for q_0 = z (see module header)."""
    p = cc.p
    w = A @ ((1.0 - Pd) * z)
    c1 = 0.5 * (dt / p) * (dt / p) * (2.0 * p * p / (cc.omega * cc.delta))
    d_prev = np.zeros_like(z)
    d = -c1 * (w + A @ (Pd * z))
    for m in range(1, p):
        c2 = (dt / p) * (dt / p) * (2.0 * p * p / cc.omega) * cc.beta_half[m]
        d_next = (1.0 + cc.beta[m]) * d - cc.beta[m] * d_prev - c2 * (w + A @ (Pd * (z + d)))
        d_prev, d = d, d_next
    return d


def lts_step(A, Pd, z_n, z_nm1, dt, cc):
    """One stabilized LF-LTS step, printed form: z_{n+1} = -z_{n-1} + 2 q_1^n."""
    return -z_nm1 + 2.0 * lts_q1(A, Pd, z_n, dt, cc)


def lts_step_inc(A, Pd, z_n, z_nm1, dt, cc):
    """The same step on increments: z_{n+1} = 2 z_n - z_{n-1} + 2 d_p."""
    return 2.0 * z_n - z_nm1 + 2.0 * lts_d1(A, Pd, z_n, dt, cc)


def lf_step(A, z_n, z_nm1, dt):
    """Plain leapfrog of Sec. 3.1 with zero forcing: z_{n+1} = 2 z_n - z_{n-1} - dt^2 A z_n."""
    return 2.0 * z_n - z_nm1 - dt * dt * (A @ z_n)


def pulse(ops: Operators, x0, width: float = 0.05) -> np.ndarray:
    """Nodal values of exp(-|x - x0|^2 / width^2) on the DOFs."""
    lv = ops.lv
    if hasattr(lv, "dof_coords"):                 # a triangle-mesh level
        px, py = lv.dof_coords()
    else:
        X, Y = np.meshgrid(lv.xs, lv.ys)
        ids = lv.dof_ids
        px, py = X.ravel()[ids], Y.ravel()[ids]
    r2 = (px - x0[0]) ** 2 + (py - x0[1]) ** 2
    return np.exp(-r2 / (width * width))


class Solver:
    """One sample on one level: Algorithm 2 in u = M^-1/2 z with start-up.

    The iterates are named z below as in the algorithm; they are nodal values
    u of the finite element function."""

    def __init__(self, ops: Operators, kappa_blocks, nu: float | None = None, p: int | None = None,
                 Pd=None):
        self.ops = ops
        self.A = mass_scaled_operator(ops, kappa_blocks)
        self.p = ops.lv.p if p is None else p
        self.nu = ops.lv.nu if nu is None else nu
        self.cc = cheb_consts(self.p, self.nu)
        self.Pd = ops.Pd if Pd is None else Pd
        self.m = ops.m

    def d1(self, z, dt):
        return lts_d1(self.A, self.Pd, z, dt, self.cc)

    def q1(self, z, dt):
        """R z = q_1(z) = z + d_p(z)."""
        return z + self.d1(z, dt)

    def run(self, u0, dt, n_steps, v0=None, keep=False, form="increment"):
        """Return u(T) (and all u_n when ``keep``).
        form = "increment" (default) or "printed" (the q-recurrence as printed)."""
        z0 = u0
        if form == "increment":
            z1 = z0 + self.d1(z0, dt)
        else:
            z1 = lts_q1(self.A, self.Pd, z0, dt, self.cc)
        if v0 is not None:
            z1 = z1 + dt * v0
        zs = [z0, z1] if keep else None
        zm, zc = z0, z1
        for _ in range(1, n_steps):
            if form == "increment":
                zn = lts_step_inc(self.A, self.Pd, zc, zm, dt, self.cc)
            else:
                zn = lts_step(self.A, self.Pd, zc, zm, dt, self.cc)
            zm, zc = zc, zn
            if keep:
                zs.append(zc)
        return (zc, zs) if keep else zc

    def run_lf(self, u0, dt, n_steps, v0=None):
        """Plain leapfrog (Sec. 3.1) in u: u_1 = u_0 + dt v_0 - dt^2/2 A_u u_0."""
        z0 = u0
        z1 = z0 - 0.5 * dt * dt * (self.A @ z0)
        if v0 is not None:
            z1 = z1 + dt * v0
        zm, zc = z0, z1
        for _ in range(1, n_steps):
            zm, zc = zc, lf_step(self.A, zc, zm, dt)
        return zc

    def energy(self, z_np1, z_n, dt):
        """E_{n+1/2} = 1/2 |u_{n+1} - u_n|_M^2 / dt^2 + 1/2 u_{n+1}^T M A_p u_n with the
        effective LTS operator A_p y = 2 (y - q_1(y)) / dt^2 (M-self-adjoint)."""
        d = z_np1 - z_n
        Apz = -2.0 * self.d1(z_n, dt) / (dt * dt)
        return 0.5 * float(d @ (self.m * d)) / (dt * dt) + 0.5 * float(z_np1 @ (self.m * Apz))


def qoi(ops: Operators, u) -> float:
    """Q = sum_i w_i u_i(T): lumped-mass quadrature of u over the QoI region."""
    return ops.qoi_w @ u
