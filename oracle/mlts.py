"""Multi-level local time stepping (MLTS), oracle side (test infrastructure
only; see the package header).

Sec. 3.5 closes with a proposal for meshes whose refined region holds ever
smaller elements: organise them into tiers of equally sized elements and let
each tier advance with the time step its own elements allow, the multi-level
LTS method the paper cites (Diaz and Grote) but does not write out.  The
scheme below is therefore a reading: Algorithm 2 nested inside itself, one
level of nesting per tier.

Tiers j = 1..T have nested fine sets S_1 >= S_2 >= ... >= S_T of elements (S_1
is the level's D_fine), projectors P_j onto the DOFs that are vertices of an
element of S_j, and integer ratios p_j.  Tier j covers a time sigma_j with the
p_j stages of Algorithm 2's stabilized recurrence (delta, omega, beta of
(p_j, nu)), sigma_1 = dt.  In the increment form of ``lts``
(d_m = q_m - z_n), for a force F held constant over tier j:

  E_j(F):  e_0 = e_{-1} = 0
           Phi_m  = F + A P_j e_m
           Phi~_m = Phi_m                                    (j = T)
                  = -(2 / sigma_{j+1}^2) E_{j+1}(Phi_m)      (j < T)
           e_{m+1} = (1 + beta_m) e_m - beta_m e_{m-1} - c_m Phi~_m,  beta_0 = 0
           result e_{p_j}
  c_0 = 1/2 (sigma_j/p_j)^2 2 p_j^2 / (omega_j delta_j),
  c_m = (sigma_j/p_j)^2 2 p_j^2 / omega_j  beta_{m+1/2}       (m >= 1)

  step:      z_{n+1} = 2 z_n - z_{n-1} + 2 E_1(A z_n)
  start-up:  z_1 = z_0 + E_1(A z_0)          (u_t(0) = 0, as in ``lts``)

For T = 1 this is Algorithm 2 (w + A P (z + d) = A z + A P d).

Why this nesting.  Because T_{m+1} + T_{m-1} = 2 delta T_m, every stage
coefficient satisfies c_m = (1 + beta_m) c_0, so stage m reads
e_{m+1} = (1 + beta_m)(e_m - c_0 Phi_m) - beta_m e_{m-1}: a three-term
combination around the increment -c_0 Phi_m, which is the leapfrog half step
from rest under the force Phi_m over the time sigma_{j+1} with
sigma_{j+1}^2 = 2 c_0 = sigma_j^2 2 / (omega_j delta_j) -- the same for every
stage (sigma_j / p_j when nu = 0).  MLTS replaces that half step by tier j+1,
which resolves the stiffer part A P_{j+1} with its own p_{j+1} stages and
holds A P_j (I - P_{j+1}) at its start value; Phi~_m above is the force that
gives the same increment.  An inner tier with A P_{j+1} = 0 (the recurrence
is exact for a constant force) or with p_{j+1} = 1 therefore changes
nothing.  The effective operator G z = -(2/dt^2) E_1(A z) comes out
M-self-adjoint (checked by the tests), so the scheme conserves ``energy``.

Tiers on the rectilinear levels (reading, ``tiers_by_leg``): an active fine
cell belongs to tier 1 + the number of j in 2..T with shorter leg < h 2^-j,
so that on the graded L-shape tier j holds the cells of shorter leg at most
h 2^-(j+1); with p_j = 2 every tier then steps at the same ratio of step to
shorter leg as the coarse cells (dt for legs h/2).
"""
from __future__ import annotations

import math

import numpy as np

from .cheby import cheb_consts
from .fem import Operators, mass_scaled_operator


def tiers_by_leg(lv, n_tiers: int) -> np.ndarray:
    """Cell tiers [nyc, nxc] of a rectilinear level: 0 for a coarse or inactive
    cell; for an active fine cell 1 + #{j in 2..n_tiers : shorter leg < h 2^-j}."""
    HX, HY = np.meshgrid(np.diff(lv.xs), np.diff(lv.ys))
    short = np.minimum(HX, HY)
    t = np.ones(short.shape, dtype=np.int64)
    for j in range(2, n_tiers + 1):
        t += (short < math.ldexp(lv.h, -j)).astype(np.int64)
    t[~(lv.cell_active & lv.cell_fine)] = 0
    return t


def tier_projectors(lv, cell_tier, n_tiers: int) -> list:
    """P_j (j = 1..n_tiers) on the DOFs as 0/1 vectors: DOFs that are vertices
    of a triangle whose cell has tier >= j."""
    ids = lv.dof_ids
    tri_t = np.asarray(cell_tier).ravel()[lv.tri_cell]
    out = []
    for j in range(1, n_tiers + 1):
        P = np.zeros(lv.nyn * lv.nxn, dtype=bool)
        P[lv.tris[tri_t >= j].ravel()] = True
        out.append(P[ids].astype(np.float64))
    return out


class MltsSolver:
    """One sample on one level with MLTS (tiers P_j, ratios p_j), in u as
    ``lts.Solver`` (A = M^-1 K applied in edge form)."""

    def __init__(self, ops: Operators, kappa_blocks, Ps, ps, nu: float | None = None):
        if len(Ps) != len(ps) or not ps:
            raise ValueError("one projector per tier")
        self.ops = ops
        self.A = mass_scaled_operator(ops, kappa_blocks)
        self.Ps = [np.asarray(P, dtype=np.float64) for P in Ps]
        self.ps = [int(p) for p in ps]
        self.nu = ops.lv.nu if nu is None else nu
        self.cc = [cheb_consts(p, self.nu) for p in self.ps]
        self.m = ops.m

    def inner_sigma(self, j: int, sigma: float) -> float:
        """sigma_{j+1} = sqrt(2 c_0) for tier j covering sigma (0-based j)."""
        p, cc = self.ps[j], self.cc[j]
        return (sigma / p) * np.sqrt(2.0 * p * p / (cc.omega * cc.delta))

    def E(self, j: int, F, sigma: float):
        """E_j(F) over the time sigma (j is 0-based here)."""
        p, cc, P = self.ps[j], self.cc[j], self.Ps[j]
        h2 = (sigma / p) * (sigma / p)
        e_prev = np.zeros_like(F)
        e = np.zeros_like(F)
        for m in range(p):
            Phi = F + self.A @ (P * e)
            if j + 1 < len(self.ps):
                s = self.inner_sigma(j, sigma)
                Phi = -(2.0 / (s * s)) * self.E(j + 1, Phi, s)
            if m == 0:
                e_next = -(0.5 * h2 * (2.0 * p * p / (cc.omega * cc.delta))) * Phi
            else:
                c = h2 * (2.0 * p * p / cc.omega) * cc.beta_half[m]
                e_next = (1.0 + cc.beta[m]) * e - cc.beta[m] * e_prev - c * Phi
            e_prev, e = e, e_next
        return e

    def d1(self, z, dt):
        """Increment of one step: q_1(z) - z = E_1(A z)."""
        return self.E(0, self.A @ z, dt)

    def run(self, u0, dt, n_steps, keep=False):
        """u(T) after n_steps steps from u_0 at rest (and all u_n when ``keep``)."""
        zm = u0
        zc = u0 + self.d1(u0, dt)
        zs = [zm, zc] if keep else None
        for _ in range(1, n_steps):
            zm, zc = zc, 2.0 * zc - zm + 2.0 * self.d1(zc, dt)
            if keep:
                zs.append(zc)
        return (zc, zs) if keep else zc

    def energy(self, z_np1, z_n, dt):
        """The discrete energy of ``lts.Solver.energy`` with this step's G."""
        d = z_np1 - z_n
        Gz = -2.0 * self.d1(z_n, dt) / (dt * dt)
        return 0.5 * float(d @ (self.m * d)) / (dt * dt) + 0.5 * float(z_np1 @ (self.m * Gz))

