"""Mass-lumped P1 Galerkin operators for the oracle (test infrastructure only).

Sec. 3.1: M_ij = (phi_j, phi_i) with mass lumping (diagonal M), K_ij =
(c grad phi_j, c grad phi_i) with the coefficient of the model problem being
c^2 (the PDE of Sec. 2.1 is u_tt - div(c^2 grad u) = f), so each element T
contributes kappa_T |T| G_T^T G_T with kappa_T = c_T^2.  The semi-discrete
system is M u'' + K u = 0; Sec. 3.1 symmetrizes it with z = M^1/2 u,
A = M^-1/2 K M^-1/2, which is the same dynamics as u'' + M^-1 K u = 0.

Assembly uses the general P1 gradient formula for an arbitrary triangle (no
use of the right-angle structure of the grids) and scipy's COO->CSR summation.
Only DOF rows/columns are kept (homogeneous Dirichlet data).

Reading (binary64 evaluation): K v is evaluated in edge form,
(K v)_i = sum_j K_ij (v_j - v_i) over the assembled off-diagonal entries of
row i, including the couplings to Dirichlet nodes (where v = 0).  For P1
elements the gradients of the barycentric coordinates sum to zero, so each
element matrix has zero row sums and K_ii = -sum_{j != i} K_ij: this is the
same matrix, but evaluated this way it annihilates constants exactly also in
floating point.  A stored diagonal (summed from element diagonals, or from the
off-diagonals) leaves row sums of O(eps K_ii), a spurious potential that is
large next to the smooth modes' eigenvalues on fine meshes and shifts their
frequencies.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .mesh import Level, finish_fplus


@dataclass
class ElementData:
    rows: np.ndarray      # [nE] DOF index of the row of each off-diagonal element entry
    cols: np.ndarray      # [nE] DOF index of the column, -1 for a Dirichlet node
    geo: np.ndarray       # [nE] |T| grad(lambda_a) . grad(lambda_b), a != b
    block: np.ndarray     # [nE] coefficient block of the entry's element
    n: int                # number of DOFs


def element_data(lv: Level) -> ElementData:
    nn = lv.nyn * lv.nxn
    X, Y = np.meshgrid(lv.xs, lv.ys)
    px, py = X.ravel(), Y.ravel()
    dof_index = -np.ones(nn, dtype=np.int64)
    ids = lv.dof_ids
    dof_index[ids] = np.arange(len(ids))

    t = lv.tris
    x = px[t]                                   # [nT, 3]
    y = py[t]
    twoA = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    area = 0.5 * np.abs(twoA)
    # gradients of the barycentric coordinates
    gx = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], axis=1) / twoA[:, None]
    gy = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], axis=1) / twoA[:, None]

    rows, cols, geo, tri = [], [], [], []
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            ra = dof_index[t[:, a]]
            cb = dof_index[t[:, b]]
            keep = ra >= 0
            rows.append(ra[keep])
            cols.append(cb[keep])
            geo.append((area * (gx[:, a] * gx[:, b] + gy[:, a] * gy[:, b]))[keep])
            tri.append(np.flatnonzero(keep))
    tri = np.concatenate(tri)
    block = lv.cell_block.ravel()[lv.tri_cell[tri]]
    return ElementData(rows=np.concatenate(rows), cols=np.concatenate(cols),
                       geo=np.concatenate(geo), block=block, n=len(ids))


class EdgeStiffness:
    """K(kappa) in edge form, K v = E^T diag(c) E v: E is the signed incidence
    matrix of the stiffness graph (one row per coupled pair i < j of DOFs, +1 at
    i and -1 at j, and one row per DOF coupled to Dirichlet nodes, +1 at the DOF),
    c_e = -K_ij the edge weights.  E v forms the differences v_i - v_j exactly
    up to one rounding, so constants are annihilated exactly."""

    def __init__(self, ed: ElementData, kappa_blocks):
        kb = np.asarray(kappa_blocks)
        vals = kb[ed.block] * ed.geo
        n = ed.n
        cols = np.where(ed.cols >= 0, ed.cols, n)
        C = sp.csr_matrix((vals, (ed.rows, cols)), shape=(n, n + 1)).tocoo()
        r, c, k = C.row, C.col, C.data
        inner = (c < n) & (r < c)
        ground = c == n
        er = np.concatenate([r[inner], r[ground]])
        ec = np.concatenate([c[inner], np.full(int(ground.sum()), -1)])
        self.w = -np.concatenate([k[inner], k[ground]])
        ne = er.size
        rows = np.concatenate([np.arange(ne), np.flatnonzero(ec >= 0)])
        colsE = np.concatenate([er, ec[ec >= 0]])
        vals_e = np.concatenate([np.ones(ne), -np.ones(int((ec >= 0).sum()))])
        self.E = sp.csr_matrix((vals_e, (rows, colsE)), shape=(ne, n))
        self.ET = self.E.T.tocsr()
        self.n = n
        self.dtype = np.result_type(self.w)

    def __matmul__(self, v):
        return self.ET @ (self.w * (self.E @ v))

    def matrix(self) -> sp.csr_matrix:
        """The same K as an explicit DOF x DOF matrix."""
        return (self.ET @ sp.diags(self.w) @ self.E).tocsr()


def stiffness(ed: ElementData, kappa_blocks) -> sp.csr_matrix:
    """K(kappa) = sum_T kappa_T |T| G_T^T G_T on the DOFs as an explicit CSR matrix
    (for tests and structure); solvers apply it through EdgeStiffness.
    ``kappa_blocks`` may be complex (complex-step differentiation)."""
    return EdgeStiffness(ed, kappa_blocks).matrix()


@dataclass
class Operators:
    lv: Level
    ed: ElementData
    m: np.ndarray          # [n] lumped mass on the DOFs
    Pd: np.ndarray         # [n] 0/1 diagonal of the projector P on the DOFs
    qoi_w: np.ndarray      # [n] QoI weights on the DOFs


def operators(lv: Level) -> Operators:
    ed = element_data(lv)
    ids = lv.dof_ids
    K1 = stiffness(ed, np.ones(lv.n_blocks))
    finish_fplus(lv, K1)
    return Operators(lv=lv, ed=ed, m=lv.mass.ravel()[ids].copy(),
                     Pd=lv.Pmask.ravel()[ids].astype(np.float64),
                     qoi_w=lv.qoi_w.ravel()[ids].copy())


class MassScaled:
    """A_u = M^-1 K applied as (K v) / m with K in edge form; its transpose applies
    K (v / m)."""

    def __init__(self, K, m):
        self.K = K
        self.m = m
        self.dtype = K.dtype

    def __matmul__(self, v):
        return (self.K @ v) / self.m

    @property
    def T(self):
        return _MassScaledT(self.K, self.m)


class _MassScaledT:
    def __init__(self, K, m):
        self.K = K
        self.m = m

    def __matmul__(self, v):
        return self.K @ (v / self.m)


def mass_scaled_operator(ops: Operators, kappa_blocks) -> MassScaled:
    """A_u = M^-1 K(kappa): the operator of u'' + A_u u = 0 (Sec. 3.1)."""
    return MassScaled(EdgeStiffness(ops.ed, kappa_blocks), ops.m)


def sym_operator(ops: Operators, kappa_blocks) -> sp.csr_matrix:
    """A = M^-1/2 K M^-1/2 (the symmetrized form of Sec. 3.1); used by tests."""
    K = stiffness(ops.ed, kappa_blocks)
    d = sp.diags(1.0 / np.sqrt(ops.m))
    return (d @ K @ d).tocsr()
