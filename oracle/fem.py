"""Mass-lumped P1 Galerkin operators for the oracle (test infrastructure only).

Sec. 3.1: M_ij = (phi_j, phi_i) with mass lumping (diagonal M), K_ij =
(c grad phi_j, c grad phi_i) with the coefficient of the model problem being
c^2 (the PDE of Sec. 2.1 is u_tt - div(c^2 grad u) = f), so each element T
contributes kappa_T |T| G_T^T G_T with kappa_T = c_T^2.  The symmetrized
operator of the same section is A = M^-1/2 K M^-1/2 acting on z = M^1/2 u.

The assembly below uses the general P1 gradient formula for an arbitrary
triangle (no use of the right-angle structure of the grids) and scipy's
COO->CSR duplicate summation.  Only DOF rows/columns are kept (homogeneous
Dirichlet data).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .mesh import Level, finish_fplus


@dataclass
class ElementData:
    rows: np.ndarray      # [nE] DOF index of the row of each element entry
    cols: np.ndarray      # [nE]
    geo: np.ndarray       # [nE] |T| grad(lambda_a) . grad(lambda_b)
    block: np.ndarray     # [nE] coefficient block of the entry's element
    tri: np.ndarray       # [nE] triangle index of the entry
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
            ra = dof_index[t[:, a]]
            cb = dof_index[t[:, b]]
            keep = (ra >= 0) & (cb >= 0)
            rows.append(ra[keep])
            cols.append(cb[keep])
            geo.append((area * (gx[:, a] * gx[:, b] + gy[:, a] * gy[:, b]))[keep])
            tri.append(np.flatnonzero(keep))
    tri = np.concatenate(tri)
    block = lv.cell_block.ravel()[lv.tri_cell[tri]]
    return ElementData(rows=np.concatenate(rows), cols=np.concatenate(cols),
                       geo=np.concatenate(geo), block=block, tri=tri, n=len(ids))


def stiffness(ed: ElementData, kappa_blocks) -> sp.csr_matrix:
    """K(kappa) = sum_T kappa_T |T| G_T^T G_T on the DOFs (CSR, duplicates summed).
    ``kappa_blocks`` may be complex (complex-step differentiation)."""
    kb = np.asarray(kappa_blocks)
    vals = kb[ed.block] * ed.geo
    return sp.csr_matrix((vals, (ed.rows, ed.cols)), shape=(ed.n, ed.n))


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


def sym_operator(ops: Operators, kappa_blocks) -> sp.csr_matrix:
    """A = M^-1/2 K M^-1/2 (Sec. 3.1, symmetrized semi-discrete system)."""
    K = stiffness(ops.ed, kappa_blocks)
    d = sp.diags(1.0 / np.sqrt(ops.m))
    return (d @ K @ d).tocsr()
