"""Levels given as triangulations, for the oracle (test infrastructure only;
see the package header).

Sec. 3.1: conforming P1 elements with mass lumping on a triangle mesh; each
element T contributes kappa_T |T| G_T^T G_T to the stiffness (G_T the
gradients of the barycentric coordinates) and |T|/3 to the lumped mass of
each of its vertices.  Sec. 3.3: P is the diagonal projector onto the DOFs
that are vertices of a fine element.  Homogeneous Dirichlet data on the
nodes the caller marks; every other node is a DOF.

The operators are assembled with the same general P1 formulas as for the
rectilinear levels (``fem``), so a tensor grid handed over as a triangle
list gives the rectilinear level's operators, and the solver, pulse and QoI
of ``lts`` apply unchanged.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem


@dataclass
class TriLevel:
    xy: np.ndarray            # [n_nodes, 2]
    tris: np.ndarray          # [n_tris, 3] node ids, counter-clockwise
    dirichlet: np.ndarray     # [n_nodes] bool
    tri_block: np.ndarray     # [n_tris] coefficient block of each element
    tri_fine: np.ndarray      # [n_tris] bool, element in D_fine
    qoi_nodes: np.ndarray     # [n_nodes] QoI weights given per node
    n_blocks: int
    h: float
    p: int
    nu: float
    # derived
    mass: np.ndarray = field(default=None)     # [n_nodes] lumped mass, every node
    Pmask: np.ndarray = field(default=None)    # [n_nodes] bool (DOFs only)
    Fplus: np.ndarray = field(default=None)    # [n_nodes] bool
    qoi_w: np.ndarray = field(default=None)    # [n_nodes] QoI weights, 0 off the DOFs

    @property
    def dof(self) -> np.ndarray:
        return ~self.dirichlet

    @property
    def dof_ids(self) -> np.ndarray:
        """Node ids of the DOFs, in increasing order."""
        return np.flatnonzero(~self.dirichlet)

    @property
    def n_dof(self) -> int:
        return int((~self.dirichlet).sum())

    def dof_coords(self):
        ids = self.dof_ids
        return self.xy[ids, 0], self.xy[ids, 1]


def tri_level(xy, tris, dirichlet, tri_block, tri_fine, qoi_nodes, n_blocks: int, h: float, p: int,
              nu: float) -> TriLevel:
    """Checks the triangulation (positive orientation, every DOF in a triangle)
    and fills the derived per-node data."""
    xy = np.asarray(xy, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    tl = TriLevel(xy=xy, tris=tris, dirichlet=np.asarray(dirichlet, dtype=bool),
                  tri_block=np.asarray(tri_block, dtype=np.int64), tri_fine=np.asarray(tri_fine, dtype=bool),
                  qoi_nodes=np.asarray(qoi_nodes, dtype=np.float64), n_blocks=n_blocks, h=h, p=p, nu=nu)
    nn = len(xy)
    px, py = xy[:, 0], xy[:, 1]
    t = tris
    x0, y0 = px[t[:, 0]], py[t[:, 0]]
    x1, y1 = px[t[:, 1]], py[t[:, 1]]
    x2, y2 = px[t[:, 2]], py[t[:, 2]]
    twoA = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    if np.any(twoA <= 0):
        raise ValueError("triangles must be counter-clockwise")
    used = np.zeros(nn, dtype=bool)
    used[t.ravel()] = True
    if np.any(~tl.dirichlet & ~used):
        raise ValueError("a DOF belongs to no triangle")
    # lumped mass: (sum over triangles T containing i of 2|T|) / 6
    acc = np.zeros(nn)
    for k in range(3):
        np.add.at(acc, t[:, k], np.abs(twoA))
    tl.mass = acc / 6.0
    P = np.zeros(nn, dtype=bool)
    P[t[tl.tri_fine].ravel()] = True
    tl.Pmask = P & tl.dof
    tl.qoi_w = np.where(tl.dof, tl.qoi_nodes, 0.0)
    return tl


def element_data(tl: TriLevel) -> fem.ElementData:
    """Off-diagonal element entries |T| grad(lambda_a) . grad(lambda_b) of every
    triangle (the general P1 formula, as fem.element_data)."""
    px, py = tl.xy[:, 0], tl.xy[:, 1]
    dof_index = -np.ones(len(tl.xy), dtype=np.int64)
    ids = tl.dof_ids
    dof_index[ids] = np.arange(len(ids))
    t = tl.tris
    x = px[t]
    y = py[t]
    twoA = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    area = 0.5 * np.abs(twoA)
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
    return fem.ElementData(rows=np.concatenate(rows), cols=np.concatenate(cols), geo=np.concatenate(geo),
                           block=tl.tri_block[tri], n=len(ids))


def operators(tl: TriLevel) -> fem.Operators:
    """Lumped mass, P, F+ (P and the DOFs coupled to P by a nonzero entry of
    K with unit coefficient) and the element data of a triangle-mesh level."""
    ed = element_data(tl)
    ids = tl.dof_ids
    K1 = fem.stiffness(ed, np.ones(tl.n_blocks))
    Pd = tl.Pmask[ids]
    touched = (abs(K1) @ Pd.astype(np.float64)) != 0.0
    F = np.zeros(len(tl.xy), dtype=bool)
    F[ids[touched | Pd]] = True
    tl.Fplus = F
    return fem.Operators(lv=tl, ed=ed, m=tl.mass[ids].copy(), Pd=Pd.astype(np.float64),
                         qoi_w=tl.qoi_w[ids].copy())


def from_grid_level(lv) -> TriLevel:
    """A rectilinear level handed over as a triangle list: its nodes, its
    triangles in order, Dirichlet = not a DOF, each triangle's cell block and
    fine flag, and the level's QoI weights per node."""
    X, Y = np.meshgrid(lv.xs, lv.ys)
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    return tri_level(xy, lv.tris, ~lv.dof.ravel(), lv.cell_block.ravel()[lv.tri_cell],
                     lv.cell_fine.ravel()[lv.tri_cell], lv.qoi_w.ravel(), lv.n_blocks, lv.h, lv.p, lv.nu)


def stiffness_full(tl: TriLevel, kappa_blocks) -> sp.csr_matrix:
    """K(kappa) over all nodes (no Dirichlet rows removed): sum over elements of
    kappa_T |T| G_T^T G_T, assembled from the element matrices directly."""
    px, py = tl.xy[:, 0], tl.xy[:, 1]
    t = tl.tris
    kb = np.asarray(kappa_blocks, dtype=np.float64)[tl.tri_block]
    rows, cols, vals = [], [], []
    for e in range(len(t)):
        v = t[e]
        x = px[v]
        y = py[v]
        twoA = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0])
        G = np.array([[y[1] - y[2], y[2] - y[0], y[0] - y[1]],
                      [x[2] - x[1], x[0] - x[2], x[1] - x[0]]]) / twoA
        Ke = kb[e] * 0.5 * abs(twoA) * (G.T @ G)
        for a in range(3):
            for b in range(3):
                rows.append(v[a])
                cols.append(v[b])
                vals.append(Ke[a, b])
    n = len(tl.xy)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
