"""Seeded triangle meshes for the triangle-mesh tests (input generation only:
node positions, triangles, Dirichlet nodes, blocks, fine flags and QoI node
weights; none of the method's arithmetic).  Used by the oracle tests and the
GPU parity tests alike."""
from __future__ import annotations

import numpy as np


def _ccw(xy, tris):
    t = np.asarray(tris, dtype=np.int64).copy()
    x, y = xy[t, 0], xy[t, 1]
    a = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    flip = a < 0
    t[flip, 1], t[flip, 2] = t[flip, 2].copy(), t[flip, 1].copy()
    return t


def _blocks(xy, tris, nbx=4, nby=4):
    c = xy[tris].mean(axis=1)
    bx = np.minimum((c[:, 0] * nbx).astype(np.int64), nbx - 1)
    by = np.minimum((c[:, 1] * nby).astype(np.int64), nby - 1)
    return by * nbx + bx


def _qoi_nodes(xy, box=(0.6, 0.8, 0.6, 0.8)):
    """Weights of the mean of the nodal values inside the box."""
    inside = (xy[:, 0] >= box[0]) & (xy[:, 0] <= box[1]) & (xy[:, 1] >= box[2]) & (xy[:, 1] <= box[3])
    return np.where(inside, 1.0 / max(int(inside.sum()), 1), 0.0)


def criss_cross(n: int = 16, box=(0.375, 0.625), ref: int = 4, jitter: float = 0.15, seed: int = 0,
                qoi_box=(0.6, 0.8, 0.6, 0.8)) -> dict:
    """Unit square, n cells per axis; per axis the cells meeting the open box are
    split into `ref` parts.  Interior nodes move by up to `jitter` of the
    smaller adjacent spacing in each coordinate; cell (a, b) is split along
    the diagonal through its lower-left corner when a + b is even, else the
    other one.  Fine elements: those of cells narrower than 1/(2n) in some
    direction.  p = ref.  Dirichlet: the boundary nodes.  QoI: the mean of the
    nodal values in qoi_box."""
    rng = np.random.default_rng(seed)
    edges = []
    for k in range(n):
        a, b = k / n, (k + 1) / n
        if b > box[0] and a < box[1]:
            edges.extend(a + (b - a) * j / ref for j in range(ref))
        else:
            edges.append(a)
    xs = np.array(edges + [1.0])
    m = len(xs)
    X, Y = np.meshgrid(xs, xs)
    gap = np.minimum(np.diff(xs)[:-1], np.diff(xs)[1:])      # smaller spacing next to interior nodes
    JX = np.zeros((m, m))
    JY = np.zeros((m, m))
    JX[:, 1:-1] = rng.uniform(-jitter, jitter, (m, m - 2)) * gap[None, :]
    JY[1:-1, :] = rng.uniform(-jitter, jitter, (m - 2, m)) * gap[:, None]
    X = X + JX
    Y = Y + JY
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    tris, fine = [], []
    h = 1.0 / n
    for bj in range(m - 1):
        for ai in range(m - 1):
            n00 = bj * m + ai
            n10, n01, n11 = n00 + 1, n00 + m, n00 + m + 1
            if (ai + bj) % 2 == 0:
                tris += [(n00, n10, n11), (n00, n11, n01)]
            else:
                tris += [(n00, n10, n01), (n10, n11, n01)]
            f = min(xs[ai + 1] - xs[ai], xs[bj + 1] - xs[bj]) < 0.5 * h
            fine += [f, f]
    tris = _ccw(xy, tris)
    bnd = np.zeros((m, m), dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    return {"xy": xy, "tris": tris, "dirichlet": bnd.ravel(), "tri_block": _blocks(xy, tris),
            "tri_fine": np.asarray(fine, dtype=bool), "qoi_nodes": _qoi_nodes(xy, qoi_box), "n_blocks": 16,
            "h": h, "p": ref, "nu": 0.01}


def delaunay_disk(n: int = 12, centre=(0.5, 0.5), radius: float = 0.15, ref: int = 3, jitter: float = 0.2,
                  seed: int = 0) -> dict:
    """Delaunay triangulation of a jittered n x n lattice on the unit square
    (boundary nodes on the boundary) whose points inside a disk are replaced by
    a jittered lattice `ref` times denser.  Fine elements: those with all three
    vertices in the disk grown by one fine spacing.  p = ref."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g)
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    inner = (P[:, 0] > 0) & (P[:, 0] < 1) & (P[:, 1] > 0) & (P[:, 1] < 1)
    P[inner] += rng.uniform(-jitter, jitter, (int(inner.sum()), 2)) * h
    r = np.hypot(P[:, 0] - centre[0], P[:, 1] - centre[1])
    P = P[~inner | (r > radius + 0.5 * h)]
    hf = h / ref
    gf = np.arange(centre[0] - radius, centre[0] + radius + 0.5 * hf, hf)
    FX, FY = np.meshgrid(gf, gf - centre[0] + centre[1])
    F = np.stack([FX.ravel(), FY.ravel()], axis=1)
    F = F[np.hypot(F[:, 0] - centre[0], F[:, 1] - centre[1]) <= radius]
    F += rng.uniform(-jitter, jitter, F.shape) * hf
    xy = np.concatenate([P, F])
    tris = _ccw(xy, Delaunay(xy).simplices)
    x, y = xy[tris, 0], xy[tris, 1]
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    tris = tris[area > 1e-12]
    rr = np.hypot(xy[:, 0] - centre[0], xy[:, 1] - centre[1]) <= radius + hf
    fine = rr[tris].all(axis=1)
    bnd = (xy[:, 0] <= 0) | (xy[:, 0] >= 1) | (xy[:, 1] <= 0) | (xy[:, 1] >= 1)
    return {"xy": xy, "tris": tris, "dirichlet": bnd, "tri_block": _blocks(xy, tris),
            "tri_fine": fine, "qoi_nodes": _qoi_nodes(xy), "n_blocks": 16, "h": h, "p": ref, "nu": 0.01}
