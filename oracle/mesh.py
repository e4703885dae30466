"""Level meshes for the oracle (test infrastructure only; see package header).

Rectilinear tensor grids, every cell [x_a, x_a+1] x [y_b, y_b+1] split along
the diagonal (x_a, y_b)-(x_a+1, y_b+1) into two P1 triangles, as needed by the
mass-lumped conforming discretization of Sec. 3.1 on the locally refined
meshes of Sec. 3.2 (fixed refined box) and Sec. 3.5 (grading toward a
reentrant corner).

Readings of the paper taken here (the paper does not fix them):
* refined box: per axis, every coarse interval that meets the open box is
  split into ``ref`` equal parts (so the fine cells form a cross of strips);
* graded L-shape: per axis the two cells next to 0 are replaced by nodes
  +-h 2^-j, j = 1..G; cells with midpoint x > 0, y < 0 are removed;
* fine elements are cells with a leg shorter than h/2 (h = the level's base
  spacing), and P marks the DOFs that are vertices of a fine element
  (Sec. 3.3 defines P as the DOFs of the refined part);
* coefficient blocks and the QoI region are decided per cell by its midpoint.

All coordinates are dyadic, so every area, mass and weight below is exact up
to the single final division by 6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# 1-D node rules
# ---------------------------------------------------------------------------

def axis_box_refined(lo: float, hi: float, n_base: int, box_lo: float, box_hi: float,
                     ref: int) -> np.ndarray:
    """Nodes of one axis: n_base uniform cells, the ones meeting (box_lo, box_hi)
    split into ``ref`` parts.  Coordinate of fine index t is lo + t*(h/ref)."""
    h = (hi - lo) / n_base
    hf = (hi - lo) / (n_base * ref)
    nodes = []
    for k in range(n_base):
        a = lo + k * h
        b = lo + (k + 1) * h
        if b > box_lo and a < box_hi:
            for t in range(ref):
                nodes.append(lo + (k * ref + t) * hf)
        else:
            nodes.append(lo + (k * ref) * hf)
    nodes.append(hi)
    return np.array(nodes, dtype=np.float64)


def axis_graded(lo: float, hi: float, n_base: int, layers: int) -> np.ndarray:
    """Nodes of one axis: uniform spacing h, with the two cells adjacent to 0
    replaced by the nodes +-h*2^-j, j = 1..layers (smallest cell h/2^layers)."""
    h = (hi - lo) / n_base
    k0 = None
    for k in range(n_base + 1):
        if lo + k * h == 0.0:
            k0 = k
    if k0 is None or k0 == 0 or k0 == n_base:
        raise ValueError("graded axis needs 0 as an interior node")
    nodes = [lo + k * h for k in range(0, k0)]
    nodes += [-math.ldexp(h, -j) for j in range(1, layers + 1)]
    nodes += [0.0]
    nodes += [math.ldexp(h, -j) for j in range(layers, 0, -1)]
    nodes += [lo + k * h for k in range(k0 + 1, n_base + 1)]
    return np.array(nodes, dtype=np.float64)


# ---------------------------------------------------------------------------
# Level
# ---------------------------------------------------------------------------

@dataclass
class Level:
    xs: np.ndarray            # [nxn] node x-coordinates
    ys: np.ndarray            # [nyn] node y-coordinates
    h: float                  # base spacing of the level
    cell_active: np.ndarray   # [nyc, nxc] bool
    cell_block: np.ndarray    # [nyc, nxc] int, coefficient block of the cell
    cell_fine: np.ndarray     # [nyc, nxc] bool, cell belongs to D_fine
    cell_qoi: np.ndarray      # [nyc, nxc] bool, midpoint inside the QoI box
    n_blocks: int
    p: int
    nu: float
    # derived
    tris: np.ndarray = field(default=None)        # [n_tri, 3] node ids (ccw)
    tri_cell: np.ndarray = field(default=None)    # [n_tri] flat cell index
    dof: np.ndarray = field(default=None)         # [nyn, nxn] bool
    mass: np.ndarray = field(default=None)        # [nyn, nxn] lumped mass (all nodes)
    qoi_w: np.ndarray = field(default=None)       # [nyn, nxn] QoI weights
    Pmask: np.ndarray = field(default=None)       # [nyn, nxn] bool
    Fplus: np.ndarray = field(default=None)       # [nyn, nxn] bool

    @property
    def nxn(self):
        return len(self.xs)

    @property
    def nyn(self):
        return len(self.ys)

    @property
    def dof_ids(self) -> np.ndarray:
        """Flat node ids (j*nxn + i) of the DOFs, in increasing order."""
        return np.flatnonzero(self.dof.ravel())

    @property
    def n_dof(self) -> int:
        return int(self.dof.sum())


def _finish(lv: Level) -> Level:
    nxn, nyn = lv.nxn, lv.nyn
    nxc, nyc = nxn - 1, nyn - 1

    # triangles of every active cell (a, b), node id = b*nxn + a
    bb, aa = np.nonzero(lv.cell_active)
    n00 = bb * nxn + aa
    n10 = n00 + 1
    n11 = n00 + nxn + 1
    n01 = n00 + nxn
    t1 = np.stack([n00, n10, n11], axis=1)
    t2 = np.stack([n00, n11, n01], axis=1)
    cell = bb * nxc + aa
    lv.tris = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int64)
    lv.tri_cell = np.repeat(cell, 2).astype(np.int64)

    X, Y = np.meshgrid(lv.xs, lv.ys)
    px, py = X.ravel(), Y.ravel()

    # a node is a DOF iff all four incident cells exist and are active
    act = lv.cell_active
    dof = np.zeros((nyn, nxn), dtype=bool)
    dof[1:-1, 1:-1] = act[1:, 1:] & act[1:, :-1] & act[:-1, 1:] & act[:-1, :-1]
    lv.dof = dof

    # lumped mass: m_i = (sum over triangles T containing i of 2|T|) / 6,
    # 2|T| from the general cross product of two edge vectors
    t = lv.tris
    x0, y0 = px[t[:, 0]], py[t[:, 0]]
    x1, y1 = px[t[:, 1]], py[t[:, 1]]
    x2, y2 = px[t[:, 2]], py[t[:, 2]]
    ta = np.abs((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0))
    in_q = lv.cell_qoi.ravel()[lv.tri_cell]
    twoA = np.zeros(nyn * nxn)
    twoA_q = np.zeros(nyn * nxn)
    for k in range(3):
        np.add.at(twoA, t[:, k], ta)
        np.add.at(twoA_q, t[:, k], np.where(in_q, ta, 0.0))
    lv.mass = (twoA / 6.0).reshape(nyn, nxn)
    qw = (twoA_q / 6.0).reshape(nyn, nxn)
    qw[~dof] = 0.0          # u = 0 on Dirichlet nodes
    lv.qoi_w = qw

    # P: DOFs that are vertices of a fine element
    P = np.zeros(nyn * nxn, dtype=bool)
    fine_t = lv.cell_fine.ravel()[lv.tri_cell]
    P[t[fine_t].ravel()] = True
    lv.Pmask = P.reshape(nyn, nxn) & dof
    return lv


def finish_fplus(lv: Level, K_full) -> None:
    """F+ = P plus every DOF coupled to P by a nonzero stiffness entry."""
    ids = lv.dof_ids
    Pd = lv.Pmask.ravel()[ids]
    Kabs = abs(K_full)
    touched = (Kabs @ Pd.astype(np.float64)) != 0.0
    F = np.zeros(lv.nyn * lv.nxn, dtype=bool)
    F[ids[touched | Pd]] = True
    lv.Fplus = F.reshape(lv.nyn, lv.nxn)


def _cells(xs, ys, h, active_fn, blo, bhi, nbx, nby, qoi_box):
    hx = np.diff(xs)
    hy = np.diff(ys)
    mx = 0.5 * (xs[:-1] + xs[1:])
    my = 0.5 * (ys[:-1] + ys[1:])
    MX, MY = np.meshgrid(mx, my)          # [nyc, nxc]
    HX, HY = np.meshgrid(hx, hy)
    active = active_fn(MX, MY)
    bx = np.minimum(np.floor((MX - blo) / (bhi - blo) * nbx).astype(np.int64), nbx - 1)
    by = np.minimum(np.floor((MY - blo) / (bhi - blo) * nby).astype(np.int64), nby - 1)
    block = by * nbx + bx
    fine = np.minimum(HX, HY) < 0.5 * h
    qx0, qx1, qy0, qy1 = qoi_box
    qoi = (qx0 <= MX) & (MX <= qx1) & (qy0 <= MY) & (MY <= qy1)
    return active, block, fine, qoi


def _p_from_mesh(xs, ys, h):
    hmin = min(np.min(np.diff(xs)), np.min(np.diff(ys)))
    return int(math.ceil(h / hmin))


def box_refined_level(n_base: int, box=(0.45, 0.55), ref: int = 4, lo: float = 0.0,
                      hi: float = 1.0, blocks=(4, 4), qoi_box=(0.6, 0.8, 0.6, 0.8),
                      p: int | None = None, nu: float = 0.01) -> Level:
    """Unit square refined ``ref`` times inside ``box`` (both axes)."""
    xs = axis_box_refined(lo, hi, n_base, box[0], box[1], ref)
    ys = xs.copy()
    h = (hi - lo) / n_base
    active, block, fine, qoi = _cells(xs, ys, h, lambda mx, my: np.ones(mx.shape, dtype=bool), lo, hi,
                                      blocks[0], blocks[1], qoi_box)
    if p is None:
        p = _p_from_mesh(xs, ys, h)
    lv = Level(xs=xs, ys=ys, h=h, cell_active=active, cell_block=block, cell_fine=fine,
               cell_qoi=qoi, n_blocks=blocks[0] * blocks[1], p=p, nu=nu)
    return _finish(lv)


def graded_L_level(n_base: int, layers: int = 6, lo: float = -1.0, hi: float = 1.0,
                   blocks=(8, 8), qoi_box=(0.5, 0.9, 0.2, 0.6), p: int | None = None,
                   nu: float = 0.01) -> Level:
    """L-shape [-1,1]^2 minus (0,1]x[-1,0), graded toward the reentrant corner."""
    xs = axis_graded(lo, hi, n_base, layers)
    ys = xs.copy()
    h = (hi - lo) / n_base
    active, block, fine, qoi = _cells(xs, ys, h, lambda mx, my: ~((mx > 0.0) & (my < 0.0)),
                                      lo, hi, blocks[0], blocks[1], qoi_box)
    if p is None:
        p = _p_from_mesh(xs, ys, h)
    lv = Level(xs=xs, ys=ys, h=h, cell_active=active, cell_block=block, cell_fine=fine,
               cell_qoi=qoi, n_blocks=blocks[0] * blocks[1], p=p, nu=nu)
    return _finish(lv)


def lf_twin(lv: Level) -> Level:
    """The standard leapfrog level that the cost comparison of Sec. 3.4 and the
    experiments of Sec. 4 set against LF-LTS: the same grid, blocks and QoI
    cells with no fine cells (P empty) and p = 1, so that Algorithm 2 is one
    plain leapfrog step over all DOFs, and nominal spacing h/p, so that a
    sample's step count (T c_max / (cfl h)) is that of the step dt/p which the
    smallest elements need."""
    tw = Level(xs=lv.xs.copy(), ys=lv.ys.copy(), h=lv.h / lv.p, cell_active=lv.cell_active.copy(),
               cell_block=lv.cell_block.copy(), cell_fine=np.zeros_like(lv.cell_fine),
               cell_qoi=lv.cell_qoi.copy(), n_blocks=lv.n_blocks, p=1, nu=lv.nu)
    return _finish(tw)


# ---------------------------------------------------------------------------
# Choice of the fine set on graded meshes (Sec. 3.5)
# ---------------------------------------------------------------------------
#
# Sec. 3.5 takes the fine region D_f of a graded mesh as the union of the q
# tiers of smallest elements; the time step of the coarse region is then set
# by its own smallest elements (tier q+1), and q is chosen to minimise the LTS
# cost, elements of D_f over h_1 plus elements of D_c over h_{q+1}
# (eq. cost_waveeq_LTSgraded, optimum by eq. ddqS).
#
# Readings for the rectilinear geometric grading of graded_L_level: tier k
# (k = 1..layers) holds the cells whose shorter leg is h 2^(k-1-layers) (tier 1
# the smallest, h 2^-layers); cells whose shorter leg is h or longer are the
# outer tier.  With q tiers fine, the fine cells are those with shorter leg
# < h 2^(q-layers).  The coarse step of the level uses the spacing
# H_q = 2 * (shortest coarse leg), and p_q = ceil(H_q / h_min): for
# q = layers - 1 this is the workload's rule (fine cells with a leg < h/2,
# H = h, p = ceil(h / h_min)), which is why the factor 2 is taken.  q = 0 has
# no fine cells (plain leapfrog, p = 1: p is ceil(H / h_min) whenever an
# active cell is fine).  The cost compared across q is the
# DOF-update rate ((N - |P_q|) + p_q |P_q|) / H_q per unit time (the step
# count is T c_max / (cfl H_q)); the smallest q wins a tie.

def graded_L_tiers(n_base: int, q: int, layers: int = 6, lo: float = -1.0, hi: float = 1.0,
                   blocks=(8, 8), qoi_box=(0.5, 0.9, 0.2, 0.6), nu: float = 0.01) -> Level:
    """The graded L-shape level with the q smallest tiers fine (0 <= q <= layers)."""
    if not 0 <= q <= layers:
        raise ValueError("q must be in 0..layers")
    xs = axis_graded(lo, hi, n_base, layers)
    ys = xs.copy()
    h = (hi - lo) / n_base
    active, block, _, qoi = _cells(xs, ys, h, lambda mx, my: ~((mx > 0.0) & (my < 0.0)),
                                   lo, hi, blocks[0], blocks[1], qoi_box)
    HX, HY = np.meshgrid(np.diff(xs), np.diff(ys))
    short = np.minimum(HX, HY)
    fine = short < math.ldexp(h, q - layers)
    coarse_short = short[active & ~fine]
    H = 2.0 * float(coarse_short.min())
    h_min = float(short[active].min())
    lv = Level(xs=xs, ys=ys, h=H, cell_active=active, cell_block=block, cell_fine=fine,
               cell_qoi=qoi, n_blocks=blocks[0] * blocks[1], p=1, nu=nu)
    lv = _finish(lv)
    if (fine & active).any():
        lv.p = int(math.ceil(H / h_min))
    return lv


def lts_cost_rate(lv: Level) -> float:
    """DOF updates per unit time and per unit T c_max / cfl: ((N - |P|) + p |P|) / H."""
    n, nP = lv.n_dof, int(lv.Pmask.sum())
    return ((n - nP) + lv.p * nP) / lv.h


def qopt_tiers(n_base: int, layers: int = 6, p_max: int = 0, **kw):
    """(q_opt, costs): the number of fine tiers minimising the LTS cost rate,
    among the q whose p is at most p_max when p_max > 0 (q = 0 always is)."""
    lvs = [graded_L_tiers(n_base, q, layers, **kw) for q in range(layers + 1)]
    costs = [lts_cost_rate(lv) for lv in lvs]
    ok = [q for q in range(layers + 1) if p_max <= 0 or lvs[q].p <= p_max]
    q = min(ok, key=lambda k: (costs[k], k))
    return q, costs


def cost_lts_graded_model(m: float, s: float, d: int, q: float) -> float:
    """eq. cost_waveeq_LTSgraded: (m^(s+d) + m^s q^d ((q+1)^s - q^s - 1)) / ((q+1)^s - q^s),
    the cost of one LTS solve on the radially graded mesh T_{m,s} with q fine layers."""
    g = (q + 1.0) ** s - q ** s
    return (m ** (s + d) + m ** s * q ** d * (g - 1.0)) / g


def speedup_graded_model(m: float, s: float, d: int, q: float) -> float:
    """eq. speedup_det_graded: C_LF / C_LTS = m^d ((q+1)^s - q^s) / (m^d + q^d ((q+1)^s - q^s - 1))."""
    g = (q + 1.0) ** s - q ** s
    return m ** d * g / (m ** d + q ** d * (g - 1.0))


def ddq_speedup_graded_model(m: float, s: float, d: int, q: float) -> float:
    """Left-hand side of eq. ddqS (proportional to the q-derivative of the speed-up)."""
    g = (q + 1.0) ** s - q ** s
    gs = (q + 1.0) ** (s - 1.0) - q ** (s - 1.0)
    return (s * gs * (m ** d + q ** d * (g - 1.0))
            - g * q ** (d - 1.0) * (d * (g - 1.0) + s * q * gs))
