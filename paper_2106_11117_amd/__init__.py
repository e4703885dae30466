"""MLMC with stabilized leapfrog local time-stepping on MI355X (gfx950).

Thin Python binding of the C ABI in ``include/lfltsmc.h``: argument
marshalling only; every step of the solve runs in the library's HIP kernels.
Host arrays are numpy arrays; device arrays are torch tensors on the
context's device (torch is used for device memory and streams only).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (LTS_BATCH_GRAPH, LTS_FP32_STEP, LTS_FP64, LTS_MLMC_BATCHED, LTS_MLMC_PLAIN,
                   LTS_NODE_DOF, LTS_NODE_FPLUS, LTS_NODE_P, LTS_PTR_DEVICE, LTS_PTR_HOST,
                   LTS_RULE_BOX, LTS_RULE_GRADED_L, LTS_RULE_LF, LtsError)

__all__ = ["Context", "gen_samples", "mesh_host", "line_rule", "line_sample_rule", "line_level_host", "gen_line_samples", "philox", "rect_level_host", "tiling_host", "lf_rule", "cheb_constants", "sample_rule", "box_rule", "graded_L_rule", "LtsError",
           "LTS_FP64", "LTS_FP32_STEP", "LTS_BATCH_GRAPH", "LTS_MLMC_BATCHED", "LTS_MLMC_PLAIN",
           "LTS_NODE_DOF", "LTS_NODE_P", "LTS_NODE_FPLUS", "LTS_RULE_LF", "LtsQoI"]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def box_rule(n_base, box=(0.45, 0.55), ref=4, lo=0.0, hi=1.0, blocks=(4, 4),
             qoi=(0.6, 0.8, 0.6, 0.8), p=0, nu=0.01) -> _lib.RectRule:
    """Square [lo,hi]^2, refined `ref` times in the coarse cells meeting the open box."""
    return _lib.RectRule(kind=LTS_RULE_BOX, lo=lo, hi=hi, n_base=n_base, box_lo=box[0], box_hi=box[1],
                         ref=ref, layers=0, nbx=blocks[0], nby=blocks[1], qx_lo=qoi[0], qx_hi=qoi[1],
                         qy_lo=qoi[2], qy_hi=qoi[3], p=p, nu=nu)


def graded_L_rule(n_base, layers=6, lo=-1.0, hi=1.0, blocks=(8, 8), qoi=(0.5, 0.9, 0.2, 0.6),
                  p=0, nu=0.01, fine_tiers=None, p_max=0) -> _lib.RectRule:
    """L-shape [lo,hi]^2 minus the quadrant x > 0, y < 0, graded toward the corner.
    fine_tiers: None (cells with a leg < h/2), an int q (the q smallest tiers)
    or "opt" (q by the LTS cost model among the q with p <= p_max if p_max > 0;
    see LTS_FINE_QOPT)."""
    rule, q = _lib.LTS_FINE_HALF_H, 0
    if fine_tiers == "opt":
        rule = _lib.LTS_FINE_QOPT
    elif fine_tiers is not None:
        rule, q = _lib.LTS_FINE_TIERS, int(fine_tiers)
    return _lib.RectRule(kind=LTS_RULE_GRADED_L, lo=lo, hi=hi, n_base=n_base, box_lo=0.0, box_hi=0.0,
                         ref=1, layers=layers, nbx=blocks[0], nby=blocks[1], qx_lo=qoi[0],
                         qx_hi=qoi[1], qy_lo=qoi[2], qy_hi=qoi[3], p=p, nu=nu, fine_rule=rule,
                         fine_tiers=q, p_max=p_max)


def lf_rule(rule) -> _lib.RectRule:
    """The standard leapfrog twin of a rule's level: same grid, no fine cells,
    p = 1, nominal spacing h/p (see LTS_RULE_LF)."""
    r = _lib.RectRule.from_buffer_copy(rule)
    r.kind = rule.kind | LTS_RULE_LF
    return r


def sample_rule(n_blocks=16, sigma=0.25, pulse=(0.2, 0.4, 0.2, 0.4), width=0.05, T=1.0,
                cfl=0.2) -> _lib.SampleRule:
    return _lib.SampleRule(n_blocks=n_blocks, sigma=sigma, px_lo=pulse[0], px_hi=pulse[1],
                           py_lo=pulse[2], py_hi=pulse[3], width=width, T=T, cfl=cfl)


def _check(code, ctx=None):
    if code != 0:
        msg = _lib.load().lts_last_error(ctx).decode() if ctx else ""
        raise LtsError(code, msg)


def philox(ctr, key):
    """Raw Philox4x64-10 block (4 words) at counter ``ctr`` and key ``key``."""
    lib = _lib.load()
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    _check(lib.lts_philox4x64_10(c, k, o))
    return [int(v) for v in o]


def gen_samples(seed, sample_level, first_index, n, rule, h_mesh):
    """Host sample generation: dict of g, kappa [n, nb], x0 [n, 2], n_steps [n], dt [n]."""
    lib = _lib.load()
    nb = rule.n_blocks
    g = np.zeros((n, nb))
    kappa = np.zeros((n, nb))
    x0 = np.zeros((n, 2))
    ns = np.zeros(n, dtype=np.int32)
    dt = np.zeros(n)
    _check(lib.lts_gen_samples(C.c_uint64(seed), sample_level, first_index, n, C.byref(rule), h_mesh,
                               _dp(g), _dp(kappa), _dp(x0), _ip(ns), _dp(dt)))
    return {"g": g, "kappa": kappa, "x0": x0, "n_steps": ns, "dt": dt}


def rect_level_host(rule) -> dict:
    """Build a rule-described level on the host only; info plus derived arrays."""
    lib = _lib.load()
    info = _lib.LevelInfo()
    _check(lib.lts_rect_level_host(C.byref(rule), C.byref(info), None, None, None, None, None, None))
    nx, ny = info.nx_nodes, info.ny_nodes
    x, y = np.zeros(nx), np.zeros(ny)
    flags = np.zeros((ny, nx), dtype=np.uint8)
    mass, qw = np.zeros((ny, nx)), np.zeros((ny, nx))
    cb = np.zeros((ny - 1, nx - 1), dtype=np.int32)
    _check(lib.lts_rect_level_host(C.byref(rule), C.byref(info), _dp(x), _dp(y),
                                   flags.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(mass), _dp(qw),
                                   _ip(cb)))
    d = {k: getattr(info, k) for k, _ in _lib.LevelInfo._fields_}
    d.update({"x": x, "y": y, "flags": flags, "mass": mass, "qoi_w": qw, "cell_block": cb})
    return d


def tiling_host(rule, tile_x, tile_y, rect) -> dict:
    """Host only: the fine-tile tiling lts_set_tiling would pick for the level of
    `rule` (0, 0, rect=False: adaptive) with the tile that writes each node back
    (`owner`, [ny, nx]: -1 none, -2 more than one)."""
    lib = _lib.load()
    lv = rect_level_host(rule)
    owner = np.zeros((lv["ny_nodes"], lv["nx_nodes"]), dtype=np.int32)
    info = _lib.TilingInfo()
    _check(lib.lts_tiling_host(C.byref(rule), tile_x, tile_y, 1 if rect else 0, C.byref(info), _ip(owner)))
    d = {k: getattr(info, k) for k, _ in _lib.TilingInfo._fields_}
    d["owner"] = owner
    d["flags"] = lv["flags"]
    return d


def cheb_constants(p, nu, dt=1.0) -> dict:
    """Library-side stabilized Chebyshev constants and per-step coefficients."""
    lib = _lib.load()
    d, w = C.c_double(), C.c_double()
    b, bh, cf = np.zeros(p), np.zeros(p), np.zeros(p + 1)
    _check(lib.lts_cheb_constants(p, nu, dt, C.byref(d), C.byref(w), _dp(b), _dp(bh), _dp(cf)))
    return {"delta": d.value, "omega": w.value, "beta": b, "beta_half": bh, "coef": cf}


def line_rule(kind="kl", level=0, nu=0.01, lf=False) -> _lib.LineRule:
    """Level `level` of a one-dimensional workload on (0, 6): kind "kl" (Sec. 4.1,
    D_fine = [5 - 1/16, 5] at 2^-8) or "jump" (Sec. 4.2, [4 - 1/16, 4] at 2^-9),
    coarse spacing H = 2^-(level+4); lf: its standard leapfrog twin."""
    f = (5.0 - 1.0 / 16, 5.0, 2.0 ** -8) if kind == "kl" else (4.0 - 1.0 / 16, 4.0, 2.0 ** -9)
    return _lib.LineRule(lo=0.0, hi=6.0, H=2.0 ** -(level + 4), fine_lo=f[0], fine_hi=f[1], h_fine=f[2], nu=nu,
                         lf=1 if lf else 0)


def line_sample_rule(kind="kl", T=None, cfl=0.5) -> _lib.LineSampleRule:
    """The random wave speed, pulse and horizon of a one-dimensional workload
    (T = 11 for "kl", 6 for "jump"; jump position uniform in [4 - 1/16, 4], c = 1 | 2)."""
    return _lib.LineSampleRule(kind=_lib.LTS_LINE_KL if kind == "kl" else _lib.LTS_LINE_JUMP,
                               jump_lo=4.0 - 1.0 / 16, jump_hi=4.0, c_left=1.0, c_right=2.0, pulse_x=3.0,
                               pulse_w2=0.09, T=(11.0 if kind == "kl" else 6.0) if T is None else T, cfl=cfl)


class _MeshArgs:
    """Marshals a triangle mesh (dict or keyword arrays: xy [n, 2], tris [t, 3]
    counter-clockwise, dirichlet [n] bool, tri_block [t], tri_fine [t] bool,
    qoi_nodes [n], n_blocks, h, p, nu) into an lts_mesh_desc."""

    def __init__(self, m):
        self.keep = [np.ascontiguousarray(m["xy"], dtype=np.float64),
                     np.ascontiguousarray(m["tris"], dtype=np.int32),
                     np.ascontiguousarray(m["dirichlet"], dtype=np.uint8),
                     np.ascontiguousarray(m["tri_block"], dtype=np.int32),
                     np.ascontiguousarray(m["tri_fine"], dtype=np.uint8),
                     np.ascontiguousarray(m["qoi_nodes"], dtype=np.float64)]
        xy, tri, dr, tb, tf, qw = self.keep
        self.n_nodes = len(xy)
        self.d = _lib.MeshDesc(n_nodes=len(xy), n_tris=len(tri), n_blocks=int(m["n_blocks"]),
                               xy=xy.ctypes.data, tri=tri.ctypes.data, dirichlet=dr.ctypes.data,
                               tri_block=tb.ctypes.data, tri_fine=tf.ctypes.data, qoi_w=qw.ctypes.data,
                               h=float(m["h"]), p=int(m["p"]), nu=float(m["nu"]))


def mesh_host(m) -> dict:
    """Host only: build a triangle-mesh level as lts_add_mesh does; its info,
    per-node LTS_NODE_* flags and lumped masses."""
    lib = _lib.load()
    a = _MeshArgs(m)
    info = _lib.MeshInfo()
    flags = np.zeros(a.n_nodes, dtype=np.uint8)
    mass = np.zeros(a.n_nodes)
    _check(lib.lts_mesh_host(C.byref(a.d), C.byref(info), flags.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(mass)))
    d = {k: getattr(info, k) for k, _ in _lib.MeshInfo._fields_}
    d.update(flags=flags, mass=mass)
    return d


def _mlts_desc(ps, cell_tier, max_region=0):
    """lts_mlts_desc for ratios ps (tier 1 first), cell tiers [ny_cells, nx_cells]
    (uint8) or None (the halving rule) and the region cap (0: 2048); returns
    (desc, keep-alive array)."""
    ps = [int(v) for v in ps]
    d = _lib.MltsDesc()
    d.n_tiers = len(ps)
    d.max_region = int(max_region)
    for j, v in enumerate(ps[:_lib.LTS_MLTS_MAX_TIERS]):
        d.p[j] = v
    ct = None
    if cell_tier is not None:
        ct = np.ascontiguousarray(cell_tier, dtype=np.uint8)
        d.cell_tier = ct.ctypes.data
    return d, ct


def _mlts_dict(info) -> dict:
    n = info.n_tiers
    return {"n_tiers": n, "p": list(info.p)[:n], "n_P": list(info.n_P)[:n], "phases": info.phases,
            "n_tiles": info.n_tiles, "max_region": info.max_region, "threads": info.threads,
            "halo_ratio": info.halo_ratio, "updates_per_step": info.updates_per_step}


def mlts_host(rule, ps, cell_tier=None, max_region=0) -> dict:
    """Host only: the tiers lts_set_mlts would attach to the level of `rule`,
    with node_tier [ny_nodes, nx_nodes] (largest j with the node in P_j)."""
    lib = _lib.load()
    lv = rect_level_host(rule)
    d, keep = _mlts_desc(ps, cell_tier, max_region)
    info = _lib.MltsInfo()
    nt = np.zeros((lv["ny_nodes"], lv["nx_nodes"]), dtype=np.uint8)
    _check(lib.lts_mlts_host(C.byref(rule), C.byref(d), C.byref(info), nt.ctypes.data_as(C.POINTER(C.c_uint8))))
    out = _mlts_dict(info)
    out["node_tier"] = nt
    return out


def line_level_host(rule) -> dict:
    lib = _lib.load()
    info = _lib.LineInfo()
    _check(lib.lts_line_level_host(C.byref(rule), C.byref(info), None, None, None))
    n = info.n_nodes
    x, m, P = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.uint8)
    _check(lib.lts_line_level_host(C.byref(rule), C.byref(info), _dp(x), _dp(m),
                                   P.ctypes.data_as(C.POINTER(C.c_uint8))))
    d = {k: getattr(info, k) for k, _ in _lib.LineInfo._fields_}
    d.update(x=x, mass=m, P=P)
    return d


def gen_line_samples(seed, sample_level, first, n, rule, mesh) -> dict:
    """Host: kappa [n, cells], n_steps [n], dt [n] of a one-dimensional workload."""
    lib = _lib.load()
    cells = line_level_host(mesh)["n_nodes"] - 1
    kap, ns, dt = np.zeros((n, cells)), np.zeros(n, dtype=np.int32), np.zeros(n)
    _check(lib.lts_gen_line_samples(C.c_uint64(seed), sample_level, first, n, C.byref(rule), C.byref(mesh),
                                    _dp(kap), _ip(ns), _dp(dt)))
    return {"kappa": kap, "n_steps": ns, "dt": dt}


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _wait_caller_stream(t):
    """Device inputs are read on the library's stream: wait for the work the
    caller queued on torch's current stream (which produced them) first."""
    import torch
    torch.cuda.current_stream(t.device).synchronize()


class _SampleArgs:
    """Marshals kappa (or g = log c when kappa is None) / x0 / n_steps / dt
    (numpy -> host, torch cuda -> device)."""

    def __init__(self, kappa, x0, n_steps, dt, width, g=None):
        coef = kappa if kappa is not None else g
        self.dev = _is_torch(coef)
        if self.dev:
            import torch
            self.keep = [coef.contiguous().to(torch.float64), x0.contiguous().to(torch.float64),
                         n_steps.contiguous().to(torch.int32), dt.contiguous().to(torch.float64)]
            ptrs = [t.data_ptr() for t in self.keep]
            n = int(self.keep[3].numel())
            _wait_caller_stream(self.keep[0])
        else:
            self.keep = [np.ascontiguousarray(coef, dtype=np.float64),
                         np.ascontiguousarray(x0, dtype=np.float64),
                         np.ascontiguousarray(n_steps, dtype=np.int32),
                         np.ascontiguousarray(dt, dtype=np.float64)]
            ptrs = [a.ctypes.data for a in self.keep]
            n = int(self.keep[3].size)
        self.n = n
        kp, gp = (ptrs[0], None) if kappa is not None else (None, ptrs[0])
        self.s = _lib.Samples(n=n, ptr_kind=LTS_PTR_DEVICE if self.dev else LTS_PTR_HOST,
                              kappa=kp, x0=ptrs[1], n_steps=ptrs[2], dt=ptrs[3], width=width, g=gp)

    def out(self, count=None):
        count = self.n if count is None else count
        if self.dev:
            import torch
            t = torch.empty(count, dtype=torch.float64, device=self.keep[0].device)
            return t, t.data_ptr()
        a = np.zeros(count)
        return a, a.ctypes.data


class Context:
    """A library context on one HIP device (see lts_create)."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = _lib.load()
        self.h = C.c_void_p()
        _check(self.lib.lts_create(C.byref(self.h), device, stream))
        self.levels = []

    def close(self):
        if self.h:
            self.lib.lts_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, code):
        _check(code, self.h)

    # --- levels -----------------------------------------------------------
    def add_rect_level(self, rule) -> int:
        lid = C.c_int32()
        self._c(self.lib.lts_build_rect_level(self.h, C.byref(rule), C.byref(lid)))
        self.levels.append(lid.value)
        return lid.value

    def add_level(self, x, y, cell_block, cell_fine, cell_qoi, n_blocks, h, p, nu, cell_active=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        cb = np.ascontiguousarray(cell_block, dtype=np.int32)
        cf = np.ascontiguousarray(cell_fine, dtype=np.uint8)
        cq = np.ascontiguousarray(cell_qoi, dtype=np.uint8)
        ca = None if cell_active is None else np.ascontiguousarray(cell_active, dtype=np.uint8)
        u8 = C.POINTER(C.c_uint8)
        d = _lib.GridDesc(nx_cells=len(x) - 1, ny_cells=len(y) - 1, x=_dp(x), y=_dp(y),
                          cell_active=ca.ctypes.data_as(u8) if ca is not None else None,
                          cell_block=_ip(cb), cell_fine=cf.ctypes.data_as(u8),
                          cell_qoi=cq.ctypes.data_as(u8), n_blocks=n_blocks, h=h, p=p, nu=nu)
        lid = C.c_int32()
        self._c(self.lib.lts_add_level(self.h, C.byref(d), C.byref(lid)))
        self.levels.append(lid.value)
        return lid.value

    def autotune(self, level) -> dict:
        """Measure the candidate fine-tile shapes of `level` and keep the fastest."""
        self._c(self.lib.lts_autotune(self.h, level))
        return self.level_info(level)

    def set_tiling(self, level, tile_x, tile_y, rect=True, mix=False):
        """Pin the fine-tile shape and mode of a level (see lts_set_tiling);
        mix=True (rect mode): coarse items and fine tiles in one launch."""
        self._c(self.lib.lts_set_tiling(self.h, level, tile_x, tile_y, (2 if mix else 1) if rect else 0))
        return self.level_info(level)

    def level_info(self, level) -> dict:
        info = _lib.LevelInfo()
        self._c(self.lib.lts_level_info_get(self.h, level, C.byref(info)))
        return {k: getattr(info, k) for k, _ in _lib.LevelInfo._fields_}

    def level_arrays(self, level) -> dict:
        i = self.level_info(level)
        nx, ny = i["nx_nodes"], i["ny_nodes"]
        x, y = np.zeros(nx), np.zeros(ny)
        flags = np.zeros((ny, nx), dtype=np.uint8)
        mass, qw = np.zeros((ny, nx)), np.zeros((ny, nx))
        cb = np.zeros((ny - 1, nx - 1), dtype=np.int32)
        self._c(self.lib.lts_level_arrays(self.h, level, _dp(x), _dp(y),
                                          flags.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(mass),
                                          _dp(qw), _ip(cb)))
        return {"x": x, "y": y, "flags": flags, "mass": mass, "qoi_w": qw, "cell_block": cb}

    # --- solves -----------------------------------------------------------
    def forward(self, level, kappa, x0, n_steps, dt, width=0.05, precision=LTS_FP64, plain=False, g=None):
        """Q of every sample; the coefficient is kappa = c^2, or g = log c with kappa=None."""
        sa = _SampleArgs(kappa, x0, n_steps, dt, width, g)
        q, qp = sa.out()
        fn = self.lib.lts_forward_plain if plain else self.lib.lts_forward
        self._c(fn(self.h, level, C.byref(sa.s), precision, qp))
        return q

    def forward_noalloc(self, level, kappa, x0, n_steps, dt, width=0.05, precision=LTS_FP64, g=None):
        """forward() through lts_forward_noalloc: no device allocation in the
        library; the batch must fit its fixed per-GPU scratch."""
        sa = _SampleArgs(kappa, x0, n_steps, dt, width, g)
        q, qp = sa.out()
        self._c(self.lib.lts_forward_noalloc(self.h, level, C.byref(sa.s), precision, qp))
        return q

    def forward_coupled(self, level_fine, level_coarse, kappa, x0, ns_f, dt_f, ns_c, dt_c, width=0.05,
                        precision=LTS_FP64):
        fa = _SampleArgs(kappa, x0, ns_f, dt_f, width)
        ca = _SampleArgs(kappa, x0, ns_c, dt_c, width)
        qf, qfp = fa.out()
        qc, qcp = fa.out()
        dq, dqp = fa.out()
        self._c(self.lib.lts_forward_coupled(self.h, level_fine, level_coarse, C.byref(fa.s),
                                             C.byref(ca.s), precision, qfp, qcp, dqp))
        return qf, qc, dq

    def batch_run(self, jobs, graph=False, precision=LTS_FP64, persist=False, sb_cap=4, auto=False, mlts=False):
        """jobs: list of (level, kappa, x0, n_steps, dt, width).  Returns the Q of all
        jobs concatenated in job order.  precision LTS_FP32_STEP steps in binary32.
        Form: per-step launches (default), their HIP graph (graph=True), one
        persistent launch (persist=True, S_b capped at sb_cap in 1, 2, 4) or the
        fastest of these by measurement (auto=True).  mlts=True: multi-level LTS
        on every job (its level's tiers), with or without the graph."""
        args, cjobs, off = [], [], 0
        for (level, kappa, x0, ns, dt, width) in jobs:
            sa = _SampleArgs(kappa, x0, ns, dt, width)
            args.append(sa)
            cjobs.append(_lib.Job(level=level, samples=sa.s, q_offset=off))
            off += sa.n
        arr = (_lib.Job * len(cjobs))(*cjobs)
        q, qp = args[0].out(off)
        flags = (LTS_BATCH_GRAPH if graph else 0) | (_lib.LTS_BATCH_FP32 if precision == LTS_FP32_STEP else 0)
        if persist:
            if sb_cap not in (1, 2, 4):
                raise ValueError("sb_cap must be 1, 2 or 4")
            flags |= _lib.LTS_BATCH_PERSIST | {1: _lib.LTS_BATCH_SB1, 2: _lib.LTS_BATCH_SB2, 4: 0}[sb_cap]
        if auto:
            flags |= _lib.LTS_BATCH_AUTO
        if mlts:
            flags |= _lib.LTS_BATCH_MLTS
        self._c(self.lib.lts_batch_run(self.h, arr, len(cjobs), flags, qp))
        return q

    def set_barrier_timeout(self, ms):
        """Bound (ms) on a persistent workgroup's wait at a step barrier."""
        self._c(self.lib.lts_set_barrier_timeout(self.h, float(ms)))

    def backward(self, level, kappa, x0, n_steps, dt, dLdQ, width=0.05, K=64, g=None):
        """(Q, dL/dg) with L = sum_s dLdQ[s] Q_s; coefficient as in forward()."""
        sa = _SampleArgs(kappa, x0, n_steps, dt, width, g)
        nb = self.level_info(level)["n_blocks"]
        q, qp = sa.out()
        if sa.dev:
            import torch
            g = torch.empty((sa.n, nb), dtype=torch.float64, device=sa.keep[0].device)
            gp = g.data_ptr()
            dl = dLdQ.contiguous().to(torch.float64)
            dlp = dl.data_ptr()
            _wait_caller_stream(dl)
        else:
            g = np.zeros((sa.n, nb))
            gp = g.ctypes.data
            dl = np.ascontiguousarray(dLdQ, dtype=np.float64)
            dlp = dl.ctypes.data
        self._c(self.lib.lts_backward(self.h, level, C.byref(sa.s), dlp, K, qp, gp))
        return q, g

    def moments(self, x):
        out = np.zeros(3)
        if _is_torch(x):
            xt = x.contiguous().to(dtype=x.new_empty(0).double().dtype)
            _wait_caller_stream(xt)
            self._c(self.lib.lts_moments(self.h, xt.data_ptr(), xt.numel(), LTS_PTR_DEVICE, _dp(out)))
        else:
            xa = np.ascontiguousarray(x, dtype=np.float64)
            self._c(self.lib.lts_moments(self.h, xa.ctypes.data, xa.size, LTS_PTR_HOST, _dp(out)))
        return out

    def mlmc(self, level_ids, rule, eps, seed=0, alpha=2.0, L_start=2, N_init=(256, 64, 16, 8, 4),
             mode=LTS_MLMC_BATCHED, max_total_samples=0, gen_rule=None, n_levels_max=0, grad_K=None,
             meshes=False, mlts=False, gen_mlts=None):
        """Algorithm 1 (lts_mlmc); meshes=True: level_ids are triangle-mesh ids
        (lts_add_mesh); mlts=True: grid levels with tiers attached, solved by
        multi-level LTS (lts_set_mlts); gen_mlts: the tier ratios attached to
        generated levels (halving rule).  With gen_rule and n_levels_max > len(level_ids)
        the hierarchy grows on demand: level l beyond the given ones is built from
        gen_rule with n_base * 2^l when the bias test first asks for it.  With
        grad_K (checkpoint interval) the gradient dE[Q]/dg is estimated alongside
        (lts_mlmc_grad): keys grad, grad_mean [L+1, nb], grad_var [L+1, nb]."""
        o = _lib.MLMCOpts()
        o.n_levels = len(level_ids)
        for k, l in enumerate(level_ids):
            o.level_ids[k] = l
        o.rule = rule
        o.seed = seed
        o.eps = eps
        o.alpha = alpha
        o.L_start = L_start
        for k in range(_lib.LTS_MAX_LEVELS):
            o.N_init[k] = N_init[k] if k < len(N_init) else N_init[-1]
        o.mode = mode
        o.max_total_samples = max_total_samples
        o.n_levels_max = n_levels_max
        if gen_rule is not None:
            o.gen_rule = gen_rule
        o.level_kind = 1 if meshes else 2 if mlts else 0
        if gen_mlts is not None:
            o.gen_mlts, _ = _mlts_desc(gen_mlts, None)
        r = _lib.MLMCResult()
        nb = rule.n_blocks
        if grad_K is not None:
            ge, gm, gv = np.zeros(nb), np.zeros((_lib.LTS_MAX_LEVELS, nb)), np.zeros((_lib.LTS_MAX_LEVELS, nb))
            self._c(self.lib.lts_mlmc_grad(self.h, C.byref(o), grad_K, C.byref(r), _dp(ge), _dp(gm), _dp(gv)))
        else:
            self._c(self.lib.lts_mlmc(self.h, C.byref(o), C.byref(r)))
        L = r.L
        out = {"estimate": r.estimate, "L": L, "N": list(r.N[:L + 1]), "mean": list(r.mean[:L + 1]),
               "var": list(r.var[:L + 1]), "cost": list(r.cost[:L + 1]), "bias": r.bias,
               "rmse": r.rmse, "converged": bool(r.converged), "seconds": r.seconds,
               "level_ids": list(r.level_ids[:L + 1])}
        if grad_K is not None:
            out.update(grad=ge, grad_mean=gm[:L + 1], grad_var=gv[:L + 1])
        return out

    # --- triangle-mesh levels ----------------------------------------------
    def add_mesh(self, m) -> int:
        """A level given as a triangulation (see _MeshArgs); returns its mesh id."""
        a = _MeshArgs(m)
        mid = C.c_int32()
        self._c(self.lib.lts_add_mesh(self.h, C.byref(a.d), C.byref(mid)))
        return mid.value

    def mesh_info(self, mesh) -> dict:
        info = _lib.MeshInfo()
        self._c(self.lib.lts_mesh_info_get(self.h, mesh, C.byref(info)))
        return {k: getattr(info, k) for k, _ in _lib.MeshInfo._fields_}

    def mesh_forward(self, mesh, kappa, x0, n_steps, dt, width=0.05, g=None):
        """Q of every sample on a triangle-mesh level (FP64)."""
        sa = _SampleArgs(kappa, x0, n_steps, dt, width, g)
        q, qp = sa.out()
        self._c(self.lib.lts_mesh_forward(self.h, mesh, C.byref(sa.s), LTS_FP64, qp))
        return q

    def mesh_forward_coupled(self, mesh_fine, mesh_coarse, kappa, x0, ns_f, dt_f, ns_c, dt_c, width=0.05):
        fa = _SampleArgs(kappa, x0, ns_f, dt_f, width)
        ca = _SampleArgs(kappa, x0, ns_c, dt_c, width)
        qf, qfp = fa.out()
        qc, qcp = fa.out()
        dq, dqp = fa.out()
        self._c(self.lib.lts_mesh_forward_coupled(self.h, mesh_fine, mesh_coarse, C.byref(fa.s), C.byref(ca.s),
                                                  LTS_FP64, qfp, qcp, dqp))
        return qf, qc, dq

    # --- multi-level LTS ------------------------------------------------------
    def set_mlts(self, level, ps, cell_tier=None, max_region=0) -> dict:
        """Attach tiers with ratios ps (tier 1 first) to a rectilinear level;
        cell_tier [ny_cells, nx_cells] or None for the halving rule; max_region
        the fine-tile region cap (512, 1024, 2048; 0: 2048).  Returns
        lts_mlts_info as a dict."""
        d, keep = _mlts_desc(ps, cell_tier, max_region)
        self._c(self.lib.lts_set_mlts(self.h, level, C.byref(d)))
        return self.mlts_info(level)

    def mlts_info(self, level) -> dict:
        info = _lib.MltsInfo()
        self._c(self.lib.lts_mlts_info_get(self.h, level, C.byref(info)))
        return _mlts_dict(info)

    def mlts_forward(self, level, kappa, x0, n_steps, dt, width=0.05, g=None, precision=LTS_FP64):
        """Q of every sample with the level's tiers (FP64, or LTS_FP32_STEP)."""
        sa = _SampleArgs(kappa, x0, n_steps, dt, width, g)
        q, qp = sa.out()
        self._c(self.lib.lts_mlts_forward(self.h, level, C.byref(sa.s), precision, qp))
        return q

    # --- one-dimensional workloads -------------------------------------------
    def add_line_level(self, rule) -> int:
        lid = C.c_int32()
        self._c(self.lib.lts_build_line_level(self.h, C.byref(rule), C.byref(lid)))
        return lid.value

    def line_forward(self, line_id, kappa, n_steps, dt, rule, n_nodes):
        """u(T) [n, n_nodes] of every sample (numpy in, numpy out; torch in, torch out)."""
        if _is_torch(kappa):
            import torch
            k = kappa.contiguous().to(torch.float64)
            ns = n_steps.contiguous().to(torch.int32)
            d = dt.contiguous().to(torch.float64)
            _wait_caller_stream(k)
            U = torch.empty((ns.numel(), n_nodes), dtype=torch.float64, device=k.device)
            self._c(self.lib.lts_line_forward(self.h, line_id, ns.numel(), LTS_PTR_DEVICE, k.data_ptr(),
                                              ns.data_ptr(), d.data_ptr(), C.byref(rule), U.data_ptr()))
            return U
        k = np.ascontiguousarray(kappa, dtype=np.float64)
        ns = np.ascontiguousarray(n_steps, dtype=np.int32)
        d = np.ascontiguousarray(dt, dtype=np.float64)
        U = np.zeros((ns.size, n_nodes))
        self._c(self.lib.lts_line_forward(self.h, line_id, ns.size, LTS_PTR_HOST, k.ctypes.data, ns.ctypes.data,
                                          d.ctypes.data, C.byref(rule), U.ctypes.data))
        return U

    def line_mlmc(self, line_ids, rule, eps, seed=0, alpha=2.0, L_start=2, N_init=(64, 32, 16, 8, 4),
                  max_nodes=4096):
        """Algorithm 1 for the L^2(D)-valued QoI u(T) on one-dimensional levels."""
        o = _lib.LineMLMCOpts()
        o.n_levels = len(line_ids)
        for k, l in enumerate(line_ids):
            o.line_ids[k] = l
        o.rule = rule
        o.seed = seed
        o.eps = eps
        o.alpha = alpha
        o.L_start = L_start
        for k in range(_lib.LTS_MAX_LEVELS):
            o.N_init[k] = N_init[k] if k < len(N_init) else N_init[-1]
        r = _lib.LineMLMCResult()
        est = np.zeros(max_nodes)
        self._c(self.lib.lts_line_mlmc(self.h, C.byref(o), C.byref(r), _dp(est)))
        L = r.L
        return {"L": L, "N": list(r.N[:L + 1]), "var": list(r.var[:L + 1]),
                "mean_norm": list(r.mean_norm[:L + 1]), "cost": list(r.cost[:L + 1]), "bias": r.bias,
                "rmse": r.rmse, "converged": bool(r.converged), "seconds": r.seconds,
                "estimate": est[:r.n_nodes].copy()}

    def set_timing(self, on=True):
        self._c(self.lib.lts_set_timing(self.h, 1 if on else 0))

    def timing(self) -> dict:
        t = _lib.Timing()
        self._c(self.lib.lts_get_timing(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _lib.Timing._fields_}


def _make_autograd():
    try:
        import torch
    except ImportError:                      # the C ABI itself does not need torch
        return None

    class LtsQoI(torch.autograd.Function):
        """Q[s] of the LF-LTS solves as a differentiable function of the block
        log-wave-speeds g[s, b] (kappa = c^2 = exp(2 g)).  Forward runs
        lts_forward (the library forms kappa = exp(2 g) on the device); backward
        runs the discrete adjoint lts_backward with the incoming gradient as
        dL/dQ, returning dL/dg at fixed step counts and dt.

        apply(g, ctx, level, x0, n_steps, dt, width=0.05, K=64): g float64 on the
        context's device, x0 [S, 2], n_steps [S] int32, dt [S] on the same device."""

        @staticmethod
        def forward(fctx, g, lctx, level, x0, n_steps, dt, width=0.05, K=64):
            gd = g.detach()
            q = lctx.forward(level, None, x0, n_steps, dt, width, g=gd)
            fctx.save_for_backward(gd, x0, n_steps, dt)
            fctx.lctx, fctx.level, fctx.width, fctx.K = lctx, level, width, K
            return q

        @staticmethod
        def backward(fctx, gq):
            g, x0, n_steps, dt = fctx.saved_tensors
            _, dg = fctx.lctx.backward(fctx.level, None, x0, n_steps, dt, gq.contiguous(), fctx.width, fctx.K,
                                       g=g)
            return dg, None, None, None, None, None, None, None

    return LtsQoI


LtsQoI = _make_autograd()
