"""Pins of the oracle's triangle-mesh levels (Sec. 3.1: mass-lumped P1
elements on a triangulation; Sec. 3.3: P and F+).

Each pin ties the assembly to something other than itself: the textbook
cotangent form of the P1 stiffness, the exact energy of linear functions,
the area of the domain, brute-force neighbour sets, the rectilinear levels'
operators (pinned elsewhere) for a tensor grid handed over as triangles, and
the conserved discrete energy of LF-LTS."""
import math

import numpy as np
import pytest

import meshgen
from oracle import fem, lts, mesh, rng, trimesh

MESHES = {"criss_cross": lambda: meshgen.criss_cross(), "delaunay": lambda: meshgen.delaunay_disk(),
          "criss_cross_s1": lambda: meshgen.criss_cross(n=12, ref=2, jitter=0.25, seed=1)}


def _level(m, **over):
    d = dict(m)
    d.update(over)
    return trimesh.tri_level(d["xy"], d["tris"], d["dirichlet"], d["tri_block"], d["tri_fine"], d["qoi_nodes"],
                             d["n_blocks"], d["h"], d["p"], d["nu"])


def test_element_weights_are_half_cotangents():
    """For P1 on a triangle, |T| grad(l_a).grad(l_b) = -cot(theta_c) / 2 with
    theta_c the angle at the third vertex: checked on random triangles with
    the angle from atan2 of the edge vectors."""
    g = np.random.default_rng(5)
    for _ in range(50):
        xy = g.uniform(-1, 1, (3, 2))
        t = np.array([[0, 1, 2]])
        x, y = xy[t, 0], xy[t, 1]
        if (x[0, 1] - x[0, 0]) * (y[0, 2] - y[0, 0]) - (x[0, 2] - x[0, 0]) * (y[0, 1] - y[0, 0]) < 0:
            t = np.array([[0, 2, 1]])
        tl = trimesh.tri_level(xy, t, np.zeros(3, bool), [0], [False], np.zeros(3), 1, 1.0, 1, 0.0)
        ed = trimesh.element_data(tl)
        for r, c, geo in zip(ed.rows, ed.cols, ed.geo):
            k = 3 - r - c                                     # the third vertex (DOF ids = node ids here)
            a, b = xy[r] - xy[k], xy[c] - xy[k]
            theta = math.atan2(abs(a[0] * b[1] - a[1] * b[0]), a @ b)
            assert abs(geo + 0.5 / math.tan(theta)) <= 1e-12 * max(1.0, abs(geo))


@pytest.mark.parametrize("name", list(MESHES))
def test_constants_linear_energy_and_mass(name):
    """No Dirichlet nodes: K 1 = 0; u^T K u = sum_T kappa_T |T| |grad u|^2 for a
    linear u (P1 reproduces linear functions exactly); the edge-form K equals
    the element-matrix assembly; the lumped masses sum to the area (1)."""
    m = MESHES[name]()
    tl = _level(m, dirichlet=np.zeros(len(m["xy"]), bool))
    ops = trimesh.operators(tl)
    kb = np.exp(2 * np.random.default_rng(1).normal(0, 0.3, m["n_blocks"]))
    K = fem.stiffness(ops.ed, kb)
    Kf = trimesh.stiffness_full(tl, kb)
    assert abs(K - Kf).max() <= 1e-13 * abs(Kf).max()
    one = np.ones(tl.n_dof)
    assert np.abs(K @ one).max() <= 1e-13 * abs(K).max()
    a, b = 0.7, -1.3
    u = a * tl.xy[:, 0] + b * tl.xy[:, 1]
    x, y = tl.xy[tl.tris, 0], tl.xy[tl.tris, 1]
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    exact = float(np.sum(kb[tl.tri_block] * area) * (a * a + b * b))
    assert abs(u @ (K @ u) - exact) <= 1e-12 * exact
    assert abs(tl.mass.sum() - 1.0) <= 1e-14


@pytest.mark.parametrize("name", list(MESHES))
def test_P_and_Fplus_by_brute_force(name):
    """P = DOF vertices of fine triangles; F+ = P and every DOF sharing an edge
    with a P DOF whose summed cotangent weight is nonzero (computed triangle
    by triangle from angles)."""
    m = MESHES[name]()
    tl = _level(m)
    trimesh.operators(tl)
    dof = ~m["dirichlet"]
    Pb = np.zeros(len(m["xy"]), bool)
    for t, f in zip(m["tris"], m["tri_fine"]):
        if f:
            Pb[t] = True
    Pb &= dof
    assert np.array_equal(Pb, tl.Pmask)
    wsum = {}
    for t in m["tris"]:
        for k in range(3):
            i, j, o = t[(k + 1) % 3], t[(k + 2) % 3], t[k]
            a, b = m["xy"][i] - m["xy"][o], m["xy"][j] - m["xy"][o]
            c = 0.5 / math.tan(math.atan2(abs(a[0] * b[1] - a[1] * b[0]), a @ b))
            e = (min(i, j), max(i, j))
            wsum[e] = wsum.get(e, 0.0) + c
    F = Pb.copy()
    for (i, j), w in wsum.items():
        if abs(w) > 1e-12:
            if Pb[i] and dof[j]:
                F[j] = True
            if Pb[j] and dof[i]:
                F[i] = True
    assert np.array_equal(F, tl.Fplus)


@pytest.mark.parametrize("make", [lambda: mesh.box_refined_level(16), lambda: mesh.graded_L_level(16)])
def test_tensor_grid_as_triangles_is_the_grid_level(make):
    """A rectilinear level handed over as its triangle list gives the
    rectilinear level's masses, P, F+, QoI weights and stiffness, and the
    same LF-LTS solution."""
    lv = make()
    ops = fem.operators(lv)
    tl = trimesh.from_grid_level(lv)
    top = trimesh.operators(tl)
    assert np.array_equal(top.m, ops.m) and np.array_equal(top.Pd, ops.Pd)
    assert np.array_equal(top.qoi_w, ops.qoi_w)
    assert np.array_equal(tl.Fplus, lv.Fplus.ravel())
    kb = np.exp(2 * np.random.default_rng(2).normal(0, 0.3, lv.n_blocks))
    assert abs(fem.stiffness(top.ed, kb) - fem.stiffness(ops.ed, kb)).max() == 0.0
    rule = rng.SampleRule(T=0.3, n_blocks=lv.n_blocks)
    smp = rng.draw(0, 0, 0, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    a = lts.Solver(ops, smp.kappa).run(lts.pulse(ops, smp.x0), dt, n)
    b = lts.Solver(top, smp.kappa).run(lts.pulse(top, smp.x0), dt, n)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["criss_cross", "delaunay"])
def test_lts_energy_conserved_on_unstructured_meshes(name):
    """LF-LTS conserves its discrete energy (M-self-adjoint effective operator)
    on unstructured triangulations too."""
    m = MESHES[name]()
    tl = _level(m)
    ops = trimesh.operators(tl)
    rule = rng.SampleRule(T=0.5)
    smp = rng.draw(0, 0, 3, rule)
    n, dt = rng.steps_for(smp, rule, tl.h)
    s = lts.Solver(ops, smp.kappa)
    _, zs = s.run(lts.pulse(ops, smp.x0), dt, n, keep=True)
    E = np.array([s.energy(zs[k + 1], zs[k], dt) for k in range(0, n, 5)])
    assert np.max(np.abs(E - E[0])) < 1e-12 * E[0]
