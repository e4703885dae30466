"""Oracle solves run in worker processes by the GPU parity tests (test
infrastructure: calls only the oracle and the seeded input generators).  Each job is a plain tuple so that it
can be sent to a spawned process; results are plain dicts."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from oracle import adjoint, fem, lts, mesh, rng

GRADED_RULE = dict(n_blocks=64, sigma=0.3, pulse_box=(-0.8, -0.4, 0.4, 0.8))


def graded_level(base, lf=False):
    lv = mesh.graded_L_level(base)
    return mesh.lf_twin(lv) if lf else lv


def solve(job):
    """('fwd', base, sample_level, i, T, lf) -> Q, sum w|u|, n_steps of that
    sample on the graded L-shape level with `base` cells across (its leapfrog
    twin when lf)."""
    _, base, slevel, i, T, lf = job
    lv = graded_level(base, lf)
    ops = fem.operators(lv)
    rule = rng.SampleRule(T=T, **GRADED_RULE)
    smp = rng.draw(0, slevel, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    u = lts.Solver(ops, smp.kappa).run(lts.pulse(ops, smp.x0), dt, n)
    return {"Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)), "n_steps": n}


def solve_tiers(job):
    """('fwdq', base, sample_level, i, T, q) -> as solve(), on the graded level
    whose q smallest tiers are fine (mesh.graded_L_tiers)."""
    _, base, slevel, i, T, q = job
    lv = mesh.graded_L_tiers(base, q)
    ops = fem.operators(lv)
    rule = rng.SampleRule(T=T, **GRADED_RULE)
    smp = rng.draw(0, slevel, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    u = lts.Solver(ops, smp.kappa).run(lts.pulse(ops, smp.x0), dt, n)
    return {"Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)), "n_steps": n}


def grad(job):
    """('adj', base, sample_level, i, T, K) -> Q and dQ/dg of that sample by the
    oracle's checkpointed discrete adjoint."""
    _, base, slevel, i, T, K = job
    lv = mesh.graded_L_level(base)
    ops = fem.operators(lv)
    rule = rng.SampleRule(T=T, **GRADED_RULE)
    smp = rng.draw(0, slevel, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    Q, _, g = adjoint.gradient(ops, smp.kappa, lts.pulse(ops, smp.x0), dt, n, K=K)
    return {"Q": float(Q), "g": np.asarray(g).tolist(), "n_steps": n}


def solve_tri(job):
    """('tri', criss_cross kwargs, sample index, T) -> Q, sum w|u|, n_steps of that
    sample (rule: 16 blocks, sigma 0.25, seed 0, MLMC level 0) on the triangle
    mesh tests/meshgen.py builds from the kwargs."""
    import meshgen
    from oracle import trimesh
    _, kw, i, T = job
    m = meshgen.criss_cross(**kw)
    tl = trimesh.tri_level(m["xy"], m["tris"], m["dirichlet"], m["tri_block"], m["tri_fine"], m["qoi_nodes"],
                           m["n_blocks"], m["h"], m["p"], m["nu"])
    ops = trimesh.operators(tl)
    rule = rng.SampleRule(T=T)
    smp = rng.draw(0, 0, i, rule)
    n, dt = rng.steps_for(smp, rule, tl.h)
    u = lts.Solver(ops, smp.kappa).run(lts.pulse(ops, smp.x0), dt, n)
    return {"Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)), "n_steps": n}


def solve_mlts(job):
    """('mlts', base, sample_level, i, T, ps) -> as solve(), with multi-level
    LTS (oracle/mlts.py) on the graded L-shape level, tiers by the halving
    rule with ratios ps."""
    from oracle import mlts
    _, base, slevel, i, T, ps = job
    lv = mesh.graded_L_level(base)
    ops = fem.operators(lv)
    ct = mlts.tiers_by_leg(lv, len(ps))
    rule = rng.SampleRule(T=T, **GRADED_RULE)
    smp = rng.draw(0, slevel, i, rule)
    n, dt = rng.steps_for(smp, rule, lv.h)
    s = mlts.MltsSolver(ops, smp.kappa, mlts.tier_projectors(lv, ct, len(ps)), ps)
    u = s.run(lts.pulse(ops, smp.x0), dt, n)
    return {"Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)), "n_steps": n}


def _run(job):
    return {"fwd": solve, "fwdq": solve_tiers, "adj": grad, "tri": solve_tri, "mlts": solve_mlts}[job[0]](job)


def run_all(jobs):
    """All jobs in parallel worker processes (spawned: they touch no GPU state)."""
    procs = max(1, min(len(jobs), 16, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.map(_run, jobs, chunksize=1)
