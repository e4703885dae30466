"""Write tests/golden/gradedL_qoi.json: oracle QoIs of a few samples on the two
finest levels of the graded L-shape hierarchy at the workload's horizon.

Workload: L-shape [-1,1]^2 minus (0,1]x[-1,0], rectilinear spacing h graded
geometrically toward the reentrant corner (ratio 1/2, 6 layers, smallest cell
h/64, Sec. 3.5), levels with 256 and 512 cells across (h = 1/128, 1/256),
p = 64, nu = 0.01; g = log c on 8x8 blocks i.i.d. N(0, 0.3^2); Gaussian
pulse of width 0.05 centred uniformly in [-0.8,-0.4]x[0.4,0.8]; T = 2;
QoI = lumped integral of u(T) over [0.5,0.9]x[0.2,0.6]; Philox seed 0, the
sample's MLMC level equal to the mesh level.

Calls only the oracle.  A level-4 sample takes about half an hour on one core,
a level-3 sample a few minutes.
Usage: python tests/golden/make_gradedL_golden.py [n_procs]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import fem, lts, mesh, rng  # noqa: E402

RULE = rng.SampleRule(n_blocks=64, sigma=0.3, pulse_box=(-0.8, -0.4, 0.4, 0.8), T=2.0, cfl=0.2)
BASES = {3: 256, 4: 512}
BATCH = 16          # the samples are picked among i = 0..BATCH-1 of each level


def pick(level):
    """Samples 0 and 1, and the longest- and shortest-running of the first BATCH."""
    lv = mesh.graded_L_level(BASES[level])
    ns = [rng.steps_for(rng.draw(0, level, i, RULE), RULE, lv.h)[0] for i in range(BATCH)]
    return sorted({0, 1, int(np.argmax(ns)), int(np.argmin(ns))})


def one(job):
    level, i = job
    lv = mesh.graded_L_level(BASES[level])
    ops = fem.operators(lv)
    smp = rng.draw(0, level, i, RULE)
    n, dt = rng.steps_for(smp, RULE, lv.h)
    t = time.time()
    u = lts.Solver(ops, smp.kappa).run(lts.pulse(ops, smp.x0, 0.05), dt, n)
    return {"level": level, "i": i, "Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)),
            "max_abs_u": float(np.max(np.abs(u))), "n_steps": n, "dt": dt, "seconds": time.time() - t}


if __name__ == "__main__":
    nproc = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    jobs = [(4, i) for i in pick(4)] + [(3, i) for i in pick(3)]
    with mp.Pool(nproc) as pool:
        res = pool.map(one, jobs, chunksize=1)
    out = {"workload": "graded L-shape [-1,1]^2 minus (0,1]x[-1,0], 6 layers ratio 1/2, levels 3 (256 cells) "
                       "and 4 (512 cells), p=64, nu=0.01, 8x8 blocks sigma 0.3, pulse w 0.05 in "
                       "[-0.8,-0.4]x[0.4,0.8], T=2, QoI [0.5,0.9]x[0.2,0.6], seed 0",
           "bases": {str(k): v for k, v in BASES.items()}, "batch": BATCH, "samples": res,
           "generator": "tests/golden/make_gradedL_golden.py (oracle only)"}
    with open(os.path.join(HERE, "gradedL_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
