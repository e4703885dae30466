"""Write tests/golden/mlts_gradedL_qoi.json: oracle QoIs of multi-level LTS
(oracle/mlts.py) for a few samples on the two finest graded L-shape levels at
the workload's horizon.

Workload: the graded L-shape levels with 256 and 512 cells across (as in
make_gradedL_golden.py: 6 layers of ratio 1/2 toward the reentrant corner,
nu = 0.01, 8x8 blocks of g ~ N(0, 0.3^2), pulse of width 0.05 centred in
[-0.8,-0.4]x[0.4,0.8], T = 2, QoI over [0.5,0.9]x[0.2,0.6], Philox seed 0,
sample level = mesh level); five tiers by the halving rule
(mlts.tiers_by_leg) with p_j = 2.  Samples: the first and last of the batch
bench.py --mlts runs (16 on level 4, 64 on level 3).

Calls only the oracle.  A level-4 sample takes about 25 minutes on one core,
a level-3 sample a few minutes.
Usage: python tests/golden/make_mlts_golden.py [n_procs]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import fem, lts, mesh, mlts, rng  # noqa: E402

RULE = rng.SampleRule(n_blocks=64, sigma=0.3, pulse_box=(-0.8, -0.4, 0.4, 0.8), T=2.0, cfl=0.2)
BASES = {3: 256, 4: 512}
PS = [2, 2, 2, 2, 2]
SAMPLES = {4: (0, 15), 3: (0, 63)}


def one(job):
    level, i = job
    lv = mesh.graded_L_level(BASES[level])
    ops = fem.operators(lv)
    Ps = mlts.tier_projectors(lv, mlts.tiers_by_leg(lv, len(PS)), len(PS))
    smp = rng.draw(0, level, i, RULE)
    n, dt = rng.steps_for(smp, RULE, lv.h)
    t = time.time()
    u = mlts.MltsSolver(ops, smp.kappa, Ps, PS).run(lts.pulse(ops, smp.x0, 0.05), dt, n)
    return {"level": level, "i": i, "Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)),
            "max_abs_u": float(np.max(np.abs(u))), "n_steps": n, "dt": dt, "seconds": time.time() - t}


if __name__ == "__main__":
    nproc = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    jobs = [(l, i) for l in (4, 3) for i in SAMPLES[l]]
    with mp.Pool(nproc) as pool:
        res = pool.map(one, jobs, chunksize=1)
    out = {"workload": "graded L-shape [-1,1]^2 minus (0,1]x[-1,0], 6 layers ratio 1/2, levels 3 (256 cells) "
                       "and 4 (512 cells), nu=0.01, 8x8 blocks sigma 0.3, pulse w 0.05 in [-0.8,-0.4]x[0.4,0.8], "
                       "T=2, QoI [0.5,0.9]x[0.2,0.6], seed 0; multi-level LTS, five tiers by halving legs, p_j = 2",
           "tiers": PS, "samples": res}
    with open(os.path.join(HERE, "mlts_gradedL_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)
