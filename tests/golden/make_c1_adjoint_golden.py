"""Write tests/golden/c1_adjoint.json: the oracle's discrete-adjoint gradients
dQ/dg (16 block log wave speeds) of four samples of the single-level
throughput workload (unit square, 512 base cells per axis, refined 8x in the
cells meeting (0.48, 0.52), p = 8, nu = 0.01, 4x4 blocks of g ~ N(0, 0.25^2),
pulse width 0.05 centred in [0.2,0.4]^2, T = 1, QoI over [0.6,0.8]^2; Philox
seed 0, MLMC level 0), checkpoints every K = 64 steps, dt and step counts
held fixed.

Calls only the oracle.  Each sample takes about an hour on one core and about
1 GB of memory.  Usage: python tests/golden/make_c1_adjoint_golden.py [n_procs]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import adjoint, fem, lts, mesh, rng  # noqa: E402

RULE = rng.SampleRule(n_blocks=16, sigma=0.25, pulse_box=(0.2, 0.4, 0.2, 0.4), T=1.0, cfl=0.2)
SAMPLES = (0, 1, 2, 3)
K = 64


def one(i):
    lv = mesh.box_refined_level(512, box=(0.48, 0.52), ref=8, nu=0.01)
    ops = fem.operators(lv)
    smp = rng.draw(0, 0, i, RULE)
    n, dt = rng.steps_for(smp, RULE, lv.h)
    t = time.time()
    Q, _, g = adjoint.gradient(ops, smp.kappa, lts.pulse(ops, smp.x0, 0.05), dt, n, K=K)
    return {"i": i, "Q": float(Q), "dQ_dg": [float(v) for v in np.asarray(g)], "n_steps": n, "dt": dt,
            "seconds": time.time() - t}


if __name__ == "__main__":
    nproc = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    with mp.Pool(nproc) as pool:
        res = pool.map(one, SAMPLES, chunksize=1)
    out = {"workload": "unit square 512 base, refined 8x in (0.48,0.52), p=8, nu=0.01, 4x4 blocks sigma 0.25, "
                       "pulse w 0.05 in [0.2,0.4]^2, T=1, QoI [0.6,0.8]^2, seed 0, level 0",
           "K": K, "samples": res, "generator": "tests/golden/make_c1_adjoint_golden.py (oracle only)"}
    with open(os.path.join(HERE, "c1_adjoint.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
