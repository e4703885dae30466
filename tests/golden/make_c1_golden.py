"""Write tests/golden/c1_qoi.json: oracle QoIs of a few samples of the
single-level throughput workload (unit square, 512 base cells per axis,
refined 8x in the cells meeting (0.48, 0.52), p = 8, nu = 0.01, 4x4 blocks of
g ~ N(0, 0.25^2), pulse width 0.05 centred in [0.2,0.4]^2, T = 1, QoI over
[0.6,0.8]^2; Philox seed 0, MLMC level 0, samples i = 0..255).

Calls only the oracle.  Each sample takes several minutes on one core.
Usage: python tests/golden/make_c1_golden.py [n_procs]
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

RULE = rng.SampleRule(n_blocks=16, sigma=0.25, pulse_box=(0.2, 0.4, 0.2, 0.4), T=1.0, cfl=0.2)
N_SAMPLES = 256


def _level():
    lv = mesh.box_refined_level(512, box=(0.48, 0.52), ref=8, nu=0.01)
    return lv, fem.operators(lv)


def pick():
    """First, second, longest-running and last sample of the batch."""
    lv = mesh.box_refined_level(512, box=(0.48, 0.52), ref=8)
    ns = [rng.steps_for(rng.draw(0, 0, i, RULE), RULE, lv.h)[0] for i in range(N_SAMPLES)]
    return sorted({0, 1, int(np.argmax(ns)), N_SAMPLES - 1}), ns


def one(i):
    lv, ops = _level()
    smp = rng.draw(0, 0, i, RULE)
    n, dt = rng.steps_for(smp, RULE, lv.h)
    t = time.time()
    u = lts.Solver(ops, smp.kappa).run(lts.pulse(ops, smp.x0, 0.05), dt, n)
    return {"i": i, "Q": float(lts.qoi(ops, u)), "abs_wu": float(ops.qoi_w @ np.abs(u)),
            "n_steps": n, "dt": dt, "seconds": time.time() - t}


if __name__ == "__main__":
    nproc = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    idx, ns = pick()
    with mp.Pool(nproc) as pool:
        res = pool.map(one, idx)
    out = {"workload": "unit square 512 base, refined 8x in (0.48,0.52), p=8, nu=0.01, 4x4 blocks "
                       "sigma 0.25, pulse w 0.05 in [0.2,0.4]^2, T=1, QoI [0.6,0.8]^2, seed 0, level 0",
           "n_samples": N_SAMPLES, "sum_n_steps": int(sum(ns)), "samples": res,
           "generator": "tests/golden/make_c1_golden.py (oracle only)"}
    with open(os.path.join(HERE, "c1_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
