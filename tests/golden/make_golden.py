"""Write oracle results at full workload sizes into tests/golden/ (calls only oracle/).

The oracle needs minutes per sample at 256x128 and about an hour at 512x256, so
the GPU parity tests at those sizes compare against these stored results for a
few sampled realisations instead of re-running the oracle.

"f1" is the paper's own stochastic model (section 4) at level 2 (128x64 cells,
192 steps over T = 6016 s), seed 5, samples 0 and 1.

"f1l3" is the paper's model on the benchmark's level-3 input (seed 1, sample 0).

"c4" holds sampled realisations of the full MLMC hierarchy (seed 3): sample 0 of level 2,
sample 0 of level 3, and the coarse partner of level-4 sample 0 (its theta solved on the
level-3 grid).

usage: python tests/golden/make_golden.py {c2|c3|c4|c5|f1|f1l3|all} [--procs N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from henry_inputs import WORKLOADS, draw_theta, level_grid  # noqa: E402
from oracle import adjoint as A  # noqa: E402
from oracle import henry as H  # noqa: E402


def _forward(args):
    name, level, seed, s = args[:4]
    theta_level = args[4] if len(args) > 4 else level   # a coupled coarse partner: the finer level's theta
    pr = H.paper_problem() if name.startswith("f1") else H.Problem()
    g = H.Grid(*level_grid(level))
    th = draw_theta(seed, s + 1, level=theta_level)[s]
    t = time.time()
    r = H.solve_sample(pr, g, th)
    out = os.path.join(HERE, f"oracle_{name}_s{s}.npz")
    np.savez_compressed(out, theta=th, c_T=r.c, p_T=r.p, qoi=r.qoi, newton_its=r.newton_its,
                        converged=r.converged, max_salt_defect=r.max_salt_defect,
                        nx=g.nx, ny=g.ny, nsteps=g.nsteps, seconds=time.time() - t)
    print(out, r.qoi, r.newton_its, f"{time.time() - t:.0f}s", flush=True)


def _adjoint(args):
    name, level, seed, s = args
    pr = H.Problem()
    g = H.Grid(*level_grid(level))
    th = draw_theta(seed, s + 1, level=level)[s]
    t = time.time()
    q, grad = A.adjoint_gradient(pr, g, th)
    out = os.path.join(HERE, f"oracle_{name}_adjoint_s{s}.npz")
    np.savez_compressed(out, theta=th, qoi=q, grad=grad, nx=g.nx, ny=g.ny, nsteps=g.nsteps,
                        seconds=time.time() - t)
    print(out, q, grad, f"{time.time() - t:.0f}s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c2", "c3", "c4", "c5", "f1", "f1l3", "all"])
    ap.add_argument("--procs", type=int, default=3)
    a = ap.parse_args()
    jobs = []
    if a.which in ("c2", "all"):
        w = WORKLOADS["c2_fp64_level3"]
        jobs += [(_forward, ("c2", w["level"], w["seed"], s)) for s in (0, 1)]
    if a.which in ("c5", "all"):
        w = WORKLOADS["c5_adjoint_level3"]
        jobs += [(_adjoint, ("c5", w["level"], w["seed"], 0))]
    if a.which in ("f1", "all"):
        jobs += [(_forward, ("f1", 2, 5, s)) for s in (0, 1)]
    if a.which in ("c4", "all"):
        w = WORKLOADS["c4_mlmc_levels0to4"]
        jobs += [(_forward, ("c4_l2", 2, w["seed"], 0)), (_forward, ("c4_l3", 3, w["seed"], 0)),
                 (_forward, ("c4_l4coarse", 3, w["seed"], 0, 4))]
    if a.which in ("f1l3", "all"):
        w = WORKLOADS["c2_fp64_level3"]
        jobs += [(_forward, ("f1l3", w["level"], w["seed"], 0))]
    if a.which in ("c3", "all"):
        w = WORKLOADS["c3_mixed_level4"]
        jobs += [(_forward, ("c3", w["level"], w["seed"], 0))]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(a.procs) as pool:
        rs = [pool.apply_async(f, (x,)) for f, x in jobs]
        for r in rs:
            r.get()


if __name__ == "__main__":
    main()
