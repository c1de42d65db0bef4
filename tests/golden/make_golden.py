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

"span" adds samples of the level-3, level-4 and adjoint workloads chosen to span theta
(the extreme recharge zeta, the largest and smallest log-permeability and the largest
porosity contrast over the grid, the last index of the batch).  Two level-3 samples also
keep the states after steps 1, 96, 192 and 288: the CPU baseline of the benchmark times
short oracle windows started from them, so that the whole horizon is represented.

"f3" runs the vertex-centred oracle (the paper's own discretisation, section 2.3) on level 1
of Table 2 (64 x 32 elements, 376 steps, T = 6016 s) with the paper's model, seed 5: the
first sample, the smallest and largest recharge zeta of the first 128 samples (7, 63) and of
all 512 (300, 389), and the last indices of both (127, 511).

usage: python tests/golden/make_golden.py {c2|c3|c4|c5|f1|f1l3|f3|span|all} [--procs N]
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


# level-3 steps after which the "span" samples with states keep (p, c)
STATE_STEPS = (1, 96, 192, 288)
# samples of the span set: level 3 (seed 1), level 4 (seed 2), adjoint at level 3 (seed 4)
SPAN_C2 = (68, 313, 342, 502, 478, 511)     # min zeta, max zeta, max / min ln K contrast, max phi contrast, last
SPAN_C2_STATES = (68, 511)
SPAN_C3 = (84, 127)                         # min zeta, last
SPAN_C5 = (108, 255)                        # min zeta, last


def _forward(args):
    name, level, seed, s = args[:4]
    theta_level = args[4] if len(args) > 4 and args[4] is not None else level   # coarse partner: finer level's theta
    keep = len(args) > 5 and args[5]
    pr = H.paper_problem() if name.startswith("f1") else H.Problem()
    g = H.Grid(*level_grid(level))
    th = draw_theta(seed, s + 1, level=theta_level)[s]
    t = time.time()
    r = H.solve_sample(pr, g, th, keep_states=keep)
    out = os.path.join(HERE, f"oracle_{name}_s{s}.npz")
    extra = {}
    if keep:
        extra = dict(state_steps=np.array(STATE_STEPS), state_p=np.stack([r.states[k][0] for k in STATE_STEPS]),
                     state_c=np.stack([r.states[k][1] for k in STATE_STEPS]))
    np.savez_compressed(out, theta=th, c_T=r.c, p_T=r.p, qoi=r.qoi, newton_its=r.newton_its,
                        converged=r.converged, max_salt_defect=r.max_salt_defect,
                        nx=g.nx, ny=g.ny, nsteps=g.nsteps, seconds=time.time() - t, **extra)
    print(out, r.qoi, r.newton_its, f"{time.time() - t:.0f}s", flush=True)


SPAN_F3 = (0, 7, 63, 127, 300, 389, 511)    # first; min, max zeta and last of 128 and of 512


def _forward_vc(args):
    level, seed, s = args
    from oracle import vertex as V
    pr = H.paper_problem()
    g = V.level_grid(level)
    th = draw_theta(seed, s + 1)[s]
    t = time.time()
    r = V.solve_sample(pr, g, th)
    out = os.path.join(HERE, f"oracle_f3_l{level}_s{s}.npz")
    np.savez_compressed(out, theta=th, c_T=r.c, p_T=r.p, qoi=r.qoi, newton_its=r.newton_its, converged=r.converged,
                        max_salt_defect=r.max_salt_defect, max_fluid_defect=r.max_fluid_defect,
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
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c2", "c3", "c4", "c5", "f1", "f1l3", "f3", "span", "all"])
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
    if a.which in ("f3", "all"):
        jobs += [(_forward_vc, (1, 5, s)) for s in SPAN_F3]
    if a.which in ("span", "all"):
        w2, w3, w5 = WORKLOADS["c2_fp64_level3"], WORKLOADS["c3_mixed_level4"], WORKLOADS["c5_adjoint_level3"]
        # longest first: the level-4 solves take hours
        jobs += [(_forward, ("c3", w3["level"], w3["seed"], s)) for s in SPAN_C3]
        jobs += [(_forward, ("c2", w2["level"], w2["seed"], s, None, s in SPAN_C2_STATES)) for s in SPAN_C2]
        jobs += [(_adjoint, ("c5", w5["level"], w5["seed"], s)) for s in SPAN_C5]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(a.procs) as pool:
        rs = [pool.apply_async(f, (x,)) for f, x in jobs]
        for r in rs:
            r.get()


if __name__ == "__main__":
    main()
