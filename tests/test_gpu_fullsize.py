"""Full-size GPU runs in the benchmark's launch configuration, checked on sampled
realisations against stored oracle results (tests/golden/make_golden.py) and, for
every sample, against invariants that hold at any size (mass balance, c in [0, 1])."""
import os

import numpy as np
import pytest
import torch

from henry_inputs import WORKLOADS, draw_theta, level_grid
from tests.oracle_runs import defect_bound

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-8


def _run(name, prec):
    import paper_2403_17018_amd as P
    w = WORKLOADS[name]
    th = draw_theta(w["seed"], w["nsamples"], level=w["level"])
    hx = P.Henry(0)
    g = P.grid(*level_grid(w["level"]))
    r = hx.solve(torch.from_numpy(th).cuda(), g, opts=P.solver_opts(mg_precision=prec), want_c=True, want_p=True)
    torch.cuda.synchronize()
    out = dict(c=r.c_T.cpu().numpy(), p=r.p_T.cpu().numpy(), q=r.qoi.cpu().numpy(), st=r.stats.cpu().numpy(),
               nfailed=r.nfailed, theta=th, nsteps=g.nsteps)
    hx.close()
    return out


def _check(out, name, samples):
    for s in samples:
        f = os.path.join(GOLD, f"oracle_{name}_s{s}.npz")
        z = np.load(f)
        assert np.array_equal(z["theta"], out["theta"][s])
        ny, nx = out["c"].shape[:2]
        c = out["c"][..., s].ravel()
        p = out["p"][..., s].ravel()
        assert np.abs(c - z["c_T"]).max() <= TOL * np.abs(z["c_T"]).max(), s
        assert np.abs(p - z["p_T"]).max() <= TOL * np.abs(z["p_T"]).max(), s
        assert abs(out["q"][s] - float(z["qoi"])) <= TOL * abs(float(z["qoi"])), s
    assert out["nfailed"] == 0
    # global balance of the accepted Newton iterate: storage change + tau * boundary flux = sum of
    # residuals, bounded by the solver tolerances (the exact discrete fixed point balances to ~1e-13)
    bound = defect_bound(out["theta"], 36000.0 / out["nsteps"], 0.5)
    assert (out["st"][:, 2] < bound).all() and (out["st"][:, 3] < bound).all()
    assert out["c"].min() >= -1e-10 and out["c"].max() <= 1 + 1e-10


def test_level3_fp64_full_batch():
    """256x128 cells, 384 steps, all 512 samples of seed 1 in one batch (the benchmark workload)."""
    _check(_run("c2_fp64_level3", 64), "c2", (0, 1))


def test_level3_fp32_multigrid_full_batch():
    """Same workload with the FP32 multigrid preconditioner inside FP64 BiCGStab/Newton."""
    _check(_run("c2_fp64_level3", 32), "c2", (0, 1))


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "oracle_c3_s0.npz")), reason="level-4 oracle result not stored")
def test_level4_fp32_multigrid_full_batch():
    """512x256 cells, 768 steps, 128 samples of seed 2 with the FP32 multigrid preconditioner."""
    _check(_run("c3_mixed_level4", 32), "c3", (0,))
